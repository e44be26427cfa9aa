"""GPU: the batched segmented form under HIP-graph capture, the
differentiable row sort, and full-size parity at the benchmarked shapes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_08648_amd import api
from paper_1608_08648_amd import native as N
from paper_1608_08648_amd import workloads
from tests.gpu_util import note, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_sortfn_forward_matches_oracle():
    x = workloads.tie_free_rows(16, 5000, seed=41)
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    vals, perm = api.sort(xd)
    want = np.stack([oracle.stable_perm(r) for r in x])
    np.testing.assert_array_equal(perm.cpu().numpy(), want)
    np.testing.assert_array_equal(vals.detach().cpu().numpy(), np.take_along_axis(x, want, 1))


def test_sortfn_backward_is_index_put_of_oracle_perm():
    """grad_x[r, perm[r, j]] = grad_y[r, j], bit for bit, with perm the
    oracle's stable permutation."""
    x = workloads.tie_free_rows(8, 3000, seed=42)
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    vals, _ = api.sort(xd)
    gy = torch.randn(vals.shape, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    vals.backward(gy)
    perm = np.stack([oracle.stable_perm(r) for r in x])
    want = oracle.scatter_grad(gy.cpu().numpy(), perm)
    np.testing.assert_array_equal(xd.grad.cpu().numpy(), want)
    # and the same through the reference's index_put formulation on the CPU
    ref = torch.zeros(x.shape, dtype=torch.float32).index_put_(
        (torch.arange(8)[:, None].expand(8, 3000), torch.from_numpy(perm)), gy.cpu())
    np.testing.assert_array_equal(xd.grad.cpu().numpy(), ref.numpy())


def test_sortfn_finite_differences_fp64():
    """Central differences on an 8 x 64 tie-free float64 slice: with a step
    far below the smallest gap the order does not change, so the loss is
    linear and the difference quotient equals the analytic gradient."""
    x = workloads.tie_free_rows(8, 64, seed=43).astype(np.float64)
    xd = torch.from_numpy(x).cuda()

    def f(t):
        return api.sort(t)[0]

    assert torch.autograd.gradcheck(f, (xd.clone().requires_grad_(True),), eps=1e-7, atol=1e-6, rtol=1e-6)
    w = torch.from_numpy(np.random.default_rng(4).standard_normal((8, 64))).cuda()
    xg = xd.clone().requires_grad_(True)
    (f(xg) * w).sum().backward()
    h = 1e-6
    fd = np.zeros_like(x)
    for r in range(8):
        for i in range(64):
            e = torch.zeros_like(xd)
            e[r, i] = h
            fd[r, i] = ((f(xd + e) * w).sum() - (f(xd - e) * w).sum()).item() / (2 * h)
    np.testing.assert_allclose(xg.grad.cpu().numpy(), fd, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("nbytes", [2, 4, 8])
def test_scatter_grad_element_sizes(nbytes):
    dt = {2: torch.float16, 4: torch.float32, 8: torch.float64}[nbytes]
    g = torch.Generator().manual_seed(nbytes)
    gy = torch.randn(5, 777, generator=g).to(dt)
    perm = torch.stack([torch.randperm(777, generator=g) for _ in range(5)])
    got = api.scatter_grad(gy.cuda(), perm.cuda()).cpu()
    want = oracle.scatter_grad(gy.numpy(), perm.numpy())
    np.testing.assert_array_equal(got.numpy(), want)


def test_segmented_graph_capture_replays():
    """One segmented sort captured in a HIP graph and replayed three times,
    with eager work (a new input written into the captured buffer) between
    replays; every replay must equal the oracle for the current input."""
    sizes = workloads.segment_sizes(600, seed=51, max_log2=17)
    off = workloads.offsets_from_sizes(sizes)
    total, max_len = int(off[-1]), int(sizes.max())
    kd = torch.empty(total, dtype=torch.int32, device="cuda")
    od = torch.from_numpy(off).cuda()
    ko = torch.empty_like(kd)
    vo = torch.empty(total, dtype=torch.int32, device="cuda")
    prm = api.params(p=64, s=8, seed=77)
    wsz = api.segmented_workspace_size(total, len(sizes), max_len, N.SS_I32, N.SS_V_IOTA32, prm)
    ws = api._workspace(wsz, kd.device)
    g = np.random.default_rng(5)
    kd.copy_(torch.from_numpy(g.integers(-2**31, 2**31, total, dtype=np.int64).astype(np.int32)))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):       # warm-up outside capture
        api.segmented_sort(kd, od, iota="int32", prm=prm, max_len=max_len, total=total, keys_out=ko,
                           vals_out=vo, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        api.segmented_sort(kd, od, iota="int32", prm=prm, max_len=max_len, total=total, keys_out=ko,
                           vals_out=vo, ws=ws)
    for rep in range(3):
        keys = g.integers(-2**31, 2**31, total, dtype=np.int64).astype(np.int32)
        if rep == 2:
            keys = (keys % 7).astype(np.int32)                      # many duplicates
        kd.copy_(torch.from_numpy(keys))
        torch.cuda.synchronize()
        note(f"graph replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        want_k, _, want_p = oracle.segmented_sort(keys, off)
        np.testing.assert_array_equal(ko.cpu().numpy(), want_k)
        np.testing.assert_array_equal(vo.cpu().numpy(), want_p)
        ko.fill_(0)                                                 # eager work between replays


def test_full_size_2p26_int32_bench_config():
    """The benchmarked configurations at full size, bit-exact: the one-pass
    split (p = 128), the wide split (p = 4096), and the wide split whose
    buckets of ~2^16 keys go one level down (p = 1024, s = 4), also in
    place."""
    keys = workloads.keys_2p26(2**26, "uniform", workloads.seed_for(1, 0), np.int32)
    want = keys[oracle.stable_perm(keys)]
    kd = torch.from_numpy(keys).cuda()
    for p, s in [(128, 16), (4096, 16), (1024, 4)]:
        note(f"2^26 int32 p={p} s={s}")
        prm = api.params(p=p, s=s, seed=1234)
        ws = api._workspace(api.workspace_size(2**26, N.SS_I32, N.SS_V_NONE, prm), kd.device)
        out = api.sort_keys(kd, prm, ws=ws)
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        if p == 1024:
            levels = api.level_stats(ws)
            assert len(levels) == 2 and levels[1]["keys"] > 0
            note("2^26 int32 p=1024 s=4 in place")
            kin = kd.clone()
            api.sort_keys(kin, prm, out=kin, ws=ws)
            np.testing.assert_array_equal(kin.cpu().numpy(), want)


def test_full_size_2p27_pairs_stable():
    """2^27 (uint64 key, uint32 payload = index) pairs, ~30% duplicates:
    keys and payloads bit-exact, i.e. stable."""
    keys, vals = workloads.pairs_dup(2**27, workloads.seed_for(2))
    perm = oracle.stable_perm(keys)
    kd, _ = to_dev(keys)
    vd, _ = to_dev(vals)
    note("2^27 pairs")
    ko, vo = api.sort_pairs(kd, vd, prm=api.params(p=1024, s=16, seed=9), key_type="u64")
    np.testing.assert_array_equal(to_host(ko, np.uint64), keys[perm])
    np.testing.assert_array_equal(to_host(vo, np.uint32), vals[perm])


def test_regular_2p20_config():
    """2^20 uint32 keys, regular oversampling p=64 s=8: stages against the
    oracle and Lemma 1's bound."""
    keys = workloads.uniform_u32(2**20, workloads.seed_for(0))
    kd, kt = to_dev(keys)
    prm = api.params(p=64, s=8, sampling="regular")
    out, st, info = api.stages(kd, prm, key_type=kt)
    assert info.p_eff == 64 and info.m == 8 * 64 * 64
    ref = oracle.stages(keys, 64, 8, oracle.REGULAR, 0)
    np.testing.assert_array_equal(st["spl_ord"], ref["spl_ord"])
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    np.testing.assert_array_equal(to_host(out, np.uint32), keys[ref["perm"]])
    assert st["counts"].max() <= oracle.lemma1_bounds(2**20, 64, 8)[1]


def test_sortfn_full_shape_64x2p18():
    """The row sort at its benchmarked shape (64 x 2^18 float32, tie-free):
    every row's permutation and values equal the oracle's, and the backward
    equals the oracle's gradient scatter, bit for bit."""
    rows, cols = 64, 1 << 18
    x = workloads.tie_free_rows(rows, cols, workloads.seed_for(4))
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    note("SortFn 64 x 2^18 forward")
    vals, perm = api.sort(xd)
    torch.cuda.synchronize()
    want = np.stack([oracle.stable_perm(r) for r in x])
    np.testing.assert_array_equal(perm.cpu().numpy(), want)
    np.testing.assert_array_equal(vals.detach().cpu().numpy(), np.take_along_axis(x, want, 1))
    gy = torch.randn(rows, cols, device="cuda", generator=torch.Generator("cuda").manual_seed(11))
    note("SortFn 64 x 2^18 backward")
    vals.backward(gy)
    np.testing.assert_array_equal(xd.grad.cpu().numpy(), oracle.scatter_grad(gy.cpu().numpy(), want))


def test_segmented_log_uniform_2000_graph_tuned():
    """The batched form at the benchmarked shape, reduced in count: 2,000
    segments of log-uniform length in [1, 2^20] (~1.5e8 int32 keys), the
    library's tuned parameters (prm = NULL), captured in a HIP graph and
    replayed twice; every segment equals the oracle's sort of it."""
    sizes = workloads.segment_sizes(2000, workloads.seed_for(3, 1))
    off = workloads.offsets_from_sizes(sizes)
    total, max_len = int(off[-1]), int(sizes.max())
    g = np.random.default_rng(6)
    keys = g.integers(-2**31, 2**31, total, dtype=np.int64).astype(np.int32)
    kd = torch.from_numpy(keys).cuda()
    od = torch.from_numpy(off).cuda()
    ko = torch.empty_like(kd)
    ws = api._workspace(api.segmented_workspace_size(total, len(sizes), max_len, N.SS_I32, N.SS_V_NONE, None),
                        kd.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        api.segmented_sort(kd, od, max_len=max_len, total=total, keys_out=ko, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        api.segmented_sort(kd, od, max_len=max_len, total=total, keys_out=ko, ws=ws)
    want, _, _ = oracle.segmented_sort(keys, off)
    for rep in range(2):
        ko.fill_(0)
        torch.cuda.synchronize()
        note(f"2000 log-uniform segments, graph replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ko.cpu().numpy(), want)
    assert api.status(ws) == ""


def test_segment_offsets_outside_the_plan_are_flagged():
    """A segment that leaves [0, total) or is longer than max_seg_len is
    skipped by the device and reported by ss_status; the other segments are
    still sorted."""
    keys = np.arange(300, 0, -1).astype(np.int32)
    kd = torch.from_numpy(keys).cuda()
    ko = torch.zeros_like(kd)
    # segment 1 ends past total = 200; segment 0 is fine
    od = torch.tensor([0, 100, 250], dtype=torch.int64, device="cuda")
    ws = api._workspace(api.segmented_workspace_size(200, 2, 100, N.SS_I32, N.SS_V_NONE, None), kd.device)
    note("segment past total")
    api.segmented_sort(kd, od, total=200, max_len=100, keys_out=ko, ws=ws)
    with pytest.raises(N.SortError, match="segment offsets"):
        api.status(ws)
    np.testing.assert_array_equal(ko[:100].cpu().numpy(), np.sort(keys[:100]))
    # segment 1 is longer than max_seg_len = 60
    od2 = torch.tensor([0, 50, 200], dtype=torch.int64, device="cuda")
    ws2 = api._workspace(api.segmented_workspace_size(200, 2, 60, N.SS_I32, N.SS_V_NONE, None), kd.device)
    note("segment longer than max_seg_len")
    api.segmented_sort(kd, od2, total=200, max_len=60, keys_out=ko, ws=ws2)
    with pytest.raises(N.SortError, match="segment offsets"):
        api.status(ws2)
    np.testing.assert_array_equal(ko[:50].cpu().numpy(), np.sort(keys[:50]))


@pytest.mark.parametrize("nbytes", [2, 4, 8])
def test_scatter_grad_vector_path(nbytes):
    """Rows whose length is a multiple of the vector width take the vector
    loads; several rows per XCD range and a tail of partial chunks."""
    dt = {2: torch.float16, 4: torch.float32, 8: torch.float64}[nbytes]
    g = torch.Generator().manual_seed(10 + nbytes)
    rows, cols = 19, 3076
    gy = torch.randn(rows, cols, generator=g).to(dt)
    perm = torch.stack([torch.randperm(cols, generator=g) for _ in range(rows)])
    got = api.scatter_grad(gy.cuda(), perm.cuda()).cpu()
    np.testing.assert_array_equal(got.numpy(), oracle.scatter_grad(gy.numpy(), perm.numpy()))
    api.grad_status()


def test_scatter_grad_flags_an_index_outside_the_row():
    cols = 1024
    gy = torch.arange(2 * cols, dtype=torch.float32).view(2, cols)
    perm = torch.stack([torch.randperm(cols), torch.randperm(cols)])
    bad = perm.clone()
    j = int((bad[1] == 5).nonzero()[0, 0])
    bad[1, j] = cols                      # outside the row: not written, flagged
    api.grad_status()                     # (clears any earlier flag)
    gx = torch.full((2, cols), -1.0, device="cuda")
    api.scatter_grad(gy.cuda(), bad.cuda(), grad_x=gx)
    with pytest.raises(N.SortError, match="outside its row"):
        api.grad_status()
    api.grad_status()                     # cleared
    want = oracle.scatter_grad(gy.numpy(), perm.numpy())
    want[1, 5] = -1.0
    np.testing.assert_array_equal(gx.cpu().numpy(), want)
