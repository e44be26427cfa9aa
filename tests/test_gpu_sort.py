"""GPU parity: the HIP sample sort against the CPU oracle, bit for bit.

Sorting has one correct answer (the stable order), so keys and payloads
must equal the oracle's exactly; the top-level stages (sorted sample,
splitters, bucket counts) must equal the oracle's step-by-step run of the
same rules."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_08648_amd import api
from paper_1608_08648_amd import native as N
from paper_1608_08648_amd import workloads
from tests.gpu_util import note, to_dev, to_host

pytestmark = pytest.mark.gpu

KEY_DTYPES = [np.uint32, np.int32, np.float32, np.uint64, np.int64, np.float64]
C_KEYS4 = 512 * 64          # one work-group holds this many 4-byte keys


def rand_keys(n, dtype, seed, dup=True):
    g = np.random.default_rng(seed)
    dt = np.dtype(dtype)
    if dt.kind == "f":
        v = g.standard_normal(n) * 1e3
        if dup:
            v = np.round(v)
        return v.astype(dt)
    info = np.iinfo(dt)
    if dup:
        v = g.integers(-50 if info.min < 0 else 0, 50, n)
        big = g.integers(info.min, info.max, n, dtype=dt, endpoint=True)
        return np.where(g.random(n) < 0.5, v.astype(dt), big).astype(dt)
    return g.integers(info.min, info.max, n, dtype=dt, endpoint=True)


def gpu_sort(keys, prm):
    kd, kt = to_dev(keys)
    out = api.sort_keys(kd, prm, key_type=kt)
    return to_host(out, keys.dtype)


def check_keys(keys, prm):
    got = gpu_sort(keys, prm)
    want = keys[oracle.stable_perm(keys)]
    np.testing.assert_array_equal(got.view(np.uint8), want.view(np.uint8))


@pytest.mark.parametrize("dtype", KEY_DTYPES)
def test_one_workgroup_sizes(dtype):
    prm = api.params(p=64, s=4)
    for n in [1, 2, 3, 63, 64, 65, 511, 512, 513, 4097, 16384, 16385, 20000]:
        note(f"direct {np.dtype(dtype)} n={n}")
        check_keys(rand_keys(n, dtype, n), prm)


@pytest.mark.parametrize("dtype", [np.int32, np.uint64, np.float64])
@pytest.mark.parametrize("vt", ["b32", "b64", "iota32", "iota64"])
def test_pairs_payload_follows_key(dtype, vt):
    for n, force in [(1000, False), (9999, False), (60000, True)]:
        note(f"pairs {np.dtype(dtype)} {vt} n={n}")
        keys = rand_keys(n, dtype, 3 * n)
        kd, kt = to_dev(keys)
        prm = api.params(p=64, s=4, flags=N.SS_F_FORCE_PIPELINE if force else 0)
        perm = oracle.stable_perm(keys)
        if vt.startswith("iota"):
            ko, vo = api.sort_pairs(kd, iota="int32" if vt == "iota32" else "int64", prm=prm, key_type=kt)
            want_v = perm
        else:
            vdt = np.uint32 if vt == "b32" else np.uint64
            vals = np.random.default_rng(n).integers(0, 2**31, n).astype(vdt)
            vd, _ = to_dev(vals)
            ko, vo = api.sort_pairs(kd, vd, prm=prm, key_type=kt)
            want_v = vals[perm]
        np.testing.assert_array_equal(to_host(ko, keys.dtype).view(np.uint8), keys[perm].view(np.uint8))
        np.testing.assert_array_equal(vo.cpu().numpy().astype(np.int64), want_v.astype(np.int64))


def _stage_check(keys, p, s, mode, seed, flags=0):
    prm = api.params(p=p, s=s, sampling="random" if mode == 0 else "regular", seed=seed,
                     flags=flags | N.SS_F_FORCE_PIPELINE)
    kd, kt = to_dev(keys)
    note(f"stages n={keys.size} p={p} s={s} mode={mode} seed={seed}")
    out, st, info = api.stages(kd, prm, key_type=kt)
    assert not info.direct
    ref = oracle.stages(keys, info.p_eff, s, mode, seed)
    np.testing.assert_array_equal(st["sample_ord"], ref["sample_ord"])
    np.testing.assert_array_equal(st["sample_tag"], ref["sample_tag"])
    np.testing.assert_array_equal(st["spl_ord"], ref["spl_ord"])
    np.testing.assert_array_equal(st["spl_tag"], ref["spl_tag"])
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    np.testing.assert_array_equal(to_host(out, keys.dtype).view(np.uint8), keys[ref["perm"]].view(np.uint8))
    return st, info


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.float32, np.uint64])
def test_stages_random(dtype):
    for n, p, s in [(50_000, 64, 4), (300_001, 256, 8), (1_000_003, 1024, 2)]:
        keys = rand_keys(n, dtype, n + p)
        _stage_check(keys, p, s, 0, seed=n * 7 + s)


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_stages_every_distribution(dist):
    keys = workloads.keys_2p26(400_000, dist, 99)
    _stage_check(keys, 256, 4, 0, seed=5)
    _stage_check(keys, 64, 4, 1, seed=0)


def test_stages_regular_lemma1():
    """Regular sampling: stages equal the oracle's and every bucket obeys
    Lemma 1's bound, for inputs that defeat naive splitting."""
    for dist in ["uniform", "all_equal", "sorted", "reverse", "distinct64"]:
        keys = workloads.keys_2p26(2**20, dist, 11, np.uint32)
        st, info = _stage_check(keys, 64, 8, 1, seed=0)
        safe, tight, final = oracle.lemma1_bounds(keys.size, info.p_eff, 8)
        assert st["counts"].max() <= tight


def test_big_sample_uses_multi_workgroup_merge():
    """p*s beyond one work-group: chunk sorts, then ranks across chunks (the
    4-byte sample of 131,071 records by chunk pairs, the 8-byte one of 16,383
    records by lane groups)."""
    keys = rand_keys(2**22, np.int32, 17)
    st, info = _stage_check(keys, 4096, 32, 0, seed=3)
    assert info.m == 4096 * 32 - 1
    keys = rand_keys(2**20, np.uint64, 18)
    _stage_check(keys, 2048, 8, 0, seed=4)


def test_big_sample_lane_ranks_and_nested_sort():
    """4-byte samples past the chunk-pair ranks: 262,143 records (128 chunks
    of 2K, ranked by lane groups on the packed records) and 2^21 - 1 records
    (sorted as 64-bit keys by a nested sort).  Sample, splitters and counts
    equal the oracle's stages."""
    keys = rand_keys(2**22, np.int32, 21)
    st, info = _stage_check(keys, 1024, 256, 0, seed=5)
    assert info.m == 1024 * 256 - 1
    keys = rand_keys(2**23, np.uint32, 22)
    st, info = _stage_check(keys, 2048, 1024, 0, seed=6)
    assert info.m == 2048 * 1024 - 1


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_distributions_2p22(dist):
    keys = workloads.keys_2p26(2**22, dist, workloads.seed_for(1, 3))
    want = keys[oracle.stable_perm(keys)]
    for p, s, mode in [(1024, 8, "random"), (4096, 16, "random"), (256, 4, "regular"), (64, 32, "random")]:
        note(f"dist {dist} p={p} s={s} {mode}")
        got = gpu_sort(keys, api.params(p=p, s=s, sampling=mode, seed=p + s))
        np.testing.assert_array_equal(got, want)


def test_recursion_and_fallback():
    keys = rand_keys(2**22, np.int32, 5)
    want = keys[oracle.stable_perm(keys)]
    note("recursion p=16")
    np.testing.assert_array_equal(gpu_sort(keys, api.params(p=16, s=8)), want)
    note("recursion p=2")
    np.testing.assert_array_equal(gpu_sort(keys, api.params(p=2, s=4)), want)
    small = keys[: 2**19]
    want_s = small[oracle.stable_perm(small)]
    note("no recursion: one-work-group fallback for large buckets")
    np.testing.assert_array_equal(gpu_sort(small, api.params(p=4, s=4, flags=N.SS_F_NO_RECURSION)), want_s)


def test_pairs_u64_duplicates_stable():
    keys, vals = workloads.pairs_dup(2**22, 21)
    perm = oracle.stable_perm(keys)
    kd, _ = to_dev(keys)
    vd, _ = to_dev(vals)
    for p, s in [(4096, 16), (1024, 8)]:
        note(f"pairs u64 p={p} s={s}")
        ko, vo = api.sort_pairs(kd, vd, prm=api.params(p=p, s=s), key_type="u64")
        np.testing.assert_array_equal(to_host(ko, np.uint64), keys[perm])
        np.testing.assert_array_equal(to_host(vo, np.uint32), vals[perm])


def test_in_place():
    keys = rand_keys(2**21, np.int32, 8)
    want = keys[oracle.stable_perm(keys)]
    kd, _ = to_dev(keys)
    api.sort_keys(kd, api.params(p=1024, s=8), out=kd)
    np.testing.assert_array_equal(kd.cpu().numpy(), want)


def test_float_total_order_specials():
    g = np.random.default_rng(4)
    specials = np.array([0xFFC00000, 0xFF800000, 0xBF800000, 0x80000000, 0x00000000, 0x3F800000,
                         0x7F800000, 0x7FC00000, 0x00000001, 0x80000001], dtype=np.uint32)
    for n in [1000, 200_000]:
        bits = specials[g.integers(0, len(specials), n)]
        keys = bits.view(np.float32)
        for force in [0, N.SS_F_FORCE_PIPELINE]:
            got = gpu_sort(keys, api.params(p=64, s=4, flags=force))
            np.testing.assert_array_equal(got.view(np.uint32), keys[oracle.stable_perm(keys)].view(np.uint32))


def test_exhaustive_weak_orderings_as_segments():
    """All weak orderings of n <= 8 items (545,835 patterns at n = 8), each
    a segment of one segmented sort; the payload (in-segment index) must be
    the oracle's stable permutation."""
    for n in range(1, 9):
        pats = workloads.weak_orderings(n).astype(np.int32)
        flat = np.ascontiguousarray(pats.reshape(-1))
        off = np.arange(0, flat.size + 1, n, dtype=np.int64)
        note(f"weak orderings n={n}: {len(pats)} segments")
        kd = torch.from_numpy(flat).cuda()
        od = torch.from_numpy(off).cuda()
        ko, vo = api.segmented_sort(kd, od, iota="int32", max_len=n, total=flat.size)
        want = oracle.segmented_perm(flat, off)
        np.testing.assert_array_equal(vo.cpu().numpy(), want)
        np.testing.assert_array_equal(ko.cpu().numpy(), flat[np.repeat(off[:-1], n) + want])


def test_segmented_log_uniform():
    keys, off = workloads.segmented_keys(1500, 31, max_log2=18)
    kd = torch.from_numpy(keys).cuda()
    od = torch.from_numpy(off).cuda()
    want_k, _, want_p = oracle.segmented_sort(keys, off)
    for prm in [None, api.params(p=64, s=8, seed=9)]:
        note(f"segmented 1500 segments prm={prm is not None}")
        ko, vo = api.segmented_sort(kd, od, iota="int32", prm=prm)
        np.testing.assert_array_equal(ko.cpu().numpy(), want_k)
        np.testing.assert_array_equal(vo.cpu().numpy(), want_p)


def test_segmented_empty_and_offset_start():
    g = np.random.default_rng(2)
    sizes = np.array([0, 5, 0, 0, 40000, 1, 0, 70000, 3], dtype=np.int64)
    off = np.concatenate([[7], 7 + np.cumsum(sizes)]).astype(np.int64)
    total = int(off[-1])
    keys = g.integers(-1000, 1000, total).astype(np.int32)
    kd = torch.from_numpy(keys).cuda()
    od = torch.from_numpy(off).cuda()
    ko = api.segmented_sort(kd, od)
    got = ko.cpu().numpy()
    for i in range(len(sizes)):
        seg = keys[off[i]:off[i + 1]]
        np.testing.assert_array_equal(got[off[i]:off[i + 1]], seg[oracle.stable_perm(seg)])


def test_status_clean_after_sort():
    keys = rand_keys(2**20, np.int32, 1)
    kd, _ = to_dev(keys)
    prm = api.params(p=1024, s=8)
    w = api._workspace(api.workspace_size(kd.numel(), N.SS_I32, N.SS_V_NONE, prm), kd.device)
    api.sort_keys(kd, prm, ws=w)
    msg = api.status(w)
    assert msg == "", msg


@pytest.mark.parametrize("dtype,vt,p,flags", [
    (np.int32, None, 512, 0),                      # one-pass split, 512-bucket kernels
    (np.int32, None, 1024, N.SS_F_NO_WIDE),        # 1024-bucket kernels
    (np.uint64, None, 512, 0),
    (np.uint64, None, 1024, 0),
    (np.int32, "b64", 512, 0),                     # stable split with payload, 512 buckets
    (np.uint64, "b32", 1024, 0),                   # 1024 buckets
    (np.float32, "b32", 2048, 0),                  # 4096-bucket kernels
])
def test_split_bucket_bounds(dtype, vt, p, flags):
    """The split kernels are built for at most 256, 512, 1024 or 4096
    buckets; each level takes the smallest bound >= its p.  2^21 + 99 keys
    with duplicates: bucket counts equal the oracle's, keys (and payloads,
    stable) bit-exact."""
    n = (1 << 21) + 99
    keys = rand_keys(n, dtype, 1000 + p)
    kd, kt = to_dev(keys)
    note(f"split bound {np.dtype(dtype)} vt={vt} p={p} flags={flags}")
    if vt is None:
        _stage_check(keys, p, 8, 0, 77, flags)
        return
    vdt = np.uint32 if vt == "b32" else np.uint64
    vals = np.random.default_rng(p).integers(0, 2**31, n).astype(vdt)
    vd, _ = to_dev(vals)
    perm = oracle.stable_perm(keys)
    ko, vo = api.sort_pairs(kd, vd, prm=api.params(p=p, s=8, seed=77, flags=flags), key_type=kt)
    np.testing.assert_array_equal(to_host(ko, keys.dtype).view(np.uint8), keys[perm].view(np.uint8))
    np.testing.assert_array_equal(to_host(vo, vdt), vals[perm])


def test_int64_index_sorted_narrow_and_widened():
    """A 64-bit index payload (IOTA64) is sorted as a 32-bit one and widened
    at the end.  Single array: the index equals the oracle's stable
    permutation.  Segments starting at offset 7 (empty ones included): the
    in-segment indices equal the oracle's, and the caller's output outside
    [offsets[0], offsets[-1]) keeps its contents."""
    n = (1 << 20) + 5
    keys = rand_keys(n, np.int32, 91)
    kd = torch.from_numpy(keys).cuda()
    note("iota64 single")
    ko, vo = api.sort_pairs(kd, iota="int64", prm=api.params(p=256, s=8))
    assert vo.dtype == torch.int64
    perm = oracle.stable_perm(keys)
    np.testing.assert_array_equal(vo.cpu().numpy(), perm.astype(np.int64))
    np.testing.assert_array_equal(ko.cpu().numpy(), keys[perm])
    sizes = np.array([0, 9, 0, 40000, 1, 0, 300000, 3, 0], dtype=np.int64)
    off = np.concatenate([[7], 7 + np.cumsum(sizes)]).astype(np.int64)
    total = int(off[-1]) + 11
    keys = rand_keys(total, np.float32, 92)
    kd = torch.from_numpy(keys).cuda()
    od = torch.from_numpy(off).cuda()
    vals_out = torch.full((total,), -7, dtype=torch.int64, device="cuda")
    note("iota64 segmented")
    ko, vo = api.segmented_sort(kd, od, iota="int64", vals_out=vals_out, total=total,
                                max_len=int(sizes.max()))
    got = vo.cpu().numpy()
    assert np.all(got[:7] == -7) and np.all(got[int(off[-1]):] == -7)
    want = oracle.segmented_perm(keys[:int(off[-1])], off).astype(np.int64)
    np.testing.assert_array_equal(got[7:int(off[-1])], want[7:])
