"""Benchmarks of the other sort forms (driven by bench.py --workload ...).

* pairs:     2^27 (uint64 key, uint32 payload) pairs, keys ~30% duplicates
* segmented: 20,000 segments of log-uniform length in [1, 2^20] (int32),
             one HIP-graph-captured segmented_sort vs one sample_sort_keys
             call per segment
* autograd:  64 x 2^18 float32 rows, SortFn forward + backward vs one call
             per row

Each returns (result dict, ok) for one JSON line; inputs are seeded and
synthetic and are resident on the GPU before timing.
"""
import ctypes
import time

import numpy as np
import torch

from . import api
from . import native as N
from . import workloads

HBM_PEAK_GBS = 8000.0


def _timed(fn, steps, warmup, stream=None):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = stream or torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _kernel_table(fn, steps):
    """Per-kernel HIP-event times of `steps` extra calls (every launch
    bracketed; outside any timed region)."""
    N.profile_enable(True, max_launches=256 * (steps + 1))
    for _ in range(steps):
        fn()
    N.profile_collect()
    rep = N.profile_report()
    N.profile_enable(False)
    return {k: {"ms_per_step": round(ms / steps, 5), "launches_per_step": round(c / steps, 3)}
            for k, (ms, c) in rep.items() if c}


def _base(metric, value, unit, args, ms, dtype, config, **extra):
    d = {"metric": metric, "value": round(value, 4), "unit": unit, "n_gpus": 1, "steps": args.steps,
         "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
         "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    d.update(extra)
    return d


def bench_pairs(args):
    n = 1 << 27
    seed = workloads.seed_for(2)
    keys, vals = workloads.pairs_dup(n, seed)
    kd = torch.from_numpy(keys.view(np.int64)).cuda()
    vd = torch.from_numpy(vals.view(np.int32)).cuda()
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    # (the stable ballot split takes p <= 256; a larger p uses the generic stable split)
    prm = api.params(p=args.p if args.p != 4096 else 256, s=args.s, seed=9)
    ws = api._workspace(api.workspace_size(n, N.SS_U64, N.SS_V_B32, prm), kd.device)

    def step():
        api.sort_pairs(kd, vd, prm=prm, keys_out=ko, vals_out=vo, ws=ws, key_type="u64")

    ms = _timed(step, args.steps, args.warmup)
    kernels = _kernel_table(step, max(1, min(args.steps, 5)))
    ko_h = ko.cpu().numpy().view(np.uint64)
    vo_h = vo.cpu().numpy().view(np.uint32)
    # stable: sorted keys, and payload (= input index) strictly increasing inside runs of equal keys
    ok = bool(np.all(ko_h[1:] >= ko_h[:-1]))
    eq = ko_h[1:] == ko_h[:-1]
    ok = ok and bool(np.all(vo_h[1:][eq] > vo_h[:-1][eq])) and bool(np.array_equal(keys[vo_h], ko_h))
    gp = n / (ms / 1e3) / 1e9
    return _base("Gpairs/s, stable sample sort of 2^27 (uint64 key, uint32 payload) pairs", gp, "Gpairs/s", args,
                 ms, "u64+u32",
                 {"workload": "2^27 uint64 keys uniform on [0, 0.7n) with uint32 payload = index, stable",
                  "p": prm.p, "s": prm.s, "seed": seed},
                 hbm_frac_56B_per_pair=round(gp * 56 / HBM_PEAK_GBS, 4), kernels=kernels,
                 check="stable order (sorted, payload increasing in equal-key runs, payload indexes the key)"
                 if ok else "FAILED"), ok


def bench_segmented(args):
    count = 20000
    seed = workloads.seed_for(3)
    sizes = workloads.segment_sizes(count, seed)
    off = workloads.offsets_from_sizes(sizes)
    total, max_len = int(off[-1]), int(sizes.max())
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(seed + 1)
    kd = torch.randint(-2**31, 2**31, (total,), dtype=torch.int32, device=dev, generator=g)
    od = torch.from_numpy(off).to(dev)
    ko = torch.empty_like(kd)
    wsz = api.segmented_workspace_size(total, count, max_len, N.SS_I32, N.SS_V_NONE, None)
    ws = api._workspace(wsz, dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        api.segmented_sort(kd, od, max_len=max_len, total=total, keys_out=ko, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        api.segmented_sort(kd, od, max_len=max_len, total=total, keys_out=ko, ws=ws)
    ms = _timed(graph.replay, args.steps, args.warmup)
    batched = ko.clone()

    # one call per segment, workspace sized for the longest one
    prm = api.params(p=1024, s=8, seed=5)
    ws1 = api._workspace(api.workspace_size(max_len, N.SS_I32, N.SS_V_NONE, prm), dev)
    L = N.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    kin, kout, wp, wn = kd.data_ptr(), ko.data_ptr(), ws1.data_ptr(), ws1.numel()
    offl = off.tolist()

    def per_segment():
        for i in range(count):
            b, e = offl[i], offl[i + 1]
            if e > b:
                L.sample_sort_keys(ctypes.c_void_p(kin + 4 * b), ctypes.c_void_p(kout + 4 * b), e - b, N.SS_I32,
                                   ctypes.byref(prm), ctypes.c_void_p(wp), wn, stream)

    steps2 = max(1, min(args.steps, 3))
    ko.zero_()
    ms_seg = _timed(per_segment, steps2, 1)
    same = bool(torch.equal(ko, batched))
    # oracle on a sample of segments (the longest, the shortest non-empty, and random ones)
    import oracle
    rng = np.random.default_rng(1)
    pick = set(rng.choice(count, 24, replace=False).tolist()) | {int(np.argmax(sizes)), int(np.argmin(sizes))}
    ok = same
    for i in sorted(pick):
        seg = kd[off[i]:off[i + 1]].cpu().numpy()
        want = seg[oracle.stable_perm(seg)]
        ok = ok and bool(np.array_equal(batched[off[i]:off[i + 1]].cpu().numpy(), want))
    gk = total / (ms / 1e3) / 1e9
    return _base("Gkeys/s, batched segmented sample sort (one graph) vs one call per segment", gk, "Gkeys/s",
                 args, ms, "i32",
                 {"workload": f"{count} segments, lengths floor(2^(20U)) in [1, 2^20], int32 uniform keys",
                  "segments": count, "total_keys": total, "max_len": max_len, "seed": seed},
                 per_segment={"ms": round(ms_seg, 3), "value": round(total / (ms_seg / 1e3) / 1e9, 4),
                              "unit": "Gkeys/s"},
                 speedup_vs_per_segment=round(ms_seg / ms, 2),
                 hbm_frac_20B_per_key=round(gk * 20 / HBM_PEAK_GBS, 4),
                 check=("batched == per-segment and == oracle on %d segments" % len(pick)) if ok else "FAILED"), ok


def bench_autograd(args):
    rows, cols = 64, 1 << 18
    seed = workloads.seed_for(4)
    x = workloads.tie_free_rows(rows, cols, seed)
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    gy = torch.randn(rows, cols, device="cuda", generator=torch.Generator("cuda").manual_seed(seed))

    def fwd():
        return api.SortFn.apply(xd)

    vals, perm = fwd()
    ms_f = _timed(fwd, args.steps, args.warmup)
    ms_b = _timed(lambda: api.scatter_grad(gy, perm), args.steps, args.warmup)

    prm = api.params(p=1024, s=8, seed=5)
    ws1 = api._workspace(api.workspace_size(cols, N.SS_F32, N.SS_V_IOTA64, prm), xd.device)
    vrow = torch.empty(rows, cols, dtype=torch.float32, device="cuda")
    prow = torch.empty(rows, cols, dtype=torch.int64, device="cuda")
    xdet = xd.detach()

    def fwd_rows():
        for r in range(rows):
            api.sort_pairs(xdet[r], iota="int64", prm=prm, keys_out=vrow[r], vals_out=prow[r], ws=ws1)

    gx = torch.empty_like(gy)

    def bwd_rows():
        for r in range(rows):
            api.scatter_grad(gy[r:r + 1], perm[r:r + 1], grad_x=gx[r:r + 1])

    ms_fr = _timed(fwd_rows, max(1, args.steps // 4), 1)
    ms_br = _timed(bwd_rows, max(1, args.steps // 4), 1)
    import oracle
    ok = bool(torch.equal(prow, perm)) and bool(torch.equal(vrow, vals.detach()))
    for r in (0, rows // 2, rows - 1):
        ok = ok and bool(np.array_equal(perm[r].cpu().numpy(), oracle.stable_perm(x[r])))
    ok = ok and bool(torch.equal(api.scatter_grad(gy, perm), torch.from_numpy(
        oracle.scatter_grad(gy.cpu().numpy(), perm.cpu().numpy())).cuda()))
    n = rows * cols
    ge = n / (ms_f / 1e3) / 1e9
    return _base("Gelem/s, differentiable row sort forward (values + permutation) of 64 x 2^18 float32", ge,
                 "Gelem/s", args, ms_f, "f32",
                 {"workload": "64 x 2^18 float32 N(0,1) tie-free rows: SortFn forward, gradient-scatter backward",
                  "rows": rows, "cols": cols, "seed": seed},
                 backward={"ms": round(ms_b, 5), "value": round(n / (ms_b / 1e3) / 1e9, 3), "unit": "Gelem/s"},
                 per_row={"forward_ms": round(ms_fr, 4), "backward_ms": round(ms_br, 4)},
                 speedup_vs_per_row={"forward": round(ms_fr / ms_f, 2), "backward": round(ms_br / ms_b, 2)},
                 check="batched == per-row == oracle permutation; backward == oracle scatter" if ok else "FAILED"), ok
