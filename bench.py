#!/usr/bin/env python
"""Benchmark of the MI355X sample sort.

Default workload: 2^26 int32 keys (uniform, seeded, synthetic), keys only,
random oversampling with p = 4096 buckets and oversampling s = 16, resident
in HBM before the timed region.  One step = one full sort: sample, sample
sort, splitters, classification and counts, the split and the bucket sorts.

Prints ONE JSON line with Gkeys/s, the roofline of the dominant kernel
(algorithmic bytes / its HIP-event time, against 8 TB/s HBM), the CPU
oracle's rate on a bounded sample of the same workload (timed first, on one
pinned host core, before anything touches the GPU), the paper's multi-core
McRan on the host's cores on the same sample (host_mcran), and -- after the
headline's timed region -- a "batched" object with the two other forms of
the metric:

* segmented: 20,000 segments of log-uniform length in [1, 2^20] (int32),
  one HIP-graph-captured segmented_sort vs one sample_sort_keys call per
  segment, both with the library's tuned parameters (prm = NULL);
* autograd: 64 x 2^18 float32 rows, SortFn forward (values + permutation)
  and the gradient-scatter backward vs one call per row.

Every output is checked without the oracle: keys non-decreasing and the
same multiset; a permutation that is a valid permutation, orders the
values and (tie-free rows) is therefore the unique sorting permutation;
the backward routes every gradient through it.

Single workloads (--workload): sort, pairs (2^27 uint64 keys + uint32
payload), segmented, autograd, strings (2^25 random 32-byte strings),
regular (2^20 uint32, regular oversampling p = 64, s = 8).
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a kernel kind, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch), scaled by what the same counters read for a
# plain device copy of the input in the same run (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0: the copy of 256 MiB reads 131,085 KiB and writes 262,144
# KiB).  Valid only for the kernel sources and the workload they were taken
# on; "traffic" is null for anything else.
MEASURED_TRAFFIC = {
    ("bucket_sort", 26, 4096, 16, "random", "uniform"): {
        "src_sha256_16": "ecf97c174e6d229b",
        "bytes_per_launch": 786305850,   # k_wide_bucket<16000, 13>: FETCH 221,542 KiB x 2 + WRITE 324,792 KiB
    },
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sort",
                    choices=["sort", "pairs", "segmented", "autograd", "strings", "regular"])
    ap.add_argument("--log2n", type=int, default=26)
    ap.add_argument("--p", type=int, default=4096)
    ap.add_argument("--s", type=int, default=16)
    ap.add_argument("--sampling", default="random", choices=["random", "regular"])
    ap.add_argument("--dist", default="uniform")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0, help="extra SS_F_* bits (tuning experiments)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the segmented and autograd forms")
    ap.add_argument("--cpu-log2n", type=int, default=25, help="CPU baseline sample size (log2)")
    ap.add_argument("--cpu-runs", type=int, default=3)
    return ap.parse_args()


# ------------------------------------------------------------ CPU baseline

def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(keys, log2n, runs):
    """The oracle (single-threaded C stable merge sort) on a prefix of the
    same input, pinned to one host core; Gkeys/s as the mean of `runs`
    runs, the fastest run beside it.  Runs before the GPU is touched."""
    import oracle
    sample = keys[: min(keys.size, 1 << log2n)].copy()
    oracle.stable_perm(sample[:1024])                # (builds / loads the oracle outside the timing)
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    try:
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.stable_perm(sample)
            ts.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, old)
    t = sum(ts) / len(ts)
    return {"value": round(sample.size / t / 1e9, 5), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first 2^{int(log2n)} keys of the same input, mean of {runs} runs "
                      f"({t:.2f} s each; fastest {min(ts):.2f} s = {sample.size / min(ts) / 1e9:.5f} Gkeys/s)",
            "pinned_core": core, "host_cpu": _cpu_model(), "host_cpu_count": os.cpu_count()}


def host_mcran(keys, log2n, runs):
    """The paper's multi-core McRan (sort-first: p blocks sorted on t
    threads, random sample, binary-search split, p-way merge per bucket) on
    this host's cores: p = 256, the paper's default s = ceil(lg^2 n), on a
    prefix of the same input.  "paper_8_threads" is the configuration of the
    paper's measurements (8 threads for step 1, step 5 on one thread; one
    run); "all_cores" spreads steps 1 and 5 over every core (mean of `runs`,
    fastest beside it).  A CPU reference point on the same machine, not the
    target."""
    import math

    import numpy as np

    from paper_1608_08648_amd import host
    sample = keys[: min(keys.size, 1 << log2n)]
    n = sample.size
    p, s = 256, math.ceil(math.log2(n) ** 2)
    cores = min(len(os.sched_getaffinity(0)), 64)
    want = np.sort(sample)
    res = {"unit": "Gkeys/s", "kind": "McRan (paper Alg. 2 with multi-core step 1), qsort as SomeSort",
           "sample": f"first 2^{int(log2n)} keys of the same input", "p": p, "s": s, "cores": cores}
    for key, t, mt, reps in (("all_cores", cores, cores, runs), ("paper_8_threads", 8, 1, 1)):
        ts, steps, ok = [], None, True
        for _ in range(reps):
            y, st = host.mcran_sort(sample, p, s, t, seed=7, merge_threads=mt)
            ts.append(st["total_s"])
            steps = st
            ok = ok and bool(np.array_equal(y, want))
        res[key] = {"threads": t, "merge_threads": mt, "value": round(n / (sum(ts) / len(ts)) / 1e9, 5),
                    "fastest": round(n / min(ts) / 1e9, 5), "runs": reps,
                    "steps_s": {k: round(v, 3) for k, v in steps.items()}, "check": "sorted" if ok else "FAILED"}
    res["value"] = res["all_cores"]["value"]
    return res


# --------------------------------------------------------------- helpers

def fingerprint(a):
    import numpy as np
    v = a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64).astype(np.uint64)
    return (int(v.sum()), int((v * v).sum()), int(np.bitwise_xor.reduce(v)))


def kernel_table(rep, steps):
    return {k: {"ms_per_step": round(ms / steps, 5), "launches_per_step": round(c / steps, 3)}
            for k, (ms, c) in rep.items() if c}


def roofline_of(rep, steps, bytes_per_step):
    """Dominant kernel: the kind with the largest HIP-event time over the
    timed region.  achieved = its algorithmic bytes per launch / its mean
    launch duration (= bytes per step / time per step, summed over the
    step's launches of that kind)."""
    tot = {k: (ms, c) for k, (ms, c) in rep.items() if c}
    dom = max(tot, key=lambda k: tot[k][0])
    ms, c = tot[dom]
    launches = c / steps
    t = ms / steps / 1e3
    b = bytes_per_step.get(dom)
    if not b:
        return dom, None
    ach = b / t / 1e9
    return dom, {"kernel": dom, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                 "bytes_per_launch": int(b / launches), "launches_per_step": launches,
                 "ms_per_launch": round(t * 1e3 / launches, 5)}


def src_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1608_08648_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind, args):
    t = MEASURED_TRAFFIC.get((kind, args.log2n, args.p, args.s, args.sampling, args.dist))
    if t is None or args.tile or args.flags or t["src_sha256_16"] != src_hash():
        return None
    return t["bytes_per_launch"]


def copy_rate(src, dst, reps=5):
    """HBM rate of a plain device copy of the input (read + write bytes per
    second); also the calibration kernel of the HBM traffic counters."""
    import torch
    dst.copy_(src)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return round(2 * src.numel() * src.element_size() / (ms / 1e3) / 1e9, 1)


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
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
    from paper_1608_08648_amd import native as N
    N.profile_enable(True, max_launches=256 * (steps + 1))
    for _ in range(steps):
        fn()
    N.profile_collect()
    rep = N.profile_report()
    N.profile_enable(False)
    return kernel_table(rep, steps)


def _segments_sorted(out, inp, off):
    """Every segment of `out` non-decreasing and a rearrangement of the same
    segment of `inp` (device tensors; checked on the GPU with torch)."""
    import torch
    n = out.numel()
    seg = torch.repeat_interleave(torch.arange(off.numel() - 1, device=out.device), off[1:] - off[:-1])
    if seg.numel() != n:
        return False
    # non-decreasing inside each segment
    inc = (out[1:] >= out[:-1]) | (seg[1:] != seg[:-1])
    if not bool(inc.all()):
        return False
    # same multiset per segment: sort (segment, key) pairs of the input with torch and compare
    ref = torch.sort(seg.to(torch.int64) * (1 << 32) + (inp.to(torch.int64) + (1 << 31)), stable=True).values
    got = seg.to(torch.int64) * (1 << 32) + (out.to(torch.int64) + (1 << 31))
    return bool(torch.equal(ref, got))


# ------------------------------------------------------- the headline sort

def bench_sort(args, keys):
    import numpy as np
    import torch

    from paper_1608_08648_amd import api, native, workloads

    n = keys.size
    dev = torch.device("cuda:0")
    seed = workloads.seed_for(1, workloads.DISTRIBUTIONS.index(args.dist))
    kd = torch.from_numpy(keys).to(dev)
    out = torch.empty_like(kd)
    prm = api.params(p=args.p, s=args.s, sampling=args.sampling, seed=1234, tile=args.tile, flags=args.flags)
    info = api.stage_layout(n, native.SS_I32, native.SS_V_NONE, prm)
    ws = api._workspace(api.workspace_size(n, native.SS_I32, native.SS_V_NONE, prm), dev)
    copy_gbs = copy_rate(kd, out)
    for _ in range(args.warmup):
        api.sort_keys(kd, prm, out=out, ws=ws)
    torch.cuda.synchronize()
    # per-kernel table: every launch bracketed by events (outside the timed
    # region: the events themselves add a few microseconds per launch)
    native.profile_enable(True, max_launches=64 * (args.steps + 1))
    for _ in range(args.steps):
        api.sort_keys(kd, prm, out=out, ws=ws)
    native.profile_collect()
    table = native.profile_report()
    dom = max((k for k in table if table[k][1]), key=lambda k: table[k][0])
    # timed region: events only around the dominant kernel's launches
    native.profile_enable(True, max_launches=64 * (args.steps + 1))
    native.profile_kinds([dom])
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.steps):
        api.sort_keys(kd, prm, out=out, ws=ws)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    native.profile_collect()
    rep = native.profile_report()
    native.profile_enable(False)
    status = api.status(ws)
    levels = api.level_stats(ws)
    got = out.cpu().numpy()
    ok = bool(np.all(got[1:] >= got[:-1])) and fingerprint(got) == fingerprint(keys)
    # algorithmic bytes: every level reads its keys to count them (classify)
    # and reads + writes them to split them (scatter); the bucket kernels
    # read + write each key once
    kb = 4
    split_keys = sum(lv["keys"] for lv in levels)
    inplace = sum(lv["bucket_keys"] for lv in levels)
    bytes_per_step = {"classify": kb * split_keys, "scatter": 2 * kb * split_keys,
                      "bucket_sort": 2 * kb * inplace, "bucket_leftover": 2 * kb * (n - inplace),
                      # wide split (p >= 1024): each of its two passes reads and writes every key
                      # (keys equal to a splitter's key stay put: counted as moved, an upper bound)
                      "split_coarse": 2 * kb * split_keys, "split_fine": 2 * kb * split_keys}
    bytes_per_step = {k: v for k, v in bytes_per_step.items() if table.get(k, (0, 0))[1]}   # kinds that ran
    dom, roof = roofline_of(rep, args.steps, bytes_per_step)
    if roof is not None:
        roof["traffic"] = measured_traffic(dom, args)
    gk = n / (ms / 1e3) / 1e9
    res = {
        "metric": "Gkeys/s and % of HBM roofline, sample sort 2^26 int32; batched vs per-segment",
        "value": round(gk, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32", "data": "synthetic",
        "config": {"workload": f"sample sort of 2^{args.log2n} int32 keys ({args.dist}), keys only",
                   "n": n, "p": args.p, "p_eff": info.p_eff, "s": args.s, "sampling": args.sampling,
                   "levels_below_top": info.levels, "dist": args.dist, "seed": seed, "flags": args.flags},
        "sort_bytes_per_key": round(sum(bytes_per_step.values()) / n, 3),
        "sort_frac_of_hbm": round(gk * sum(bytes_per_step.values()) / n / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "copy_GBs": copy_gbs,
        "levels": levels,
        "kernels": kernel_table(table, args.steps),
        "check": "sorted+multiset" if ok else "FAILED",
        "device_status": status,
    }
    del kd, out, ws
    torch.cuda.empty_cache()
    return res, ok


# ------------------------------------------------------------ other forms

def bench_pairs(args):
    import numpy as np
    import torch

    from paper_1608_08648_amd import api, native as N, workloads

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
    # stable: sorted keys, payload (= input index) a permutation that indexes
    # the keys and increases inside runs of equal keys
    ok = bool(np.all(ko_h[1:] >= ko_h[:-1]))
    eq = ko_h[1:] == ko_h[:-1]
    ok = ok and bool(np.all(vo_h[1:][eq] > vo_h[:-1][eq])) and bool(np.array_equal(keys[vo_h], ko_h))
    ok = ok and bool(np.bincount(vo_h, minlength=n).max() == 1)
    gp = n / (ms / 1e3) / 1e9
    return {"metric": "Gpairs/s, stable sample sort of 2^27 (uint64 key, uint32 payload) pairs",
            "value": round(gp, 4), "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64+u32", "data": "synthetic",
            "config": {"workload": "2^27 uint64 keys uniform on [0, 0.7n) with uint32 payload = index, stable",
                       "p": prm.p, "s": prm.s, "seed": seed},
            "hbm_frac_56B_per_pair": round(gp * 56 / HBM_PEAK_GBS, 4), "kernels": kernels,
            "check": "stable order (sorted, payload a permutation increasing in equal-key runs, indexing the keys)"
            if ok else "FAILED"}, ok


def bench_segmented(steps, warmup, per_segment_steps=2):
    """20,000 log-uniform segments: one graph-captured batched call vs one
    call per segment, both with the library's tuned parameters (prm = NULL)."""
    import numpy as np
    import torch

    from paper_1608_08648_amd import api, native as N, workloads

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
    ms = _timed(graph.replay, steps, warmup)
    status = api.status(ws)
    batched = ko.clone()
    del ws
    # one call per segment (prm = NULL: the same tuned parameters), workspace
    # sized for the longest segment
    ws1 = api._workspace(api.workspace_size(max_len, N.SS_I32, N.SS_V_NONE, None), dev)
    L = N.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    kin, kout, wp, wn = kd.data_ptr(), ko.data_ptr(), ws1.data_ptr(), ws1.numel()
    offl = off.tolist()

    def per_segment():
        for i in range(count):
            b, e = offl[i], offl[i + 1]
            if e > b:
                N.check(L.sample_sort_keys(ctypes.c_void_p(kin + 4 * b), ctypes.c_void_p(kout + 4 * b), e - b,
                                           N.SS_I32, None, ctypes.c_void_p(wp), wn, stream))

    ko.zero_()
    ms_seg = _timed(per_segment, per_segment_steps, 1)
    same = bool(torch.equal(ko, batched))
    ok = same and _segments_sorted(batched, kd, od) and status == ""
    gk = total / (ms / 1e3) / 1e9
    res = {"workload": f"{count} segments, lengths floor(2^(20U)) in [1, 2^20], int32 uniform keys",
           "segments": count, "total_keys": total, "max_len": max_len, "seed": seed,
           "params": "tuned (prm = NULL) in both legs",
           "batched_ms": round(ms, 4), "batched_Gkeys_s": round(gk, 3),
           "per_segment_ms": round(ms_seg, 3), "per_segment_Gkeys_s": round(total / (ms_seg / 1e3) / 1e9, 3),
           "speedup": round(ms_seg / ms, 2), "hbm_frac_20B_per_key": round(gk * 20 / HBM_PEAK_GBS, 4),
           "check": "batched == per-segment; every segment sorted and the same multiset" if ok else "FAILED"}
    del kd, ko, batched, ws1, od
    torch.cuda.empty_cache()
    return res, ok


def bench_autograd(steps, warmup):
    """64 x 2^18 float32 rows: SortFn forward and the gradient-scatter
    backward vs one call per row."""
    import torch

    from paper_1608_08648_amd import api, native as N, workloads

    rows, cols = 64, 1 << 18
    seed = workloads.seed_for(4)
    x = workloads.tie_free_rows(rows, cols, seed)
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    gy = torch.randn(rows, cols, device="cuda", generator=torch.Generator("cuda").manual_seed(seed))

    def fwd():
        return api.SortFn.apply(xd)

    vals, perm = fwd()
    ms_f = _timed(fwd, steps, warmup)
    gx = api.scatter_grad(gy, perm)
    ms_b = _timed(lambda: api.scatter_grad(gy, perm, grad_x=gx), steps, warmup)

    ws1 = api._workspace(api.workspace_size(cols, N.SS_F32, N.SS_V_IOTA64, None), xd.device)
    vrow = torch.empty(rows, cols, dtype=torch.float32, device="cuda")
    prow = torch.empty(rows, cols, dtype=torch.int64, device="cuda")
    xdet = xd.detach()
    L = N.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def fwd_rows():
        for r in range(rows):
            N.check(L.sample_sort_pairs(ctypes.c_void_p(xdet[r].data_ptr()), None,
                                        ctypes.c_void_p(vrow[r].data_ptr()), ctypes.c_void_p(prow[r].data_ptr()),
                                        cols, N.SS_F32, N.SS_V_IOTA64, None, ctypes.c_void_p(ws1.data_ptr()),
                                        ws1.numel(), stream))

    gxr = torch.empty_like(gy)

    def bwd_rows():
        for r in range(rows):
            api.scatter_grad(gy[r:r + 1], perm[r:r + 1], grad_x=gxr[r:r + 1])

    ms_fr = _timed(fwd_rows, max(1, steps // 2), 1)
    ms_br = _timed(bwd_rows, max(1, steps // 2), 1)
    # checks: per-row == batched; perm a permutation of every row that orders
    # its values (unique on tie-free rows); values == x[perm]; the backward
    # puts grad_y[r, j] at grad_x[r, perm[r, j]] and nowhere else
    v = vals.detach()
    ok = bool(torch.equal(prow, perm)) and bool(torch.equal(vrow, v)) and bool(torch.equal(gxr, gx))
    ok = ok and bool((v[:, 1:] > v[:, :-1]).all())
    ok = ok and bool(torch.equal(torch.sort(perm, dim=1).values,
                                 torch.arange(cols, device="cuda").expand(rows, cols)))
    ok = ok and bool(torch.equal(torch.gather(xdet, 1, perm), v))
    ok = ok and bool(torch.equal(torch.gather(gx, 1, perm), gy))
    n = rows * cols
    res = {"workload": "64 x 2^18 float32 N(0,1) tie-free rows: SortFn forward, gradient-scatter backward",
           "rows": rows, "cols": cols, "seed": seed, "params": "tuned (prm = NULL) in both legs",
           "forward_ms": round(ms_f, 4), "forward_Gelem_s": round(n / (ms_f / 1e3) / 1e9, 3),
           "backward_ms": round(ms_b, 4), "backward_Gelem_s": round(n / (ms_b / 1e3) / 1e9, 3),
           "backward_frac_of_hbm_16B": round(n * 16 / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "per_row_forward_ms": round(ms_fr, 4), "per_row_backward_ms": round(ms_br, 4),
           "speedup_forward": round(ms_fr / ms_f, 2), "speedup_backward": round(ms_br / ms_b, 2),
           "check": "batched == per-row; perm a permutation ordering each row; backward routes every gradient"
           if ok else "FAILED"}
    del xd, gy, vals, perm, gx, gxr, vrow, prow, ws1
    torch.cuda.empty_cache()
    return res, ok


def bench_strings(args):
    """2^25 random 32-byte strings (1 GiB, the paper's workload shape):
    stable memcmp-order sort through the index, permutation and sorted
    strings; checked without the oracle (the sorted strings do not decrease
    as big-endian words, and the permutation is one)."""
    import numpy as np
    import torch

    from paper_1608_08648_amd import api, workloads

    n = 1 << (args.log2n if args.log2n != 26 else 25)
    seed = workloads.seed_for(7, 0)
    recs = workloads.strings32(n, seed, "random")
    rd = torch.from_numpy(recs).cuda()
    out = torch.empty_like(rd)
    ws = api._workspace(api.strings_workspace_size(n, 32, None), rd.device)

    def step():
        api.sort_strings(rd, recs_out=out, ws=ws)

    ms = _timed(step, args.steps, args.warmup)
    perm, _ = api.sort_strings(rd, recs_out=out, ws=ws)
    w = out.view(torch.int64).view(n, 4).cpu().numpy().view(np.uint64).byteswap()
    srt = np.lexsort((w[:, 3], w[:, 2], w[:, 1], w[:, 0]))
    ok = bool(np.array_equal(srt, np.arange(n)))
    pp = perm.cpu().numpy()
    ok = ok and bool(np.array_equal(np.sort(pp), np.arange(n))) and bool(np.array_equal(recs[pp], out.cpu().numpy()))
    gs = n / (ms / 1e3) / 1e9
    return {"metric": "Gstrings/s, stable sample sort of 2^25 random 32-byte strings (memcmp order)",
            "value": round(gs, 4), "unit": "Gstrings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u8x32", "data": "synthetic",
            "config": {"workload": f"{n} random 32-byte strings, permutation and sorted strings", "n": n,
                       "params": "tuned (prm = NULL)", "seed": seed},
            "check": "sorted strings non-decreasing, a permutation, recs[perm] == sorted" if ok else "FAILED"}, ok


def bench_regular(args):
    """2^20 uint32 keys uniform on [0, 2^32), regular oversampling (Alg. 1)
    with p = 64, s (the paper's r) = 8: the small configuration.  Checked
    without the oracle: sorted, same multiset, and the largest bucket
    within Lemma 1's bound (S + p - 1) * x, S = s p, x = ceil(ceil(n/p)/S)."""
    import numpy as np
    import torch

    from paper_1608_08648_amd import api, native as N, workloads

    n, p, s = 1 << 20, 64, 8
    seed = workloads.seed_for(0)
    keys = workloads.uniform_u32(n, seed)
    kd = torch.from_numpy(keys.view(np.int32)).cuda()
    out = torch.empty_like(kd)
    prm = api.params(p=p, s=s, sampling="regular", seed=1234)
    ws = api._workspace(api.workspace_size(n, N.SS_U32, N.SS_V_NONE, prm), kd.device)

    def step():
        api.sort_keys(kd, prm, out=out, ws=ws, key_type="u32")

    ms = _timed(step, args.steps, args.warmup)
    kernels = _kernel_table(step, max(1, min(args.steps, 5)))
    o, st, info = api.stages(kd, prm, key_type="u32")
    got = o.cpu().numpy().view(np.uint32)
    ok = bool(np.all(got[1:] >= got[:-1])) and fingerprint(got) == fingerprint(keys)
    S = s * p
    x = -(-(-(-n // p)) // S)
    bound = (S + p - 1) * x
    mx = int(st["counts"].max())
    ok = ok and mx <= bound
    gk = n / (ms / 1e3) / 1e9
    return {"metric": "Gkeys/s, sample sort of 2^20 uint32 keys, regular oversampling p = 64, s = 8",
            "value": round(gk, 4), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic",
            "config": {"workload": "2^20 uint32 uniform, keys only, regular oversampling (Alg. 1)", "n": n, "p": p,
                       "s": s, "sample": int(info.m), "seed": seed},
            "largest_bucket": mx, "lemma1_bound": bound, "mean_bucket": n // p, "kernels": kernels,
            "check": "sorted+multiset, largest bucket within Lemma 1" if ok else "FAILED"}, ok


def _single_line(name, res, args):
    d = {"metric": {"segmented": "Gkeys/s, batched segmented sample sort (one graph) vs one call per segment",
                    "autograd": "Gelem/s, differentiable row sort forward of 64 x 2^18 float32"}[name],
         "value": res["batched_Gkeys_s"] if name == "segmented" else res["forward_Gelem_s"],
         "unit": "Gkeys/s" if name == "segmented" else "Gelem/s", "n_gpus": 1, "steps": args.steps,
         "warmup": args.warmup, "ms_per_step": res["batched_ms"] if name == "segmented" else res["forward_ms"],
         "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": "i32" if name == "segmented" else "f32", "data": "synthetic",
         "config": {"workload": res["workload"]}}
    d[name] = res
    return d


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: the sort of one GPU's share is what it "
                                   "measures; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "sort":
        import numpy as np

        from paper_1608_08648_amd import workloads
        seed = workloads.seed_for(1, workloads.DISTRIBUTIONS.index(args.dist))
        keys = workloads.keys_2p26(1 << args.log2n, args.dist, seed, np.int32)
        # the CPU baseline first: one pinned core, before anything touches the GPU
        cpu = None if args.no_cpu else cpu_baseline(keys, args.cpu_log2n, args.cpu_runs)
        mc = None if args.no_cpu else host_mcran(keys, args.cpu_log2n, args.cpu_runs)
        res, ok = bench_sort(args, keys)
        if cpu is not None:
            res["cpu_baseline"] = cpu
            res["host_mcran"] = mc
        if not args.no_batched:
            seg, ok1 = bench_segmented(max(2, args.steps // 4), 1)
            ag, ok2 = bench_autograd(max(4, args.steps // 2), 2)
            res["batched"] = {"segmented": seg, "autograd": ag}
            ok = ok and ok1 and ok2
    elif args.workload == "pairs":
        res, ok = bench_pairs(args)
    elif args.workload == "strings":
        res, ok = bench_strings(args)
    elif args.workload == "regular":
        res, ok = bench_regular(args)
    elif args.workload == "segmented":
        seg, ok = bench_segmented(args.steps, args.warmup)
        res = _single_line("segmented", seg, args)
    else:
        ag, ok = bench_autograd(args.steps, args.warmup)
        res = _single_line("autograd", ag, args)
    print(json.dumps(res), flush=True)
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
