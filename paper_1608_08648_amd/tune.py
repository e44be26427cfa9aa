"""Autotuner of the sample sort's parameters (p, s, tile) per size class.

The paper fixes p for the machine after some calibration and ties the
sample size to n (Section 2.1, Section 3): its default oversampling factor
for random sampling is s = ceil(lg^2 n) (Alg. 2 with w_n^2 = lg n / 2), its
sample-size study varies s = lg^(1+a) n for a = 0.2 .. 1.8 (Table 2), and
the deterministic rule takes r = 1 .. 5 (Table 8).  This module times, on the
GPU, a grid of (p, s) per size class and form, seeded with those priors,
keeps the fastest and installs it in the library (ss_set_tuning), so that
calls with prm = None use it.  Beside every choice it reports the priors'
own times and Claim 1's imbalance bound for the chosen p and s.

Results are cached as JSON, keyed by the GPU's architecture and compute-unit
count; every entry names its form, key width, payload width and size class
(class c: lengths in (2^(c-1), 2^c]).  A cache file that does not parse or
does not match the schema is ignored, and the next run rewrites it.

Usage: ``python -m paper_1608_08648_amd.tune [--quick] [--out FILE]``.
"""
import argparse
import ctypes
import json
import math
import os
import time

from . import native as N

SCHEMA = 1
FORM_SINGLE, FORM_SEGMENTED = 0, 1


# ------------------------------------------------------------------ Claim 1

def claim1_epsilon(n, p, s, rho=1.0):
    """Smallest eps for which Claim 1 (Section 2.3) holds at these n, p, s:
    s >= (1 + eps) / eps^2 * K with K = 2 rho ln n + ln(2 pi p^2 (ps - 1)
    e^(1/(3(ps - 1)))), i.e. eps = (K + sqrt(K^2 + 4 s K)) / (2 s).  Then
    with probability at least 1 - n^-rho no bucket exceeds
    ceil((1 + eps)(n - p + 1) / p).  The claim needs 0 < eps < 1 (and
    p s < n / 2); eps >= 1 means the claim says nothing at this s."""
    m = p * s - 1
    if m < 1:
        return math.inf
    K = 2.0 * rho * math.log(n) + math.log(2.0 * math.pi * p * p * m) + 1.0 / (3.0 * m)
    return (K + math.sqrt(K * K + 4.0 * s * K)) / (2.0 * s)


def claim1_bound(n, p, s, rho=1.0):
    """(eps, largest bucket Claim 1 allows, or None when eps >= 1)."""
    eps = claim1_epsilon(n, p, s, rho)
    if not eps < 1.0:
        return eps, None
    return eps, math.ceil((1.0 + eps) * (n - p + 1) / p)


def claim1_min_s(n, p, eps, rho=1.0):
    """Smallest integer s with which Claim 1 gives imbalance eps (the
    sample size ps - 1 enters the claim's logarithm, hence the search)."""
    s = 1
    while claim1_epsilon(n, p, s, rho) > eps:
        s *= 2
        if s > 1 << 40:
            return None
    lo, hi = s // 2 + 1, s
    while lo < hi:
        mid = (lo + hi) // 2
        if claim1_epsilon(n, p, mid, rho) <= eps:
            hi = mid
        else:
            lo = mid + 1
    return lo


def paper_priors(n):
    """The paper's sample-size choices for n keys: the default s = ceil(lg^2 n),
    the study's s = ceil(lg^(1+a) n) for a = 0.2, 0.6, 1.0, 1.4, 1.8, and
    r = 1..5 for regular sampling."""
    lg = math.log2(n)
    return {"default_s": math.ceil(lg * lg),
            "a_sweep": {f"{a:.1f}": math.ceil(lg ** (1.0 + a)) for a in (0.2, 0.6, 1.0, 1.4, 1.8)},
            "regular_r": [1, 2, 3, 4, 5]}


# -------------------------------------------------------------------- cache

def cache_path():
    return os.environ.get("SS_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1608_08648_amd", "tune.json")


def device_key(index=0):
    import torch
    pr = torch.cuda.get_device_properties(index)
    arch = getattr(pr, "gcnArchName", "") or pr.name
    return f"{arch.split(':')[0]}:{pr.multi_processor_count}cu"


_FIELDS = ("form", "key_bytes", "val_bytes", "size_class", "p", "s", "tile")


def _valid_entry(e):
    if not isinstance(e, dict) or any(not isinstance(e.get(k), int) for k in _FIELDS):
        return False
    p = e["p"]
    return (e["form"] in (0, 1) and e["key_bytes"] in (4, 8) and e["val_bytes"] in (0, 4, 8)
            and 0 <= e["size_class"] <= 32 and 1 <= e["s"] <= 4096 and 0 <= e["tile"] <= 1 << 24
            and ((p == 0 and e["form"] == 1) or (2 <= p <= 4096 and p & (p - 1) == 0)))


def load_cache(path=None, key=None):
    """The cached entries for this device, or None when the file is missing,
    does not parse, or does not match the schema (a corrupt cache is
    ignored, never trusted)."""
    path = path or cache_path()
    try:
        with open(path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        return None
    if not isinstance(doc, dict) or doc.get("schema") != SCHEMA or not isinstance(doc.get("devices"), dict):
        return None
    dev = doc["devices"].get(key or device_key())
    if not isinstance(dev, dict) or not isinstance(dev.get("entries"), list):
        return None
    ents = dev["entries"]
    if not ents or not all(_valid_entry(e) for e in ents):
        return None
    return ents


def save_cache(entries, report, path=None, key=None):
    """Write (or merge into) the cache; a corrupt file is replaced."""
    path = path or cache_path()
    key = key or device_key()
    doc = None
    try:
        with open(path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        doc = None
    if not isinstance(doc, dict) or doc.get("schema") != SCHEMA or not isinstance(doc.get("devices"), dict):
        doc = {"schema": SCHEMA, "devices": {}}
    doc["devices"][key] = {"tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S"), "entries": entries, "report": report}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def install(entries):
    """Install entries (dicts with _FIELDS) as the library's tuned table."""
    arr = (N.TuneEntry * max(len(entries), 1))()
    for i, e in enumerate(entries):
        arr[i] = N.TuneEntry(*(int(e[k]) for k in _FIELDS))
    N.check(N.lib().ss_set_tuning(arr, len(entries)))


def reset():
    """Back to the library's built-in table."""
    N.check(N.lib().ss_set_tuning(None, 0))


_installed = False


def ensure_installed():
    """Install this device's cached table once per process, if a valid cache
    exists (nothing is measured here)."""
    global _installed
    if _installed:
        return
    _installed = True
    try:
        ents = load_cache()
    except Exception:
        ents = None
    if ents:
        install(ents)


# ------------------------------------------------------------------- timing

def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _single_case(n, kw, vw, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    if kw == 4:
        keys = torch.randint(-2**31, 2**31, (n,), dtype=torch.int32, device="cuda", generator=g)
        kt = N.SS_I32
    else:
        keys = torch.randint(0, int(0.7 * n) + 1, (n,), dtype=torch.int64, device="cuda", generator=g)
        kt = N.SS_U64
    vt = {0: N.SS_V_NONE, 4: N.SS_V_B32, 8: N.SS_V_B64}[vw]
    return keys, kt, vt


def _time_single(keys, kt, vt, prm, reps):
    import torch
    from . import api
    n = keys.numel()
    ws = api._workspace(api.workspace_size(n, kt, vt, prm), keys.device)
    out = torch.empty_like(keys)
    L = N.lib()
    if vt == N.SS_V_NONE:
        def fn():
            N.check(L.sample_sort_keys(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, kt,
                                       ctypes.byref(prm), ctypes.c_void_p(ws.data_ptr()), ws.numel(), api._stream()))
    else:
        vdt = torch.int64 if vt == N.SS_V_B64 else torch.int32
        vals = torch.arange(n, dtype=vdt, device=keys.device)
        vout = torch.empty(n, dtype=vdt, device=keys.device)

        def fn():
            N.check(L.sample_sort_pairs(ctypes.c_void_p(keys.data_ptr()),
                                        ctypes.c_void_p(vals.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(vout.data_ptr()), n, kt, vt,
                                        ctypes.byref(prm), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        api._stream()))
    return _time(fn, reps)


def tune_single(kw, vw, classes, reps=3, log=print):
    """Fastest (p, s) per size class for single arrays; the paper's priors
    timed at the best p and reported beside it."""
    import torch
    from . import api
    entries, report = [], []
    for c in classes:
        n = 1 << c
        keys, kt, vt = _single_case(n, kw, vw, 1000 + c)
        pmax = 4096 if vw == 0 and kw == 4 else (1024 if vw == 0 else 1024)
        ps = [p for p in (64, 128, 256, 512, 1024, 2048, 4096) if p <= pmax and 32 * p <= n]
        grid = {}
        for p in ps:
            for s in (4, 8, 16, 32):
                if 2 * p * s >= n:
                    continue
                prm = api.params(p=p, s=s, seed=0x5EED)
                grid[(p, s)] = _time_single(keys, kt, vt, prm, reps)
        (bp, bs), bt = min(grid.items(), key=lambda kv: kv[1])
        pri = paper_priors(n)
        prior_t = {}
        for name, s in [("default_s", pri["default_s"])] + [(f"a={a}", v) for a, v in pri["a_sweep"].items()]:
            s = min(s, 4096)
            key = (name, s)
            prm = api.params(p=bp, s=s, seed=0x5EED)
            prior_t[key] = _time_single(keys, kt, vt, prm, reps)
        reg_t = {}
        for r in pri["regular_r"]:
            prm = api.params(p=bp, s=r, sampling="regular", seed=0x5EED)
            reg_t[r] = _time_single(keys, kt, vt, prm, reps)
        eps, bound = claim1_bound(n, bp, bs)
        entries.append({"form": FORM_SINGLE, "key_bytes": kw, "val_bytes": vw, "size_class": c,
                        "p": bp, "s": bs, "tile": 0})
        report.append({"form": "single", "key_bytes": kw, "val_bytes": vw, "size_class": c, "n": n,
                       "best": {"p": bp, "s": bs, "ms": round(bt, 4), "Gkeys_s": round(n / bt / 1e6, 2),
                                "claim1_eps": round(eps, 3), "claim1_bucket_bound": bound},
                       "grid_ms": {f"p={p},s={s}": round(t, 4) for (p, s), t in sorted(grid.items())},
                       "paper_priors_at_best_p": {f"{nm} (s={s})": round(t, 4) for (nm, s), t in prior_t.items()},
                       "regular_r_at_best_p": {f"r={r}": round(t, 4) for r, t in reg_t.items()},
                       "claim1_min_s_eps_0.5": claim1_min_s(n, bp, 0.5)})
        log(f"single kw={kw} vw={vw} 2^{c}: p={bp} s={bs} {bt:.4f} ms "
            f"(paper default s={pri['default_s']}: {prior_t[('default_s', min(pri['default_s'], 4096))]:.4f} ms)")
        del keys
        torch.cuda.empty_cache()
    return entries, report


def _segmented_case(c, kw, vw, total_log2, seed):
    """Segments of lengths uniform in (2^(c-1), 2^c], about 2^total_log2 keys."""
    import numpy as np
    import torch
    g = np.random.default_rng(seed)
    lo, hi = (1 << (c - 1)) + 1, 1 << c
    count = max(1, (1 << total_log2) // ((lo + hi) // 2))
    sizes = g.integers(lo, hi + 1, count)
    off = np.zeros(count + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    total = int(off[-1])
    tg = torch.Generator(device="cuda").manual_seed(seed)
    keys = torch.randint(-2**31, 2**31, (total,), dtype=torch.int32, device="cuda", generator=tg)
    return keys, torch.from_numpy(off).cuda(), total, int(sizes.max())


def tune_segmented(kw, vw, classes, base_entries, reps=3, total_log2=25, log=print):
    """Fastest (p, s) per size class for segments (p = 0: sized from the
    length), timed through the prm = NULL path with a candidate table."""
    import torch
    from . import api
    assert kw == 4, "segmented tuning runs on 4-byte keys"
    vt = {0: N.SS_V_NONE, 4: N.SS_V_IOTA32}[vw]
    entries, report = [], []
    for c in classes:
        keys, off, total, max_len = _segmented_case(c, kw, vw, total_log2, 2000 + c)
        out = torch.empty_like(keys)
        vout = torch.empty(total, dtype=torch.int32, device="cuda") if vw else None
        grid = {}
        for p in (0, 8, 16, 32, 64, 128, 256, 512):
            if p and 64 * p > (1 << c):
                continue
            for s in (4, 8, 16):
                cand = base_entries + [{"form": FORM_SEGMENTED, "key_bytes": kw, "val_bytes": vw,
                                        "size_class": c, "p": p, "s": s, "tile": 0}]
                install(cand)
                ws = api._workspace(api.segmented_workspace_size(total, off.numel() - 1, max_len, N.SS_I32, vt,
                                                                 None), keys.device)

                def fn():
                    if vw:
                        api.segmented_sort(keys, off, iota="int32", max_len=max_len, total=total, keys_out=out,
                                           vals_out=vout, ws=ws)
                    else:
                        api.segmented_sort(keys, off, max_len=max_len, total=total, keys_out=out, ws=ws)
                grid[(p, s)] = _time(fn, reps)
                del ws
        (bp, bs), bt = min(grid.items(), key=lambda kv: kv[1])
        entries.append({"form": FORM_SEGMENTED, "key_bytes": kw, "val_bytes": vw, "size_class": c,
                        "p": bp, "s": bs, "tile": 0})
        report.append({"form": "segmented", "key_bytes": kw, "val_bytes": vw, "size_class": c,
                       "segments": off.numel() - 1, "total": total,
                       "best": {"p": bp or "auto", "s": bs, "ms": round(bt, 4),
                                "Gkeys_s": round(total / bt / 1e6, 2)},
                       "grid_ms": {f"p={p or 'auto'},s={s}": round(t, 4) for (p, s), t in sorted(grid.items())}})
        log(f"segmented kw={kw} vw={vw} 2^{c}: p={bp or 'auto'} s={bs} {bt:.4f} ms for {total} keys")
        del keys, out, vout
        torch.cuda.empty_cache()
    install(base_entries)
    return entries, report


def run(quick=False, path=None, log=print):
    """Measure every form and size class, install the result, write the cache;
    returns (entries, report)."""
    reps = 2 if quick else 3
    single_cls = [16, 20, 24, 26] if quick else [16, 18, 20, 22, 24, 26, 27]
    entries, report = [], []
    for kw, vw, cls in [(4, 0, single_cls), (8, 4, [20, 24] if quick else [20, 23, 26]),
                        (4, 4, [18] if quick else [16, 18, 20, 22])]:
        e, r = tune_single(kw, vw, cls, reps, log)
        entries += e
        report += r
    seg_cls = [16, 18, 20] if quick else [16, 17, 18, 19, 20]
    for kw, vw, cls in [(4, 0, seg_cls), (4, 4, [18] if quick else [15, 16, 17, 18, 19, 20])]:
        e, r = tune_segmented(kw, vw, cls, entries, reps, log=log)
        entries += e
        report += r
    entries = _fill_classes(entries)
    install(entries)
    save_cache(entries, report, path)
    return entries, report


def _fill_classes(entries):
    """Every class of a measured (form, key, payload) group takes the entry of
    the nearest measured class (below the smallest: that one; the segmented
    form only from its smallest measured class up)."""
    out = list(entries)
    groups = {}
    for e in entries:
        groups.setdefault((e["form"], e["key_bytes"], e["val_bytes"]), {})[e["size_class"]] = e
    for (form, kw, vw), by_c in groups.items():
        meas = sorted(by_c)
        for c in range(0, 33):
            if c in by_c or (form == FORM_SEGMENTED and c < meas[0]):
                continue
            near = min(meas, key=lambda m: (abs(m - c), m))
            e = dict(by_c[near])
            e["size_class"] = c
            if form == FORM_SINGLE and c > near:
                # keep the bucket size of the nearest class: p grows with n
                e["p"] = min(4096 if (kw == 4 and vw == 0) else 1024, e["p"] << (c - near))
            if form == FORM_SINGLE and c < near:
                e["p"] = max(2, e["p"] >> (near - c))
            out.append(e)
    return out


def emit_c(entries, device, path):
    """Write the measured entries as the C table the library builds in
    (csrc/ss_tuned.h), so that a fresh process without a cache uses them."""
    lines = ["// Tuned (p, s, tile) per form, key width, payload width and size class,",
             f"// measured on {device} by `python -m paper_1608_08648_amd.tune --emit-c <this file>`",
             "// (classes between and beyond the measured ones take the nearest measured",
             "// class's bucket size).  Fields: form, key_bytes, val_bytes, size_class, p, s, tile.",
             "#pragma once", "", "namespace ss {", "", "constexpr uint32_t TUNED[][7] = {"]
    for e in sorted(entries, key=lambda e: tuple(e[k] for k in _FIELDS)):
        lines.append("    {" + ", ".join(str(int(e[k])) for k in _FIELDS) + "},")
    lines += ["};", "", "}  // namespace ss", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None, help="cache file (default: $SS_TUNE_CACHE or ~/.cache/...)")
    ap.add_argument("--report", default=None, help="also write the report as JSON here")
    ap.add_argument("--emit-c", default=None, help="also write the table as a C header (the built-in table)")
    args = ap.parse_args()
    entries, report = run(quick=args.quick, path=args.out)
    if args.emit_c:
        emit_c(entries, device_key(), args.emit_c)
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"device": device_key(), "entries": entries, "report": report}, f, indent=1)
    print(json.dumps({"device": device_key(), "classes": len(entries)}))


if __name__ == "__main__":
    main()
