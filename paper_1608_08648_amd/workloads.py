"""Seeded synthetic inputs for the sample sort.

This module only draws input arrays (numpy PCG64, host side); it contains
none of the sorting method's arithmetic, so the CPU oracle and the HIP path
can both be fed from it.

The paper measures on random 32-byte strings (Section 3); the integer and
float workloads below stand in for that, with the shapes and value
distributions of the sort's own workloads:

* :func:`keys_2p26` -- int32/uint32 keys in six distributions: uniform,
  Gaussian (mean 0, sd 2^28, rounded half-to-even, clamped to int32),
  all-equal, already sorted, reverse sorted, 64 distinct values.
* :func:`pairs_dup` -- uint64 keys uniform on [0, floor(0.7 n)) (about 30%
  duplicates) with a uint32 payload equal to the input index.
* :func:`segment_sizes` -- segment lengths floor(2^(20 U)) clamped to
  [1, 2^20] (log-uniform), with int64 offsets.
* :func:`tie_free_rows` -- float32 rows drawn from N(0, 1), each row
  redrawn until its values are pairwise distinct.
* :func:`strings32` -- n records of 32 bytes: uniformly random bytes (the
  paper's random strings), or records that share 8-, 16- or 24-byte
  prefixes, or repeat a few whole records (ties at every word).
"""
import numpy as np

DISTRIBUTIONS = ("uniform", "gaussian", "all_equal", "sorted", "reverse", "distinct64")

SEED_BASE = 0x5EED0000


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def seed_for(config, dist_index=0):
    """Fixed seed per (config, distribution), recorded in bench output."""
    return SEED_BASE + 16 * config + dist_index


def keys_2p26(n, dist, seed, dtype=np.int32):
    """n keys of `dtype` (int32 or uint32) in one of DISTRIBUTIONS."""
    g = rng(seed)
    dtype = np.dtype(dtype)
    if dtype == np.int32:
        lo, hi = -(2**31), 2**31
    elif dtype == np.uint32:
        lo, hi = 0, 2**32
    else:
        raise TypeError("keys_2p26: int32 or uint32")
    if dist == "uniform":
        return g.integers(lo, hi, size=n, dtype=np.int64).astype(dtype)
    if dist == "gaussian":
        v = np.round(g.normal(0.0, 2.0**28, size=n))          # numpy rounds half to even
        v = np.clip(v, lo, hi - 1)
        if dtype == np.uint32:
            v = v - lo if lo < 0 else v
        return v.astype(np.int64).astype(dtype)
    if dist == "all_equal":
        v = g.integers(lo, hi, dtype=np.int64)
        return np.full(n, v, dtype=np.int64).astype(dtype)
    if dist in ("sorted", "reverse"):
        v = np.sort(g.integers(lo, hi, size=n, dtype=np.int64))
        if dist == "reverse":
            v = v[::-1]
        return np.ascontiguousarray(v.astype(dtype))
    if dist == "distinct64":
        vals = g.choice(2**32, size=64, replace=False).astype(np.int64) + (lo if lo < 0 else 0)
        return vals[g.integers(0, 64, size=n)].astype(dtype)
    raise ValueError(f"unknown distribution {dist!r}")


def uniform_u32(n, seed):
    return rng(seed).integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)


def pairs_dup(n, seed):
    """(uint64 keys on [0, floor(0.7 n)), uint32 payload = arange(n))."""
    hi = int(0.7 * n)
    keys = rng(seed).integers(0, max(hi, 1), size=n, dtype=np.uint64)
    return keys, np.arange(n, dtype=np.uint32)


def segment_sizes(count, seed, max_log2=20):
    """Log-uniform lengths floor(2^(max_log2 * U)) clamped to [1, 2^max_log2]."""
    u = rng(seed).random(count)
    sizes = np.floor(np.exp2(max_log2 * u)).astype(np.int64)
    return np.clip(sizes, 1, 2**max_log2)


def offsets_from_sizes(sizes):
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def segmented_keys(count, seed, dtype=np.int32, max_log2=20):
    """(keys, offsets) for `count` log-uniform segments of uniform keys."""
    sizes = segment_sizes(count, seed, max_log2)
    off = offsets_from_sizes(sizes)
    total = int(off[-1])
    g = rng(seed + 1)
    if np.dtype(dtype) == np.int32:
        keys = g.integers(-(2**31), 2**31, size=total, dtype=np.int64).astype(np.int32)
    else:
        keys = g.integers(0, 2**32, size=total, dtype=np.uint64).astype(np.uint32)
    return keys, off


def tie_free_rows(rows, cols, seed):
    """float32 [rows, cols] from N(0,1) with no two equal values in a row:
    entries that repeat an earlier value of their row are drawn again until
    none does (at 2^18 values per row a float32 row has ~30 ties, so
    redrawing whole rows would not terminate)."""
    g = rng(seed)
    out = g.standard_normal((rows, cols)).astype(np.float32)
    for r in range(rows):
        row = out[r]
        while True:
            order = np.argsort(row, kind="stable")
            srt = row[order]
            dup = order[1:][srt[1:] == srt[:-1]]
            if dup.size == 0:
                break
            row[dup] = g.standard_normal(dup.size).astype(np.float32)
    return out


def weak_orderings(n):
    """Every weak ordering of n items as a key vector over 0..k-1 with no
    unused value (an ordered set partition): 1, 1, 3, 13, 75, 541, 4683,
    47293, 545835 vectors for n = 0..8 (the ordered Bell numbers)."""
    import itertools
    if n == 0:
        return np.zeros((1, 0), dtype=np.int32)
    # restricted growth strings = unordered set partitions, grouped by block count
    by_k = {}

    def rec(prefix, maxv):
        if len(prefix) == n:
            by_k.setdefault(maxv + 1, []).append(list(prefix))
            return
        for v in range(maxv + 2):
            prefix.append(v)
            rec(prefix, max(maxv, v))
            prefix.pop()

    rec([], -1)
    out = []
    for k, rgs in by_k.items():
        rgs = np.array(rgs, dtype=np.int32)                              # [m, n]
        perms = np.array(list(itertools.permutations(range(k))), dtype=np.int32)  # [k!, k]
        # each ordering of the k blocks gives a distinct weak ordering
        out.append(perms[:, rgs].transpose(1, 0, 2).reshape(-1, n))
    return np.concatenate(out, axis=0)


STRING_KINDS = ("random", "prefix", "dup")


def strings32(n, seed, kind="random"):
    """uint8 [n, 32] records.  random: every byte uniform; prefix: a quarter
    of the records each share their first 8, 16 or 24 bytes with many
    others (16 distinct prefixes per length); dup: 64 distinct records
    repeated."""
    g = rng(seed)
    recs = g.integers(0, 256, size=(n, 32), dtype=np.uint8)
    if kind == "prefix":
        for q, plen in enumerate((8, 16, 24)):
            rows = np.arange(q, n, 4)
            pre = g.integers(0, 256, size=(16, plen), dtype=np.uint8)
            recs[rows, :plen] = pre[g.integers(0, 16, size=rows.size)]
    elif kind == "dup":
        base = g.integers(0, 256, size=(64, 32), dtype=np.uint8)
        recs = base[g.integers(0, 64, size=n)]
    elif kind != "random":
        raise ValueError(kind)
    return np.ascontiguousarray(recs)
