"""CPU oracle for the oversampling sample sort (arXiv 1608.08648).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package; the product path never imports it.

The arithmetic lives in ``oracle.c`` (plain C, single-threaded, built with
gcc).  This module only marshals numpy arrays to it:

* :func:`stable_perm` / :func:`stable_sort` -- the definition of the result
  (Section 1: a stable sort keeps equal keys in input order).
* :func:`stages` -- one top-level pass of the method in the paper's order:
  sample (Alg. 1 step 2 / Alg. 2 step 2), sort the sample, take splitters
  (step 3), split the keys with key-then-tag comparisons (step 4 and
  Section 2.2), then sort each bucket and concatenate.
* :func:`p_eff`, :func:`splitmix64`, :func:`lemma1_bounds` -- the parameter
  rule, the counter-based generator behind random sampling, and the bucket
  bound of Lemma 1.
* :func:`stable_perm_bytes` -- the stable order of fixed-width byte strings
  in memcmp order (the paper's 32-byte string keys, Section 3).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

RANDOM = 0
REGULAR = 1

_KT = {
    np.dtype(np.uint32): 0,
    np.dtype(np.int32): 1,
    np.dtype(np.float32): 2,
    np.dtype(np.uint64): 3,
    np.dtype(np.int64): 4,
    np.dtype(np.float64): 5,
}


def build(so_path=_SO, plant=0):
    """Compile ``oracle.c`` (gcc, -O2).  ``plant`` != 0 builds a variant with a
    deliberate mistake, used only to show that the pin tests catch it."""
    tmp = so_path + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", f"-DORC_PLANT={int(plant)}", _SRC, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, so_path)



def _bind(so_path):
    lib = ctypes.CDLL(so_path)
    P = ctypes.c_void_p
    U64 = ctypes.c_uint64
    lib.orc_stable_sort.argtypes = [P, U64, ctypes.c_int, P]
    lib.orc_stable_sort.restype = ctypes.c_int
    lib.orc_segmented_sort.argtypes = [P, P, U64, ctypes.c_int, P]
    lib.orc_segmented_sort.restype = ctypes.c_int
    lib.orc_splitmix64.argtypes = [U64, U64, P]
    lib.orc_splitmix64.restype = None
    lib.orc_p_eff.argtypes = [U64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
    lib.orc_p_eff.restype = ctypes.c_uint32
    lib.orc_sample_count.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
    lib.orc_sample_count.restype = U64
    lib.orc_stages.argtypes = [P, U64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_int, U64, P, P, P, P, P, P]
    lib.orc_stages.restype = ctypes.c_int
    lib.orc_ord_array.argtypes = [P, U64, ctypes.c_int, P]
    lib.orc_ord_array.restype = None
    lib.orc_lemma1.argtypes = [U64, ctypes.c_uint32, ctypes.c_uint32, P, P]
    lib.orc_lemma1.restype = None
    lib.orc_stable_sort_bytes.argtypes = [P, U64, ctypes.c_uint32, P]
    lib.orc_stable_sort_bytes.restype = ctypes.c_int
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _kt(keys):
    try:
        return _KT[keys.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {keys.dtype}")


class Oracle:
    """The oracle's functions bound to one compiled copy of ``oracle.c``."""

    def __init__(self, so_path):
        self.lib = _bind(so_path)

    def ord_keys(self, keys):
        """The order-preserving unsigned image of each key (uint64)."""
        keys = np.ascontiguousarray(keys)
        out = np.empty(keys.size, dtype=np.uint64)
        self.lib.orc_ord_array(_ptr(keys), keys.size, _kt(keys), _ptr(out))
        return out

    def stable_perm(self, keys):
        """perm[r] = input index of the r-th element of the stable ascending order."""
        keys = np.ascontiguousarray(keys)
        perm = np.empty(keys.size, dtype=np.uint64)
        rc = self.lib.orc_stable_sort(_ptr(keys), keys.size, _kt(keys), _ptr(perm))
        if rc != 0:
            raise MemoryError("oracle: out of memory")
        return perm.astype(np.int64)

    def stable_sort(self, keys, vals=None):
        """(sorted keys, payload carried along or None, permutation)."""
        perm = self.stable_perm(keys)
        return keys[perm], (vals[perm] if vals is not None else None), perm

    def segmented_perm(self, keys, offsets):
        """Per-segment stable permutation; perm holds in-segment indices."""
        keys = np.ascontiguousarray(keys)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        perm = np.empty(keys.size, dtype=np.uint64)
        rc = self.lib.orc_segmented_sort(_ptr(keys), _ptr(offsets), offsets.size - 1, _kt(keys),
                                         _ptr(perm))
        if rc != 0:
            raise ValueError(f"oracle: segmented sort failed ({rc})")
        return perm.astype(np.int64)

    def segmented_sort(self, keys, offsets, vals=None):
        """Sort each segment [offsets[g], offsets[g+1]) on its own."""
        offsets = np.asarray(offsets, dtype=np.int64)
        perm = self.segmented_perm(keys, offsets)
        seg_start = np.repeat(offsets[:-1], np.diff(offsets))
        gperm = seg_start + perm
        return keys[gperm], (vals[gperm] if vals is not None else None), perm

    def splitmix64(self, seed, count):
        """The first `count` outputs of a SplitMix64 generator with state `seed`."""
        out = np.empty(count, dtype=np.uint64)
        self.lib.orc_splitmix64(ctypes.c_uint64(seed & (2**64 - 1)), count, _ptr(out))
        return out

    def p_eff(self, n, p, s, mode):
        """Effective bucket count under the paper's preconditions (1 = sort directly)."""
        return int(self.lib.orc_p_eff(n, p, s, mode))

    def sample_count(self, p, s, mode):
        return int(self.lib.orc_sample_count(p, s, mode))

    def stages(self, keys, p, s, mode, seed):
        """One top-level pass of the method, step by step (p = effective p).

        Returns a dict with the sorted sample (ord, tag), the p-1 splitters
        (ord, tag), the per-bucket key counts and the output permutation."""
        keys = np.ascontiguousarray(keys)
        n = keys.size
        m = self.sample_count(p, s, mode)
        so = np.empty(m, np.uint64)
        st = np.empty(m, np.uint64)
        po = np.empty(max(p - 1, 0), np.uint64)
        pt = np.empty(max(p - 1, 0), np.uint64)
        cnt = np.empty(p, np.uint64)
        perm = np.empty(n, np.uint64)
        rc = self.lib.orc_stages(_ptr(keys), n, _kt(keys), p, s, mode,
                                 ctypes.c_uint64(seed & (2**64 - 1)),
                                 _ptr(so), _ptr(st), _ptr(po), _ptr(pt), _ptr(cnt), _ptr(perm))
        if rc != 0:
            raise ValueError(f"oracle: stages failed ({rc})")
        return {"sample_ord": so, "sample_tag": st, "spl_ord": po, "spl_tag": pt,
                "counts": cnt.astype(np.int64), "perm": perm.astype(np.int64)}

    def stable_perm_bytes(self, recs):
        """Stable ascending permutation of the rows of a uint8 [n, width]
        array in memcmp order (the paper's string keys, Section 3)."""
        recs = np.ascontiguousarray(recs, dtype=np.uint8)
        n, width = recs.shape
        perm = np.empty(n, dtype=np.uint64)
        if self.lib.orc_stable_sort_bytes(_ptr(recs), n, width, _ptr(perm)) != 0:
            raise MemoryError("oracle: out of memory")
        return perm.astype(np.int64)

    def lemma1_bounds(self, n, p, s):
        """Bucket-size bounds of Lemma 1 (Section 2.1) for regular
        oversampling with factor s (the paper's r) and p buckets: with
        S = s*p samples per block and segment length x = ceil(ceil(n/p)/S),
        returns (safe, tight, final): safe = (S+p)*x, tight = (S+p-1)*x
        (the difference bound b_{i+1}-b_i), final = (1+1/s)*n/p + s*p (the
        lemma's closing expression)."""
        u = np.zeros(2, np.uint64)
        d = np.zeros(1, np.float64)
        self.lib.orc_lemma1(n, p, s, _ptr(u), _ptr(d))
        return int(u[0]), int(u[1]), float(d[0])


def lemma1_bounds(n, p, s):
    return _get().lemma1_bounds(n, p, s)


def stable_perm_bytes(recs):
    return _get().stable_perm_bytes(recs)


_default = None


def _get():
    global _default
    if _default is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _default = Oracle(_SO)
    return _default


def planted(plant, directory):
    """An Oracle built with deliberate mistake number `plant` (tests only)."""
    so = os.path.join(directory, f"liboracle_plant{int(plant)}.so")
    build(so, plant)
    return Oracle(so)


def ord_keys(keys):
    return _get().ord_keys(keys)


def stable_perm(keys):
    return _get().stable_perm(keys)


def stable_sort(keys, vals=None):
    return _get().stable_sort(keys, vals)


def segmented_perm(keys, offsets):
    return _get().segmented_perm(keys, offsets)


def segmented_sort(keys, offsets, vals=None):
    return _get().segmented_sort(keys, offsets, vals)


def splitmix64(seed, count):
    return _get().splitmix64(seed, count)


def p_eff(n, p, s, mode):
    return _get().p_eff(n, p, s, mode)


def sample_count(p, s, mode):
    return _get().sample_count(p, s, mode)


def stages(keys, p, s, mode, seed):
    return _get().stages(keys, p, s, mode, seed)


def scatter_grad(grad_y, perm):
    """Backward of a row-wise sort: grad_x[r, perm[r, j]] = grad_y[r, j]
    (a sort is a permutation, so the gradient is routed back through it)."""
    gx = np.zeros_like(grad_y)
    rows = np.arange(grad_y.shape[0])[:, None]
    gx[rows, perm] = grad_y
    return gx
