"""Host (CPU) comparator: the paper's multi-core McRan on this machine's
cores (``mcran.c``, plain C with pthreads, built with gcc).

It gives the GPU sort's benchmark an apples-to-apples CPU reference on the
same host: the paper's own method and organisation (sort the p blocks on t
threads, sample, split by binary search, p-way merge per bucket).  Nothing
in the GPU sort calls it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcran.c")
_SO = os.path.join(_HERE, "libmcran.so")
_lib = None


def build(verbose=False):
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P, U64, U32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        L.mcran_sort_i32.argtypes = [P, P, U64, U32, U32, U64, U32, U32, P]
        L.mcran_sort_i32.restype = ctypes.c_int
        _lib = L
    return _lib


def mcran_sort(keys, p, s, threads, seed=1, merge_threads=1):
    """Sort int32 keys with McRan: returns (sorted copy, seconds per step:
    blocks, sample, split, merge, total).  The input is not modified."""
    x = np.array(keys, dtype=np.int32, copy=True)
    y = np.empty_like(x)
    t = np.zeros(5, dtype=np.float64)
    rc = lib().mcran_sort_i32(x.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p), x.size, p, s,
                              seed & (2**64 - 1), threads, merge_threads, t.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError("mcran: bad arguments or out of memory")
    return y, {"blocks_s": t[0], "sample_s": t[1], "split_s": t[2], "merge_s": t[3], "total_s": t[4]}
