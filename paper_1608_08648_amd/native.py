"""ctypes binding of ``libsamplesort.so`` (the C ABI in include/samplesort.h).

The library is built in-tree by :mod:`paper_1608_08648_amd.build`; if it
is missing, :func:`lib` raises instead of falling back to anything else.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libsamplesort.so")

# key types
SS_U32, SS_I32, SS_F32, SS_U64, SS_I64, SS_F64 = range(6)
# payload types
SS_V_NONE, SS_V_B32, SS_V_B64, SS_V_IOTA32, SS_V_IOTA64 = range(5)
# sampling
SS_RANDOM, SS_REGULAR = 0, 1
# flags
SS_F_EXPORT_STAGES = 1
SS_F_FORCE_PIPELINE = 2
SS_F_NO_RECURSION = 4
SS_F_NO_WIDE = 8
SS_F_SORT_FIRST = 16
SS_F_SF_MERGE = 32
# return codes
SS_OK, SS_EINVAL, SS_EWORKSPACE, SS_EHIP, SS_EDEVICE = 0, -1, -2, -3, -4
SS_P_MAX = 4096
SS_MAX_LEVELS = 6

EXPORTS = ("ss_last_error", "ss_workspace_size", "ss_stage_layout", "sample_sort_keys", "sample_sort_pairs",
           "ss_segmented_workspace_size", "segmented_sort", "ss_scatter_grad", "ss_status", "ss_level_stats",
           "ss_set_tuning", "ss_get_tuning", "ss_grad_status", "sample_sort_keys_noalloc",
           "ss_noalloc_capacity_bytes", "ss_strings_workspace_size", "sample_sort_strings",
           "ss_profile_enable", "ss_profile_kinds", "ss_profile_collect", "ss_profile_report")


class Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint32), ("s", ctypes.c_uint32), ("sampling", ctypes.c_int32),
                ("stable", ctypes.c_int32), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("tile", ctypes.c_uint32)]


class StageInfo(ctypes.Structure):
    _fields_ = [("p_eff", ctypes.c_uint32), ("stride", ctypes.c_uint32), ("m", ctypes.c_uint64),
                ("sample_ord", ctypes.c_uint64), ("sample_tag", ctypes.c_uint64), ("spl_ord", ctypes.c_uint64),
                ("spl_tag", ctypes.c_uint64), ("counts", ctypes.c_uint64), ("direct", ctypes.c_uint32),
                ("levels", ctypes.c_uint32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("form", ctypes.c_uint32), ("key_bytes", ctypes.c_uint32), ("val_bytes", ctypes.c_uint32),
                ("size_class", ctypes.c_uint32),
                ("p", ctypes.c_uint32), ("s", ctypes.c_uint32), ("tile", ctypes.c_uint32)]


class LevelInfo(ctypes.Structure):
    _fields_ = [("segments", ctypes.c_uint32), ("buckets", ctypes.c_uint32), ("keys", ctypes.c_uint64),
                ("bucket_keys", ctypes.c_uint64)]


class SortError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"samplesort error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise RuntimeError(f"{SO} is missing: build it with paper_1608_08648_amd.build.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(SO)
        P, SZ, I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        PP = ctypes.POINTER(Params)
        L.ss_last_error.restype = ctypes.c_char_p
        L.ss_last_error.argtypes = []
        L.ss_workspace_size.argtypes = [SZ, I, I, PP, ctypes.POINTER(SZ)]
        L.ss_stage_layout.argtypes = [SZ, I, I, PP, ctypes.POINTER(StageInfo)]
        L.sample_sort_keys.argtypes = [P, P, SZ, I, PP, P, SZ, P]
        L.sample_sort_pairs.argtypes = [P, P, P, P, SZ, I, I, PP, P, SZ, P]
        L.ss_segmented_workspace_size.argtypes = [SZ, SZ, SZ, I, I, PP, ctypes.POINTER(SZ)]
        L.segmented_sort.argtypes = [P, P, P, P, P, SZ, SZ, SZ, I, I, PP, P, SZ, P]
        L.ss_scatter_grad.argtypes = [P, P, P, SZ, SZ, I, P]
        L.ss_status.argtypes = [P, P]
        L.ss_grad_status.argtypes = [P]
        L.sample_sort_keys_noalloc.argtypes = [P, P, SZ, I, PP, P]
        L.ss_noalloc_capacity_bytes.argtypes = []
        L.ss_strings_workspace_size.argtypes = [SZ, ctypes.c_uint32, PP, ctypes.POINTER(SZ)]
        L.sample_sort_strings.argtypes = [P, P, P, SZ, ctypes.c_uint32, PP, P, SZ, P]
        L.ss_level_stats.argtypes = [P, I, ctypes.POINTER(LevelInfo), P]
        L.ss_set_tuning.argtypes = [ctypes.POINTER(TuneEntry), SZ]
        L.ss_get_tuning.argtypes = [I, I, I, SZ, PP]
        L.ss_profile_enable.argtypes = [I, I]
        L.ss_profile_kinds.argtypes = [ctypes.c_uint]
        L.ss_profile_collect.argtypes = []
        L.ss_profile_report.argtypes = [I, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_uint64)]
        for name in EXPORTS:
            if name != "ss_last_error":
                getattr(L, name).restype = I
        L.ss_noalloc_capacity_bytes.restype = SZ
        _lib = L
    return _lib


def check(rc):
    if rc != SS_OK:
        raise SortError(rc, lib().ss_last_error().decode())
    return rc


def last_error():
    return lib().ss_last_error().decode()


def profile_enable(on, max_launches=4096):
    check(lib().ss_profile_enable(1 if on else 0, max_launches))


def profile_kinds(names=None):
    """Bracket only the named kernel kinds (None: every kind)."""
    if names is None:
        check(lib().ss_profile_kinds(0xFFFFFFFF))
        return
    idx = {}
    i = 0
    while True:
        name = ctypes.c_char_p()
        if lib().ss_profile_report(i, ctypes.byref(name), None, None) != SS_OK:
            break
        idx[name.value.decode()] = i
        i += 1
    mask = 0
    for nm in names:
        mask |= 1 << idx[nm]
    check(lib().ss_profile_kinds(mask))


def profile_collect():
    check(lib().ss_profile_collect())


def profile_report():
    """{kernel kind: (total ms, launches)} accumulated since profile_enable."""
    out = {}
    i = 0
    while True:
        name = ctypes.c_char_p()
        ms = ctypes.c_double()
        cnt = ctypes.c_uint64()
        if lib().ss_profile_report(i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(cnt)) != SS_OK:
            break
        out[name.value.decode()] = (ms.value, cnt.value)
        i += 1
    return out
