"""The C ABI library: loads, exports what include/samplesort.h declares, and
its host-only logic (planning, argument checks) behaves -- no GPU needed,
nothing here launches a kernel."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle
from paper_1608_08648_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "samplesort.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    assert set(names) == set(N.EXPORTS), names


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", N.SO], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for name in declared_functions():
        assert name in exported, name


def _ws(n, kt, vt=N.SS_V_NONE, **kw):
    prm = N.Params(p=kw.get("p", 1024), s=kw.get("s", 8), sampling=kw.get("sampling", 0), stable=1,
                   seed=1, flags=kw.get("flags", 0), tile=kw.get("tile", 0))
    out = ctypes.c_size_t()
    rc = N.lib().ss_workspace_size(n, kt, vt, ctypes.byref(prm), ctypes.byref(out))
    return rc, out.value


def _layout(n, kt, vt=N.SS_V_NONE, **kw):
    prm = N.Params(p=kw.get("p", 1024), s=kw.get("s", 8), sampling=kw.get("sampling", 0), stable=1,
                   seed=1, flags=kw.get("flags", 0), tile=0)
    info = N.StageInfo()
    rc = N.lib().ss_stage_layout(n, kt, vt, ctypes.byref(prm), ctypes.byref(info))
    return rc, info


def test_workspace_sizes():
    rc, b = _ws(2**26, N.SS_I32, p=4096, s=16)
    assert rc == 0 and b >= 4 * 2**26            # at least one copy of the keys
    rc, b2 = _ws(2**26, N.SS_I32, p=256, s=16)
    assert rc == 0 and b2 >= 4 * 2**26
    rc, b3 = _ws(2**27, N.SS_U64, N.SS_V_B32, p=4096, s=16)
    assert rc == 0 and b3 >= 12 * 2**27
    rc, b4 = _ws(100, N.SS_I32)                   # fits one work-group: no workspace data copy
    assert rc == 0 and b4 < 4096


@pytest.mark.parametrize("mode", [0, 1])
def test_effective_p_matches_the_oracle_rule(mode):
    """The library's p_eff is the oracle's: the largest power of two <= p
    with p <= n, p*s < n/2 (random) or 4*s*p^2 <= n (regular)."""
    for n in [40000, 100000, 2**20, 2**22 + 17, 2**26]:
        for p in [2, 64, 256, 1024, 4096]:
            for s in [1, 4, 8, 32]:
                rc, info = _layout(n, N.SS_U32, p=p, s=s, sampling=mode, flags=N.SS_F_FORCE_PIPELINE)
                assert rc == 0
                want = oracle.p_eff(n, p, s, mode)
                if want < 2:
                    assert info.direct == 1
                else:
                    assert info.p_eff == want, (n, p, s, mode)
                    assert info.m == oracle.sample_count(want, s, mode)
                    assert info.stride == (s if mode == 0 else s * want)


def test_small_inputs_sort_directly():
    rc, info = _layout(1000, N.SS_I32, p=64, s=4)
    assert rc == 0 and info.direct == 1 and info.p_eff == 1
    rc, info = _layout(1000, N.SS_I32, p=64, s=4, flags=N.SS_F_FORCE_PIPELINE)
    assert rc == 0 and info.direct == 0 and info.p_eff == 64


def test_levels_are_planned_for_large_buckets():
    rc, info = _layout(2**26, N.SS_I32, p=256, s=8)
    assert rc == 0 and info.levels >= 1          # 2^18-key buckets need another split
    rc, info = _layout(2**26, N.SS_I32, p=256, s=8, flags=N.SS_F_NO_RECURSION)
    assert rc == 0 and info.levels == 0


@pytest.mark.parametrize("bad", [dict(p=3), dict(p=1), dict(p=8192), dict(s=0), dict(sampling=7)])
def test_bad_parameters_rejected(bad):
    rc, _ = _ws(1 << 20, N.SS_I32, **bad)
    assert rc == N.SS_EINVAL
    assert N.last_error()


def test_bad_types_rejected():
    assert _ws(100, 9)[0] == N.SS_EINVAL
    assert _ws(100, N.SS_I32, 9)[0] == N.SS_EINVAL


def test_sort_first_flag():
    """SS_F_SORT_FIRST (the organisation of Alg. 1 / Alg. 2: blocks sorted
    first) plans no level below, and its workspace holds the sorted blocks
    (keys and in-block indices) and the p x (p + 1) run table; 8-byte keys
    and payloads plan the gathered buckets' segmented sort too, and the
    pairwise merge of step 5 (SS_F_SF_MERGE) takes 4-byte keys without
    payload only."""
    SF = N.SS_F_SORT_FIRST
    for kt in (N.SS_I32, N.SS_U32, N.SS_F32):
        rc, b = _ws(2**26, kt, p=4096, s=16, flags=SF)
        assert rc == 0 and b >= 3 * 4 * 2**26 + 4 * 4096 * 4097
        for mode in (0, 1):
            rc, info = _layout(2**22, kt, p=256, s=4, sampling=mode, flags=SF)
            assert rc == 0 and info.levels == 0 and info.p_eff == 256
    for kt, vt in ((N.SS_U64, N.SS_V_NONE), (N.SS_I32, N.SS_V_B32), (N.SS_F64, N.SS_V_B64),
                   (N.SS_I64, N.SS_V_IOTA64)):
        rc, b = _ws(2**22, kt, vt, p=1024, s=8, flags=SF)
        kw = 4 if kt in (N.SS_U32, N.SS_I32, N.SS_F32) else 8
        # sorted blocks + in-block index, the stage, the run table
        assert rc == 0 and b >= (2 * kw + 4) * 2**22 + 4 * 1024 * 1025
        rc, info = _layout(2**22, kt, p=256, s=4, flags=SF)
        assert rc == 0 and info.levels == 0 and info.p_eff == 256
        assert _ws(2**22, kt, vt, p=1024, s=8, flags=SF | N.SS_F_SF_MERGE)[0] == N.SS_EINVAL
        assert "SF_MERGE" in N.last_error()


def _prm():
    return N.Params(p=1024, s=8, sampling=0, stable=1, seed=0, flags=0, tile=0)


def test_calls_rejected_before_any_launch():
    L = N.lib()
    P = ctypes.c_void_p
    prm = _prm()
    # n = 0 is a no-op
    assert L.sample_sort_keys(None, None, 0, N.SS_I32, ctypes.byref(prm), None, 0, None) == 0
    # NULL keys
    assert L.sample_sort_keys(None, P(4096), 10, N.SS_I32, ctypes.byref(prm), None, 0, None) == N.SS_EINVAL
    # workspace too small (checked on the host)
    rc = L.sample_sort_keys(P(1 << 20), P(1 << 30), 1 << 20, N.SS_I32, ctypes.byref(prm), P(1 << 40), 16, None)
    assert rc == N.SS_EWORKSPACE
    # partial overlap of input and output
    rc = L.sample_sort_keys(P(1 << 20), P((1 << 20) + 64), 1000, N.SS_I32, ctypes.byref(prm), P(1 << 40),
                            1 << 30, None)
    assert rc == N.SS_EINVAL
    # pairs: no payload type / iota with a payload pointer / missing payload
    assert L.sample_sort_pairs(P(4096), P(8192), P(1 << 20), P(1 << 21), 10, N.SS_I32, N.SS_V_NONE,
                               ctypes.byref(prm), None, 0, None) == N.SS_EINVAL
    assert L.sample_sort_pairs(P(4096), P(8192), P(1 << 20), P(1 << 21), 10, N.SS_I32, N.SS_V_IOTA32,
                               ctypes.byref(prm), None, 0, None) == N.SS_EINVAL
    assert L.sample_sort_pairs(P(4096), None, P(1 << 20), P(1 << 21), 10, N.SS_I32, N.SS_V_B32,
                               ctypes.byref(prm), None, 0, None) == N.SS_EINVAL
    # scatter_grad: element size / aliasing / empty
    assert L.ss_scatter_grad(P(4096), P(8192), P(1 << 20), 2, 3, 3, None) == N.SS_EINVAL
    assert L.ss_scatter_grad(P(4096), P(8192), P(4096), 2, 3, 4, None) == N.SS_EINVAL
    assert L.ss_scatter_grad(None, None, None, 0, 5, 4, None) == 0
    # segmented: no segments is a no-op; NULL offsets rejected
    assert L.segmented_sort(P(4096), None, P(8192), None, None, 0, 0, 0, N.SS_I32, 0, None, None, 0, None) == 0
    assert L.segmented_sort(P(4096), None, P(8192), None, None, 3, 10, 5, N.SS_I32, 0, None, None, 0,
                            None) == N.SS_EINVAL


def test_segmented_workspace():
    out = ctypes.c_size_t()
    L = N.lib()
    # every segment fits one work-group: only the control block and the small list
    assert L.ss_segmented_workspace_size(20000 * 100, 20000, 100, N.SS_I32, 0, None, ctypes.byref(out)) == 0
    small = out.value
    assert L.ss_segmented_workspace_size(20000 * 100, 20000, 2**20, N.SS_I32, 0, None, ctypes.byref(out)) == 0
    assert out.value > small


def test_int64_index_payload_planned_narrow():
    """A 64-bit index payload (IOTA64) is planned as a 32-bit one plus a
    buffer of n 32-bit indices that is widened at the end: its workspace is
    the IOTA32 plan's plus 4n bytes (rounded to the 256-byte alignment), for
    single arrays and for segments."""
    for n, p in [(2**20 + 5, 256), (2**26, 4096), (1000, 64)]:
        rc32, b32 = _ws(n, N.SS_F32, N.SS_V_IOTA32, p=p)
        rc64, b64 = _ws(n, N.SS_F32, N.SS_V_IOTA64, p=p)
        assert rc32 == 0 and rc64 == 0
        assert b64 - b32 == ((b32 + 255) // 256 * 256 - b32) + 4 * n
    L = N.lib()
    out32, out64 = ctypes.c_size_t(), ctypes.c_size_t()
    total, nseg, maxlen = 64 * 2**18, 64, 2**18
    assert L.ss_segmented_workspace_size(total, nseg, maxlen, N.SS_F32, N.SS_V_IOTA32, None, ctypes.byref(out32)) == 0
    assert L.ss_segmented_workspace_size(total, nseg, maxlen, N.SS_F32, N.SS_V_IOTA64, None, ctypes.byref(out64)) == 0
    assert out64.value - out32.value == ((out32.value + 255) // 256 * 256 - out32.value) + 4 * total


def _tuned(form, kt, vt, n):
    out = N.Params()
    assert N.lib().ss_get_tuning(form, kt, vt, n, ctypes.byref(out)) == 0, N.last_error()
    return out.p, out.s, out.tile


def test_tuning_table_set_get_restore():
    L = N.lib()
    try:
        assert L.ss_set_tuning(None, 0) == 0
        # built-in: keys-only int32 at 2^26 takes 4096 buckets
        assert _tuned(0, N.SS_I32, N.SS_V_NONE, 2**26)[0] == 4096
        E = (N.TuneEntry * 2)(N.TuneEntry(0, 4, 0, 20, 512, 8, 65536), N.TuneEntry(1, 4, 0, 18, 16, 4, 0))
        assert L.ss_set_tuning(E, 2) == 0
        assert _tuned(0, N.SS_I32, N.SS_V_NONE, 2**20) == (512, 8, 65536)
        assert _tuned(0, N.SS_U32, N.SS_V_NONE, 2**19 + 1) == (512, 8, 65536)     # same class (2^19, 2^20]
        assert _tuned(0, N.SS_I32, N.SS_V_NONE, 2**19) != (512, 8, 65536)
        assert _tuned(1, N.SS_I32, N.SS_V_NONE, 2**18)[:2] == (16, 4)
        assert _tuned(0, N.SS_I32, N.SS_V_B32, 2**20) != (512, 8, 65536)          # other payload width
        # a 64-bit index payload is tuned as a 4-byte one
        assert _tuned(0, N.SS_F32, N.SS_V_IOTA64, 2**20) == _tuned(0, N.SS_F32, N.SS_V_B32, 2**20)
        # an invalid entry is refused and the table stays as it was
        bad = (N.TuneEntry * 1)(N.TuneEntry(0, 4, 0, 20, 3, 8, 0))
        assert L.ss_set_tuning(bad, 1) == N.SS_EINVAL
        assert _tuned(0, N.SS_I32, N.SS_V_NONE, 2**20) == (512, 8, 65536)
        bad = (N.TuneEntry * 1)(N.TuneEntry(0, 4, 0, 33, 64, 8, 0))
        assert L.ss_set_tuning(bad, 1) == N.SS_EINVAL
        bad = (N.TuneEntry * 1)(N.TuneEntry(0, 4, 0, 20, 0, 8, 0))                # p = 0: segmented only
        assert L.ss_set_tuning(bad, 1) == N.SS_EINVAL
        # workspace sizes follow the table when prm is NULL
        out = ctypes.c_size_t()
        assert L.ss_workspace_size(2**20, N.SS_I32, N.SS_V_NONE, None, ctypes.byref(out)) == 0
        prm = N.Params(p=512, s=8, sampling=0, stable=1, seed=0x5EED, flags=0, tile=65536)
        out2 = ctypes.c_size_t()
        assert L.ss_workspace_size(2**20, N.SS_I32, N.SS_V_NONE, ctypes.byref(prm), ctypes.byref(out2)) == 0
        assert out.value == out2.value
    finally:
        assert L.ss_set_tuning(None, 0) == 0
    assert _tuned(0, N.SS_I32, N.SS_V_NONE, 2**20) != (512, 8, 65536)


def test_strings_workspace_and_refusals():
    L = N.lib()
    out = ctypes.c_size_t()
    assert L.ss_strings_workspace_size(1 << 20, 32, None, ctypes.byref(out)) == 0
    assert out.value >= (1 << 20) * 32                   # words, index, runs and the sorts' workspaces
    for w in (0, 7, 12, 264):
        assert L.ss_strings_workspace_size(1000, w, None, ctypes.byref(out)) == N.SS_EINVAL
    P = ctypes.c_void_p
    # unaligned strings, or no permutation output: refused before any launch
    assert L.sample_sort_strings(P(4097), None, P(8192), 10, 32, None, P(1 << 20), 1 << 30, None) == N.SS_EINVAL
    assert L.sample_sort_strings(P(4096), None, None, 10, 32, None, P(1 << 20), 1 << 30, None) == N.SS_EINVAL
    assert L.sample_sort_strings(P(4096), P(4096), P(8192), 10, 32, None, P(1 << 20), 1 << 30, None) == N.SS_EINVAL
    assert L.sample_sort_strings(P(4096), None, P(8192), 10, 32, None, None, 0, None) == N.SS_EWORKSPACE
