"""GPU: split-level recursion (buckets beyond one work-group's sort are
sample-sorted again) and the per-level counts the library reports."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_08648_amd import api
from paper_1608_08648_amd import native as N
from paper_1608_08648_amd import workloads
from tests.gpu_util import note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _check_levels(levels, n, p_eff):
    assert levels, "no split level reported"
    assert levels[0]["segments"] == 1 and levels[0]["keys"] == n and levels[0]["buckets"] == p_eff
    for up, lo in zip(levels, levels[1:]):
        # only keys that a level did not sort in place can reach the next one
        assert lo["keys"] <= up["keys"] - up["bucket_keys"]
    assert sum(lv["bucket_keys"] for lv in levels) <= n


@pytest.mark.parametrize("kind", ["keys", "pairs"])
def test_oversize_buckets_go_one_level_down(kind):
    """2^22 int32 keys with p = 32: buckets of ~2^17 keys exceed what one
    work-group sorts (65535 keys for the keys-only slot sort), so every
    bucket is split again by the next level; the result stays bit-exact
    (stable for pairs)."""
    n = 1 << 22
    keys = workloads.keys_2p26(n, "uniform", workloads.seed_for(1, 0), np.int32)
    perm = oracle.stable_perm(keys)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=32, s=16, seed=21)
    vt = N.SS_V_NONE if kind == "keys" else N.SS_V_IOTA32
    ws = api._workspace(api.workspace_size(n, N.SS_I32, vt, prm), kd.device)
    note(f"levels {kind} 2^22 p=32")
    if kind == "keys":
        out = api.sort_keys(kd, prm, ws=ws)
        np.testing.assert_array_equal(out.cpu().numpy(), keys[perm])
    else:
        ko, vo = api.sort_pairs(kd, iota="int32", prm=prm, ws=ws)
        np.testing.assert_array_equal(ko.cpu().numpy(), keys[perm])
        np.testing.assert_array_equal(vo.cpu().numpy(), perm.astype(np.int32))
    levels = api.level_stats(ws)
    _check_levels(levels, n, 32)
    assert len(levels) >= 2 and levels[1]["keys"] == n
    assert api.status(ws) == ""


def test_level_counts_without_recursion_flag():
    """SS_F_NO_RECURSION keeps every bucket at level 0 (oversize buckets are
    sorted by the in-work-group fallbacks): one level, output still exact."""
    n = 1 << 20
    keys = workloads.uniform_u32(n, workloads.seed_for(0))
    kd, kt = to_dev(keys)
    prm = api.params(p=32, s=8, seed=3, flags=N.SS_F_NO_RECURSION)
    ws = api._workspace(api.workspace_size(n, N.SS_U32, N.SS_V_NONE, prm), kd.device)
    note("no recursion 2^20 p=32")
    out = api.sort_keys(kd, prm, ws=ws, key_type=kt)
    np.testing.assert_array_equal(to_host(out, np.uint32), np.sort(keys))
    levels = api.level_stats(ws)
    _check_levels(levels, n, 32)
    assert len(levels) == 1


@pytest.mark.parametrize("dtype", [np.int32, np.uint64])
def test_pairs_without_recursion_merge_in_one_work_group(dtype):
    """Stable pairs with SS_F_NO_RECURSION and p = 16 on 2^20 keys with many
    duplicates: every bucket (~2^16 pairs) is past the stable slot sort, so
    one work-group sorts it in LDS chunks and merges them through global
    memory (reading back what it wrote); keys and an explicit payload must
    equal the oracle's stable order."""
    n = 1 << 20
    g = np.random.default_rng(workloads.seed_for(7))
    keys = g.integers(0, n // 8, size=n).astype(dtype)
    vals = g.integers(0, 2**31 - 1, size=n).astype(np.int32)
    perm = oracle.stable_perm(keys)
    kd = torch.from_numpy(keys.view(np.int64) if dtype == np.uint64 else keys).cuda()
    vd = torch.from_numpy(vals).cuda()
    kt = N.SS_U64 if dtype == np.uint64 else N.SS_I32
    prm = api.params(p=16, s=8, seed=5, flags=N.SS_F_NO_RECURSION)
    ws = api._workspace(api.workspace_size(n, kt, N.SS_V_B32, prm), kd.device)
    note(f"pairs no recursion 2^20 p=16 {np.dtype(dtype).name}")
    ko, vo = api.sort_pairs(kd, vd, prm=prm, ws=ws, key_type="u64" if dtype == np.uint64 else None)
    got = ko.cpu().numpy().view(dtype) if dtype == np.uint64 else ko.cpu().numpy()
    np.testing.assert_array_equal(got, keys[perm])
    np.testing.assert_array_equal(vo.cpu().numpy(), vals[perm])
    levels = api.level_stats(ws)
    assert len(levels) == 1
    # the status notes the fallback (and nothing else): the path was taken
    assert "0x2 " in api.status(ws), api.status(ws)


def test_small_input_reports_no_level():
    """An input that one work-group sorts directly runs no split level."""
    keys = workloads.uniform_u32(1000, 5)
    kd, kt = to_dev(keys)
    prm = api.params(p=64, s=8)
    ws = api._workspace(api.workspace_size(1000, N.SS_U32, N.SS_V_NONE, prm), kd.device)
    out = api.sort_keys(kd, prm, ws=ws, key_type=kt)
    np.testing.assert_array_equal(to_host(out, np.uint32), np.sort(keys))
    assert api.level_stats(ws) == []


def test_level_below_buckets_in_rounds():
    """2^26 int32 keys, p = 256, s = 4: the level below splits the 2^18-key
    buckets with only 4 samples per bucket, so some of its buckets exceed the
    30,464 keys of one slot-sort round.  Those sit in the output buffer (odd
    levels write their buckets there) and must be sorted from a copy: a
    second round re-reads the keys after the first one wrote.  Bit-exact."""
    keys = workloads.keys_2p26(2**26, "uniform", workloads.seed_for(7, 1), np.int32)
    want = keys[oracle.stable_perm(keys)]
    kd = torch.from_numpy(keys).cuda()
    for s, inplace in [(4, False), (4, True)]:
        note(f"levels 2^26 p=256 s={s} in_place={inplace}")
        prm = api.params(p=256, s=s, seed=1234)
        ws = api._workspace(api.workspace_size(2**26, N.SS_I32, N.SS_V_NONE, prm), kd.device)
        src = kd.clone() if inplace else kd
        out = api.sort_keys(src, prm, ws=ws, out=src if inplace else None)
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        lv = api.level_stats(ws)
        assert len(lv) == 2 and lv[1]["keys"] == 2**26
