"""GPU: the sort-first organisation (SS_F_SORT_FIRST), Alg. 1 / Alg. 2 as
stated: blocks sorted first (step 1), the splitters placed in every sorted
block by binary search (step 4), bucket j formed from the runs X_{k,j} and
sorted (step 5).  Bit-exact against the oracle; bucket counts against the
oracle's stages (the same (key, index) order decides both)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_08648_amd import api
from paper_1608_08648_amd import native as N
from paper_1608_08648_amd import workloads
from tests.gpu_util import note, to_dev, to_host

pytestmark = pytest.mark.gpu

SF = N.SS_F_SORT_FIRST


def _sorted_by_oracle(keys):
    return keys[oracle.stable_perm(keys)]


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_sort_first_six_distributions(dist):
    """2^22 + 12345 int32 keys (ragged blocks) in each distribution, p =
    1024, s = 8, random sampling: bit-exact, every key in a bucket."""
    n = (1 << 22) + 12345
    keys = workloads.keys_2p26(n, dist, workloads.seed_for(6, workloads.DISTRIBUTIONS.index(dist)), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=1024, s=8, seed=72, flags=SF)
    ws = api._workspace(api.workspace_size(n, N.SS_I32, N.SS_V_NONE, prm), kd.device)
    note(f"sort-first {dist} n={n}")
    out = api.sort_keys(kd, prm, ws=ws)
    np.testing.assert_array_equal(out.cpu().numpy(), _sorted_by_oracle(keys))


@pytest.mark.parametrize("mode,p,s", [(oracle.RANDOM, 256, 4), (oracle.REGULAR, 256, 4), (oracle.RANDOM, 4096, 2)])
@pytest.mark.parametrize("mod", [0, 1000])
def test_sort_first_counts_equal_oracle(mode, p, s, mod):
    """Bucket counts (the sizes of the concatenated runs X_{k,j}) and
    splitters equal the oracle's, with distinct keys and with heavy
    duplicates (keys mod 1000), under both sampling rules."""
    n = 1 << 20
    keys = workloads.uniform_u32(n, workloads.seed_for(0) + 11 + mod)
    if mod:
        keys = (keys % np.uint32(mod)).astype(np.uint32)
    kd, kt = to_dev(keys)
    sampling = "regular" if mode == oracle.REGULAR else "random"
    prm = api.params(p=p, s=s, seed=5, sampling=sampling, flags=SF)
    note(f"sort-first stages mode={mode} p={p} s={s} mod={mod}")
    out, st, info = api.stages(kd, prm, key_type=kt)
    ref = oracle.stages(keys, p, s, mode, 5)
    assert info.p_eff == p
    np.testing.assert_array_equal(st["spl_ord"], ref["spl_ord"])
    np.testing.assert_array_equal(st["spl_tag"], ref["spl_tag"])
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    np.testing.assert_array_equal(to_host(out, np.uint32), keys[ref["perm"]])


@pytest.mark.parametrize("dtype", [np.float32, np.uint32])
def test_sort_first_key_types(dtype):
    """float32 (totalOrder image: negatives, -0.0/+0.0) and uint32 keys."""
    n = (1 << 21) + 7
    g = np.random.default_rng(13)
    if dtype == np.float32:
        keys = g.standard_normal(n).astype(np.float32)
        keys[::1000] = -0.0
        keys[1::1000] = 0.0
    else:
        keys = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    kd, kt = to_dev(keys)
    prm = api.params(p=512, s=16, seed=4, flags=SF)
    note(f"sort-first {np.dtype(dtype).name}")
    out = api.sort_keys(kd, prm, key_type=kt)
    want = _sorted_by_oracle(keys)
    np.testing.assert_array_equal(to_host(out, dtype).view(np.uint32), want.view(np.uint32))


def test_sort_first_in_place_and_large_blocks():
    """keys_in == keys_out, and blocks of 64K keys (p = 64 on 2^22 keys):
    the splitter search then runs on the sorted block in global memory (no
    LDS copy past 16K keys) and buckets of ~64K keys take the slot sort in
    rounds, some with 32-bit counters."""
    n = 1 << 22
    keys = workloads.keys_2p26(n, "gaussian", workloads.seed_for(6, 9), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=64, s=16, seed=8, flags=SF)
    note("sort-first in place p=64")
    out = api.sort_keys(kd, prm, out=kd)
    assert out.data_ptr() == kd.data_ptr()
    np.testing.assert_array_equal(kd.cpu().numpy(), _sorted_by_oracle(keys))


def test_sort_first_full_size():
    """2^26 int32 keys, p = 4096, s = 16, random and regular sampling (the
    benchmarked size): bit-exact."""
    keys = workloads.keys_2p26(2**26, "uniform", workloads.seed_for(1, 0), np.int32)
    want = keys[oracle.stable_perm(keys)]
    kd = torch.from_numpy(keys).cuda()
    for sampling, p, s in [("random", 4096, 16), ("regular", 1024, 4)]:
        note(f"sort-first 2^26 {sampling} p={p} s={s}")
        prm = api.params(p=p, s=s, seed=1234, sampling=sampling, flags=SF)
        ws = api._workspace(api.workspace_size(2**26, N.SS_I32, N.SS_V_NONE, prm), kd.device)
        out = api.sort_keys(kd, prm, ws=ws)
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        assert api.status(ws) == ""


@pytest.mark.parametrize("n,p,s,mode", [(5000, 4096, 8, oracle.RANDOM), (3001, 64, 2, oracle.RANDOM),
                                        (40000, 32, 4, oracle.REGULAR), (1 << 16, 2, 1, oracle.RANDOM)])
def test_sort_first_small_inputs(n, p, s, mode):
    """Small inputs forced through the pipeline (SS_F_FORCE_PIPELINE): the
    effective p shrinks by the paper's preconditions (here to 256, 64, 32
    and 2), blocks hold a few dozen keys, n is not a multiple of p.  Bucket
    counts and output equal the oracle's."""
    keys = workloads.uniform_u32(n, workloads.seed_for(0) + n)
    keys[::7] = keys[3]                      # duplicates across blocks
    kd, kt = to_dev(keys)
    sampling = "regular" if mode == oracle.REGULAR else "random"
    prm = api.params(p=p, s=s, seed=19, sampling=sampling, flags=SF | N.SS_F_FORCE_PIPELINE)
    note(f"sort-first small n={n} p={p} s={s} mode={mode}")
    out, st, info = api.stages(kd, prm, key_type=kt)
    pe = oracle.p_eff(n, p, s, mode)
    assert info.p_eff == pe
    ref = oracle.stages(keys, pe, s, mode, 19)
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    np.testing.assert_array_equal(to_host(out, np.uint32), keys[ref["perm"]])


SFM = SF | N.SS_F_SF_MERGE


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_sort_first_merge_six_distributions(dist):
    """Step 5 as the paper states it (SS_F_SF_MERGE: each bucket's p runs
    merged pairwise in lg p rounds): 2^22 + 12345 int32 keys in each
    distribution, p = 1024, s = 8, bit-exact."""
    n = (1 << 22) + 12345
    keys = workloads.keys_2p26(n, dist, workloads.seed_for(6, workloads.DISTRIBUTIONS.index(dist)), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=1024, s=8, seed=72, flags=SFM)
    note(f"sort-first merge {dist} n={n}")
    out = api.sort_keys(kd, prm)
    np.testing.assert_array_equal(out.cpu().numpy(), _sorted_by_oracle(keys))


@pytest.mark.parametrize("mode,p,s", [(oracle.RANDOM, 256, 4), (oracle.REGULAR, 256, 4), (oracle.RANDOM, 4096, 2),
                                      (oracle.RANDOM, 2, 1)])
def test_sort_first_merge_counts_and_large_buckets(mode, p, s):
    """Bucket counts equal the oracle's; p = 256 on 2^20 keys gives buckets
    around 4K keys, and p = 2 buckets of 2^19 keys, past the merge's LDS
    (gathered and sorted by the leftover sort instead)."""
    n = 1 << 20
    keys = workloads.uniform_u32(n, workloads.seed_for(0) + 31 + p)
    keys[::5] = keys[1]
    kd, kt = to_dev(keys)
    sampling = "regular" if mode == oracle.REGULAR else "random"
    prm = api.params(p=p, s=s, seed=5, sampling=sampling, flags=SFM)
    note(f"sort-first merge stages mode={mode} p={p} s={s}")
    out, st, info = api.stages(kd, prm, key_type=kt)
    pe = oracle.p_eff(n, p, s, mode)
    assert info.p_eff == pe
    ref = oracle.stages(keys, pe, s, mode, 5)
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    np.testing.assert_array_equal(to_host(out, np.uint32), keys[ref["perm"]])


def test_sort_first_merge_full_size_in_place():
    """2^26 int32 keys, p = 4096, s = 16, step 5 by merging, in place."""
    keys = workloads.keys_2p26(2**26, "uniform", workloads.seed_for(1, 0), np.int32)
    want = keys[oracle.stable_perm(keys)]
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=4096, s=16, seed=1234, flags=SFM)
    ws = api._workspace(api.workspace_size(2**26, N.SS_I32, N.SS_V_NONE, prm), kd.device)
    note("sort-first merge 2^26 p=4096 in place")
    api.sort_keys(kd, prm, out=kd, ws=ws)
    np.testing.assert_array_equal(kd.cpu().numpy(), want)
    assert api.status(ws) == ""


# 8-byte keys and payloads: step 5 gathers each bucket's runs with the
# payload of every key and sorts the p buckets as segments.

def _keys64(n, kind, seed):
    g = np.random.default_rng(seed)
    if kind == "u64":
        k = g.integers(0, 2**64 - 1, n, dtype=np.uint64, endpoint=True)
        k[::9] = k[4]                            # duplicates across blocks
    elif kind == "i64":
        k = g.integers(-2**40, 2**40, n, dtype=np.int64)
        k[::11] = -7
    else:
        k = g.standard_normal(n) * 1e6
        k[::1000] = -0.0
        k[1::1000] = 0.0
        k[2::13] = 3.5
    return k


@pytest.mark.parametrize("kind", ["u64", "i64", "f64"])
@pytest.mark.parametrize("mode,p,s", [(oracle.RANDOM, 1024, 8), (oracle.REGULAR, 256, 4), (oracle.RANDOM, 64, 16)])
def test_sort_first_8byte_keys_counts(kind, mode, p, s):
    """8-byte keys under both sampling rules: splitters and bucket counts
    (sizes of the concatenated runs) equal the oracle's, the output is the
    oracle's stable order bit for bit.  2^20 + 333 keys: ragged blocks; p =
    64 gives blocks of 16K 8-byte keys, past the search's LDS copy."""
    n = (1 << 20) + 333
    keys = _keys64(n, kind, 100 + p + mode)
    kd, kt = to_dev(keys)
    sampling = "regular" if mode == oracle.REGULAR else "random"
    prm = api.params(p=p, s=s, seed=23, sampling=sampling, flags=SF)
    note(f"sort-first 8-byte {kind} mode={mode} p={p} s={s}")
    out, st, info = api.stages(kd, prm, key_type=kt)
    pe = oracle.p_eff(n, p, s, mode)
    assert info.p_eff == pe
    ref = oracle.stages(keys, pe, s, mode, 23)
    np.testing.assert_array_equal(st["spl_ord"], ref["spl_ord"])
    np.testing.assert_array_equal(st["spl_tag"], ref["spl_tag"])
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    np.testing.assert_array_equal(to_host(out, keys.dtype).view(np.uint64), keys[ref["perm"]].view(np.uint64))


@pytest.mark.parametrize("kdt,vform", [(np.int32, "b32"), (np.int32, "iota64"), (np.uint64, "b64"),
                                       (np.float64, "iota32"), (np.uint64, "b32"), (np.float32, "b64")])
@pytest.mark.parametrize("sampling", ["random", "regular"])
def test_sort_first_pairs(kdt, vform, sampling):
    """Pairs under sort-first: every payload width (stored 4 / 8 bytes, the
    stable permutation as 32- or 64-bit index) with 4- and 8-byte keys.
    Keys and payloads equal the oracle's stable order element by element."""
    n = (1 << 21) + 4099
    g = np.random.default_rng([np.dtype(kdt).itemsize, len(vform), int(vform[-2:]), len(sampling)])
    if kdt in (np.float32, np.float64):
        keys = g.standard_normal(n).astype(kdt)
    elif kdt == np.int32:
        keys = g.integers(-5000, 5000, n, dtype=np.int32)         # many equal keys
    else:
        keys = g.integers(0, 2**64 - 1, n, dtype=np.uint64, endpoint=True)
        keys[::3] = keys[10]
    kd, kt = to_dev(keys)
    perm = oracle.stable_perm(keys)
    prm = api.params(p=512, s=8, seed=9, sampling=sampling, flags=SF)
    note(f"sort-first pairs {np.dtype(kdt).name} {vform} {sampling}")
    if vform.startswith("iota"):
        ko, vo = api.sort_pairs(kd, None, prm, iota="int32" if vform == "iota32" else "int64", key_type=kt)
        np.testing.assert_array_equal(vo.cpu().numpy().astype(np.int64), perm)
    else:
        vdt = np.uint32 if vform == "b32" else np.uint64
        vals = g.integers(0, np.iinfo(vdt).max, n, dtype=vdt, endpoint=True)
        vd, _ = to_dev(vals)
        ko, vo = api.sort_pairs(kd, vd, prm, key_type=kt)
        np.testing.assert_array_equal(to_host(vo, vdt), vals[perm])
    w = np.uint32 if np.dtype(kdt).itemsize == 4 else np.uint64
    np.testing.assert_array_equal(to_host(ko, kdt).view(w), keys[perm].view(w))


def test_sort_first_pairs_in_place_full_size():
    """2^26 uint64 keys with a 4-byte payload (the duplicate-heavy pairs
    workload: keys on [0, 0.7 n)), p = 4096, s = 16, keys and payload
    sorted in place (keys_out == keys_in, vals_out == vals_in)."""
    n = 1 << 26
    keys, vals = workloads.pairs_dup(n, workloads.seed_for(3, 1))
    vals ^= np.uint32(0x5A5A5A5A)
    perm = oracle.stable_perm(keys)
    kd, kt = to_dev(keys)
    vd, _ = to_dev(vals)
    prm = api.params(p=4096, s=16, seed=3, flags=SF)
    ws = api._workspace(api.workspace_size(n, N.SS_U64, N.SS_V_B32, prm), kd.device)
    note("sort-first pairs 2^26 u64/u32 in place")
    api.sort_pairs(kd, vd, prm, keys_out=kd, vals_out=vd, ws=ws, key_type=kt)
    np.testing.assert_array_equal(to_host(kd, np.uint64), keys[perm])
    np.testing.assert_array_equal(to_host(vd, np.uint32), vals[perm])
    assert api.status(ws) == ""
