"""GPU: the wide split (keys only, 4-byte keys, p >= 1024): the same
buckets as the paper's one-pass split of step 4, moved in two passes, tie
keys written back as runs.  Bit-exact against the oracle; bucket counts
against the oracle's stages and against the one-pass split (SS_F_NO_WIDE)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_08648_amd import api
from paper_1608_08648_amd import native as N
from paper_1608_08648_amd import workloads
from tests.gpu_util import note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _sorted_by_oracle(keys):
    return keys[oracle.stable_perm(keys)]


@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_wide_six_distributions(dist):
    """2^22 + 12345 int32 keys (a ragged last tile) in each distribution,
    p = 1024, s = 8: bit-exact."""
    n = (1 << 22) + 12345
    keys = workloads.keys_2p26(n, dist, workloads.seed_for(5, workloads.DISTRIBUTIONS.index(dist)), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=1024, s=8, seed=71)
    ws = api._workspace(api.workspace_size(n, N.SS_I32, N.SS_V_NONE, prm), kd.device)
    note(f"wide {dist} n={n}")
    out = api.sort_keys(kd, prm, ws=ws)
    np.testing.assert_array_equal(out.cpu().numpy(), _sorted_by_oracle(keys))
    lv = api.level_stats(ws)
    assert len(lv) == 1 and lv[0]["buckets"] == 1024 and lv[0]["keys"] == n


@pytest.mark.parametrize("mod", [0, 1000, 3])
def test_wide_stage_counts_equal_oracle(mod):
    """Bucket counts of the wide split equal the oracle's (key, position)
    classification, also with heavy duplicates (keys mod 1000, mod 3), where
    most keys are ties of a splitter."""
    n = 1 << 20
    keys = workloads.uniform_u32(n, workloads.seed_for(0) + mod)
    if mod:
        keys = (keys % np.uint32(mod)).astype(np.uint32)
    kd, kt = to_dev(keys)
    prm = api.params(p=1024, s=4, seed=99)
    note(f"wide stages mod={mod}")
    out, st, info = api.stages(kd, prm, key_type=kt)
    ref = oracle.stages(keys, 1024, 4, oracle.RANDOM, 99)
    assert info.p_eff == 1024
    np.testing.assert_array_equal(st["spl_ord"], ref["spl_ord"])
    np.testing.assert_array_equal(st["spl_tag"], ref["spl_tag"])
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    np.testing.assert_array_equal(to_host(out, np.uint32), keys[ref["perm"]])


def test_wide_equals_one_pass_split():
    """The wide split and the one-pass split give the same buckets and the
    same output."""
    n = (1 << 21) + 3
    keys = workloads.keys_2p26(n, "gaussian", workloads.seed_for(5, 1), np.int32)
    kd = torch.from_numpy(keys).cuda()
    outs, counts = [], []
    for flags in (0, N.SS_F_NO_WIDE):
        prm = api.params(p=2048, s=8, seed=5, flags=flags)
        note(f"wide vs one-pass flags={flags}")
        out, st, _ = api.stages(kd, prm)
        outs.append(out.cpu().numpy())
        counts.append(st["counts"])
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(counts[0], counts[1])
    np.testing.assert_array_equal(outs[0], np.sort(keys))


def test_wide_in_place():
    """keys_in == keys_out: the stage is the workspace copy and the bucket
    sort runs in place."""
    n = (1 << 22) + 1
    keys = workloads.keys_2p26(n, "uniform", workloads.seed_for(5, 0), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=4096, s=8, seed=8)
    note("wide in place")
    out = api.sort_keys(kd, prm, out=kd)
    assert out.data_ptr() == kd.data_ptr()
    np.testing.assert_array_equal(kd.cpu().numpy(), _sorted_by_oracle(keys))


@pytest.mark.parametrize("dtype", [np.float32, np.uint32])
def test_wide_key_types(dtype):
    """float32 (totalOrder image: negatives, -0.0/+0.0) and uint32 keys."""
    n = 1 << 21
    g = np.random.default_rng(12)
    if dtype == np.float32:
        keys = g.standard_normal(n).astype(np.float32)
        keys[::1000] = -0.0
        keys[1::1000] = 0.0
    else:
        keys = g.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    kd, kt = to_dev(keys)
    prm = api.params(p=1024, s=16, seed=3)
    note(f"wide {np.dtype(dtype).name}")
    out = api.sort_keys(kd, prm, key_type=kt)
    want = _sorted_by_oracle(keys)
    np.testing.assert_array_equal(to_host(out, dtype).view(np.uint32), want.view(np.uint32))


def test_wide_large_buckets_sorted_in_rounds():
    """2^24 + 777 keys with p = 1024, s = 16: buckets average 16K keys, so
    the bucket sort takes its two-work-groups-per-CU layout (16,000 keys a
    round); the largest pass 30K keys and take two or three rounds."""
    n = (1 << 24) + 777
    keys = workloads.keys_2p26(n, "uniform", workloads.seed_for(5, 2), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=1024, s=16, seed=17)
    note("wide rounds 2^24 p=1024")
    out, st, _ = api.stages(kd, prm)
    assert st["counts"].max() > 30720 - 48
    np.testing.assert_array_equal(out.cpu().numpy(), _sorted_by_oracle(keys))


def test_wide_regular_sampling():
    """Regular oversampling (Alg. 1) with p = 1024, s = 1 on 2^22 keys:
    splitters and counts equal the oracle's, buckets within Lemma 1."""
    n = 1 << 22
    keys = workloads.uniform_u32(n, workloads.seed_for(0) + 7)
    kd, kt = to_dev(keys)
    prm = api.params(p=1024, s=1, sampling="regular")
    note("wide regular 2^22 p=1024 s=1")
    out, st, info = api.stages(kd, prm, key_type=kt)
    assert info.p_eff == 1024
    ref = oracle.stages(keys, 1024, 1, oracle.REGULAR, 0)
    np.testing.assert_array_equal(st["spl_ord"], ref["spl_ord"])
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    assert st["counts"].max() <= oracle.lemma1_bounds(n, 1024, 1)[1]
    np.testing.assert_array_equal(to_host(out, np.uint32), keys[ref["perm"]])


def test_wide_buckets_beyond_16_bit_counters():
    """No level below (SS_F_NO_RECURSION), p = 1024, s = 4 on 2^25 + 12345
    keys: buckets average 32K keys and many exceed 65535, which the bucket
    sort takes with 32-bit slot counters in several rounds.  Counts equal
    the oracle's; output bit-exact."""
    n = (1 << 25) + 12345
    keys = workloads.keys_2p26(n, "uniform", workloads.seed_for(5, 3), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=1024, s=4, seed=29, flags=N.SS_F_NO_RECURSION)
    note("wide 2^25 p=1024 s=4 no recursion")
    out, st, info = api.stages(kd, prm)
    ref = oracle.stages(keys, 1024, 4, oracle.RANDOM, 29)
    assert info.p_eff == 1024
    np.testing.assert_array_equal(st["counts"], ref["counts"])
    assert st["counts"].max() > 65535
    np.testing.assert_array_equal(out.cpu().numpy(), keys[ref["perm"]])


def test_wide_in_place_buckets_in_rounds():
    """keys_in == keys_out without a level below (SS_F_NO_RECURSION), p =
    1024, s = 4 on 2^25 + 3 keys: buckets average 32K keys, so the bucket
    sort re-reads most of them in several rounds (some with 32-bit slot
    counters) while it writes the output; it must read a copy the output
    does not overwrite."""
    n = (1 << 25) + 3
    keys = workloads.keys_2p26(n, "uniform", workloads.seed_for(5, 4), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=1024, s=4, seed=31, flags=N.SS_F_NO_RECURSION)
    note("wide in place 2^25 p=1024 s=4 rounds")
    out = api.sort_keys(kd, prm, out=kd)
    assert out.data_ptr() == kd.data_ptr()
    np.testing.assert_array_equal(kd.cpu().numpy(), _sorted_by_oracle(keys))


@pytest.mark.parametrize("in_place", [False, True])
def test_wide_small_layout_many_rounds(in_place):
    """2^25 + 5 keys with p = 1024, s = 16: a mean bucket of 32K keys with
    s >= 16 still takes the layout of 16,000 keys a round, and the largest
    buckets need three rounds or more (each re-reading the bucket while
    earlier rounds wrote their part of the output).  In place too."""
    n = (1 << 25) + 5
    keys = workloads.keys_2p26(n, "uniform", workloads.seed_for(5, 6), np.int32)
    kd = torch.from_numpy(keys).cuda()
    prm = api.params(p=1024, s=16, seed=37)
    note(f"wide small layout 2^25 p=1024 s=16 in_place={in_place}")
    if in_place:
        out = api.sort_keys(kd, prm, out=kd)
        assert out.data_ptr() == kd.data_ptr()
        got = kd.cpu().numpy()
    else:
        out, st, _ = api.stages(kd, prm)
        assert st["counts"].max() > 2 * (16000 - 256)   # three rounds or more
        got = out.cpu().numpy()
    np.testing.assert_array_equal(got, _sorted_by_oracle(keys))


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_wide_unaligned_input(offset):
    """Keys starting 4, 8 or 12 bytes past a 16-byte boundary (a view into a
    larger tensor) take the count pass's one-key-at-a-time loads; the result
    is the same bit-exact sort."""
    n = (1 << 21) + 777
    keys = workloads.keys_2p26(n + offset, "gaussian", workloads.seed_for(5, 9), np.int32)
    big = torch.from_numpy(keys).cuda()
    kd = big[offset:]
    assert kd.data_ptr() % 16 != 0
    prm = api.params(p=2048, s=16, seed=5)
    note(f"wide unaligned offset={offset}")
    out = api.sort_keys(kd, prm)
    np.testing.assert_array_equal(out.cpu().numpy(), _sorted_by_oracle(keys[offset:]))
