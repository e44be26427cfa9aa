"""Pins for the CPU oracle: each check rests on something other than the
oracle itself (brute force, a library routine, a closed form, a published
value or a hand-derived example from the paper's rules)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1608_08648_amd import workloads
from tests import golden_io




# ---------------------------------------------------------------- the result

def _bruteforce_perm(keys):
    """The unique permutation pi with (key[pi(r)], pi(r)) strictly
    increasing, found by trying every permutation (Section 1's stability)."""
    n = len(keys)
    perms = np.array(list(itertools.permutations(range(n))), dtype=np.int64)
    comp = keys[perms].astype(np.int64) * n + perms          # (key, index) as one integer
    ok = np.all(np.diff(comp, axis=1) > 0, axis=1) if n > 1 else np.ones(len(perms), bool)
    assert ok.sum() == 1
    return perms[np.argmax(ok)]


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_bruteforce_all_weak_orderings(n):
    """Every weak ordering of n <= 6 items: the oracle's permutation equals the
    one exhaustive search over all n! permutations finds."""
    for keys in workloads.weak_orderings(n):
        keys = np.ascontiguousarray(keys, dtype=np.int32)
        got = oracle.stable_perm(keys)
        if n == 0:
            assert got.size == 0
            continue
        np.testing.assert_array_equal(got, _bruteforce_perm(keys))


@pytest.mark.parametrize("n", [7, 8])
def test_definition_all_weak_orderings(n):
    """n = 7, 8 (47,293 and 545,835 patterns), checked against the
    definition: keys non-decreasing, a permutation, equal keys in input order."""
    pats = workloads.weak_orderings(n)
    flat = np.ascontiguousarray(pats.reshape(-1), dtype=np.int32)
    off = np.arange(0, flat.size + 1, n, dtype=np.int64)
    perm = oracle.segmented_perm(flat, off).reshape(-1, n)
    assert np.all(np.sort(perm, axis=1) == np.arange(n))
    rows = np.arange(len(pats))[:, None]
    k = pats[rows, perm]
    d = np.diff(k, axis=1)
    assert np.all(d >= 0)
    assert np.all((d > 0) | (np.diff(perm, axis=1) > 0))


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.uint64, np.int64, np.float32, np.float64])
def test_matches_numpy_stable_argsort(dtype):
    """numpy's stable argsort computes the same unique permutation (a library
    routine independent of the oracle); keys drawn with many duplicates."""
    g = np.random.default_rng(7)
    for n in [1, 2, 17, 1000, 65537]:
        if np.dtype(dtype).kind == "f":
            keys = (g.integers(-50, 50, n) * 0.25 + 0.125).astype(dtype)   # no zeros, no NaN
        elif np.dtype(dtype).kind == "i":
            info = np.iinfo(dtype)
            keys = np.concatenate([g.integers(-20, 20, n // 2), g.integers(info.min, info.max, n - n // 2)])
            keys = g.permutation(keys).astype(dtype)
        else:
            info = np.iinfo(dtype)
            keys = np.concatenate([g.integers(0, 40, n // 2),
                                   g.integers(0, info.max, n - n // 2, dtype=dtype)]).astype(dtype)
            keys = g.permutation(keys)
        np.testing.assert_array_equal(oracle.stable_perm(keys), np.argsort(keys, kind="stable"))


def test_float_total_order():
    """IEEE 754 totalOrder: -NaN < -inf < -1 < -0 < +0 < 1 < +inf < +NaN."""
    bits = np.array([0xFFC00000, 0xFF800000, 0xBF800000, 0x80000000,
                     0x00000000, 0x3F800000, 0x7F800000, 0x7FC00000], dtype=np.uint32)
    vals = bits.view(np.float32)
    o = oracle.ord_keys(vals)
    assert np.all(np.diff(o.astype(np.float64)) > 0) and np.all(np.diff(o) > 0)
    sh = np.random.default_rng(3).permutation(len(vals))
    np.testing.assert_array_equal(vals[sh][oracle.stable_perm(vals[sh])].view(np.uint32), bits)


def test_double_total_order():
    """IEEE 754 totalOrder for binary64: -NaN < -inf < -1 < -0 < +0 < 1 < +inf < +NaN."""
    bits = np.array([0xFFF8000000000000, 0xFFF0000000000000, 0xBFF0000000000000, 0x8000000000000000,
                     0x0000000000000000, 0x3FF0000000000000, 0x7FF0000000000000, 0x7FF8000000000000],
                    dtype=np.uint64)
    vals = bits.view(np.float64)
    o = oracle.ord_keys(vals)
    assert np.all(np.diff(o) > 0)
    sh = np.random.default_rng(4).permutation(len(vals))
    np.testing.assert_array_equal(vals[sh][oracle.stable_perm(vals[sh])].view(np.uint64), bits)
    # -0 and +0 compare equal as floats but sort apart, each keeping input order
    z = np.array([0.0, -0.0, 0.0, -0.0], dtype=np.float64)
    np.testing.assert_array_equal(oracle.stable_perm(z), [1, 3, 0, 2])


def test_segmented_matches_numpy():
    keys, off = workloads.segmented_keys(50, 11, max_log2=10)
    perm = oracle.segmented_perm(keys, off)
    for g in range(len(off) - 1):
        seg = keys[off[g]:off[g + 1]]
        np.testing.assert_array_equal(perm[off[g]:off[g + 1]], np.argsort(seg, kind="stable"))


def test_scatter_grad_is_transpose_of_permutation():
    """For y = P x (rows sorted by a permutation), dL/dx = P^T dL/dy."""
    g = np.random.default_rng(5)
    x = g.standard_normal((3, 9))
    gy = g.standard_normal((3, 9))
    perm = np.stack([np.argsort(r, kind="stable") for r in x])
    gx = oracle.scatter_grad(gy, perm)
    for r in range(3):
        P = np.zeros((9, 9))
        P[np.arange(9), perm[r]] = 1.0                   # y = P x
        np.testing.assert_allclose(gx[r], P.T @ gy[r], rtol=0, atol=0)


# ---------------------------------------------------------------- SplitMix64

def test_splitmix64_published_vector():
    seed, vals = golden_io.splitmix64_vectors()
    np.testing.assert_array_equal(oracle.splitmix64(seed, len(vals)), np.array(vals, dtype=np.uint64))


def test_random_positions_scale_exactly():
    """Sample tags are floor(r * n / 2^64) for the SplitMix64 draws, checked
    with Python integers at an n that needs the full 128-bit product."""
    keys = np.zeros(12345, dtype=np.uint32)        # all equal: sample order = tag order
    for seed in [0, 1, 99, 2**63 + 5]:
        st = oracle.stages(keys, 8, 3, oracle.RANDOM, seed)
        r = oracle.splitmix64(seed, 8 * 3 - 1)
        want = sorted((int(v) * 12345) >> 64 for v in r)
        np.testing.assert_array_equal(st["sample_tag"], np.array(want, dtype=np.uint64))


# ---------------------------------------------------------------- the steps

@pytest.mark.parametrize("case", golden_io.stage_cases(), ids=lambda c: c["name"])
def test_golden_stages(case):
    st = oracle.stages(case["keys"], case["p"], case["s"], case["mode"], case["seed"])
    assert list(zip(st["sample_ord"].tolist(), st["sample_tag"].tolist())) == case["sample"]
    assert list(zip(st["spl_ord"].tolist(), st["spl_tag"].tolist())) == case["splitters"]
    assert st["counts"].tolist() == case["counts"]


def _bruteforce_counts(keys, spl):
    """Step 4 by exhaustive comparison: bucket = number of splitters
    (key, index) strictly below the key's own (key, index)."""
    cnt = [0] * (len(spl) + 1)
    for i, k in enumerate(keys.tolist()):
        b = sum(1 for (so, sp) in spl if (so, sp) < (k, i))
        cnt[b] += 1
    return cnt


@pytest.mark.parametrize("mode", [oracle.RANDOM, oracle.REGULAR])
def test_counts_bruteforce(mode):
    g = np.random.default_rng(21)
    for trial in range(40):
        n = int(g.integers(40, 400))
        p = int(2 ** g.integers(1, 4))
        s = int(g.integers(1, 4))
        if oracle.p_eff(n, p, s, mode) < p:
            continue
        kind = trial % 4
        keys = [g.integers(0, 2**32, n), g.integers(0, 3, n), np.sort(g.integers(0, 50, n)),
                np.full(n, 9)][kind].astype(np.uint32)
        st = oracle.stages(keys, p, s, mode, int(g.integers(0, 2**32)))
        spl = list(zip(st["spl_ord"].tolist(), st["spl_tag"].tolist()))
        assert spl == sorted(spl)
        assert st["counts"].tolist() == _bruteforce_counts(keys, spl)
        np.testing.assert_array_equal(st["perm"], np.argsort(keys, kind="stable"))


@pytest.mark.parametrize("mode", [oracle.RANDOM, oracle.REGULAR])
def test_method_reaches_the_sorted_result(mode):
    """The concatenation of the sorted buckets is the stable sorted order."""
    for dist in workloads.DISTRIBUTIONS:
        keys = workloads.keys_2p26(20000, dist, 77)
        for p, s in [(4, 2), (16, 4), (64, 1)]:
            q = oracle.p_eff(keys.size, p, s, mode)
            if q < 2:
                continue
            st = oracle.stages(keys, q, s, mode, 1234)
            np.testing.assert_array_equal(st["perm"], oracle.stable_perm(keys))
            assert st["counts"].sum() == keys.size


def test_lemma1_bucket_bound_regular():
    """Lemma 1: with regular oversampling no bucket exceeds the bound,
    for any input (uniform, few values, sorted, reverse, all equal,
    periodic), because tags make every key distinct (Section 2.2)."""
    g = np.random.default_rng(5)
    checked = 0
    for trial in range(300):
        p = int(2 ** g.integers(1, 5))
        s = int(g.integers(1, 6))
        n = int(g.integers(4 * s * p * p, 4 * s * p * p + 3000))
        kind = trial % 6
        keys = [g.integers(0, 2**32, n), g.integers(0, 4, n), np.arange(n), np.arange(n)[::-1],
                np.full(n, 3), np.arange(n) % 7][kind].astype(np.uint32)
        keys = np.ascontiguousarray(keys)
        assert oracle.p_eff(n, p, s, oracle.REGULAR) == p
        st = oracle.stages(keys, p, s, oracle.REGULAR, 0)
        safe, tight, final = oracle.lemma1_bounds(n, p, s)
        mx = int(st["counts"].max())
        assert mx <= tight <= safe, (n, p, s, kind, mx, tight)
        assert mx <= final + 1e-9, (n, p, s, kind, mx, final)
        checked += 1
    assert checked == 300


def test_lemma1_bounds_hand_worked():
    """The bound the Lemma 1 tests check against, pinned to values worked by
    hand from the lemma's proof (tests/golden/lemma1.txt)."""
    cases = golden_io.lemma1_cases()
    assert len(cases) >= 4
    for n, p, r, safe, tight, final in cases:
        got = oracle.lemma1_bounds(n, p, r)
        assert got[0] == safe and got[1] == tight, (n, p, r, got)
        assert abs(got[2] - final) < 1e-9, (n, p, r, got)


def test_p_eff_closed_forms():
    R, G = oracle.RANDOM, oracle.REGULAR
    # 2^20 keys, p=64, s=8 regular: 4*8*64^2 = 2^17 <= 2^20
    assert oracle.p_eff(2**20, 64, 8, G) == 64
    # 2^26 keys regular: p^2 s <= 2^24
    assert oracle.p_eff(2**26, 256, 32, G) == 256
    assert oracle.p_eff(2**26, 1024, 16, G) == 1024
    assert oracle.p_eff(2**26, 1024, 32, G) == 512
    assert oracle.p_eff(2**26, 4096, 4, G) == 2048
    assert oracle.p_eff(2**26, 4096, 8, G) == 1024
    # random: p*s < n/2
    assert oracle.p_eff(2**26, 4096, 32, R) == 4096
    assert oracle.p_eff(100, 64, 1, R) == 32
    assert oracle.p_eff(100, 64, 2, R) == 16
    assert oracle.p_eff(4, 64, 1, R) == 1          # 2*2*1 = 4 is not < 4
    assert oracle.p_eff(5, 64, 1, R) == 2
    assert oracle.p_eff(1, 2, 1, R) == 1
    # p is rounded down to a power of two
    assert oracle.p_eff(2**20, 100, 4, R) == 64


# ------------------------------------------------------------ string keys

def _strings(n, width, alphabet, g, prefix=0):
    recs = g.integers(0, alphabet, (n, width)).astype(np.uint8)
    if prefix:
        recs[:, :prefix] = recs[0, :prefix]          # a common prefix: ties in the leading words
    return recs


def test_bytes_order_matches_python_sorted():
    """The stable memcmp order equals Python's sort of (bytes, index) tuples
    (bytes compare as unsigned byte strings), on tiny alphabets with many
    ties and on full-range bytes."""
    g = np.random.default_rng(21)
    for n, width, alphabet in [(1, 4, 2), (6, 3, 2), (50, 5, 3), (400, 32, 256), (300, 9, 2)]:
        recs = _strings(n, width, alphabet, g)
        want = sorted(range(n), key=lambda i: (bytes(recs[i]), i))
        np.testing.assert_array_equal(oracle.stable_perm_bytes(recs), want)


def test_bytes_order_brute_force_tiny():
    """n <= 5: the permutation is the only one whose (record, index) sequence
    strictly increases, found by trying every permutation."""
    g = np.random.default_rng(22)
    for n in range(1, 6):
        for _ in range(20):
            recs = _strings(n, 2, 2, g)
            key = [(bytes(recs[i]), i) for i in range(n)]
            good = [pm for pm in itertools.permutations(range(n))
                    if all(key[pm[k]] < key[pm[k + 1]] for k in range(n - 1))]
            assert len(good) == 1
            np.testing.assert_array_equal(oracle.stable_perm_bytes(recs), good[0])


def test_bytes_order_matches_numpy_lexsort_on_words():
    """32-byte strings with a shared 16-byte prefix: equal to numpy's stable
    lexsort on the four big-endian 64-bit words (a library routine that
    never compares bytes)."""
    g = np.random.default_rng(23)
    recs = _strings(20000, 32, 4, g, prefix=16)
    words = recs.view(">u8").astype(np.uint64)           # [n, 4] big-endian words
    want = np.lexsort((words[:, 3], words[:, 2], words[:, 1], words[:, 0]))
    np.testing.assert_array_equal(oracle.stable_perm_bytes(recs), want)
