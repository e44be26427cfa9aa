"""The pins catch plausible mistakes: each test builds the oracle with one
deliberate error (on the CPU) and shows that a pin from test_oracle.py
rejects it.  The correct oracle passes the same checks."""
import numpy as np
import pytest

import oracle
from tests import golden_io


def _golden_ok(orc):
    for c in golden_io.stage_cases():
        st = orc.stages(c["keys"], c["p"], c["s"], c["mode"], c["seed"])
        if list(zip(st["sample_ord"].tolist(), st["sample_tag"].tolist())) != c["sample"]:
            return False
        if list(zip(st["spl_ord"].tolist(), st["spl_tag"].tolist())) != c["splitters"]:
            return False
        if st["counts"].tolist() != c["counts"]:
            return False
    return True


def _stable_ok(orc):
    g = np.random.default_rng(1)
    for n in [5, 50, 500]:
        keys = g.integers(-3, 3, n).astype(np.int32)
        if not np.array_equal(orc.stable_perm(keys), np.argsort(keys, kind="stable")):
            return False
    return True


def _lemma1_ok(orc):
    for n, p, r, safe, tight, final in golden_io.lemma1_cases():
        got = orc.lemma1_bounds(n, p, r)
        if got[0] != safe or got[1] != tight or abs(got[2] - final) > 1e-9:
            return False
    return True


def _bytes_ok(orc):
    g = np.random.default_rng(9)
    recs = g.integers(0, 3, (500, 32)).astype(np.uint8)
    recs[:, :10] = 1                                   # shared 10-byte prefix
    want = sorted(range(500), key=lambda i: (bytes(recs[i]), i))
    return bool(np.array_equal(orc.stable_perm_bytes(recs), want))


CASES = {
    1: ("merge takes the right run on equal keys", _stable_ok),
    2: ("splitter rank off by one", _golden_ok),
    3: ("a splitter opens its bucket instead of closing it", _golden_ok),
    4: ("padded segment length rounded down", _golden_ok),
    5: ("tags ignored when keys are equal", _golden_ok),
    6: ("signed keys compared without the sign flip", _stable_ok),
    7: ("Lemma 1 segment length rounded down", _lemma1_ok),
    8: ("string keys compared on their first 8 bytes only", _bytes_ok),
}


def test_correct_oracle_passes():
    assert _golden_ok(oracle._get()) and _stable_ok(oracle._get()) and _lemma1_ok(oracle._get()) \
        and _bytes_ok(oracle._get())


@pytest.mark.parametrize("plant", sorted(CASES))
def test_planted_mistake_is_caught(plant, tmp_path):
    what, check = CASES[plant]
    bad = oracle.planted(plant, str(tmp_path))
    assert not check(bad), f"planted mistake not caught: {what}"
