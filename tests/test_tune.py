"""The autotuner's host logic: its JSON cache (round trip, corrupt files
ignored and replaced), installing a table into the library, filling the
unmeasured size classes, and the paper's priors and Claim 1 arithmetic it
reports.  No GPU needed."""
import ctypes
import json
import math

from paper_1608_08648_amd import native as N
from paper_1608_08648_amd import tune

KEY = "gfx950:256cu"


def _e(form, kw, vw, c, p, s, tile=0):
    return {"form": form, "key_bytes": kw, "val_bytes": vw, "size_class": c, "p": p, "s": s, "tile": tile}


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    ents = [_e(0, 4, 0, 26, 4096, 16), _e(1, 4, 0, 18, 0, 8)]
    tune.save_cache(ents, [{"note": 1}], path, KEY)
    assert tune.load_cache(path, KEY) == ents
    assert tune.load_cache(path, "gfx942:304cu") is None            # another device


def test_corrupt_cache_is_ignored_and_replaced(tmp_path):
    path = str(tmp_path / "t.json")
    for bad in ["{not json", json.dumps([1, 2]), json.dumps({"schema": 99, "devices": {}}),
                json.dumps({"schema": tune.SCHEMA, "devices": {KEY: {"entries": [_e(0, 4, 0, 20, 3, 8)]}}}),
                json.dumps({"schema": tune.SCHEMA, "devices": {KEY: {"entries": [_e(0, 4, 0, 20, 0, 8)]}}}),
                json.dumps({"schema": tune.SCHEMA, "devices": {KEY: {"entries": [{"p": 64}]}}}),
                json.dumps({"schema": tune.SCHEMA, "devices": {KEY: {"entries": []}}})]:
        with open(path, "w") as f:
            f.write(bad)
        assert tune.load_cache(path, KEY) is None, bad
    ents = [_e(0, 4, 0, 20, 512, 8)]
    tune.save_cache(ents, [], path, KEY)                               # rewrites the corrupt file
    assert tune.load_cache(path, KEY) == ents


def test_install_sets_the_library_table():
    try:
        tune.install([_e(0, 4, 0, 21, 256, 4, 65536)])
        out = N.Params()
        assert N.lib().ss_get_tuning(0, N.SS_I32, N.SS_V_NONE, 2**21, ctypes.byref(out)) == 0
        assert (out.p, out.s, out.tile) == (256, 4, 65536)
    finally:
        tune.reset()
    out = N.Params()
    N.lib().ss_get_tuning(0, N.SS_I32, N.SS_V_NONE, 2**21, ctypes.byref(out))
    assert (out.p, out.s, out.tile) != (256, 4, 65536)


def test_fill_classes():
    ents = tune._fill_classes([_e(0, 4, 0, 20, 64, 8), _e(0, 4, 0, 24, 1024, 16), _e(1, 4, 0, 16, 8, 8)])
    single = {e["size_class"]: e for e in ents if e["form"] == 0}
    assert sorted(single) == list(range(33))
    assert single[21]["p"] == 128 and single[21]["s"] == 8          # nearest below (20), bucket size kept
    assert single[23]["p"] == 512 and single[23]["s"] == 16         # nearest above (24)
    assert single[30]["p"] == 4096                                   # capped
    assert single[3]["p"] == 2
    seg = {e["size_class"] for e in ents if e["form"] == 1}
    assert seg == set(range(16, 33))
    assert all(tune._valid_entry(e) for e in ents)


def test_paper_priors():
    pr = tune.paper_priors(2**26)
    assert pr["default_s"] == 676                                    # ceil(26^2)
    assert pr["a_sweep"]["1.0"] == 676 and pr["a_sweep"]["0.2"] == math.ceil(26 ** 1.2)
    assert pr["regular_r"] == [1, 2, 3, 4, 5]


def test_claim1_arithmetic():
    """Claim 1 at n = 2^26, rho = 1: eps = 1 needs s >= 119 for p = 256 and
    s >= 136 for p = 4096 (worked by hand: K = 2 ln n + ln(2 pi p^2 (ps-1))
    + 1/(3(ps-1)) and s >= 2K at eps = 1)."""
    assert tune.claim1_min_s(2**26, 256, 1.0) == 119
    assert tune.claim1_min_s(2**26, 4096, 1.0) == 136
    n, p, s = 2**26, 1024, 200
    eps = tune.claim1_epsilon(n, p, s)
    K = 2 * math.log(n) + math.log(2 * math.pi * p * p * (p * s - 1)) + 1 / (3 * (p * s - 1))
    assert abs(s - (1 + eps) / eps ** 2 * K) < 1e-6                   # the claim's condition, at equality
    e2, bound = tune.claim1_bound(n, p, s)
    assert e2 == eps and bound == math.ceil((1 + eps) * (n - p + 1) / p)
    assert tune.claim1_bound(2**26, 4096, 16)[1] is None             # vacuous at the bench's s
