"""The host McRan comparator sorts: its output equals numpy's sort for
uniform, duplicate-heavy, sorted and reverse inputs, any p (1, small, = n),
threads above p, and a parallel merge step."""
import numpy as np
import pytest

from paper_1608_08648_amd import host


@pytest.mark.parametrize("n,p,s,t,mt", [(1, 4, 4, 2, 1), (1000, 1, 8, 4, 1), (1000, 16, 8, 4, 1),
                                        (5000, 64, 3, 8, 1), (777, 777, 1, 3, 2), (200_000, 256, 16, 8, 4),
                                        (65_537, 32, 1000, 40, 1)])
def test_mcran_equals_numpy(n, p, s, t, mt):
    g = np.random.default_rng(n + p)
    for kind in range(4):
        keys = [g.integers(-2**31, 2**31, n), g.integers(-3, 3, n), np.arange(n), np.arange(n)[::-1]][kind]
        keys = keys.astype(np.int32)
        y, times = host.mcran_sort(keys, p, s, t, seed=kind, merge_threads=mt)
        np.testing.assert_array_equal(y, np.sort(keys))
        assert times["total_s"] >= 0.0


def test_mcran_rejects_bad_arguments():
    with pytest.raises(ValueError):
        host.mcran_sort(np.arange(10, dtype=np.int32), 0, 4, 2)
