"""GPU: fixed-width byte strings (the paper's 32-byte string keys, memcmp
order), sorted through their index: the permutation equals the oracle's
stable order and the sorted strings are the input permuted by it."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_08648_amd import api
from paper_1608_08648_amd import workloads
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def _check(recs, prm=None):
    rd = torch.from_numpy(recs).cuda()
    perm, out = api.sort_strings(rd, prm=prm)
    torch.cuda.synchronize()
    want = oracle.stable_perm_bytes(recs)
    np.testing.assert_array_equal(perm.cpu().numpy(), want)
    np.testing.assert_array_equal(out.cpu().numpy(), recs[want])


@pytest.mark.parametrize("kind", workloads.STRING_KINDS)
def test_strings32_kinds(kind):
    """Random strings (one round), strings sharing 8/16/24-byte prefixes
    (runs refined by words 1..3) and 64 distinct strings repeated (runs
    equal in every word: input order kept)."""
    n = (1 << 19) + 123
    recs = workloads.strings32(n, workloads.seed_for(7, workloads.STRING_KINDS.index(kind)), kind)
    note(f"strings32 {kind} n={n}")
    _check(recs)


@pytest.mark.parametrize("n,width", [(1, 32), (2, 8), (100, 16), (5000, 40), (70001, 24)])
def test_strings_sizes_and_widths(n, width):
    g = np.random.default_rng(n + width)
    recs = g.integers(0, 3, (n, width)).astype(np.uint8)       # three byte values: many ties
    note(f"strings n={n} width={width}")
    _check(recs)


def test_strings_user_params_and_no_output():
    recs = workloads.strings32(200_000, workloads.seed_for(7, 5), "prefix")
    rd = torch.from_numpy(recs).cuda()
    note("strings p=64 s=4, permutation only")
    perm, out = api.sort_strings(rd, prm=api.params(p=64, s=4, seed=3), want_sorted=False)
    assert out is None
    np.testing.assert_array_equal(perm.cpu().numpy(), oracle.stable_perm_bytes(recs))


def test_strings32_full_size():
    """2^24 random 32-byte strings (512 MiB)."""
    n = 1 << 24
    recs = workloads.strings32(n, workloads.seed_for(7, 6), "random")
    note("strings32 2^24")
    _check(recs)
