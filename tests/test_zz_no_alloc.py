"""The no-allocation entry point (sample_sort_keys_noalloc, static scratch)
against the workspace entry point (sample_sort_keys) through the C ABI: two
calls in a row, the second on a smaller input, each bit-exact to the
workspace call; an input too large for the static array is refused before
anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1608_08648_amd import api
from paper_1608_08648_amd import native as N
from paper_1608_08648_amd import workloads
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def _ws_sort(kd, kt):
    n = kd.numel()
    out = torch.empty_like(kd)
    ws = api._workspace(api.workspace_size(n, kt, N.SS_V_NONE, None), kd.device)
    N.check(N.lib().sample_sort_keys(ctypes.c_void_p(kd.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, kt, None,
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), api._stream()))
    return out


def _noalloc_sort(kd, kt, out):
    N.check(N.lib().sample_sort_keys_noalloc(ctypes.c_void_p(kd.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             kd.numel(), kt, None, api._stream()))
    return out


def test_noalloc_matches_the_workspace_entry_point_twice():
    L = N.lib()
    cap = L.ss_noalloc_capacity_bytes()
    assert cap == 64 << 20
    cases = [(1 << 22, np.int32, N.SS_I32, 1), (100_003, np.float32, N.SS_F32, 2)]
    for n, dt, kt, seed in cases:
        assert api.workspace_size(n, kt, N.SS_V_NONE, None) <= cap
        g = np.random.default_rng(seed)
        if dt == np.int32:
            keys = workloads.keys_2p26(n, "uniform", workloads.seed_for(9, seed), np.int32)
        else:
            keys = g.standard_normal(n).astype(np.float32)
        kd = torch.from_numpy(keys).cuda()
        note(f"noalloc n={n} {np.dtype(dt).name}")
        want = _ws_sort(kd, kt)
        got = torch.full_like(kd, 7)
        _noalloc_sort(kd, kt, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        np.testing.assert_array_equal(got.cpu().numpy(), np.sort(keys, kind="stable"))


def test_noalloc_refuses_inputs_beyond_the_scratch():
    L = N.lib()
    n = 1 << 24
    assert api.workspace_size(n, N.SS_I32, N.SS_V_NONE, None) > L.ss_noalloc_capacity_bytes()
    kd = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = torch.full_like(kd, 3)
    rc = L.sample_sort_keys_noalloc(ctypes.c_void_p(kd.data_ptr()), ctypes.c_void_p(out.data_ptr()), n, N.SS_I32,
                                    None, api._stream())
    assert rc == N.SS_EWORKSPACE and "static scratch" in N.last_error()
    torch.cuda.synchronize()
    assert bool((out == 3).all())
