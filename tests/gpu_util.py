"""Helpers for the GPU tests: numpy <-> device tensors for every key type."""
import numpy as np
import torch

_VIEW = {np.dtype(np.uint32): (np.int32, "u32"), np.dtype(np.uint64): (np.int64, "u64")}


def to_dev(a):
    """(device tensor, key_type override or None) holding a's bytes."""
    a = np.ascontiguousarray(a)
    if a.dtype in _VIEW:
        v, kt = _VIEW[a.dtype]
        return torch.from_numpy(a.view(v)).cuda(), kt
    return torch.from_numpy(a).cuda(), None


def to_host(t, dtype):
    return t.cpu().numpy().view(dtype)


def note(msg):
    """Name the case before a GPU step (shows with -s; the test id shows with -v)."""
    import sys
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()
