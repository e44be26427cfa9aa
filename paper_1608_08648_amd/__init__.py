"""MI355X-native oversampling sample sort (arXiv 1608.08648).

The sort runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/samplesort.h``; this package only marshals torch
tensors to it.  The public functions are re-exported from :mod:`.api`.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]


def __getattr__(name):
    # the torch-facing API loads the native library on first use
    from . import api
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)
