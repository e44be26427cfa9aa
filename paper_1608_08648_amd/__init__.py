"""MI355X-native oversampling sample sort (arXiv 1608.08648).

The sort runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/samplesort.h``; :mod:`.api` only marshals torch
tensors to it (``sort_keys``, ``sort_pairs``, ``segmented_sort``,
``scatter_grad``, ``SortFn``/``sort``).
"""
import importlib

_SUBMODULES = ("api", "native", "workloads", "build", "tune")


def __getattr__(name):
    if name in _SUBMODULES:
        return importlib.import_module(f"{__name__}.{name}")
    api = importlib.import_module(f"{__name__}.api")
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)
