"""MI355X-native IB-LBM time step (arXiv 2002.08855) behind a C ABI.

The compute path lives in ``csrc/`` (HIP kernels for gfx950 and the C-ABI host
library ``libiblbm.so``); ``binding`` marshals arguments to it through ctypes.  The
binding is loaded lazily so that ``inputs`` (seeded synthetic inputs) can be imported
without touching the GPU library.
"""
import importlib

__all__ = ["binding", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
