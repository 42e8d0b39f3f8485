"""MI355X library for the row/column-sampling Monte Carlo estimator of
matrix functions on sparse graphs (subgraph centrality diag(f(sA)) and total
communicability f(sA) v).

The compute path is the HIP library ``libmcmf.so`` (sources in ``csrc/``,
C ABI in ``include/mcmf.h``); :mod:`paper_2308_01037_amd.mcmf` is its
ctypes binding.  ``python -m paper_2308_01037_amd.build`` compiles it.
"""
import importlib

__all__ = ["mcmf", "build"]


def __getattr__(name):
    if name in ("mcmf", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    mod = importlib.import_module(f"{__name__}.mcmf")
    try:
        return getattr(mod, name)
    except AttributeError:
        raise AttributeError(f"module {__name__!r} has no attribute {name!r}") from None
