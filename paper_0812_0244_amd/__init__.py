"""MI355X-native factorised vdW-DF nonlocal correlation (Roman-Perez & Soler).

The compute path is the HIP library ``libvdwnl.so`` (C ABI in
``include/vdwnl.h``); this package only marshals arguments to it.
"""
from .binding import VdwNl, VdwNlError, load_library  # noqa: F401

__all__ = ["VdwNl", "VdwNlError", "load_library", "NonlocalCorrelation", "VdwDF", "VdwNlEnergy"]


def __getattr__(name):
    if name in ("NonlocalCorrelation", "VdwDF", "VdwNlEnergy"):
        from . import torch_fn
        return getattr(torch_fn, name)
    raise AttributeError(name)
