"""MI355X-native lensless RF volumetric rendering (GeRaF, arXiv 2605.29097).

The compute lives in ``librfvr.so`` (HIP, gfx950) behind the C ABI of
``include/rfvr.h``; :mod:`.rfvr` is its thin ctypes binding and
:mod:`.autograd` wraps the forward/adjoint pairs as torch autograd functions.
"""
from . import rfvr  # noqa: F401

__all__ = ["rfvr"]
