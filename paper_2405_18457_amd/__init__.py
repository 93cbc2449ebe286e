"""MI355X-native hot path of iterative-GP marginal-likelihood optimisation.

The numerical work lives in ``libgpmi.so`` (hand-written HIP for gfx950, C ABI
in ``include/gp.h``); ``api`` is a thin ctypes binding that passes torch
device pointers and torch's current stream.
"""
from . import _native  # noqa: F401

__all__ = ["api", "build", "_native"]
