"""MI355X (gfx950) SPOD hot path: HIP kernels behind the C ABI of include/spod.h.

The Python layer only marshals arguments; see `spod.Plan`.
"""
from .spod import Batch, OutOfCore, Plan, PRECISIONS, lib, shape  # noqa: F401
from ._native import SpodError  # noqa: F401
from .autograd import spod, SpodFunction  # noqa: F401
