"""MI355X-native staggered-grid incompressible Navier-Stokes hot path (arXiv 2604.18536).

The computation lives in the gfx950 HIP library ``libins.so`` behind the C ABI
of ``include/ins.h``; this package only marshals torch tensors to it.
"""
from ._lib import InsError, LIB_PATH  # noqa: F401
from .solver import Solver  # noqa: F401

__all__ = ["Solver", "InsError", "LIB_PATH"]
