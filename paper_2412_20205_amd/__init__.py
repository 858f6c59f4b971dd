"""MI355X (gfx950) extrapolated geometric multigrid for B-spline IGA Poisson problems.

The solver is libigamg.so (HIP kernels + C ABI, include/igamg.h); this package
holds its sources (csrc/), its build script and a thin ctypes binding.
"""
from . import igamg  # noqa: F401
from .igamg import Solver, lib  # noqa: F401
