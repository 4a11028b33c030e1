"""MI355X-native explicit finite-volume shallow-water step (Delmas &
Soulaimani, arXiv 2010.14416, sections 2-3): HIP kernels for gfx950 behind the
C interface of include/swe.h, with a thin ctypes binding (``swe``)."""
from . import swe  # noqa: F401
from .swe import Ensemble, Solver, SweError, load  # noqa: F401

__all__ = ["swe", "Ensemble", "Solver", "SweError", "load"]
