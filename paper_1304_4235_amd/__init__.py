"""MI355X reverse ray tracer: self-shielded photoionisation rates of SPH gas.

The work runs in librrt.so (hand-written HIP kernels for gfx950, C ABI in
include/rrt.h); this package only binds it.  Importing fails if the library
has not been built (python paper_1304_4235_amd/build.py).
"""
from .rrt import RRTError, Solver, healpix_dirs, lib, LIB_PATH, SIGNATURES  # noqa: F401

__all__ = ["Solver", "RRTError", "healpix_dirs", "lib", "LIB_PATH", "SIGNATURES"]
