"""MI355X (gfx950) library for the coupled ferrofluid compound-droplet time step of
arXiv:2410.11129: hybrid finite-difference magnetic potential + phase-field MRT lattice
Boltzmann, as hand-written HIP kernels behind the C ABI of include/fcd.h.

The Python side only marshals arguments (``fcd``) and allocates device memory with
torch (``sim.Channel``).  Importing ``fcd`` functions needs the built ``libfcd.so``;
there is no fallback implementation.
"""
from . import fcd  # noqa: F401

__all__ = ["fcd"]
