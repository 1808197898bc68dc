"""MI355X (gfx950) hybrid low-Mach lattice-Boltzmann / finite-difference time step of
Hosseini, Darabiha, Thevenin (arXiv 2207.11567): HIP kernels behind the C ABI of
include/lbm.h, with a thin Python binding (``Solver``)."""
from .solver import Solver  # noqa: F401
