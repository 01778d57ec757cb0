"""MI355X (gfx950) implementation of the coupled Grand-Potential phase-field /
lattice-Boltzmann time step: HIP kernels behind the C ABI of include/gpf.h,
with a thin ctypes binding (gpf.Sim)."""
from . import workloads  # noqa: F401

__all__ = ["workloads", "gpf"]
