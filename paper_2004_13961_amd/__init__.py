"""MI355X (gfx950) preconditioned Legendre-Galerkin PCG solver.

C ABI: include/lgpcg.h, built into liblgpcg.so by paper_2004_13961_amd.build.
Python: lgpcg (ctypes binding), solver (Problem, Factor, pcg_solve),
workload (nodal data of the benchmark coefficient family).
"""
from .lgpcg import LgpError, gauss_legendre, lib  # noqa: F401

__all__ = ["LgpError", "gauss_legendre", "lib"]
