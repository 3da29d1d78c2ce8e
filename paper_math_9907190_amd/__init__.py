"""Diagonally oriented multigrid V-cycle for the Poisson equation on MI355X.

The solver is libdmg.so (HIP kernels for gfx950 behind the C ABI in
include/dmg.h); ``paper_math_9907190_amd.dmg`` is its Python binding.
Importing the package itself loads nothing, so the input generators in
``paper_math_9907190_amd.workloads`` work on machines without a GPU.
"""

__all__ = ["dmg", "workloads"]
