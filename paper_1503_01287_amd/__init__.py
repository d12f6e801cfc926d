"""MI355X (gfx950) algebraic multigrid for hierarchical quadratic finite
element systems (Yang, arXiv:1503.01287): separated linear/quadratic
coarsening, Galerkin coarse operators on the GPU, AMG-preconditioned CG and
flexible Krylov solves. The compute path is the HIP library libamgp2.so
(C ABI in include/amg_p2.h); this package binds it and builds its inputs.
"""
from . import problems
from ._lib import AmgError, lib
from .solver import AMGSolver, BatchedSolver, SolveResult, parse_smoother

__all__ = ["AMGSolver", "BatchedSolver", "SolveResult", "AmgError", "lib", "problems", "parse_smoother"]
