"""Plain FP64 CPU oracle for the algebraic multigrid method of Yang,
"An algebraic multigrid method for quadratic finite element equations of
elliptic and saddle point systems in 3D" (arXiv:1503.01287).

TEST INFRASTRUCTURE ONLY. Nothing in the GPU library or its Python binding
may import, call, link or execute anything in this package; only the tests,
the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle is written to be read against the paper: slow, direct and in FP64.
It shares no code with the GPU path. Modules:

* ``mesh``    Kuhn tetrahedral mesh of the unit cube and P2 node numbering.
* ``fem``     hierarchical quadratic / Taylor-Hood assembly with exact
              barycentric integration, Neumann loads, Dirichlet elimination
              (Section 2, equations for the weak forms and block systems).
* ``amg``     separated coarsening, block-diagonal prolongation, Galerkin
              coarse operators, smoothers and Algorithm 1 (Section 3).
* ``krylov``  PCG, flexible CG and flexible GMRES drivers.
* ``mlp``     FP64 reference of the damping-weight network (gradient checks).
* ``reduced`` the cycle on operators rounded as a reduced-precision
              preconditioner stores them (FP32 finest, BF16 with row
              scales below), computed in FP64.
* ``loops.c`` the inherently sequential loops (greedy independent set,
              greedy colouring, Gauss-Seidel sweeps) in plain C.
* ``threaded`` (with ``omp_loops.c``) the order-independent loops (block and
              transfer products, Gauss-Seidel within a colour, Jacobi) on
              every host core, for timing the oracle there; the results
              equal the sequential ones (bit for bit for the sweeps).

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
