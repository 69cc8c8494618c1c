"""CPU oracle for the AMG-preconditioned reduced-Hessian solve.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
statement of what the GPU library computes, written from the paper
(Barker & Draganescu, "Algebraic multigrid preconditioning of the Hessian in
PDE-constrained optimization", arXiv:2001.11533).  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the GPU
library and its Python binding never do, and share no code with it.

Modules
  csr     minimal CSR container, ordered (left-to-right) segment sums, stable
          transpose
  fem     P1 finite-element assembly of the stiffness and mass matrices
          (Section 2: the matrices A, M_y, M_u, M_yu)
  sa      smoothed-aggregation hierarchy (Section 3.1 names smoothed
          aggregation as the AMG used to fix ideas; eqs. coarsestiffness and
          coarsemass give the Galerkin coarse matrices)
  solve   V-cycle, PCG, state/adjoint solves, Hessian action, the multilevel
          Hessian preconditioner (Section 3.2, Algorithm MLAS, and its
          practical form of Section 5.2) and the outer CG (Section 5.3)
  dense   explicit dense operators for tiny meshes (reduced Hessian,
          two-grid and multilevel preconditioners in the paper's own
          M_u-inner-product form) used to pin the sparse code

Every function states the passage it follows.  See the test-suite for the
pins (closed forms, invariants, brute force) that tie this code to the paper.
"""
