"""amghess: AMG-preconditioned reduced-Hessian solves on MI355X (gfx950).

Barker & Draganescu, "Algebraic multigrid preconditioning of the Hessian in
PDE-constrained optimization" (arXiv:2001.11533): the linear-quadratic
elliptic control problem min 1/2||y - y_d||^2 + beta/2||u||^2 subject to
-div(kappa grad y) = u, solved through (K^T M_y K + beta M_u) u = K^T M_y y_d
by CG with the multilevel Hessian preconditioner built from a
smoothed-aggregation hierarchy.  The computation lives in the HIP library
libamghess.so (C ABI in include/amghess.h); this package is its binding.
"""
from ._lib import AmgError, LIB_PATH  # noqa: F401


def __getattr__(name):
    if name in ("HessianSolver", "assemble_p1", "assemble_p1_device", "default_opts", "release_memory"):
        from . import solver
        return getattr(solver, name)
    if name in ("StateSolve", "MassQuad", "reduced_functional"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
