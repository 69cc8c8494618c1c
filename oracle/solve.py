"""Solve phase of the oracle (test infrastructure only).

What is solved (paper, Section 5.2, eq. firstorderpractice): the symmetric
practical form (K^T M_y K + beta M_u) u = K^T M_y y_d with K = A^{-1} M_yu
(eq. solutionopdef), i.e. H_0 u = b.  H_j := M_{u,j} G_j at every level j.

  * inner solves with A_j: CG preconditioned by one AMG V-cycle from level j
    (Section 5.2 uses AMG-preconditioned CG for every application of K and
    K^*); the V-cycle uses nu l1-Jacobi pre/post sweeps and the dense Cholesky
    solve on the coarsest AMG level;
  * mass solves M_{u,j}^{-1}: CG preconditioned by the diagonal of M_{u,j}
    (the paper uses a symmetric Gauss-Seidel sweep; Jacobi is the
    order-independent choice for a GPU, only iteration counts change);
  * the multilevel preconditioner B_j ~ H_j^{-1} (Section 3.2, eqs.
    twogridinmulti, twogridinmultiactual, twogridinmultiactualfine and
    Algorithm MLAS, in the practical form announced in Section 5.2):
        C_j(r)  = P_j B_{j+1}(P_j^T r) + beta^{-1}(M_{u,j}^{-1} r
                  - P_j M_{u,j+1}^{-1} P_j^T r)
        B_{l-1} = H_{l-1}^{-1}  (dense, exact as the theory assumes)
        B_j(r)  = z + C_j(r - H_j z), z = C_j(r)     for 0 < j < l-1
        B_0     = C_0;
  * the outer CG on H_0 preconditioned by B_0 (Section 5.3: CG to relative
    residual 1e-8).

All residuals are Euclidean 2-norms relative to the right-hand side; every CG
starts from zero, except the outer CG after a dropped Hessian level, which
restarts from its last iterate.  A mixed-precision twin (float32 V-cycle and CG inside FP64
iterative refinement, FP64 dense coarse solve) is provided beside the FP64
path.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import sa
from .csr import CSR


class Indefinite(RuntimeError):
    """The preconditioner met a direction of non-positive curvature; x is the
    last iterate (every step taken had p.q > 0) and iters the steps taken."""

    def __init__(self, msg, x=None, iters=0):
        super().__init__(msg)
        self.x = x
        self.iters = iters


class NoConvergence(RuntimeError):
    pass


# Chebyshev smoother: degree and the interval of the spectrum of D_l1^{-1} A it
# damps (the top, 1, bounds that spectrum on every level)
CHEB_DEGREE = 2
CHEB_LO, CHEB_HI = 0.3, 1.0

@dataclass
class Counters:
    inner_iters: int = 0
    inner_solves: int = 0
    inner_max: int = 0
    mass_iters: int = 0
    outer_iters: int = 0
    refine_steps: int = 0
    coarse_cg_iters: int = 0
    history: list = field(default_factory=list)


def pcg(apply_A, apply_B, b, rtol, maxit, indefinite_check=False, x0=None):
    """Preconditioned conjugate gradients (Hestenes-Stiefel) from x_0 (zero
    when not given), stop at ||r||_2 <= rtol ||b||_2 on the recursive residual
    (r_0 = b - A x_0).  Returns (x, iters)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return np.zeros_like(b), 0
    r = b.copy() if x0 is None else b - apply_A(x)
    if float(np.linalg.norm(r)) <= rtol * bn:
        return x, 0
    z = apply_B(r)
    rho = float(r @ z)
    if indefinite_check and not rho > 0.0:
        raise Indefinite("r.z <= 0", x, 0)
    p = z.copy()
    for it in range(1, maxit + 1):
        q = apply_A(p)
        pq = float(p @ q)
        if indefinite_check and not pq > 0.0:
            raise Indefinite("p.q <= 0", x, it - 1)
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        if float(np.linalg.norm(r)) <= rtol * bn:
            return x, it
        z = apply_B(r)
        rho_new = float(r @ z)
        if indefinite_check and not rho_new > 0.0:
            raise Indefinite("r.z <= 0", x, it)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    raise NoConvergence(f"CG did not reach {rtol} in {maxit} iterations")


def cg_mass_inner(apply_H, mass_solve, b, rtol, maxit):
    """CG for the practical-form system H x = b carried out in the inner
    product of the mass matrix M: the paper states its operators on L^2, where
    H = M G and the coarsest-level solve of Section 5.2 is CG on G with the L^2
    inner product.  In coordinates that is CG on H preconditioned by M^{-1}
    (each step's M^{-1} r is the vector of G x - g).  From x_0 = 0, it stops
    when ||G x - g||_M <= rtol ||g||_M, g = M^{-1} b, i.e. when r.M^{-1}r <=
    rtol^2 b.M^{-1}b.  Returns (x, iters)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = mass_solve(r)
    rho = float(r @ z)
    if rho == 0.0:
        return x, 0
    tol2 = rtol * rtol * rho
    p = z.copy()
    for it in range(1, maxit + 1):
        q = apply_H(p)
        alpha = rho / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = mass_solve(r)
        rho_new = float(r @ z)
        if rho_new <= tol2:
            return x, it
        p = z + (rho_new / rho) * p
        rho = rho_new
    raise NoConvergence(f"CG in the M inner product did not reach {rtol} in {maxit} iterations")


class Oracle:
    """FP64 reference solver on a hierarchy built by oracle.sa.build."""

    def __init__(self, h: sa.Hierarchy, mixed: bool = False):
        self.h = h
        self.o = h.opts
        self.beta = h.opts.beta
        self.cnt = Counters()
        self.mixed = mixed
        if mixed:
            self.l32 = [dict(A=lev.A.astype32(), S=None if lev.S is None else lev.S.astype32(),
                             St=None if lev.St is None else lev.St.astype32(),
                             dl1=lev.dl1.astype(np.float32)) for lev in h.levels]

    # ---- smoothers ----
    def smooth(self, A, dl1, b, x):
        """One smoothing pass for A x = b from x (None = zero): nu l1-Jacobi
        sweeps, or the Chebyshev iteration of degree CHEB_DEGREE preconditioned
        by the l1 diagonal on the interval [CHEB_LO, CHEB_HI] of the spectrum of
        D_l1^{-1} A, whose top is at most 1 because the l1 diagonal bounds each
        row's absolute sum (Chebyshev acceleration as in Saad, Iterative
        Methods for Sparse Linear Systems).  Works in the dtype of b."""
        if self.o.smoother == 0:
            x = b / dl1 if x is None else x + (b - A.matvec(x)) / dl1
            for _ in range(self.o.nu - 1):
                x = x + (b - A.matvec(x)) / dl1
            return x
        t = b.dtype.type
        theta = (CHEB_HI + CHEB_LO) / 2
        delta = (CHEB_HI - CHEB_LO) / 2
        sigma = theta / delta
        rho = 1.0 / sigma
        r = b / dl1 if x is None else (b - A.matvec(x)) / dl1
        d = r * t(1.0 / theta)
        x = d if x is None else x + d
        for _ in range(CHEB_DEGREE - 1):
            rho_new = 1.0 / (2.0 * sigma - rho)
            r = (b - A.matvec(x)) / dl1
            d = t(rho_new * rho) * d + t(2.0 * rho_new / delta) * r
            x = x + d
            rho = rho_new
        return x

    # ---- V-cycle (AMG preconditioner for A_j) ----
    def vcycle(self, l: int, b: np.ndarray) -> np.ndarray:
        """One V(nu, nu) cycle from level l; it ends with an exact solve at the
        coarsest level or at the first coarse level small enough to hold a
        dense factor of A_l (n_l <= dense_solve_max)."""
        h = self.h
        if l == h.L - 1:
            return sla.cho_solve(h.chol_A, b)
        lev = h.levels[l]
        if lev.chol_A is not None:
            return sla.cho_solve(lev.chol_A, b)
        A = lev.A
        x = self.smooth(A, lev.dl1, b, None)
        r = b - A.matvec(x)
        e = self.vcycle(l + 1, lev.St.matvec(r))
        x = x + lev.S.matvec(e)
        return self.smooth(A, lev.dl1, b, x)

    def vcycle32(self, l: int, b: np.ndarray) -> np.ndarray:
        h = self.h
        if l == h.L - 1:
            return sla.cho_solve(h.chol_A, b.astype(np.float64)).astype(np.float32)
        if h.levels[l].chol_A is not None:
            return sla.cho_solve(h.levels[l].chol_A, b.astype(np.float64)).astype(np.float32)
        m = self.l32[l]
        A, dl1 = m["A"], m["dl1"]
        x = self.smooth(A, dl1, b, None)
        r = b - A.matvec(x)
        e = self.vcycle32(l + 1, m["St"].matvec(r))
        x = x + m["S"].matvec(e)
        return self.smooth(A, dl1, b, x)

    # ---- inner solves ----
    def solve_A(self, j: int, f: np.ndarray, rtol: float) -> np.ndarray:
        """x = A_j^{-1} f by V-cycle-preconditioned CG (FP64), or the mixed
        refinement loop; the coarsest AMG level is solved densely."""
        h = self.h
        if j == h.L - 1:
            return sla.cho_solve(h.chol_A, f)
        if h.levels[j].chol_A is not None:
            return sla.cho_solve(h.levels[j].chol_A, f)
        if self.mixed and self.o.mixed_mode == 1:
            return self._solve_A_mixed(j, f, rtol)
        A = h.levels[j].A
        if self.mixed:
            # FP64 CG whose preconditioner is the float32 V-cycle applied to
            # the residual rounded to float32
            x, it = pcg(A.matvec, lambda r: self.vcycle32(j, r.astype(np.float32)).astype(np.float64), f, rtol,
                        self.o.inner_maxit)
            self._count_inner(it)
            return x
        x, it = pcg(A.matvec, lambda r: self.vcycle(j, r), f, rtol, self.o.inner_maxit)
        self._count_inner(it)
        return x

    def _count_inner(self, it):
        self.cnt.inner_iters += it
        self.cnt.inner_solves += 1
        self.cnt.inner_max = max(self.cnt.inner_max, it)

    def pcg32(self, j: int, b32: np.ndarray, rtol: float):
        """CG in float32 with float64 dot products and float64 scalars."""
        m = self.l32[j]
        A = m["A"]
        d64 = lambda a, c: float(a.astype(np.float64) @ c.astype(np.float64))
        x = np.zeros_like(b32)
        bn = np.sqrt(d64(b32, b32))
        if bn == 0.0:
            return x, 0
        r = b32.copy()
        z = self.vcycle32(j, r)
        rho = d64(r, z)
        p = z.copy()
        for it in range(1, self.o.inner_maxit + 1):
            q = A.matvec(p)
            alpha = rho / d64(p, q)
            a32 = np.float32(alpha)
            x = x + a32 * p
            r = r - a32 * q
            if np.sqrt(d64(r, r)) <= rtol * bn:
                return x, it
            z = self.vcycle32(j, r)
            rho_new = d64(r, z)
            beta = rho_new / rho
            rho = rho_new
            p = z + np.float32(beta) * p
        raise NoConvergence("float32 CG did not converge")

    def _solve_A_mixed(self, j: int, f: np.ndarray, rtol: float) -> np.ndarray:
        """FP64 iterative refinement around the float32 CG: x += s d,
        d = CG32(fp32(r/s)), s = ||r||, r = f - A x in FP64."""
        A = self.h.levels[j].A
        x = np.zeros_like(f)
        fn = float(np.linalg.norm(f))
        if fn == 0.0:
            return x
        r = f.copy()
        s = fn
        for step in range(self.o.refine_maxit):
            d, it = self.pcg32(j, (r / s).astype(np.float32), self.o.inner32_rtol)
            self._count_inner(it)
            self.cnt.refine_steps += 1
            x = x + s * d.astype(np.float64)
            r = f - A.matvec(x)
            s_new = float(np.linalg.norm(r))
            if s_new <= rtol * fn:
                return x
            if s_new > 0.5 * s:
                raise NoConvergence("refinement stagnated")
            s = s_new
        raise NoConvergence("refinement did not converge")

    def mass_solve(self, j: int, r: np.ndarray) -> np.ndarray:
        if self.h.levels[j].chol_M is not None:
            return sla.cho_solve(self.h.levels[j].chol_M, r)
        M = self.h.levels[j].M
        d = M.diag()
        x, it = pcg(M.matvec, lambda v: v / d, r, self.o.mass_rtol, self.o.mass_maxit)
        self.cnt.mass_iters += it
        return x

    # ---- operators (Section 2 and Section 5.2) ----
    def state_solve(self, j: int, u: np.ndarray, rtol=None) -> np.ndarray:
        """y = K_j u = A_j^{-1} M_{yu,j} u."""
        return self.solve_A(j, sa.mass_yu(self.h, j, u), rtol or self.o.inner_rtol)

    def adjoint_solve(self, j: int, w: np.ndarray, rtol=None) -> np.ndarray:
        """K_j^T w = M_{yu,j}^T A_j^{-1} w (A_j symmetric)."""
        return sa.mass_yu_t(self.h, j, self.solve_A(j, w, rtol or self.o.inner_rtol))

    def hessian_apply(self, j: int, u: np.ndarray, rtol=None) -> np.ndarray:
        """H_j u = K_j^T M_{y,j} K_j u + beta M_{u,j} u."""
        return self.hessian_apply_t(j, u, rtol)[0]

    def hessian_apply_t(self, j: int, u: np.ndarray, rtol=None):
        """(H_j u, t) with t = A_j^{-1} M_{y,j} K_j u, so that
        H_j u = M_{yu,j}^T t + beta M_{u,j} u."""
        y = self.state_solve(j, u, rtol)
        t = self.solve_A(j, sa.mass_y(self.h, j, y), rtol or self.o.inner_rtol)
        return sa.mass_yu_t(self.h, j, t) + self.beta * sa.mass_u(self.h, j, u), t

    def rhs(self, yd: np.ndarray) -> np.ndarray:
        """b = K_0^T M_{y,0} y_d."""
        return self.adjoint_solve(0, sa.mass_y(self.h, 0, yd))

    # ---- multilevel preconditioner ----
    def C(self, j: int, r: np.ndarray, mr=None) -> np.ndarray:
        """C_j r (practical form, Section 5.2); mr: M_{u,j}^{-1} r when the
        caller has it."""
        lev = self.h.levels[j]
        q = lev.St.matvec(r)
        v = self.B(j + 1, q) - (1.0 / self.beta) * self.mass_solve(j + 1, q)
        if mr is None:
            mr = self.mass_solve(j, r)
        return lev.S.matvec(v) + (1.0 / self.beta) * mr

    def B(self, j: int, r: np.ndarray) -> np.ndarray:
        h = self.h
        if j == h.ell - 1:
            if h.chol_H is not None:
                return sla.cho_solve(h.chol_H, r)
            # Section 5.2: the coarsest Hessian level solved by CG (on G, in
            # the L^2 inner product) to a loose relative residual (1e-4)
            x, it = cg_mass_inner(lambda v: self.hessian_apply(j, v, self.o.precond_inner_rtol),
                                  lambda v: self.mass_solve(j, v), r, self.o.coarse_hess_rtol, self.o.outer_maxit)
            self.cnt.coarse_cg_iters += it
            return x
        if j == 0:
            return self.C(0, r)
        # Algorithm MLAS: B_j r = z + C_j (r - H_j z), z = C_j r.  At j >= 1 the
        # mass matrices are all M_j, so H_j z = M_j (t + beta z) with t the
        # Hessian's inner result, and the second C_j's mass solve is
        # M_j^{-1} (r - H_j z) = M_j^{-1} r - (t + beta z), from the first's.
        mr = self.mass_solve(j, r)
        z = self.C(j, r, mr)
        hz, t = self.hessian_apply_t(j, z, self.o.precond_inner_rtol)
        return z + self.C(j, r - hz, mr - (t + self.beta * z))

    def precond(self, r: np.ndarray) -> np.ndarray:
        return self.B(0, r) if self.o.precond else r.copy()

    # ---- hierarchy quality (Section 4: eqs. ajnumerical and aj-tilde) ----
    def quality_apply(self, j: int, v: np.ndarray, transpose: bool) -> np.ndarray:
        """E v or E^T v for E = K_j - S_j K_{j+1} Pi_j, Pi_j = M_{u,j+1}^{-1}
        S_j^T M_{u,j} (the control projection with P_j = S_j)."""
        h = self.h
        lev = h.levels[j]
        if not transpose:
            pv = self.mass_solve(j + 1, lev.St.matvec(sa.mass_u(h, j, v)))
            return self.state_solve(j, v) - lev.S.matvec(self.state_solve(j + 1, pv))
        q = self.mass_solve(j + 1, self.adjoint_solve(j + 1, lev.St.matvec(v)))
        return self.adjoint_solve(j, v) - sa.mass_u(h, j, lev.S.matvec(q))

    def quality(self, j: int, v0: np.ndarray, iters: int) -> float:
        """a~_j = ||E||_2 estimated, as the paper does, by the power method on
        E^T E from v0: iters steps, the last Rayleigh quotient's square root."""
        v = v0 / np.linalg.norm(v0)
        lam = 0.0
        for _ in range(iters):
            y = self.quality_apply(j, self.quality_apply(j, v, False), True)
            lam = float(v @ y)
            v = y / np.linalg.norm(y)
        return float(np.sqrt(max(lam, 0.0)))

    # ---- outer solve (Section 5.3) ----
    def reduced_solve(self, yd: np.ndarray, rtol: float = 1e-8):
        """Solve H_0 u = b for one desired state; on an indefinite
        preconditioner with auto_levels, drop one Hessian level and restart CG
        from the last iterate (the paper drops levels when definiteness is
        lost, Sections 5.5 and 5.6; every step taken before had p.q > 0, so
        that iterate is no worse than zero).  Returns (u, outer iterations
        over all attempts)."""
        b = self.rhs(yd)
        x0, total = None, 0
        while True:
            try:
                u, it = pcg(lambda v: self.hessian_apply(0, v), self.precond, b, rtol,
                            self.o.outer_maxit, indefinite_check=True, x0=x0)
                total += it
                self.cnt.outer_iters += total
                return u, total
            except Indefinite as e:
                if not self.o.auto_levels or self.h.ell <= 1:
                    raise
                total += e.iters
                x0 = e.x
                sa.set_hessian_levels(self.h, self.h.ell - 1)

    def objective(self, u: np.ndarray, yd: np.ndarray) -> float:
        """J(u) = 1/2 (Ku - y_d)^T M_y (Ku - y_d) + beta/2 u^T M_u u (eq. functional)."""
        e = self.state_solve(0, u) - yd
        return 0.5 * float(e @ sa.mass_y(self.h, 0, e)) + 0.5 * self.beta * float(u @ sa.mass_u(self.h, 0, u))

    def gradient(self, u: np.ndarray, yd: np.ndarray) -> np.ndarray:
        """grad J(u) = K^T M_y (K u - y_d) + beta M_u u."""
        e = self.state_solve(0, u) - yd
        return self.adjoint_solve(0, sa.mass_y(self.h, 0, e)) + self.beta * sa.mass_u(self.h, 0, u)


def build_problem(prob, opts: sa.Opts | None = None):
    """Assemble and build the hierarchy for an inputs.Problem."""
    from . import fem
    opts = opts or sa.Opts(beta=prob.beta)
    A, M = fem.assemble(prob.mesh.coords, prob.mesh.elems, prob.kappa)
    bc = prob.dirichlet.astype(bool)
    A0 = fem.dirichlet_stiffness(A, bc)
    h = sa.build(A0, M, bc, opts)
    return h, A, M
