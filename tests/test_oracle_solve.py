"""Pins for the oracle's solve phase: dense brute force on tiny meshes, the
paper's closed-form optimal control (eq. test-state), the structural facts of
Section 3 (T symmetric positive definite, P Pi a projection, the stated
inverse of T), the exact-quadratic identities of the reduced functional and
the equivalence of the practical-form preconditioner with the paper's W_j."""
import math

import numpy as np
import pytest

import inputs
from oracle import dense, fem, sa, solve


def build(name, n, **kw):
    p = inputs.config(name, n=n)
    opts = sa.Opts(beta=kw.pop("beta", p.beta), **kw)
    h, A, M = solve.build_problem(p, opts)
    return p, h


def tight(**kw):
    base = dict(inner_rtol=1e-13, mass_rtol=1e-14, precond_inner_rtol=1e-13)
    base.update(kw)
    return base


def test_vcycle_is_symmetric_and_contracts():
    p, h = build("c2", 12, max_coarse=12)
    assert h.L >= 3
    o = solve.Oracle(h)
    n = h.levels[0].n
    B = dense.vcycle_matrix(lambda e: o.vcycle(0, e), n)
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    A = h.levels[0].A.dense()
    ev = np.linalg.eigvals(B @ A).real
    assert ev.min() > 0 and ev.max() < 2.0       # ||I - BA||_A < 1


def test_chebyshev_smoother_is_the_scaled_chebyshev_polynomial():
    # one pass from any x maps the error e to p(D^{-1} A) e with
    # p(l) = T_2((theta - l) / delta) / T_2(theta / delta), T_2(z) = 2 z^2 - 1,
    # theta, delta the centre and half-width of [CHEB_LO, CHEB_HI]
    p, h = build("c1", 6, smoother=1)
    o = solve.Oracle(h)
    lev = h.levels[0]
    A, d = lev.A.dense(), lev.dl1
    rng = np.random.default_rng(5)
    xt, x0 = rng.standard_normal(lev.n), rng.standard_normal(lev.n)
    x1 = o.smooth(lev.A, d, A @ xt, x0)
    s = 1.0 / np.sqrt(d)
    lam, V = np.linalg.eigh(s[:, None] * A * s[None, :])     # D^{-1/2} A D^{-1/2}
    assert lam.max() <= 1.0 + 1e-12                          # the l1 bound
    th = (solve.CHEB_HI + solve.CHEB_LO) / 2
    de = (solve.CHEB_HI - solve.CHEB_LO) / 2
    T2 = lambda z: 2 * z * z - 1
    pl = T2((th - lam) / de) / T2(th / de)
    e0 = (x0 - xt) / s                                       # D^{1/2} e
    e1 = s * (V @ (pl * (V.T @ e0)))
    assert np.max(np.abs((x1 - xt) - e1)) <= 1e-12 * np.max(np.abs(x0 - xt))
    # from zero it is the same polynomial applied to e = -x_true
    z1 = o.smooth(lev.A, d, A @ xt, None)
    ez = s * (V @ (pl * (V.T @ (-xt / s))))
    assert np.max(np.abs((z1 - xt) - ez)) <= 1e-12 * np.max(np.abs(xt))


def test_chebyshev_vcycle_symmetric_contracting_same_solution():
    p, h = build("c2", 12, max_coarse=12, smoother=1)
    o = solve.Oracle(h)
    n = h.levels[0].n
    B = dense.vcycle_matrix(lambda e: o.vcycle(0, e), n)
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    ev = np.linalg.eigvals(B @ h.levels[0].A.dense()).real
    assert ev.min() > 0 and ev.max() < 2.0
    yd = p.yd[:, 0]
    u1, _ = o.reduced_solve(yd, rtol=1e-10)
    h.opts.smoother = 0
    u0, _ = solve.Oracle(h).reduced_solve(yd, rtol=1e-10)
    assert np.linalg.norm(u1 - u0) <= 1e-8 * np.linalg.norm(u0)


@pytest.mark.parametrize("name,n", [("c1", 8), ("c3", 4)])
def test_state_adjoint_hessian_against_dense(name, n):
    p, h = build(name, n, max_coarse=10, **tight())
    o = solve.Oracle(h)
    ops = dense.level_ops(h, 0)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(h.levels[0].n)
    np.testing.assert_allclose(o.state_solve(0, u), ops["K"] @ u, rtol=1e-10, atol=1e-12 * np.abs(ops["K"] @ u).max())
    w = rng.standard_normal(h.levels[0].n)
    np.testing.assert_allclose(o.adjoint_solve(0, w), ops["K"].T @ w, rtol=1e-10,
                               atol=1e-12 * np.abs(ops["K"].T @ w).max())
    H = dense.hessian_practical(h)
    Hu = o.hessian_apply(0, u)
    np.testing.assert_allclose(Hu, H @ u, rtol=1e-9, atol=1e-11 * np.abs(H @ u).max())
    # the paper's two forms: H = M_u G
    np.testing.assert_allclose(H, ops["Mu"] @ ops["G"], rtol=1e-9, atol=1e-12 * np.abs(H).max())


def test_dense_hessian_spectrum_bounds_and_closed_form():
    # (G u, u)_M >= beta (u, u)_M, and for kappa = 1 in 2D the top of the
    # spectrum of K^*K approaches 1/(2 pi^2)^2 (first Dirichlet eigenvalue of
    # the Laplacian on the unit square is 2 pi^2).
    p, h = build("c1", 16)
    H = dense.hessian_practical(h)
    Mu = dense.level_ops(h, 0)["Mu"]
    assert np.array_equal(H, H) and np.max(np.abs(H - H.T)) < 1e-12 * np.abs(H).max()
    import scipy.linalg as sla
    lam = sla.eigh(H, Mu, eigvals_only=True)
    beta = p.beta
    assert lam.min() >= beta * (1 - 1e-10)
    assert np.linalg.eigvalsh(H).min() >= beta * np.linalg.eigvalsh(Mu).min() * (1 - 1e-10)
    top = beta + 1.0 / (2 * math.pi ** 2) ** 2
    assert abs(lam.max() - top) / top < 0.03


@pytest.mark.parametrize("name,n,mc", [("c2", 12, 12), ("c3", 5, 8)])
def test_practical_preconditioner_equals_paper_multilevel_operator(name, n, mc):
    p, h = build(name, n, max_coarse=mc, beta=1e-2, **tight())
    assert h.ell >= 3, "need an intermediate level to exercise the W recursion"
    o = solve.Oracle(h)
    N = h.levels[0].n
    B = dense.vcycle_matrix(o.precond, N)
    W0 = dense.W(h, 0, h.ell)
    Mu = dense.level_ops(h, 0)["Mu"]
    ref = W0 @ np.linalg.inv(Mu)
    assert np.max(np.abs(B - ref)) <= 1e-8 * np.max(np.abs(ref))
    # B_0 W-cycle form equals 2C - C H C at level 1 (Algorithm MLAS)
    assert np.max(np.abs(ref - ref.T)) <= 1e-8 * np.max(np.abs(ref))


@pytest.mark.parametrize("name,n,mc", [("c2", 12, 12), ("c3", 5, 8)])
def test_coarse_mass_solve_of_hessian_is_its_inner_result(name, n, mc):
    """At levels j >= 1 the state, control and mixed mass matrices are all M_j,
    so M_j^{-1} H_j z = t + beta z with t = A_j^{-1} M_j A_j^{-1} M_j z: checked
    against a dense solve with M_j, at every intermediate level.  B_j uses it for
    the mass solve of its second C_j."""
    p, h = build(name, n, max_coarse=mc, beta=1e-2, **tight())
    assert h.ell >= 3
    o = solve.Oracle(h)
    rng = np.random.default_rng(11)
    for j in range(1, h.ell - 1):
        z = rng.standard_normal(h.levels[j].n)
        hz, t = o.hessian_apply_t(j, z, 1e-13)
        Mj = h.levels[j].M.dense()
        lhs = np.linalg.solve(Mj, hz)
        rhs = t + h.opts.beta * z
        assert np.linalg.norm(lhs - rhs) <= 1e-10 * np.linalg.norm(rhs)
        # and t is not a neighbouring intermediate (K z, or M^{-1} H z without beta z)
        y = o.state_solve(j, z, 1e-13)
        assert np.linalg.norm(lhs - (y + h.opts.beta * z)) > 1e-3 * np.linalg.norm(rhs)
        assert np.linalg.norm(lhs - t) > 1e-3 * np.linalg.norm(rhs)


def test_multilevel_preconditioner_with_fresh_second_mass_solve():
    """B_j with the second C_j's mass solve taken from the first (the identity
    above) equals B_j with that mass solve done afresh, to the inner tolerances."""
    p, h = build("c3", 5, max_coarse=8, beta=1e-2, **tight())
    assert h.ell >= 3
    o = solve.Oracle(h)
    r = np.random.default_rng(12).standard_normal(h.levels[1].n)

    def B_fresh(j, v):
        z = o.C(j, v)
        return z + o.C(j, v - o.hessian_apply(j, z, o.o.precond_inner_rtol))

    ref = B_fresh(1, r)
    got = o.B(1, r)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_two_grid_identities():
    p, h = build("c2", 12, max_coarse=12, beta=1e-3)
    P = h.levels[0].S.dense()
    Pi = dense.projection(h, 0)
    np.testing.assert_allclose(Pi @ P, np.eye(P.shape[1]), atol=1e-10)          # Pi P = I
    PP = P @ Pi
    np.testing.assert_allclose(PP @ PP, PP, atol=1e-10 * np.abs(PP).max())     # projection
    T, Tinv = dense.two_grid_T(h, 0)
    np.testing.assert_allclose(T @ Tinv, np.eye(T.shape[0]), atol=1e-8)        # eq. twogrid
    Mu = dense.level_ops(h, 0)["Mu"]
    MT = Mu @ T                                                                 # M_u-self-adjoint
    assert np.max(np.abs(MT - MT.T)) < 1e-9 * np.abs(MT).max()
    assert np.linalg.eigvalsh(0.5 * (MT + MT.T)).min() > 0                      # T is SPD


def test_one_level_preconditioner_converges_in_one_iteration():
    p, h = build("c1", 8, hess_levels=1, **tight())
    assert h.ell == 1
    o = solve.Oracle(h)
    u, it = o.reduced_solve(p.yd[:, 0])
    assert it == 1


def test_two_level_preconditioner_is_spd():
    p, h = build("c1", 12, max_coarse=30, hess_levels=2, **tight())
    o = solve.Oracle(h)
    B = dense.vcycle_matrix(o.precond, h.levels[0].n)
    assert np.max(np.abs(B - B.T)) < 1e-9 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


@pytest.mark.parametrize("name,n,mc", [("c1", 10, 20), ("c2", 12, 12), ("c3", 4, 8)])
def test_reduced_solve_matches_dense_solution(name, n, mc):
    p, h = build(name, n, max_coarse=mc)
    o = solve.Oracle(h)
    yd = p.yd[:, 0]
    u, it = o.reduced_solve(yd, rtol=1e-10)
    H = dense.hessian_practical(h)
    b = dense.rhs_practical(h, yd)
    ref = np.linalg.solve(H, b)
    assert np.linalg.norm(u - ref) <= 1e-8 * np.linalg.norm(ref)
    # the preconditioner does not change the solution (Section 5.3)
    h.opts.precond = 0
    o2 = solve.Oracle(h)
    u2, it2 = o2.reduced_solve(yd, rtol=1e-10)
    assert np.linalg.norm(u2 - ref) <= 1e-8 * np.linalg.norm(ref)
    assert it2 >= it


def _mass_norm(M, v):
    return math.sqrt(float(v @ M.matvec(v)))


def test_closed_form_control_2d_second_order():
    # 2D analogue of eq. test-state: y_d = sin(pi x) sin(pi y) gives
    # u* = c sin sin with c = 1/(2 pi^2 beta + 1/(2 pi^2)).
    beta = 1e-2
    c = 1.0 / (2 * math.pi ** 2 * beta + 1.0 / (2 * math.pi ** 2))
    errs = []
    for n in (8, 16, 32, 64):
        p, h = build("c1", n)
        o = solve.Oracle(h)
        u, _ = o.reduced_solve(p.yd[:, 0], rtol=1e-11)
        ustar = inputs.yd_sin(p.mesh, c)
        errs.append(_mass_norm(h.levels[0].M, u - ustar) / _mass_norm(h.levels[0].M, ustar))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert errs[2] < 1e-2
    assert all(3.5 < r < 4.5 for r in ratios), ratios


def test_manufactured_solution_3d_converges():
    # eq. test-state: y_d = (1/(3 pi^2) + 3 pi^2 beta) sin sin sin has the
    # optimal control u* = sin sin sin (kappa = 1).
    beta = 1e-2
    errs = []
    for n in (4, 8, 16):
        m = inputs.mesh3d(n)
        p = inputs.Problem("m", m, inputs.kappa_const(m), beta,
                           inputs.yd_manufactured(m, beta).reshape(-1, 1), m.boundary)
        h, A, M = solve.build_problem(p)
        o = solve.Oracle(h)
        u, _ = o.reduced_solve(p.yd[:, 0], rtol=1e-11)
        ustar = inputs.yd_sin(m)
        errs.append(_mass_norm(M, u - ustar) / _mass_norm(M, ustar))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[2] > 3.0, errs


def test_exact_quadratic_identities_and_gradient():
    p, h = build("c2", 12, max_coarse=12, **tight())
    o = solve.Oracle(h)
    yd = p.yd[:, 0]
    rng = np.random.default_rng(11)
    u = rng.standard_normal(h.levels[0].n)
    d = rng.standard_normal(h.levels[0].n)
    d /= np.linalg.norm(d)
    g = o.gradient(u, yd)
    H = dense.hessian_practical(h)
    b = dense.rhs_practical(h, yd)
    np.testing.assert_allclose(g, H @ u - b, rtol=1e-9, atol=1e-11 * np.abs(g).max())
    step = 1e-2
    Jp, J0, Jm = o.objective(u + step * d, yd), o.objective(u, yd), o.objective(u - step * d, yd)
    fd = (Jp - Jm) / (2 * step)
    assert abs(fd - g @ d) <= 1e-9 * max(abs(g @ d), 1e-30) + 1e-12 * abs(J0) / step
    sd = (Jp - 2 * J0 + Jm) / step ** 2
    assert abs(sd - d @ H @ d) <= 1e-6 * abs(d @ H @ d) + 1e-12 * abs(J0) / step ** 2


@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_precision_twin_matches_fp64(mode):
    # both float32 forms reach the FP64 answer to 1e-8: the FP64 CG with the
    # float32 V-cycle (mode 0) and float32 CG inside refinement (mode 1)
    p, h = build("c3", 8, max_coarse=30, mixed_mode=mode)
    o64 = solve.Oracle(h)
    o32 = solve.Oracle(h, mixed=True)
    yd = p.yd[:, 0]
    u64, _ = o64.reduced_solve(yd)
    u32, _ = o32.reduced_solve(yd)
    assert np.linalg.norm(u32 - u64) <= 1e-8 * np.linalg.norm(u64)
    assert (o32.cnt.refine_steps > 0) == (mode == 1)


def test_indefinite_fallback_drops_levels():
    # a preconditioner may lose definiteness with many levels (Section 3.2);
    # the fallback drops Hessian levels until CG runs.  Force it with an
    # absurdly small beta on a coarse hierarchy and check that the answer is
    # still the dense solution.
    p, h = build("c2", 16, max_coarse=6, beta=1e-9)
    o = solve.Oracle(h)
    yd = p.yd[:, 0]
    ell0 = h.ell
    u, it = o.reduced_solve(yd, rtol=1e-9)
    assert h.ell < ell0
    H = dense.hessian_practical(h)
    ref = np.linalg.solve(H, dense.rhs_practical(h, yd))
    assert np.linalg.norm(u - ref) <= 1e-6 * np.linalg.norm(ref)


def test_cg_in_mass_inner_product_is_textbook_cg_on_G():
    # The coarsest-level solve of Section 5.2 is CG on G = M^{-1} H in the L^2
    # (M) inner product.  Written out plainly on the dense G with <u, v>_M, a
    # textbook CG run for the same number of steps must give the practical-form
    # routine's iterate (CG on H preconditioned by M^{-1}), and the routine's
    # stopping rule is the relative M-norm of G x - g.
    p, h = build("c2", 10, max_coarse=20, **tight())
    j = 1
    lev = h.levels[j]
    H = dense.hessian_practical(h, j)
    Mj = lev.M.dense()
    G = np.linalg.solve(Mj, H)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(lev.n)
    g = np.linalg.solve(Mj, b)
    ip = lambda u, v: float(u @ (Mj @ v))

    def textbook(steps):
        x = np.zeros_like(g)
        r = g.copy()
        d = r.copy()
        for _ in range(steps):
            Gd = G @ d
            a = ip(r, r) / ip(d, Gd)
            x = x + a * d
            r_new = r - a * Gd
            d = r_new + (ip(r_new, r_new) / ip(r, r)) * d
            r = r_new
        return x

    for rtol in (1e-1, 1e-2, 1e-4, 1e-8):
        x, it = solve.cg_mass_inner(lambda v: H @ v, lambda v: np.linalg.solve(Mj, v), b, rtol, 500)
        assert it >= 1
        xt = textbook(it)
        assert np.linalg.norm(x - xt) <= 1e-9 * np.linalg.norm(xt), rtol
        e = G @ x - g
        assert math.sqrt(ip(e, e)) <= rtol * math.sqrt(ip(g, g)) * (1 + 1e-9), rtol
        if it > 1:   # it is the first step count that meets the rule
            e = G @ textbook(it - 1) - g
            assert math.sqrt(ip(e, e)) > rtol * math.sqrt(ip(g, g)) * (1 - 1e-9), rtol


def test_coarsest_hessian_by_loose_cg():
    # Section 5.2 solves the coarsest Hessian level by CG (on G in the L^2
    # inner product) to 1e-4 instead of exactly; forcing that path (dense_max
    # below the coarsest Hessian level) must leave the solution of H_0 u = b
    # unchanged
    p, h = build("c2", 16, max_coarse=30, dense_max=30, hess_levels=2, beta=1e-3)
    assert h.levels[h.ell - 1].n > 30 and h.chol_H is None
    o = solve.Oracle(h)
    yd = p.yd[:, 0]
    u, it = o.reduced_solve(yd, rtol=1e-10)
    assert o.cnt.coarse_cg_iters > 0
    H = dense.hessian_practical(h)
    ref = np.linalg.solve(H, dense.rhs_practical(h, yd))
    assert np.linalg.norm(u - ref) <= 1e-8 * np.linalg.norm(ref)


def test_exact_small_coarse_solves_do_not_change_the_solution():
    # exact dense A_j / M_j solves on small coarse levels return what the
    # iterative inner solves approximate: same outer solution to tolerance
    p, h1 = build("c2", 32, max_coarse=20)
    assert any(lev.chol_A is not None for lev in h1.levels[1:-1])
    p, h0 = build("c2", 32, max_coarse=20, dense_solve_max=0)
    assert all(lev.chol_A is None for lev in h0.levels)
    yd = p.yd[:, 0]
    u1, _ = solve.Oracle(h1).reduced_solve(yd, rtol=1e-11)
    u0, _ = solve.Oracle(h0).reduced_solve(yd, rtol=1e-11)
    assert np.linalg.norm(u1 - u0) <= 1e-9 * np.linalg.norm(u0)


def test_hierarchy_quality_power_method_and_ajnumerical():
    # Section 4: a~_j = ||K_j - S_j K_{j+1} Pi_j||_2 by the power method equals
    # the largest singular value of the explicit E, and approximates
    # a_j = ||M_y^{1/2} E M_u^{-1/2}||_2 up to the mass matrices' spectral
    # scale (the paper's argument for using a~_j): the ratio a_j / a~_j lies in
    # [sqrt(lmin(M_y)) / sqrt(lmax(M_u)), sqrt(lmax(M_y)) / sqrt(lmin(M_u))]
    p, h = build("c2", 16, max_coarse=12, **tight())
    assert h.L >= 3
    o = solve.Oracle(h)
    rng = np.random.default_rng(23)
    for j in range(h.L - 1):
        a, at = dense.quality(h, j)
        est = o.quality(j, rng.standard_normal(h.levels[j].n), 300)
        assert abs(est - at) <= 1e-6 * at
        ops = dense.level_ops(h, j)
        ly = np.linalg.eigvalsh(ops["My"])
        lu = np.linalg.eigvalsh(ops["Mu"])
        lo = np.sqrt(max(ly.min(), 0.0) / lu.max())
        hi = np.sqrt(ly.max() / lu.min())
        assert lo * at * (1 - 1e-9) <= a <= hi * at * (1 + 1e-9)
