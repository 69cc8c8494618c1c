"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.

Integer setup outputs (roots, aggregates, every sparsity pattern) must be
bit-exact; setup values are formed in the same order on both sides and must be
bit-identical too; dense coarse data within 1e-12; solve-phase FP64 results
within the tolerances stated per test (the reduced solve to 1e-8 relative,
the target of the method)."""
import numpy as np
import pytest

import inputs
from oracle import dense as odense
from oracle import sa as osa
from oracle import solve as osolve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


ORACLE_KEYS = ("hess_levels", "max_coarse", "inner_rtol", "mass_rtol", "precond_inner_rtol", "precond", "dense_max", "dense_solve_max",
               "inner32_rtol", "mixed_mode", "smoother", "theta0")


def make(name, n, nb_max=1, **opts):
    _need_gpu()
    import paper_2001_11533_amd as amg
    p = inputs.config(name, n=n)
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    beta = opts.pop("beta", p.beta)
    g = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, beta=beta, nb_max=nb_max, **opts)
    oo = osa.Opts(beta=beta, **{k: v for k, v in opts.items() if k in ORACLE_KEYS})
    h, A, M = osolve.build_problem(p, oo)
    mixed = opts.get("inner_precision", 64) == 32
    return p, g, osolve.Oracle(h, mixed=mixed)


def cuda(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel(a, b):
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# theta0 = 0.3 on the 64^2 mesh coarsens slowly (4225 -> 2253 -> 1218 -> 883 ->
# 179 nodes): the level-0 products have fewer than 8192 rows and more than 2048
# output columns, the case of the hash-table product kernels for few rows (the
# other few-row products use dense accumulators)
SETUP_CASES = [("c1", None, {}), ("c2", 64, {}), ("c3", 16, {}), ("c3", 20, {"max_coarse": 50}),
               ("c2", 48, {"max_coarse": 10}), ("c2", 64, {"theta0": 0.3})]


@pytest.mark.parametrize("name,n,opts", SETUP_CASES)
def test_setup_bit_exact(name, n, opts):
    p, g, o = make(name, n, **opts)
    h = o.h
    L, ell = g.levels()
    assert L == h.L and ell == h.ell
    for j in range(L):
        lev = h.levels[j]
        nj, nnzA, nnzS, nnzM = g.level_size(j)
        assert nj == lev.n and nnzA == lev.A.nnz and nnzM == lev.M.nnz
        for which, ref in ((0, lev.A), (3, lev.M)):
            rp, ci, v = g.csr(j, which)
            assert np.array_equal(rp, ref.rowptr) and np.array_equal(ci, ref.col), (j, which)
            assert np.array_equal(v.view(np.uint64), ref.val.view(np.uint64)), (j, which, np.abs(v - ref.val).max())
        if j < L - 1:
            agg, root = g.aggregates(j)
            assert np.array_equal(root.astype(bool), lev.root)
            assert np.array_equal(agg, lev.agg)
            for which, ref in ((1, lev.S), (2, lev.St)):
                rp, ci, v = g.csr(j, which)
                assert np.array_equal(rp, ref.rowptr) and np.array_equal(ci, ref.col), (j, which)
                assert np.array_equal(v.view(np.uint64), ref.val.view(np.uint64)), (j, which)
    Ainv = g.dense(0)
    ref = np.linalg.inv(h.levels[-1].A.dense())
    assert np.max(np.abs(Ainv - ref)) <= 1e-12 * np.max(np.abs(ref))
    H = g.dense(1)
    assert np.max(np.abs(H - h.H_dense)) <= 1e-12 * np.max(np.abs(h.H_dense))
    Hinv = g.dense(2)
    assert np.max(np.abs(Hinv @ H - np.eye(H.shape[0]))) < 1e-9


def test_mass_operators():
    p, g, o = make("c2", 32, nb_max=4)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((p.mesh.nverts, 3))
    fns = [osa.mass_u, osa.mass_y, osa.mass_yu, osa.mass_yu_t]
    for which, f in enumerate(fns):
        y = g.mass_apply(cuda(x), which)
        assert rel(y, f(o.h, 0, x)) < 1e-14, which
    q = g.mass_quad(cuda(x), 1).numpy()
    ref = np.einsum("ic,ic->c", x, osa.mass_y(o.h, 0, x))
    assert np.max(np.abs(q - ref) / np.abs(ref)) < 1e-13


TIGHT = dict(inner_rtol=1e-13, mass_rtol=1e-14, precond_inner_rtol=1e-13)


@pytest.mark.parametrize("name,n,mc", [("c1", None, 200), ("c2", 40, 20), ("c3", 12, 40)])
def test_state_adjoint_hessian(name, n, mc):
    p, g, o = make(name, n, max_coarse=mc, **TIGHT)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(p.mesh.nverts)
    assert rel(g.state_solve(cuda(u)), o.state_solve(0, u)) < 1e-11
    assert rel(g.adjoint_solve(cuda(u)), o.adjoint_solve(0, u)) < 1e-11
    assert rel(g.hessian_apply(cuda(u)), o.hessian_apply(0, u)) < 1e-11
    L, _ = g.levels()
    if L > 2:
        u1 = rng.standard_normal(g.level_size(1)[0])
        assert rel(g.hessian_apply(cuda(u1), level=1), o.hessian_apply(1, u1)) < 1e-11


@pytest.mark.parametrize("name,n,mc", [("c2", 40, 20), ("c3", 12, 40)])
def test_precond_apply(name, n, mc):
    p, g, o = make(name, n, max_coarse=mc, **TIGHT)
    assert g.levels()[1] >= 3
    rng = np.random.default_rng(9)
    r = rng.standard_normal(p.mesh.nverts)
    assert rel(g.precond_apply(cuda(r)), o.precond(r)) < 1e-10


@pytest.mark.parametrize("name,n,mc", [("c1", None, 200), ("c2", 64, 200), ("c3", 16, 200)])
def test_reduced_solve(name, n, mc):
    p, g, o = make(name, n, max_coarse=mc)
    yd = p.yd[:, 0]
    u, info = g.reduced_solve(cuda(yd), rtol=1e-8)
    uo, it = o.reduced_solve(yd, rtol=1e-12)
    assert info[0]["rel_resid"] <= 1e-8
    assert rel(u, uo) < 1e-8, (rel(u, uo), info[0])
    assert abs(info[0]["outer_iters"] - it) <= 3


def test_reduced_solve_tiny_against_dense():
    # inner solves far below the comparison tolerance: the dense Hessian is exact
    p, g, o = make("c1", 10, max_coarse=20, **TIGHT)
    yd = p.yd[:, 0]
    u, info = g.reduced_solve(cuda(yd), rtol=1e-11)
    H = odense.hessian_practical(o.h)
    ref = np.linalg.solve(H, odense.rhs_practical(o.h, yd))
    assert rel(u, ref) < 1e-9


@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_precision_solve(mode):
    # mode 0: FP64 CG preconditioned by the float32 V-cycle; mode 1: float32
    # CG inside FP64 refinement.  Both against the FP64 oracle to 1e-8, and
    # the inner iteration counts against the oracle's own float32 emulation.
    p, g, o = make("c3", 16, inner_precision=32, mixed_mode=mode)
    o64 = osolve.Oracle(o.h)
    yd = p.yd[:, 0]
    u, info = g.reduced_solve(cuda(yd), rtol=1e-8)
    uo, _ = o64.reduced_solve(yd, rtol=1e-12)
    assert (info[0]["refine_steps"] > 0) == (mode == 1)
    assert rel(u, uo) < 1e-8
    um, _ = o.reduced_solve(yd, rtol=1e-8)
    assert rel(um, uo) < 1e-8
    assert abs(info[0]["inner_iters_total"] - o.cnt.inner_iters) <= 0.2 * o.cnt.inner_iters + 5


@pytest.mark.parametrize("prec", [64, 32])
def test_chebyshev_smoother_solve(prec):
    # the V-cycle with the degree-2 Chebyshev smoother: same solution as the
    # oracle with the same smoother, and the same inner iteration counts (the
    # FP64 case compares at 1e-10: K and K* applied with inner solves to 1e-10)
    p, g, o = make("c3", 16, smoother=1, inner_precision=prec, inner_rtol=1e-10 if prec == 64 else 1e-8)
    yd = p.yd[:, 0]
    u, info = g.reduced_solve(cuda(yd), rtol=1e-10 if prec == 64 else 1e-8)
    uo, _ = osolve.Oracle(o.h).reduced_solve(yd, rtol=1e-12)
    assert rel(u, uo) < (1e-10 if prec == 64 else 1e-8)
    o.reduced_solve(yd, rtol=1e-10 if prec == 64 else 1e-8)
    assert abs(info[0]["inner_iters_total"] - o.cnt.inner_iters) <= 0.2 * o.cnt.inner_iters + 5


def test_batched_matches_single_columns():
    p, g, o = make("c2", 48, nb_max=4)
    yd = np.stack([inputs.yd_bumps(p.mesh, s) for s in (2, 3, 4)], axis=1)   # nb = 3 (padded to 4)
    U, infos = g.reduced_solve(cuda(yd), rtol=1e-10)
    for k in range(3):
        uk, _ = g.reduced_solve(cuda(yd[:, k]), rtol=1e-10)
        assert rel(U[:, k], uk.cpu().numpy()) < 1e-8
        uo, _ = o.reduced_solve(yd[:, k], rtol=1e-12)
        assert rel(U[:, k], uo) < 1e-8


def test_unpreconditioned_matches_preconditioned():
    p, g, o = make("c2", 32, precond=0)
    yd = p.yd[:, 0]
    u0, i0 = g.reduced_solve(cuda(yd), rtol=1e-10)
    p2, g2, _ = make("c2", 32)
    u1, i1 = g2.reduced_solve(cuda(yd), rtol=1e-10)
    assert rel(u0, u1.cpu().numpy()) < 1e-8
    assert i0[0]["outer_iters"] >= i1[0]["outer_iters"]


def test_gradient_autograd_and_objective():
    from paper_2001_11533_amd import reduced_functional
    p, g, o = make("c2", 32, nb_max=2, **TIGHT)
    rng = np.random.default_rng(4)
    U = rng.standard_normal((p.mesh.nverts, 2))
    yd = np.repeat(p.yd, 2, axis=1)
    u = cuda(U).requires_grad_(True)
    J = reduced_functional(u, cuda(yd), g)
    J.sum().backward()
    for k in range(2):
        gref = o.gradient(U[:, k], yd[:, k])
        assert rel(u.grad[:, k], gref) < 1e-10
        assert abs(float(J[k]) - o.objective(U[:, k], yd[:, k])) <= 1e-11 * abs(o.objective(U[:, k], yd[:, k]))
    Jl, gl = g.objective(cuda(U), cuda(yd))
    assert rel(gl, u.grad.detach().cpu().numpy()) < 1e-11
    # exact quadratic: central difference along a direction
    d = rng.standard_normal(p.mesh.nverts)
    d /= np.linalg.norm(d)
    h = 1e-2
    Jp, _ = g.objective(cuda(U[:, 0] + h * d), cuda(yd[:, 0]), grad=False)
    Jm, _ = g.objective(cuda(U[:, 0] - h * d), cuda(yd[:, 0]), grad=False)
    fd = (float(Jp[0]) - float(Jm[0])) / (2 * h)
    gd = float(u.grad[:, 0].cpu().numpy() @ d)
    assert abs(fd - gd) <= 1e-8 * abs(gd) + 1e-12


def test_error_paths():
    _need_gpu()
    import paper_2001_11533_amd as amg
    from paper_2001_11533_amd import AmgError
    p = inputs.config("c1", n=12)
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    bad = va.copy()
    bad[np.nonzero(ci == 1)[0][0]] += 1e-3          # breaks exact symmetry
    with pytest.raises(AmgError) as e:
        amg.HessianSolver((rp, ci, bad), (rp, ci, vm), p.dirichlet, beta=1e-2)
    assert e.value.code == -2
    neg = va.copy()
    d = np.nonzero(ci == np.repeat(np.arange(len(rp) - 1), np.diff(rp)))[0]
    interior = np.nonzero(p.dirichlet == 0)[0][0]
    neg[d[interior]] = -neg[d[interior]]
    with pytest.raises(AmgError) as e:
        amg.HessianSolver((rp, ci, neg), (rp, ci, vm), p.dirichlet, beta=1e-2, max_coarse=10)
    assert e.value.code == -3
    g = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, beta=1e-2, max_coarse=10, inner_maxit=1)
    with pytest.raises(AmgError) as e:
        g.state_solve(cuda(np.ones(p.mesh.nverts)))
    assert e.value.code == -4
    with pytest.raises(AmgError) as e:
        g.state_solve(cuda(np.ones((p.mesh.nverts, 2))))    # nb above nb_max
    assert e.value.code == -1


def test_indefinite_coarse_level_is_not_spd():
    # A - sigma M with sigma = 1.5 lambda_min(M^-1 A): every diagonal entry on
    # every level stays positive, but the dense levels (18 and 2 rows) are
    # indefinite, so the dense inverse meets a non-positive pivot; the oracle's
    # Cholesky factorisation of the same level fails too
    _need_gpu()
    import scipy.linalg as sla
    import paper_2001_11533_amd as amg
    from paper_2001_11533_amd import AmgError
    from oracle import fem
    p = inputs.config("c1", n=12)
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    dA, dM = np.zeros((n, n)), np.zeros((n, n))
    dA[rows, ci], dM[rows, ci] = va, vm
    inner = np.nonzero(p.dirichlet == 0)[0]
    lam = sla.eigh(dA[np.ix_(inner, inner)], dM[np.ix_(inner, inner)], eigvals_only=True)[0]
    sigma = 1.5 * lam
    shifted = va - sigma * vm
    assert np.all(shifted[rows == ci] > 0)
    A0 = fem.dirichlet_stiffness(fem.CSR(rp, ci, shifted, n), p.dirichlet)
    with pytest.raises(np.linalg.LinAlgError):
        osa.build(A0, fem.CSR(rp, ci, vm, n), p.dirichlet, osa.Opts(max_coarse=10))
    print(f"[parity] indefinite shift sigma={sigma:.3f}", flush=True)
    with pytest.raises(AmgError) as e:
        amg.HessianSolver((rp, ci, shifted), (rp, ci, vm), p.dirichlet, beta=1e-2, max_coarse=10)
    assert e.value.code == -3 and "pivot" in str(e.value)


def test_graph_replay_matches_eager_launches():
    # the captured CG iterations are replayed many times, with eager work and
    # host synchronisations in between; every replay must reproduce the eager
    # launches bit for bit
    # (graphs for every CG, and for the mass-matrix CGs only)
    pe, ge, _ = make("c3", 12, max_coarse=40, use_graphs=0)
    for mode in (1, 2):
        pg, gg, o = make("c3", 12, max_coarse=40, use_graphs=mode)
        rng = np.random.default_rng(21)
        for k in range(3):
            u = cuda(rng.standard_normal(pg.mesh.nverts))
            a = gg.hessian_apply(u)
            b = ge.hessian_apply(u)
            assert torch.equal(a, b), (mode, k)
            za = gg.precond_apply(u)
            zb = ge.precond_apply(u)
            assert torch.equal(za, zb), (mode, k)
        ua, _ = gg.reduced_solve(cuda(pg.yd[:, 0]))
        ub, _ = ge.reduced_solve(cuda(pg.yd[:, 0]))
        assert torch.equal(ua, ub), mode


def test_coarsest_hessian_by_loose_cg():
    # coarsest Hessian level above dense_max: unpreconditioned CG to 1e-4 on it
    # (the practice of Section 5.2), on both sides
    p, g, o = make("c2", 16, max_coarse=30, dense_max=30, hess_levels=2, beta=1e-3)
    assert g.levels()[1] == 2 and o.h.chol_H is None
    assert g.dense(1).size == 0
    yd = p.yd[:, 0]
    u, info = g.reduced_solve(cuda(yd), rtol=1e-10)
    uo, it = o.reduced_solve(yd, rtol=1e-12)
    assert rel(u, uo) < 1e-8


def test_hierarchy_quality_against_oracle():
    # a~_j of Section 4 by the same power method from the same start vector on
    # both sides, and near the largest singular value of the explicit E
    p, g, o = make("c2", 24, max_coarse=12, **TIGHT)
    rng = np.random.default_rng(29)
    L = g.levels()[0]
    assert L >= 3
    for j in range(L - 1):
        v0 = rng.standard_normal(p.mesh.nverts if j == 0 else g.level_n(j))
        at_gpu = g.hierarchy_quality(j, cuda(v0), iters=40)
        at_orc = o.quality(j, v0, 40)
        assert abs(at_gpu - at_orc) <= 1e-8 * at_orc
        a, at = odense.quality(o.h, j)
        assert at_orc <= at * (1 + 1e-9) and at_orc >= 0.99 * at


def test_time_kernel_entries():
    # every entry of amg_time_kernel times its launches and reports algorithmic
    # bytes; the level-0 entries run with and without the XCD rotation of the
    # sliced-ELL kernel, which must leave the solver's own launches untouched
    import paper_2001_11533_amd as amg
    from paper_2001_11533_amd import AmgError
    p, g, o = make("c3", 12, max_coarse=40, inner_precision=32, smoother=1)
    yd = cuda(p.yd[:, 0])
    u0, _ = g.reduced_solve(yd)
    for which in range(4):
        ms, by = g.time_kernel(which, prec=32, nb=1, reps=3)
        assert ms > 0 and by > 0, which
    ms, by = g.time_kernel(3, prec=64, nb=1, reps=3)
    assert ms > 0 and by > 0
    # the FP64 CG product (FP64 only), and a grid barrier against a kernel boundary
    ms, by = g.time_kernel(4, prec=64, nb=1, reps=3)
    assert ms > 0 and by > 0
    with pytest.raises(AmgError):
        g.time_kernel(4, prec=32, nb=1, reps=3)
    for which in (5, 6):
        ms, by = g.time_kernel(which, prec=64, nb=1, reps=20)
        assert ms > 0, which
    with pytest.raises(AmgError):
        g.time_kernel(7, prec=32, nb=1, reps=3)
    u1, _ = g.reduced_solve(yd)
    assert torch.equal(u0, u1)


def test_solve_info_fields():
    # amg_info of a reduced solve: the true residual recomputed at exit agrees
    # with the recursive one, the phase times add up to about the call, and the
    # algorithmic bytes grow with the work
    p, g, o = make("c3", 12, max_coarse=40, inner_precision=32, smoother=1, true_resid=1)
    yd = cuda(p.yd[:, 0])
    u, info = g.reduced_solve(yd, rtol=1e-8)
    f = info[0]
    assert 0 < f["true_rel_resid"] <= 1e-7 and abs(f["true_rel_resid"] - f["rel_resid"]) <= 1e-8
    ph = f["ms_phase"]
    assert all(v >= 0 for v in ph.values()) and ph["hessian"] > 0 and ph["precond"] > 0 and ph["true_resid"] > 0
    assert sum(ph.values()) <= f["ms_total"] * 1.05 + 0.5
    assert f["bytes_moved"] > 0
    _, info2 = g.reduced_solve(yd, rtol=1e-4)
    assert 0 < info2[0]["bytes_moved"] < f["bytes_moved"]
    # without the option nothing is recomputed
    p, g2, _ = make("c3", 12, max_coarse=40)
    _, info3 = g2.reduced_solve(yd, rtol=1e-8)
    assert info3[0]["true_rel_resid"] == -1.0 and info3[0]["ms_phase"]["true_resid"] == 0.0


def test_wide_slices_fall_back_to_csr():
    # a randomly numbered 41^3 mesh: a slice of 64 rows then spans ~68,900
    # columns, beyond 16-bit offsets, so level 0 keeps no sliced-ELL copy and
    # its products run on CSR.  The hierarchy depends on the numbering, the
    # reduced solution (to a tight tolerance) does not.
    import paper_2001_11533_amd as amg
    _need_gpu()
    p = inputs.config("c3", n=40)
    rng = np.random.default_rng(41)
    perm = rng.permutation(p.mesh.nverts)          # new index -> old index
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))

    def solver(coords, elems, dirichlet):
        rp, ci, va, vm = amg.assemble_p1(coords, elems, p.kappa)
        return amg.HessianSolver((rp, ci, va), (rp, ci, vm), dirichlet, beta=p.beta,
                                 inner_precision=32, smoother=1)

    g0 = solver(p.mesh.coords, p.mesh.elems, p.dirichlet)
    g1 = solver(np.ascontiguousarray(p.mesh.coords[perm]), inv[p.mesh.elems].astype(p.mesh.elems.dtype),
                np.ascontiguousarray(p.dirichlet[perm]))
    yd = p.yd[:, 0]
    u0, _ = g0.reduced_solve(cuda(yd), rtol=1e-10)
    u1, _ = g1.reduced_solve(cuda(yd[perm]), rtol=1e-10)
    back = torch.empty_like(u1)
    back[torch.as_tensor(perm, device="cuda")] = u1
    assert rel(back, u0.cpu().numpy()) < 1e-7
    # without the copy the timed pre-sweep residual counts 4-byte columns: its
    # algorithmic bytes exceed the natural numbering's by 2 nnz(A_0)
    _, b0 = g0.time_kernel(1, prec=32, nb=1, reps=1)
    _, b1 = g1.time_kernel(1, prec=32, nb=1, reps=1)
    assert b1 > b0


def test_wide_rows_take_sixteen_loads():
    # Interior nodes of the 14^3 Kuhn cube moved by up to 0.1 h per coordinate:
    # no stiffness entry is exactly zero any more, so A_0 keeps the 15-entry
    # rows of the tetrahedral mesh graph and the level-0 sliced-ELL products
    # (V-cycle sweeps, the FP64 CG product) take sixteen loads per lane instead
    # of eight.  The reduced solve of the headline configuration against the
    # oracle on the same mesh.  (Heights of a Kuhn tetrahedron are at least
    # h / sqrt(2); nodes moving by at most 0.1 sqrt(3) h keep every element's
    # orientation.)
    import dataclasses

    import paper_2001_11533_amd as amg
    _need_gpu()
    p = inputs.config("c3", n=14)
    m = p.mesh
    rng = np.random.default_rng(1411)
    h = 1.0 / m.n
    move = rng.uniform(-0.1 * h, 0.1 * h, size=m.coords.shape) * (m.boundary == 0)[:, None]
    m = dataclasses.replace(m, coords=np.ascontiguousarray(m.coords + move))
    p = dataclasses.replace(p, mesh=m)
    rp, ci, va, vm = amg.assemble_p1(m.coords, m.elems, p.kappa)
    g = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, beta=p.beta, inner_precision=32, smoother=1)
    n0, nnz0, _, _ = g.level_size(0)
    assert np.diff(g.csr(0, 0)[0]).max() == 15   # interior rows: the vertex and its 14 neighbours
    h_, _, _ = osolve.build_problem(p, osa.Opts(beta=p.beta, smoother=1))
    yd = p.yd[:, 0]
    print(f"[parity] wide rows: N={m.nverts} nnz(A_0)={nnz0}", flush=True)
    u, info = g.reduced_solve(cuda(yd), rtol=1e-8)
    uo, _ = osolve.Oracle(h_).reduced_solve(yd, rtol=1e-12)
    assert rel(u, uo) < 1e-8
    o = osolve.Oracle(h_, mixed=True)
    o.reduced_solve(yd, rtol=1e-8)
    assert abs(info[0]["inner_iters_total"] - o.cnt.inner_iters) <= 0.2 * o.cnt.inner_iters + 5
