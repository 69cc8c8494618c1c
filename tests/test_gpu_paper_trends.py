"""The paper's qualitative results on synthetic meshes (Section 5.3): with the
multilevel Hessian preconditioner the outer CG needs few iterations that fall
as beta grows and do not grow with N (Table 3), far fewer than plain CG with
the same inner solves (Table 4), and with two Hessian levels the counts stay
bounded as h -> 0 (Table 5).  The paper's own counts (BoomerAMG hierarchies,
its meshes) are context, not targets; these are the properties its tables show,
with bounds that leave room for the different hierarchy."""
import numpy as np
import pytest

import inputs
from inputs import Problem, kappa_const, mesh2d, mesh3d, yd_manufactured, yd_sin

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def outer_iters(p, beta, **opts):
    import paper_2001_11533_amd as amg
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    g = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, beta=beta, **opts)
    u, info = g.reduced_solve(torch.tensor(p.yd[:, 0], device="cuda"), rtol=1e-8)
    g.close()
    return info[0]["outer_iters"], u


def cube(n, beta):
    m = mesh3d(n)
    return Problem("cube", m, kappa_const(m), beta, np.ascontiguousarray(yd_manufactured(m, beta)[:, None]),
                   m.boundary)


def test_multilevel_counts_follow_table3_and_beat_plain_cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bound = {1e-4: 12, 1e-2: 5, 1.0: 3, 100.0: 3}
    for beta, top in bound.items():
        its = []
        for n in (16, 32):
            p = cube(n, beta)
            ml, u_ml = outer_iters(p, beta)
            plain, u_plain = outer_iters(p, beta, precond=0)
            print(f"3D n={n} beta={beta:g}: multilevel {ml}, plain CG {plain}", flush=True)
            assert ml <= top
            assert 2 * ml <= plain
            assert float(torch.linalg.norm(u_ml - u_plain) / torch.linalg.norm(u_plain)) < 1e-5
            its.append(ml)
        assert its[1] <= its[0] + 1          # no growth with N


def test_two_level_counts_bounded_in_h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for beta in (1e-4, 1e-2):
        its = []
        for n in (32, 64, 128, 256):
            m = mesh2d(n)
            p = Problem("square", m, kappa_const(m), beta, np.ascontiguousarray(yd_sin(m)[:, None]), m.boundary)
            it, _ = outer_iters(p, beta, hess_levels=2)
            its.append(it)
        print(f"2D two-level beta={beta:g}: {its}", flush=True)
        assert max(its) - min(its) <= 2
        assert max(its) <= 10
