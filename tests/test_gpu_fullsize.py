"""Parity at the benchmark's full size (3D 64^3, N = 274,625) in the launch
configuration bench.py times (float32 inner solves in FP64 refinement, nb = 1):
the GPU hierarchy is bit-exact with the oracle's and the reduced solve agrees
with the oracle's FP64 solution to 1e-8."""
import numpy as np
import pytest

import inputs
from oracle import sa as osa
from oracle import solve as osolve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_full_size_64cube_against_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_11533_amd as amg
    p = inputs.config("c3")
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    g = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, beta=p.beta, inner_precision=32)
    h, A, M = osolve.build_problem(p, osa.Opts(beta=p.beta))
    L, ell = g.levels()
    assert L == h.L == 4 and ell == h.ell
    for j in range(L):
        lev = h.levels[j]
        rpj, cij, vj = g.csr(j, 0)
        assert np.array_equal(rpj, lev.A.rowptr) and np.array_equal(cij, lev.A.col)
        assert np.array_equal(vj.view(np.uint64), lev.A.val.view(np.uint64))
        if j < L - 1:
            agg, root = g.aggregates(j)
            assert np.array_equal(agg, lev.agg)
    yd = torch.tensor(p.yd[:, 0], device="cuda")
    u, info = g.reduced_solve(yd, rtol=1e-8)
    o = osolve.Oracle(h)
    uo, it = o.reduced_solve(p.yd[:, 0], rtol=1e-11)
    err = float(np.linalg.norm(u.cpu().numpy() - uo) / np.linalg.norm(uo))
    print(f"64^3 mixed-precision GPU solve vs FP64 oracle: rel. error {err:.3e}, outer {info[0]['outer_iters']} vs {it}")
    assert err < 1e-8
