"""Parity at the benchmark's full size (3D 64^3, N = 274,625, log-normal kappa,
beta = 1e-3) in the configuration bench.py times: inner A-solves by FP64 CG
preconditioned with float32 V-cycles smoothed by the degree-2 Chebyshev
iteration (inner_precision = 32, mixed_mode = 0, smoother = 1), nb = 1.

* the GPU hierarchy is bit-exact with the oracle's at every level: A_j, M_j,
  S_j, S_j^T, aggregates and roots;
* the reduced solve agrees with the oracle's FP64 solution (same smoother,
  solved to 1e-11) to 1e-8, and so does the FP64 GPU path."""
import numpy as np
import pytest

import inputs
from oracle import sa as osa
from oracle import solve as osolve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.timeout(900)
def test_full_size_64cube_bench_configuration_against_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_11533_amd as amg
    p = inputs.config("c3")
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    print("[fullsize] 64^3 bench configuration: setup", flush=True)
    g = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, beta=p.beta, inner_precision=32, smoother=1)
    h, A, M = osolve.build_problem(p, osa.Opts(beta=p.beta, smoother=1))
    L, ell = g.levels()
    assert L == h.L == 4 and ell == h.ell
    for j in range(L):
        lev = h.levels[j]
        mats = [(0, lev.A), (3, lev.M)] + ([(1, lev.S), (2, lev.St)] if j < L - 1 else [])
        for which, ref in mats:
            rpj, cij, vj = g.csr(j, which)
            assert np.array_equal(rpj, ref.rowptr) and np.array_equal(cij, ref.col), (j, which)
            assert np.array_equal(vj.view(np.uint64), ref.val.view(np.uint64)), (j, which)
        if j < L - 1:
            agg, root = g.aggregates(j)
            assert np.array_equal(agg, lev.agg) and np.array_equal(root.astype(bool), lev.root), j
    print("[fullsize] hierarchy bit-exact; solves", flush=True)
    yd = torch.tensor(p.yd[:, 0], device="cuda")
    u, info = g.reduced_solve(yd, rtol=1e-8)
    g.close()
    g64 = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, beta=p.beta, inner_precision=64, smoother=1)
    u64, info64 = g64.reduced_solve(yd, rtol=1e-8)
    g64.close()
    o = osolve.Oracle(h)
    uo, it = o.reduced_solve(p.yd[:, 0], rtol=1e-11)
    err = float(np.linalg.norm(u.cpu().numpy() - uo) / np.linalg.norm(uo))
    err64 = float(np.linalg.norm(u64.cpu().numpy() - uo) / np.linalg.norm(uo))
    print(f"[fullsize] 64^3 vs FP64 oracle: float32-preconditioned {err:.3e} (outer {info[0]['outer_iters']}), "
          f"FP64 {err64:.3e} (outer {info64[0]['outer_iters']}), oracle outer {it}", flush=True)
    assert info[0]["rel_resid"] <= 1e-8 and info64[0]["rel_resid"] <= 1e-8
    assert err < 1e-8 and err64 < 1e-8
