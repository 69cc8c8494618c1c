"""The sparse-product autotuner (amg_autotune): it times the lanes-per-row
choices of every CSR product, records them in the process-wide table (and a
JSON file), applies them, and later contexts built with autotune = 1 take them
from the table.  A tuned choice changes the order in which a row's entries are
summed, so the parity checks against the oracle are repeated under tuned
choices: one V-cycle, the Hessian action, and reduced solves of one and of
sixteen columns."""
import json

import numpy as np
import pytest

import inputs
from oracle import sa as osa
from oracle import solve as osolve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def cuda(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel(a, b):
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("nb", [1, 16])
def test_autotuned_products_keep_oracle_parity(nb, tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_11533_amd as amg
    p = inputs.config("c3", n=16, nb=nb)
    rp, ci, va, vm = amg.assemble_p1(p.mesh.coords, p.mesh.elems, p.kappa)
    kw = dict(beta=p.beta, nb_max=nb, inner_precision=32, smoother=1, max_coarse=40, inner_rtol=1e-13,
              mass_rtol=1e-14, precond_inner_rtol=1e-13)
    print(f"[autotune] c3 n=16 nb={nb}", flush=True)
    g = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, **kw)
    path = str(tmp_path / "tune.json")
    timed = g.autotune(reps=3, cache_path=path)
    assert timed > 0
    entries = json.load(open(path))["entries"]
    assert len(entries) >= timed and all(0 <= e["lg"] <= 6 and len(e["us"]) >= 1 for e in entries)
    assert g.autotune(reps=3, cache_path=path) == 0           # everything is in the table now
    # a new context of the same shapes takes the table's choices at setup
    g2 = amg.HessianSolver((rp, ci, va), (rp, ci, vm), p.dirichlet, autotune=1, **kw)
    h, _, _ = osolve.build_problem(p, osa.Opts(beta=p.beta, smoother=1, max_coarse=40, inner_rtol=1e-13,
                                                mass_rtol=1e-14, precond_inner_rtol=1e-13))
    o = osolve.Oracle(h)
    rng = np.random.default_rng(3)
    for gg in (g, g2):
        L, _ = gg.levels()
        for j in range(L):
            b = rng.standard_normal(gg.level_n(j))
            assert rel(gg.vcycle_apply(cuda(b), level=j, prec=64), o.vcycle(j, b)) < 1e-13, j
        u = rng.standard_normal(p.mesh.nverts)
        assert rel(gg.hessian_apply(cuda(u)), o.hessian_apply(0, u)) < 1e-11
        U, infos = gg.reduced_solve(cuda(p.yd), rtol=1e-10)
        U = U.reshape(p.mesh.nverts, -1)
        for c in range(nb):
            uo, _ = o.reduced_solve(p.yd[:, c], rtol=1e-12)
            assert rel(U[:, c], uo) < 1e-8, c
    g.close()
    g2.close()
