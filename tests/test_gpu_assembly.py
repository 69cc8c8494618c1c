"""P1 assembly on the GPU (amg_p1_pattern_device / amg_p1_assemble_device)
against the host assembler, bit for bit, and its argument checks.  The host
assembler is itself pinned to the oracle's assembly (tests/test_lib_host.py)."""
import ctypes as C

import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype=dt, device="cuda")


def renumbered(m, seed):
    # the same mesh with a random vertex numbering: element lists around a
    # vertex arrive out of order, and rows gather far-apart columns
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m.nverts)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    return np.ascontiguousarray(m.coords[perm]), inv[m.elems].astype(np.int32)


@pytest.mark.parametrize("kind", ["2d", "2dj", "3d", "3d_renumbered", "3d64"])
def test_device_assembly_bit_identical_to_host(kind):
    _need_gpu()
    import paper_2001_11533_amd as amg
    m = {"2d": lambda: inputs.mesh2d(9), "2dj": lambda: inputs.mesh2d(40, jitter=0.2),
         "3d": lambda: inputs.mesh3d(7), "3d_renumbered": lambda: inputs.mesh3d(9),
         "3d64": lambda: inputs.mesh3d(64)}[kind]()
    kappa = inputs.kappa_lognormal(m, 1.0)
    coords, elems = m.coords, m.elems
    if kind == "3d_renumbered":
        coords, elems = renumbered(m, 7)
    print(f"[assembly] {kind}: nv={len(coords)} ne={len(elems)}", flush=True)
    rp, ci, va, vm = amg.assemble_p1(coords, elems, kappa)
    r2, c2, a2, m2 = amg.assemble_p1_device(dev(coords, torch.float64), dev(elems, torch.int32),
                                            dev(kappa, torch.float64))
    assert np.array_equal(r2.cpu().numpy(), rp)
    assert np.array_equal(c2.cpu().numpy(), ci)
    # the same operations in the same order: equal to the last bit
    assert np.array_equal(a2.cpu().numpy().view(np.int64), va.view(np.int64))
    assert np.array_equal(m2.cpu().numpy().view(np.int64), vm.view(np.int64))


def test_device_assembly_rejects_bad_input():
    _need_gpu()
    import paper_2001_11533_amd as amg
    from paper_2001_11533_amd import AmgError
    from paper_2001_11533_amd._lib import lib
    m = inputs.mesh2d(6)
    kappa = inputs.kappa_lognormal(m, 1.0)
    coords, elems, kap = dev(m.coords, torch.float64), dev(m.elems, torch.int32), dev(kappa, torch.float64)
    bad = elems.clone()
    bad[3, 1] = m.nverts                       # vertex id out of range
    with pytest.raises(AmgError) as e:
        amg.assemble_p1_device(coords, bad, kap)
    assert e.value.code == -1
    bad[3, 1] = -1
    with pytest.raises(AmgError) as e:
        amg.assemble_p1_device(coords, bad, kap)
    assert e.value.code == -1
    # an nnz that is not the mesh graph's is refused before anything is written
    rp, ci, va, vm = amg.assemble_p1_device(coords, elems, kap)
    nnz = int(ci.numel())
    col = torch.full((nnz,), -7, dtype=torch.int32, device="cuda")
    L = lib()
    rc = L.amg_p1_assemble_device(2, m.nverts, coords.data_ptr(), len(m.elems), elems.data_ptr(), kap.data_ptr(),
                                  nnz - 1, rp.data_ptr(), col.data_ptr(), va.data_ptr(), vm.data_ptr(), None)
    assert rc == -1
    assert bool((col == -7).all())
    n = C.c_int32(0)
    assert L.amg_p1_pattern_device(4, m.nverts, len(m.elems), elems.data_ptr(), C.byref(n), None) == -1
    assert L.amg_p1_pattern_device(2, m.nverts, len(m.elems), None, C.byref(n), None) == -1
