"""The allocation-free GPU assembly (amg_p1_assemble_device_noalloc) against the
allocating one (amg_p1_assemble_device), both called through the C ABI:
bit-identical pattern and values on two calls in a row, the second with a
smaller mesh (the static workspace keeps the first call's contents, which
must not leak into the second), and the refusal of a mesh whose workspace
exceeds the static array, before anything runs."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype=dt, device="cuda")


def _assemble(fn_name, m, kappa):
    from paper_2001_11533_amd._lib import check, lib
    import ctypes as C
    L = lib()
    coords, elems, kap = _dev(m.coords, torch.float64), _dev(m.elems, torch.int32), _dev(kappa, torch.float64)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    nnz = C.c_int32(0)
    check(L.amg_p1_pattern_device(m.dim, m.nverts, m.nelems, elems.data_ptr(), C.byref(nnz), stream))
    rp = torch.full((m.nverts + 1,), -3, dtype=torch.int32, device="cuda")
    col = torch.full((nnz.value,), -3, dtype=torch.int32, device="cuda")
    va = torch.full((nnz.value,), np.nan, dtype=torch.float64, device="cuda")
    vm = torch.full((nnz.value,), np.nan, dtype=torch.float64, device="cuda")
    check(getattr(L, fn_name)(m.dim, m.nverts, coords.data_ptr(), m.nelems, elems.data_ptr(), kap.data_ptr(),
                              nnz.value, rp.data_ptr(), col.data_ptr(), va.data_ptr(), vm.data_ptr(), stream))
    return [t.cpu().numpy() for t in (rp, col, va, vm)]


def test_noalloc_assembly_matches_allocating_one():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # the 64^3 cube (the largest the static workspace holds), then a smaller 2D mesh
    for m in (inputs.mesh3d(64), inputs.mesh2d(37, jitter=0.2)):
        kappa = inputs.kappa_lognormal(m, 1.0)
        print(f"[no-alloc] dim={m.dim} nv={m.nverts} ne={m.nelems}", flush=True)
        ref = _assemble("amg_p1_assemble_device", m, kappa)
        got = _assemble("amg_p1_assemble_device_noalloc", m, kappa)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2].view(np.uint64), ref[2].view(np.uint64))
        assert np.array_equal(got[3].view(np.uint64), ref[3].view(np.uint64))


def test_noalloc_assembly_refuses_a_mesh_beyond_its_workspace():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2001_11533_amd._lib import lib
    # the 128^3 cube's sizes need about 225 MB of workspace: refused on the host
    # from the sizes alone, before any pointer is read or any kernel runs
    nv, ne = 129 ** 3, 6 * 128 ** 3
    small = torch.zeros(16, dtype=torch.float64, device="cuda")
    ids = torch.zeros(16, dtype=torch.int32, device="cuda")
    rc = lib().amg_p1_assemble_device_noalloc(3, nv, small.data_ptr(), ne, ids.data_ptr(), small.data_ptr(), 16,
                                              ids.data_ptr(), ids.data_ptr(), small.data_ptr(), small.data_ptr(),
                                              None)
    assert rc == -1
