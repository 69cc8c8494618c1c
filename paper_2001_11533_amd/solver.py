"""Python binding of the amghess C ABI.

Every computation runs in the HIP library; this module only moves arguments:
torch tensors supply device memory (``data_ptr``) and the HIP stream
(``torch.cuda.current_stream().cuda_stream``).  There is no CPU fallback: the
calls raise if the library or a GPU is missing.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import Csr, Info, Opts, check, lib


def assemble_p1(coords: np.ndarray, elems: np.ndarray, kappa: np.ndarray):
    """P1 stiffness A and mass M of a simplicial mesh by the library's host
    assembler (paper, Section 2).  Returns numpy (rowptr, col, valA, valM)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    elems = np.ascontiguousarray(elems, dtype=np.int32)
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    dim = coords.shape[1]
    nv, ne = coords.shape[0], elems.shape[0]
    if elems.shape[1] != dim + 1 or kappa.shape[0] != ne:
        raise ValueError("mesh arrays have inconsistent shapes")
    L = lib()
    nnz = C.c_int32(0)
    check(L.amg_p1_pattern(dim, nv, ne, elems.ctypes.data, C.byref(nnz)))
    rowptr = np.empty(nv + 1, dtype=np.int32)
    col = np.empty(nnz.value, dtype=np.int32)
    valA = np.empty(nnz.value, dtype=np.float64)
    valM = np.empty(nnz.value, dtype=np.float64)
    check(L.amg_p1_assemble(dim, nv, coords.ctypes.data, ne, elems.ctypes.data, kappa.ctypes.data, nnz.value,
                            rowptr.ctypes.data, col.ctypes.data, valA.ctypes.data, valM.ctypes.data))
    return rowptr, col, valA, valM


def assemble_p1_device(coords, elems, kappa):
    """The same assembly on the GPU (amg_p1_pattern_device / amg_p1_assemble_device),
    bit-identical to assemble_p1.  coords (nv x dim, float64), elems (ne x (dim+1),
    int32) and kappa (ne, float64) are CUDA tensors; returns CUDA tensors (rowptr,
    col, valA, valM), computed on torch's current stream."""
    import torch
    if not (coords.is_cuda and elems.is_cuda and kappa.is_cuda):
        raise ValueError("assemble_p1_device takes device tensors")
    coords = coords.to(torch.float64).contiguous()
    elems = elems.to(torch.int32).contiguous()
    kappa = kappa.to(torch.float64).contiguous()
    dim = coords.shape[1]
    nv, ne = coords.shape[0], elems.shape[0]
    if elems.shape[1] != dim + 1 or kappa.shape[0] != ne:
        raise ValueError("mesh arrays have inconsistent shapes")
    L = lib()
    stream = C.c_void_p(torch.cuda.current_stream(coords.device).cuda_stream)
    nnz = C.c_int32(0)
    check(L.amg_p1_pattern_device(dim, nv, ne, elems.data_ptr(), C.byref(nnz), stream))
    dev = coords.device
    rowptr = torch.empty(nv + 1, dtype=torch.int32, device=dev)
    col = torch.empty(nnz.value, dtype=torch.int32, device=dev)
    valA = torch.empty(nnz.value, dtype=torch.float64, device=dev)
    valM = torch.empty(nnz.value, dtype=torch.float64, device=dev)
    check(L.amg_p1_assemble_device(dim, nv, coords.data_ptr(), ne, elems.data_ptr(), kappa.data_ptr(), nnz.value,
                                   rowptr.data_ptr(), col.data_ptr(), valA.data_ptr(), valM.data_ptr(), stream))
    return rowptr, col, valA, valM


def release_memory() -> None:
    """Return the device memory that ended contexts keep cached for later ones
    to the driver (amg_release_memory)."""
    check(lib().amg_release_memory(), None)


def default_opts(**kw) -> Opts:
    o = Opts()
    check(lib().amg_opts_default(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k!r}")
        setattr(o, k, v)
    return o


def _to_dev(x, dtype, device):
    if isinstance(x, torch.Tensor):
        if x.dtype != dtype:
            raise TypeError(f"expected {dtype}")
        return x.to(device).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32 if dtype == torch.int32 else
                                                np.float64 if dtype == torch.float64 else np.uint8)).to(device)


def _dev_csr(rowptr, col, val, device):
    """CSR arrays (numpy, or tensors already resident on the device) as an amg_csr."""
    rp = _to_dev(rowptr, torch.int32, device)
    ci = _to_dev(col, torch.int32, device)
    v = _to_dev(val, torch.float64, device)
    n = rp.numel() - 1
    return Csr(n, n, ci.numel(), rp.data_ptr(), ci.data_ptr(), v.data_ptr()), (rp, ci, v)


@dataclass
class SolveInfo:
    outer_iters: int
    inner_solves: int
    inner_iters_total: int
    inner_iters_max: int
    mass_iters_total: int
    refine_steps: int
    levels: int
    ell: int
    rel_resid: float
    ms_total: float


class HessianSolver:
    """A setup of the library: the smoothed-aggregation hierarchy, the dense
    coarse factors and the solve workspaces for batches of up to nb_max."""

    def __init__(self, A, M, dirichlet=None, beta: float = 1e-2, device="cuda", **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("HessianSolver needs a ROCm GPU")
        self.device = torch.device(device)
        self.opts = default_opts(beta=beta, **opts)
        Ac, self._A = _dev_csr(*A, self.device)
        Mc, self._M = _dev_csr(*M, self.device)
        self.N = Ac.nrows
        if dirichlet is not None:
            self._mask = _to_dev(dirichlet, torch.uint8, self.device)
            mptr = self._mask.data_ptr()
        else:
            self._mask, mptr = None, None
        # every call of the context runs on this stream: inputs and outputs are
        # made and used on it, so torch and the library see the same order
        self._stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = lib().amg_setup(C.byref(Ac), C.byref(Mc), mptr, C.byref(self.opts), self._stream.cuda_stream,
                             C.byref(h))
        check(rc, None)
        self._h = h
        self.beta = beta
        self.nb_max = self.opts.nb_max

    # ---- helpers ----
    def close(self):
        if getattr(self, "_h", None):
            lib().amg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_stream(self):
        """The library enqueues on the stream current at construction; a call
        made while another stream is current would let torch allocate, copy and
        read its tensors out of order with the library's work."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self._stream:
            raise RuntimeError("HessianSolver calls must run on the stream that was current when it was built "
                               f"(built on {self._stream}, called on {cur})")

    def _vec(self, x: torch.Tensor, n: int):
        self._check_stream()
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
            raise TypeError("expected a float64 GPU tensor")
        squeeze = x.dim() == 1
        x2 = x.reshape(n, -1).contiguous() if not squeeze else x.reshape(n, 1).contiguous()
        if x2.shape[0] != n:
            raise ValueError(f"expected {n} rows")
        return x2, squeeze

    def level_n(self, level: int) -> int:
        n = C.c_int32()
        check(lib().amg_level_size(self._h, level, C.byref(n), None, None, None), self._h)
        return n.value

    def _call(self, fn, level, x, with_level=True):
        n = self.level_n(level)
        x2, sq = self._vec(x, n)
        nb = x2.shape[1]
        out = torch.empty_like(x2)
        info = Info()
        if with_level:
            rc = fn(self._h, level, x2.data_ptr(), out.data_ptr(), nb, C.byref(info))
        else:
            rc = fn(self._h, x2.data_ptr(), out.data_ptr(), nb, C.byref(info))
        check(rc, self._h)
        self.last_info = info.as_dict()
        return out.reshape(-1) if sq else out

    # ---- the calls of the C ABI ----
    def state_solve(self, u, level: int = 0):
        """y = K u = A^{-1} M_yu u."""
        return self._call(lib().state_solve, level, u)

    def adjoint_solve(self, w, level: int = 0):
        """z = K^T w = M_yu^T A^{-1} w."""
        return self._call(lib().adjoint_solve, level, w)

    def hessian_apply(self, u, level: int = 0):
        """H u = (K^T M_y K + beta M_u) u."""
        return self._call(lib().hessian_apply, level, u)

    def precond_apply(self, r):
        """z = B_0 r, the multilevel Hessian preconditioner."""
        return self._call(lib().hessian_precond_apply, 0, r, with_level=False)

    def reduced_solve(self, yd, u0=None, rtol: float = 1e-8):
        """Solve (K^T M_y K + beta M_u) u = K^T M_y y_d; returns (u, [info per column])."""
        y2, sq = self._vec(yd, self.N)
        nb = y2.shape[1]
        u = torch.empty_like(y2)
        infos = (Info * nb)()
        u0p = None
        if u0 is not None:
            u0c, _ = self._vec(u0, self.N)
            u0p = u0c.data_ptr()
        rc = lib().reduced_solve(self._h, y2.data_ptr(), u0p, u.data_ptr(), nb, rtol, infos)
        check(rc, self._h)
        return (u.reshape(-1) if sq else u), [i.as_dict() for i in infos]

    def objective(self, u, yd, grad: bool = True):
        """(J per column as a CPU float64 tensor, gradient or None)."""
        u2, sq = self._vec(u, self.N)
        y2, _ = self._vec(yd, self.N)
        nb = u2.shape[1]
        J = np.zeros(nb, dtype=np.float64)
        g = torch.empty_like(u2) if grad else None
        info = Info()
        rc = lib().reduced_objective(self._h, u2.data_ptr(), y2.data_ptr(), J.ctypes.data,
                                     g.data_ptr() if grad else None, nb, C.byref(info))
        check(rc, self._h)
        if g is not None and sq:
            g = g.reshape(-1)
        return torch.from_numpy(J), g

    def mass_apply(self, x, which: int = 0, level: int = 0):
        """M x with which = 0: M_u, 1: M_y, 2: M_yu, 3: M_yu^T."""
        n = self.level_n(level)
        x2, sq = self._vec(x, n)
        out = torch.empty_like(x2)
        check(lib().amg_mass_apply(self._h, level, which, x2.data_ptr(), out.data_ptr(), x2.shape[1]), self._h)
        return out.reshape(-1) if sq else out

    def mass_quad(self, x, which: int = 0):
        """x_c^T M x_c per column (CPU float64 tensor)."""
        x2, sq = self._vec(x, self.N)
        q = np.zeros(x2.shape[1], dtype=np.float64)
        check(lib().amg_mass_quad(self._h, which, x2.data_ptr(), q.ctypes.data, x2.shape[1]), self._h)
        return torch.from_numpy(q)

    # ---- introspection ----
    def levels(self):
        L, ell = C.c_int32(), C.c_int32()
        check(lib().amg_num_levels(self._h, C.byref(L), C.byref(ell)), self._h)
        return L.value, ell.value

    def level_size(self, level: int):
        n, a, s, m = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().amg_level_size(self._h, level, C.byref(n), C.byref(a), C.byref(s), C.byref(m)), self._h)
        return n.value, a.value, s.value, m.value

    def aggregates(self, level: int):
        n = self.level_n(level)
        agg = np.empty(n, dtype=np.int32)
        root = np.empty(n, dtype=np.uint8)
        check(lib().amg_copy_aggregates(self._h, level, agg.ctypes.data, root.ctypes.data), self._h)
        return agg, root

    def csr(self, level: int, which: int):
        """which: 0 = A_j, 1 = S_j, 2 = S_j^T, 3 = M_j; numpy (rowptr, col, val)."""
        n, nnzA, nnzS, nnzM = self.level_size(level)
        nrows = {0: n, 1: n, 2: self.level_n(level + 1) if which == 2 else n, 3: n}[which]
        nnz = {0: nnzA, 1: nnzS, 2: nnzS, 3: nnzM}[which]
        rp = np.empty(nrows + 1, dtype=np.int32)
        ci = np.empty(nnz, dtype=np.int32)
        v = np.empty(nnz, dtype=np.float64)
        check(lib().amg_copy_csr(self._h, level, which, rp.ctypes.data, ci.ctypes.data, v.ctypes.data), self._h)
        return rp, ci, v

    def dense(self, which: int):
        """which: 0 = inverse of the coarsest A, 1 = coarsest dense Hessian, 2 = its inverse."""
        n = C.c_int32()
        check(lib().amg_copy_dense(self._h, which, C.byref(n), None), self._h)
        out = np.empty((n.value, n.value), dtype=np.float64)
        check(lib().amg_copy_dense(self._h, which, C.byref(n), out.ctypes.data), self._h)
        return out

    def autotune(self, reps: int = 20, cache_path: str | None = None) -> int:
        """Time the lanes-per-row choices of this context's sparse products (amg_autotune);
        returns how many products were timed.  The choices go to the process-wide table
        (and to cache_path as JSON when given); contexts made with autotune=1 apply them."""
        self._check_stream()
        n = C.c_int32(0)
        path = cache_path.encode() if cache_path else None
        check(lib().amg_autotune(self._h, reps, path, C.byref(n)), self._h)
        return n.value

    def vcycle_apply(self, b, level: int = 0, prec: int = 64):
        """x = V_j b, one AMG V-cycle from level j (FP64, or the float32 cycle)."""
        n = self.level_n(level)
        b2, sq = self._vec(b, n)
        out = torch.empty_like(b2)
        check(lib().amg_vcycle_apply(self._h, level, prec, b2.data_ptr(), out.data_ptr(), b2.shape[1]), self._h)
        return out.reshape(-1) if sq else out

    def set_hess_levels(self, ell: int):
        check(lib().amg_set_hess_levels(self._h, ell), self._h)

    def hierarchy_quality(self, level: int, v0, iters: int = 30) -> float:
        """a~_j = ||K_j - S_j K_{j+1} Pi_j||_2 by the power method from v0 (a
        float64 GPU tensor of n_level entries)."""
        self._check_stream()
        v, _ = self._vec(v0, self.level_n(level))
        a = C.c_double()
        check(lib().amg_hierarchy_quality(self._h, level, v.data_ptr(), iters, C.byref(a)), self._h)
        return a.value

    def time_kernel(self, which: int, prec: int = 64, nb: int = 1, reps: int = 50):
        """(ms per launch, algorithmic bytes per launch) of 0: level-0 SpMV, 1: pre-sweep
        residual, 2: V-cycle, 3: fused coarse correction and first post step at level 0,
        4: level-0 product of the float32-preconditioned FP64 CG; 5 / 6: ms per round of a
        grid-wide synchronisation by a barrier in a cooperative launch / by kernel boundaries."""
        self._check_stream()
        ms, by = C.c_double(), C.c_double()
        check(lib().amg_time_kernel(self._h, which, prec, nb, reps, C.byref(ms), C.byref(by)), self._h)
        return ms.value, by.value
