"""ctypes declarations of the C ABI in include/amghess.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamghess.so")

AMG_OK = 0
ERRORS = {
    -1: "AMG_ERR_ARG", -2: "AMG_ERR_NOT_SYMMETRIC", -3: "AMG_ERR_NOT_SPD", -4: "AMG_ERR_NOCONV",
    -5: "AMG_ERR_INDEFINITE", -6: "AMG_ERR_HIP", -7: "AMG_ERR_OOM", -8: "AMG_ERR_DENSE_TOO_LARGE",
    -9: "AMG_ERR_CAPACITY",
}


class AmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Csr(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int32),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("beta", C.c_double), ("hess_levels", C.c_int32), ("auto_levels", C.c_int32),
                ("max_levels", C.c_int32), ("max_coarse", C.c_int32), ("dense_max", C.c_int32),
                ("theta0", C.c_double), ("agg_seed", C.c_uint64), ("nu", C.c_int32),
                ("inner_rtol", C.c_double), ("mass_rtol", C.c_double), ("precond_inner_rtol", C.c_double),
                ("inner_maxit", C.c_int32), ("mass_maxit", C.c_int32), ("outer_maxit", C.c_int32),
                ("inner_precision", C.c_int32), ("inner32_rtol", C.c_double), ("refine_maxit", C.c_int32),
                ("nb_max", C.c_int32), ("precond", C.c_int32), ("check_every", C.c_int32),
                ("use_graphs", C.c_int32), ("coarse_hess_rtol", C.c_double),
                ("dense_solve_max", C.c_int32), ("mixed_mode", C.c_int32),
                ("smoother", C.c_int32), ("true_resid", C.c_int32), ("autotune", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("inner_solves", C.c_int32), ("inner_iters_total", C.c_int32),
                ("inner_iters_max", C.c_int32), ("mass_iters_total", C.c_int32), ("refine_steps", C.c_int32),
                ("levels", C.c_int32), ("ell", C.c_int32), ("status_detail", C.c_int32), ("pad_", C.c_int32),
                ("rel_resid", C.c_double), ("ms_total", C.c_double), ("true_rel_resid", C.c_double),
                ("ms_phase", C.c_double * 8), ("bytes_moved", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("pad_", "ms_phase")}
        d["ms_phase"] = dict(zip(("rhs", "hessian", "precond", "outer_vector", "true_resid"), list(self.ms_phase)[:5]))
        return d


P = C.c_void_p
I32 = C.c_int32
PI32 = C.POINTER(C.c_int32)
PD = C.POINTER(C.c_double)

SIGNATURES = {
    "amg_opts_default": (C.c_int, [C.POINTER(Opts)]),
    "amg_p1_pattern": (C.c_int, [C.c_int, I32, I32, P, PI32]),
    "amg_p1_assemble": (C.c_int, [C.c_int, I32, P, I32, P, P, I32, P, P, P, P]),
    "amg_p1_pattern_device": (C.c_int, [C.c_int, I32, I32, P, PI32, P]),
    "amg_p1_assemble_device": (C.c_int, [C.c_int, I32, P, I32, P, P, I32, P, P, P, P, P]),
    "amg_p1_assemble_device_noalloc": (C.c_int, [C.c_int, I32, P, I32, P, P, I32, P, P, P, P, P]),
    "amg_setup": (C.c_int, [C.POINTER(Csr), C.POINTER(Csr), P, C.POINTER(Opts), P, C.POINTER(P)]),
    "amg_destroy": (C.c_int, [P]),
    "amg_release_memory": (C.c_int, []),
    "state_solve": (C.c_int, [P, C.c_int, P, P, C.c_int, C.POINTER(Info)]),
    "adjoint_solve": (C.c_int, [P, C.c_int, P, P, C.c_int, C.POINTER(Info)]),
    "hessian_apply": (C.c_int, [P, C.c_int, P, P, C.c_int, C.POINTER(Info)]),
    "hessian_precond_apply": (C.c_int, [P, P, P, C.c_int, C.POINTER(Info)]),
    "reduced_solve": (C.c_int, [P, P, P, P, C.c_int, C.c_double, C.POINTER(Info)]),
    "reduced_objective": (C.c_int, [P, P, P, P, P, C.c_int, C.POINTER(Info)]),
    "amg_mass_apply": (C.c_int, [P, C.c_int, C.c_int, P, P, C.c_int]),
    "amg_mass_quad": (C.c_int, [P, C.c_int, P, P, C.c_int]),
    "amg_num_levels": (C.c_int, [P, PI32, PI32]),
    "amg_level_size": (C.c_int, [P, C.c_int, PI32, PI32, PI32, PI32]),
    "amg_copy_aggregates": (C.c_int, [P, C.c_int, P, P]),
    "amg_copy_csr": (C.c_int, [P, C.c_int, C.c_int, P, P, P]),
    "amg_copy_dense": (C.c_int, [P, C.c_int, PI32, P]),
    "amg_set_hess_levels": (C.c_int, [P, C.c_int]),
    "amg_last_error": (C.c_char_p, [P]),
    "amg_time_kernel": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int, PD, PD]),
    "amg_hierarchy_quality": (C.c_int, [P, C.c_int, C.c_void_p, C.c_int, PD]),
    "amg_vcycle_apply": (C.c_int, [P, C.c_int, C.c_int, P, P, C.c_int]),
    "amg_autotune": (C.c_int, [P, C.c_int, C.c_char_p, PI32]),
}

_lib = None


def lib():
    """Load libamghess.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python __graft_entry__.py build` "
                               "or paper_2001_11533_amd._build.build()")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(rc: int, ctx=None):
    if rc != AMG_OK:
        msg = lib().amg_last_error(ctx)
        raise AmgError(rc, msg.decode() if msg else "")
