"""ctypes binding of libmgr's C ABI (include/mgr.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  The library must have been built (``paper_1801_08464_amd.build``);
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgr.so")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_ZERO_FDIAG, E_SINGULAR_BLOCK, E_BREAKDOWN, E_HIP, E_OOM = -1, -2, -3, -4, -5, -6

EXPORTS = [
    "mgr_default_options", "mgr_setup", "mgr_solve", "mgr_pattern_outer", "mgr_apply_preconditioner", "mgr_spmv",
    "mgr_destroy", "mgr_status_string", "mgr_last_error", "mgr_num_levels", "mgr_get_matrix", "mgr_get_vector",
    "mgr_set_kernel_timing", "mgr_kernel_time", "mgr_ncp_eval", "mgr_ncp_jacobian", "mgr_ncp_eval_noalloc",
    "mgr_update_values",
]


class MgrCsr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("values", C.c_void_p)]


class MgrOptions(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("precision", C.c_int), ("restart", C.c_int), ("max_iter", C.c_int),
                ("rp_type", C.c_int), ("global_relax", C.c_int), ("f_sweeps", C.c_int), ("amg_theta", C.c_double),
                ("amg_pre", C.c_int), ("amg_post", C.c_int), ("amg_max_levels", C.c_int),
                ("amg_coarse_max", C.c_int), ("dense_max", C.c_int), ("pmis_seed", C.c_uint64),
                ("transpose", C.c_int), ("use_x0", C.c_int), ("frelax_amg_mask", C.c_int),
                ("frelax_amg_pre", C.c_int), ("frelax_amg_post", C.c_int), ("cycle_post", C.c_int),
                ("index16", C.c_int)]


class MgrStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("rel_residual", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("n_levels", C.c_int), ("level_n", C.c_int64 * 64),
                ("level_nnz", C.c_int64 * 64), ("res_history", C.POINTER(C.c_double)),
                ("res_history_cap", C.c_int), ("res_history_len", C.c_int)]


class MGRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{status_string(code)}: {msg}")
        self.code = code


_lib = None


def load_library(build_if_missing: bool = True):
    """Load libmgr.so (building it in-tree first if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"{LIB_PATH} is not built")
        from . import build as _b
        _b.build()
    L = C.CDLL(LIB_PATH)
    P, vp, i64, i32 = C.POINTER, C.c_void_p, C.c_int64, C.c_int
    L.mgr_default_options.argtypes = [P(MgrOptions)]
    L.mgr_default_options.restype = None
    L.mgr_setup.argtypes = [P(MgrCsr), i32, vp, P(MgrOptions), P(vp)]
    L.mgr_solve.argtypes = [vp, vp, vp, C.c_double, P(MgrStats)]
    L.mgr_update_values.argtypes = [vp, vp]
    L.mgr_pattern_outer.argtypes = [vp, vp, vp, vp]
    L.mgr_apply_preconditioner.argtypes = [vp, vp, vp]
    L.mgr_spmv.argtypes = [vp, vp, vp]
    L.mgr_destroy.argtypes = [vp]
    L.mgr_destroy.restype = None
    L.mgr_status_string.argtypes = [i32]
    L.mgr_status_string.restype = C.c_char_p
    L.mgr_last_error.argtypes = [vp]
    L.mgr_last_error.restype = C.c_char_p
    L.mgr_num_levels.argtypes = [vp, P(i32), P(i32)]
    L.mgr_get_matrix.argtypes = [vp, i32, i32, P(i64), P(i64), P(i64), vp, vp, vp]
    L.mgr_get_vector.argtypes = [vp, i32, i32, vp, P(i64)]
    L.mgr_set_kernel_timing.argtypes = [vp, i32]
    L.mgr_kernel_time.argtypes = [vp, i32, P(C.c_double), P(i64), P(C.c_double)]
    L.mgr_ncp_eval.argtypes = [P(MgrCsr), vp, vp, vp, vp, C.c_double, vp, vp, P(C.c_double), P(i64), P(i64), vp]
    L.mgr_ncp_eval_noalloc.argtypes = [P(MgrCsr), vp, vp, vp, vp, C.c_double, vp, vp, P(C.c_double), P(i64), P(i64),
                                       vp]
    L.mgr_ncp_jacobian.argtypes = [P(MgrCsr), vp, vp, vp, vp, vp, i64, P(i64), vp]
    _lib = L
    return L


def status_string(code: int) -> str:
    return load_library().mgr_status_string(code).decode()


def last_error(handle=None) -> str:
    return load_library().mgr_last_error(handle).decode()


def default_options() -> MgrOptions:
    o = MgrOptions()
    load_library().mgr_default_options(C.byref(o))
    return o
