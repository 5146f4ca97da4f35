"""ctypes declarations of libslamg.so (include/slamg.h and include/slamg_ops.h).

Loading fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslamg.so")

SLAMG_OK, SLAMG_NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "E_INVALID", -2: "E_OOM", -3: "E_BUDGET", -4: "E_DEVICE",
                -5: "E_NUMERIC", -6: "E_BUSY"}
STATUS_BUSY = -6
KIND = {"svd": 0, "spd": 1}
TARGET = {"dominant": 0, "minimal": 1}
PRECISION = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16": 2}


class Csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("on_device", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("theta", C.c_double), ("strength_rule", C.c_int32), ("top_s", C.c_int32),
                ("df_filter", C.c_double), ("n_t", C.c_int32), ("mu_t", C.c_int32), ("mu_b", C.c_int32),
                ("omega_J", C.c_double), ("n_mult", C.c_int32), ("max_add", C.c_int32),
                ("coarse_max", C.c_int32), ("max_levels", C.c_int32), ("stall_ratio", C.c_double),
                ("tol", C.c_double), ("seed", C.c_uint64), ("precision", C.c_int32),
                ("ritz_in_mult", C.c_int32), ("coarse_pinv", C.c_int32), ("profile_mask", C.c_int32),
                ("verbose", C.c_int32), ("graphs", C.c_int32), ("square_coarsening", C.c_int32),
                ("n_guard", C.c_int32), ("mu_tJ", C.c_int32), ("mu_bJ", C.c_int32),
                ("kaczmarz_order", C.c_int32), ("coarse_dense_max", C.c_int32),
                ("redo_p", C.c_int32), ("redo_tol", C.c_double), ("cycle_gamma", C.c_int32),
                ("ritz_coarse", C.c_int32),
                ("solve_phase", C.c_int32), ("fmg", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("levels", C.c_int32), ("mult_cycles", C.c_int32), ("add_iters", C.c_int32),
                ("converged", C.c_int32), ("rows", C.c_int64 * 32), ("cols", C.c_int64 * 32),
                ("nnz", C.c_int64 * 32), ("colours", C.c_int32 * 32), ("capped", C.c_int32 * 32),
                ("anorm", C.c_double), ("resid", C.c_double * 16), ("rho_history", C.c_double * 256),
                ("mult_sigma", (C.c_double * 16) * 32), ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("err_bound", C.c_double * 16), ("prof_ms", C.c_double * 8), ("prof_launches", C.c_int64 * 8),
                ("prof_bytes", C.c_double * 8), ("graph_iters", C.c_int32), ("redo_count", C.c_int32),
                ("device_bytes", C.c_int64), ("t_queue_ms", C.c_double), ("t_latency_ms", C.c_double),
                ("p_dropped", C.c_int32), ("reserved_r", C.c_int32)]


_P = C.c_void_p
_I = C.c_int32
_D = C.c_double

# name: (restype, argtypes)
SIGNATURES = {
    "slamg_params_init": (_I, [C.POINTER(Params), _I, _I]),
    "slamg_create": (_I, [C.POINTER(_P), C.c_int, _P, C.c_size_t]),
    "slamg_destroy": (None, [_P]),
    "slamg_solve": (_I, [_P, C.POINTER(Csr), _I, _I, _I, C.POINTER(Params), _P, _P, _P, _P, C.POINTER(Report)]),
    "slamg_matrix_create": (_I, [_P, C.POINTER(Csr), _I, C.POINTER(_P)]),
    "slamg_matrix_destroy": (None, [_P]),
    "slamg_solve_matrix": (_I, [_P, _P, _I, _I, C.POINTER(Params), _P, _P, _P, _P, _I, C.POINTER(Report)]),
    "slamg_submit": (_I, [_P, C.POINTER(Csr), _I, _I, _I, C.POINTER(Params), C.POINTER(C.c_uint64)]),
    "slamg_poll": (_I, [_P, C.c_uint64, C.POINTER(_I)]),
    "slamg_wait": (_I, [_P, C.c_uint64]),
    "slamg_serve_start": (_I, [_P, _I]),
    "slamg_serve_stop": (_I, [_P]),
    "slamg_fetch": (_I, [_P, C.c_uint64, _P, _P, _P, C.POINTER(Report)]),
    "slamg_status_string": (C.c_char_p, [_I]),
    "slamg_last_error": (C.c_char_p, [_P]),
    "slamg_op_spmm": (_I, [_I, _I, _P, _P, _P, _P, _P, _D, _P]),
    "slamg_op_spmm_f32": (_I, [_I, _I, _P, _P, _P, _P, _P, _D, _P]),
    "slamg_op_spmm_bf16": (_I, [_I, _I, _P, _P, _P, _P, _P, _D, _P]),
    "slamg_op_cast_bf16": (_I, [C.c_int64, _P, _P, _P]),
    "slamg_op_relax_test": (_I, [_I, _I, _I, _I] + [_P] * 12 + [_D, _P, _P, _P]),
    "slamg_op_relax_boot": (_I, [_I, _I, _I, _I] + [_P] * 12 + [_P, _P, _P, _D, _P, _P, _P]),
    "slamg_op_kaczmarz": (_I, [_I, _I, _I, _P, _P, _P, _P, _P, _P, _P, _I, _P, _P, _P]),
    "slamg_op_residual": (_I, [_I, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "slamg_op_dots": (_I, [_I, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "slamg_op_gram": (_I, [_I, _I, _P, _P, _P, _P]),
    "slamg_op_gram_noalloc": (_I, [_I, _I, _P, _P, _P, _P]),
    "slamg_op_gram_noalloc_scratch_bytes": (C.c_size_t, []),
    "slamg_op_ritz": (_I, [_I, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P, _P]),
    "slamg_op_ls_fit": (_I, [_I, _P, _P, _P, _I, _P, _P, _I, _P, _P, _P, _P, _P]),
    "slamg_op_spgemm": (_I, [_I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "slamg_op_topsel": (_I, [_I, _P, _P, _P, _I, _P, _P, _P]),
    "slamg_op_coarse_gsvd": (_I, [_I, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P]),
    "slamg_op_coarse_solve": (_I, [_I, _I, _I, _P, _P, _P, _P, _P]),
    "slamg_op_proj_svd": (_I, [_I, _I, _I, _P, _P, _P, _P]),
    "slamg_graph_strength": (_I, [_I, _P, _P, _P, _D, _I, _I, _P, _P]),
    "slamg_graph_rs": (_I, [_I, _P, _P, _P]),
    "slamg_graph_interp": (_I, [_I, _P, _P, _P, _P, _P, _P, _I, _P, _P, _P]),
    "slamg_graph_colour": (_I, [_I, _I, _P, _P, _P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libslamg.so and declare its entry points.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libslamg.so not found at {path}: build it with "
                           "`python -m paper_1102_0919_amd.build` (there is no fallback path)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
