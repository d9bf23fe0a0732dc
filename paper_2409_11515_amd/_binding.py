"""ctypes binding of libcondest.so -- argument marshalling only.

Every step of the estimator runs inside the C/HIP library; this module only
converts numpy arrays and torch tensors to pointers and sizes and raises on a
non-zero status. There is no fallback: if the library is missing, every call
raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcondest.so")

COND_OK = 0
COND_EINVAL = -1
COND_ESINGULAR = -2
COND_ENOMEM = -3
COND_EHIP = -4
COND_ENUMERIC = -5
COND_ESTATE = -6
COND_ETIMEOUT = -7
COND_MIN_LU = 0
COND_MIN_SPMV = 1
COND_MIN_NONE = 2
COND_SCALE_NONE = 0
COND_SCALE_COL = 1
COND_F_COLSCALED = 8
COND_F_NUMSING = 1
COND_F_MAXITER = 2
COND_F_SINGULAR = 4


class CondError(RuntimeError):
    def __init__(self, status: int, where: str, text: str):
        super().__init__(f"{where}: status {status}: {text}")
        self.status = status


class CsrT(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class OptsT(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("max_iter", C.c_int64), ("stop_rtol", C.c_double),
                ("stop_window", C.c_int64), ("sigma_min_method", C.c_int32), ("chunk", C.c_int32),
                ("col_perm", C.c_void_p), ("pivot_tol", C.c_double), ("profile", C.c_int32),
                ("alpha_min", C.c_double), ("alpha_decay", C.c_double), ("scaling", C.c_int32)]


class BoundsT(C.Structure):
    _fields_ = [(f, C.c_double) for f in (
        "res_norm", "b_norm", "x_norm", "rel_residual", "err_x_lower", "err_x_upper",
        "err_xhat_lower", "err_xhat_upper", "err_x_tight", "roundoff_floor")]


class ResultT(C.Structure):
    _fields_ = [("sigma_max", C.c_double), ("sigma_min", C.c_double), ("kappa", C.c_double),
                ("iters_max", C.c_int64), ("iters_min", C.c_int64), ("flags", C.c_uint32),
                ("status_max", C.c_int32), ("status_min", C.c_int32), ("ms_max", C.c_double),
                ("ms_min", C.c_double), ("setup_ms", C.c_double), ("nnz_l", C.c_int64),
                ("nnz_u", C.c_int64)]


_lib = None

#: every symbol include/condest.h declares
EXPORTS = (
    "cond_strerror", "cond_last_error", "cond_opts_default", "cond_version", "cond_csr_check",
    "cond_csr_transpose", "cond_order_nd", "cond_lu_factor", "cond_lu_destroy", "cond_lu_info",
    "cond_lu_export", "cond_lu_solve_host", "cond_plan_create", "cond_plan_workspace_bytes",
    "cond_plan_bind", "cond_plan_destroy", "cond_plan_run", "cond_plan_spmv",
    "cond_plan_inverse_apply", "cond_estimate", "cond_plan_kernel_stats", "cond_plan_solve_info",
    "cond_plan_solve_replay",
    "cond_batch_create",
    "cond_batch_info", "cond_batch_bind", "cond_batch_run", "cond_batch_destroy",
    "cond_cnn_param_count", "cond_cnn_create", "cond_cnn_set_params", "cond_cnn_get_params",
    "cond_cnn_predict", "cond_cnn_gradients", "cond_cnn_train_step", "cond_cnn_activation",
    "cond_cnn_destroy", "cond_plan_error_bounds", "cond_plan_column_norms",
    "cond_batch_run_min", "cond_batch_fill", "cond_estimate_batched", "cond_batch_solve_replay",
    "cond_stream_triad", "cond_error_bounds_noalloc", "cond_plan_inject_timeout",
)

BATCH_K = 8

KERNEL_NAMES = ("normalise", "spmv_A", "spmv_At", "sumsq", "trsv_L", "trsv_U", "trsv_Ut",
                "trsv_Lt", "adam_pass1", "adam_pass2")


def lib():
    """The loaded library; raises ImportError if it was never built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_11515_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.cond_strerror.restype = C.c_char_p
    L.cond_strerror.argtypes = [C.c_int]
    L.cond_last_error.restype = C.c_char_p
    L.cond_last_error.argtypes = []
    L.cond_opts_default.argtypes = [C.POINTER(OptsT)]
    L.cond_opts_default.restype = None
    L.cond_version.restype = C.c_int
    L.cond_csr_check.argtypes = [C.POINTER(CsrT)]
    L.cond_csr_transpose.argtypes = [C.POINTER(CsrT), vp, vp, vp]
    L.cond_order_nd.argtypes = [C.POINTER(CsrT), vp]
    L.cond_lu_factor.argtypes = [C.POINTER(CsrT), vp, dbl, C.POINTER(vp)]
    L.cond_lu_destroy.argtypes = [vp]
    L.cond_lu_destroy.restype = None
    L.cond_lu_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i64)]
    L.cond_lu_export.argtypes = [vp] + [vp] * 9
    L.cond_lu_solve_host.argtypes = [vp, C.c_int, vp, vp]
    L.cond_plan_create.argtypes = [C.POINTER(CsrT), C.POINTER(OptsT), C.POINTER(vp)]
    L.cond_plan_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.cond_plan_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.cond_plan_destroy.argtypes = [vp]
    L.cond_plan_destroy.restype = None
    L.cond_plan_run.argtypes = [vp, C.POINTER(OptsT), vp, vp, C.POINTER(ResultT), vp, vp, vp, vp]
    L.cond_plan_spmv.argtypes = [vp, C.c_int, vp, vp]
    L.cond_plan_inverse_apply.argtypes = [vp, vp, vp, vp]
    L.cond_estimate.argtypes = [C.POINTER(CsrT), C.POINTER(OptsT), vp, vp, vp, C.POINTER(ResultT)]
    L.cond_plan_kernel_stats.argtypes = [vp, vp, vp, vp]
    L.cond_plan_solve_info.argtypes = [vp, vp, vp, vp]
    L.cond_plan_solve_replay.argtypes = [vp, vp, vp, vp]
    L.cond_batch_create.argtypes = [vp, i32, C.POINTER(OptsT), C.POINTER(vp)]
    L.cond_batch_info.argtypes = [vp, vp, C.POINTER(C.c_size_t), C.POINTER(i32), C.POINTER(i32)]
    L.cond_batch_bind.argtypes = [vp, vp, C.c_size_t, vp, i32, i32]
    L.cond_batch_run.argtypes = [vp, C.POINTER(OptsT), vp, vp, vp, vp, vp, vp, vp,
                                 C.POINTER(dbl)]
    L.cond_batch_destroy.argtypes = [vp]
    L.cond_batch_destroy.restype = None
    L.cond_cnn_param_count.argtypes = []
    L.cond_cnn_create.argtypes = [i32, i32, i32, vp, C.POINTER(vp)]
    L.cond_cnn_set_params.argtypes = [vp, vp]
    L.cond_cnn_get_params.argtypes = [vp, vp]
    L.cond_cnn_predict.argtypes = [vp, vp, i32, i32, vp]
    L.cond_cnn_gradients.argtypes = [vp, vp, vp, i32, i32, vp, vp]
    L.cond_cnn_train_step.argtypes = [vp, vp, vp, i32, i32, C.c_float, C.POINTER(C.c_float)]
    L.cond_cnn_activation.argtypes = [vp, i32, i32, i32, vp]
    L.cond_cnn_destroy.argtypes = [vp]
    L.cond_cnn_destroy.restype = None
    L.cond_plan_column_norms.argtypes = [vp, vp]
    L.cond_batch_run_min.argtypes = [vp, C.POINTER(OptsT), vp, vp, vp, vp, vp, vp, vp,
                                     C.POINTER(dbl)]
    L.cond_batch_solve_replay.argtypes = [vp, vp, vp, vp]
    L.cond_plan_inject_timeout.argtypes = [vp]
    L.cond_stream_triad.argtypes = [i64, vp, vp, vp, dbl, i32, i32, vp, C.POINTER(dbl)]
    L.cond_batch_fill.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(dbl)]
    L.cond_estimate_batched.argtypes = [vp, i32, C.POINTER(OptsT), vp, vp, vp, vp]
    L.cond_plan_error_bounds.argtypes = [vp, vp, vp, dbl, dbl, C.POINTER(BoundsT)]
    L.cond_error_bounds_noalloc.argtypes = [i32, i64, vp, vp, vp, vp, vp, dbl, dbl, vp,
                                            C.POINTER(BoundsT)]
    for name in EXPORTS:
        getattr(L, name)  # raises AttributeError if a declared symbol is missing
    _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != COND_OK:
        L = lib()
        raise CondError(status, where, (L.cond_last_error() or b"").decode() or
                        L.cond_strerror(status).decode())


def _ptr(a) -> int:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


class HostCsr:
    """Keeps the int64/int32/float64 host arrays alive behind a CsrT."""

    def __init__(self, n, rowptr, col, val):
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = int(n)
        self.struct = CsrT(self.n, int(self.rowptr[-1]) if self.rowptr.size else 0,
                           self.rowptr.ctypes.data, self.col.ctypes.data, self.val.ctypes.data)


def make_opts(**kw) -> OptsT:
    o = OptsT()
    lib().cond_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "col_perm":
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o
