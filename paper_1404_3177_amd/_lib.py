"""ctypes binding of libmnl.so (the C ABI declared in include/mnl.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  Importing this module never falls back to another implementation:
if the library is missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmnl.so")

MNL_OK = 0
ERRORS = {
    -1: "MNL_ERR_ARG", -2: "MNL_ERR_OOM", -3: "MNL_ERR_NOT_PD",
    -4: "MNL_ERR_NONFINITE", -5: "MNL_ERR_LS_FAIL", -6: "MNL_ERR_HIP",
    -7: "MNL_ERR_UNSUPPORTED",
}
STOP_NONE, STOP_GTOL, STOP_FTOL, STOP_MAXITER = 0, 1, 2, 3
STOP_LS_FAIL, STOP_NOT_PD, STOP_NONFINITE = 4, 5, 6
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
METHOD = {"newton": 0, "newton-cg": 1}

EXPORTS = [
    "mnl_version", "mnl_strerror", "mnl_default_opts", "mnl_num_params",
    "mnl_create", "mnl_destroy", "mnl_workspace_bytes", "mnl_last_error",
    "mnl_loglik_grad", "mnl_loglik_grad_noalloc", "mnl_hessian",
    "mnl_newton_step", "mnl_fit", "mnl_fit_batch", "mnl_batch_eligible",
    "mnl_hessvec", "mnl_collinear", "mnl_select_columns", "mnl_predict",
    "mnl_stderr", "mnl_covariance", "mnl_quadform", "mnl_chi2_sf",
    "mnl_lrtest",
    "mnl_fit_footprint", "mnl_server_now_ms", "mnl_server_create",
    "mnl_server_destroy", "mnl_server_submit", "mnl_server_wait",
    "mnl_server_get_stats",
]


class MnlProblem(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("K", ctypes.c_int32), ("p", ctypes.c_int32),
        ("g", ctypes.c_int32), ("a", ctypes.c_int32),
        ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("Z", ctypes.c_void_p),
        ("choice", ctypes.c_void_p), ("w", ctypes.c_void_p),
    ]


class MnlFitOpts(ctypes.Structure):
    _fields_ = [
        ("maxiter", ctypes.c_int32), ("ftol", ctypes.c_double),
        ("gtol", ctypes.c_double), ("prec", ctypes.c_int32),
        ("ls_max", ctypes.c_int32), ("ls_tol_ulps", ctypes.c_double),
        ("validate", ctypes.c_int32), ("method", ctypes.c_int32),
        ("cg_maxiter", ctypes.c_int32), ("graph", ctypes.c_int32),
    ]


class MnlFitInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("ls_iters", ctypes.c_int32),
        ("ls_backtracks", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
        ("hess_fallbacks", ctypes.c_int32), ("n_hess", ctypes.c_int32),
        ("loglik", ctypes.c_double), ("grad_norm", ctypes.c_double),
        ("loglik_diff", ctypes.c_double), ("t_total", ctypes.c_double),
        ("t_loglik_grad", ctypes.c_double), ("t_hessian", ctypes.c_double),
        ("t_chol", ctypes.c_double), ("t_ls", ctypes.c_double),
        ("t_hess_kernel", ctypes.c_double), ("t_pass_kernel", ctypes.c_double),
        ("n_pass", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_
                if f != "reserved"}


class MnlServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t),
                ("host_only", ctypes.c_int32), ("max_group", ctypes.c_int32),
                ("host_fit_ms", ctypes.c_double)]


class MnlServerResult(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64), ("status", ctypes.c_int32),
        ("slot", ctypes.c_int32), ("t_arrival", ctypes.c_double),
        ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
        ("footprint", ctypes.c_size_t), ("info", MnlFitInfo),
    ]


class MnlServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
        ("queued", ctypes.c_int32), ("running", ctypes.c_int32),
        ("max_running", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("budget", ctypes.c_size_t), ("in_use", ctypes.c_size_t),
        ("peak_in_use", ctypes.c_size_t),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmnl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with paper_1404_3177_amd/build.py")
    # torch ships its own HIP runtime (same soname as ROCm's).  Loading torch
    # first makes libmnl.so bind to that runtime, so both share one device
    # context, one allocator view and the same stream objects.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.mnl_version.restype = ctypes.c_char_p
    lib.mnl_strerror.restype = ctypes.c_char_p
    lib.mnl_strerror.argtypes = [ctypes.c_int]
    lib.mnl_default_opts.argtypes = [ctypes.POINTER(MnlFitOpts)]
    lib.mnl_default_opts.restype = None
    lib.mnl_num_params.argtypes = [I32, I32, I32, I32]
    lib.mnl_num_params.restype = I64
    lib.mnl_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t]
    lib.mnl_destroy.argtypes = [P]
    lib.mnl_destroy.restype = None
    lib.mnl_workspace_bytes.argtypes = [P]
    lib.mnl_workspace_bytes.restype = ctypes.c_size_t
    lib.mnl_last_error.argtypes = [P]
    lib.mnl_last_error.restype = ctypes.c_char_p
    prob = ctypes.POINTER(MnlProblem)
    lib.mnl_loglik_grad.argtypes = [P, prob, P, P, P, P, P]
    lib.mnl_loglik_grad_noalloc.argtypes = [P, prob, P, P, P, P, P]
    lib.mnl_hessian.argtypes = [P, prob, P, I32, P, P]
    lib.mnl_newton_step.argtypes = [P, prob, P, ctypes.POINTER(MnlFitOpts),
                                    ctypes.POINTER(MnlFitInfo), P]
    lib.mnl_fit.argtypes = [P, prob, P, ctypes.POINTER(MnlFitOpts), P,
                            ctypes.POINTER(MnlFitInfo), P]
    lib.mnl_fit_batch.argtypes = [P, I32, prob, P, ctypes.POINTER(MnlFitOpts),
                                  P, ctypes.POINTER(MnlFitInfo), P]
    lib.mnl_batch_eligible.argtypes = [prob, ctypes.POINTER(MnlFitOpts)]
    lib.mnl_batch_eligible.restype = ctypes.c_int
    lib.mnl_hessvec.argtypes = [P, prob, P, P, P, P]
    lib.mnl_collinear.argtypes = [P, prob, ctypes.c_double, P, P, P, P]
    lib.mnl_covariance.argtypes = [P, prob, P, P, I32, P, P]
    lib.mnl_quadform.argtypes = [P, P, P, P, P, I64, I32,
                                 ctypes.POINTER(ctypes.c_double), P]
    lib.mnl_chi2_sf.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.mnl_chi2_sf.restype = ctypes.c_double
    lib.mnl_lrtest.argtypes = [ctypes.c_double, ctypes.c_double,
                               ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)]
    lib.mnl_lrtest.restype = ctypes.c_int
    lib.mnl_select_columns.argtypes = [P, prob, P, P, P, P, P, P, P]
    lib.mnl_predict.argtypes = [P, prob, P, P, P]
    lib.mnl_stderr.argtypes = [P, prob, P, P, P, P, P]
    lib.mnl_fit_footprint.argtypes = [prob, I32]
    lib.mnl_fit_footprint.restype = I64
    lib.mnl_server_now_ms.argtypes = []
    lib.mnl_server_now_ms.restype = ctypes.c_double
    lib.mnl_server_create.argtypes = [ctypes.POINTER(P),
                                      ctypes.POINTER(MnlServerOpts)]
    lib.mnl_server_destroy.argtypes = [P]
    lib.mnl_server_destroy.restype = None
    lib.mnl_server_submit.argtypes = [P, prob, P, ctypes.POINTER(MnlFitOpts),
                                      P, ctypes.c_double,
                                      ctypes.POINTER(I64)]
    lib.mnl_server_wait.argtypes = [P, ctypes.POINTER(MnlServerResult), I32,
                                    ctypes.c_double, ctypes.POINTER(I32)]
    lib.mnl_server_get_stats.argtypes = [P, ctypes.POINTER(MnlServerStats)]
    for name in ("mnl_create", "mnl_loglik_grad", "mnl_loglik_grad_noalloc",
                 "mnl_hessian",
                 "mnl_newton_step", "mnl_fit", "mnl_fit_batch", "mnl_hessvec",
                 "mnl_predict",
                 "mnl_collinear", "mnl_select_columns", "mnl_covariance",
                 "mnl_quadform",
                 "mnl_stderr",
                 "mnl_server_create",
                 "mnl_server_submit", "mnl_server_wait",
                 "mnl_server_get_stats"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class MnlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
