"""ctypes loader for ``libexageo.so`` (argument marshalling only).

The library is built in-tree by ``paper_1908_06936_amd/build.py``.  There is
no fallback: if the shared object is missing or fails to load, every entry
point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexageo.so")

OK, EINVAL, ENOTPD, ENOMEM, EDEVICE, ENOCONV = 0, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
EUCLIDEAN, GREAT_CIRCLE = 0, 1
DFO, LBFGSB, LBFGSB_FP64_FINISH = 0, 1, 2

STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOTPD: "ENOTPD", ENOMEM: "ENOMEM",
                EDEVICE: "EDEVICE", ENOCONV: "ENOCONV"}


class MleStats(ctypes.Structure):
    _fields_ = [("n_evals", ctypes.c_int64), ("n_grad_evals", ctypes.c_int64), ("iters", ctypes.c_int64),
                ("total_s", ctypes.c_double), ("per_eval_s", ctypes.c_double), ("status", ctypes.c_int32),
                ("n_fp64_finish_evals", ctypes.c_int64)]


EXPORTS = [
    "exageo_create", "exageo_destroy", "exageo_set_stream", "exageo_workspace_bytes", "exageo_set_workspace",
    "exageo_set_mixed_policy", "exageo_set_mixed_fp64_band", "exageo_set_mixed_correlation",
    "exageo_set_mixed_refinement", "exageo_set_mixed_bf16_block", "exageo_set_dst_band", "exageo_set_distance", "exageo_set_nugget", "exageo_set_verbose", "exageo_last_error",
    "exageo_matern_cov",
    "exageo_simulate", "exageo_loglik",
    "exageo_loglik_grad", "exageo_loglik_grad_noalloc", "exageo_mle", "exageo_predict", "exageo_fisher", "exageo_get_timings", "exageo_set_profiling",
]

_lib = None


def load():
    """Load the library once; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1908_06936_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, i32, d, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_int32
    pd = ctypes.POINTER(ctypes.c_double)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    lib.exageo_create.restype = st
    lib.exageo_create.argtypes = [ctypes.POINTER(p), i32, i64, p]
    lib.exageo_destroy.restype = None
    lib.exageo_destroy.argtypes = [p]
    lib.exageo_set_stream.restype = st
    lib.exageo_set_stream.argtypes = [p, p]
    lib.exageo_workspace_bytes.restype = ctypes.c_size_t
    lib.exageo_workspace_bytes.argtypes = [i64, i64, i32, i32]
    lib.exageo_set_workspace.restype = st
    lib.exageo_set_workspace.argtypes = [p, p, ctypes.c_size_t]
    lib.exageo_set_mixed_policy.restype = st
    lib.exageo_set_mixed_policy.argtypes = [p, d]
    lib.exageo_set_mixed_fp64_band.restype = st
    lib.exageo_set_mixed_fp64_band.argtypes = [p, d]
    lib.exageo_set_mixed_correlation.restype = st
    lib.exageo_set_mixed_correlation.argtypes = [p, d, d]
    lib.exageo_set_mixed_refinement.restype = st
    lib.exageo_set_mixed_refinement.argtypes = [p, i32]
    lib.exageo_set_mixed_bf16_block.restype = st
    lib.exageo_set_mixed_bf16_block.argtypes = [p, i32]
    lib.exageo_set_dst_band.restype = st
    lib.exageo_set_dst_band.argtypes = [p, i64]
    lib.exageo_set_distance.restype = st
    lib.exageo_set_distance.argtypes = [p, i32]
    lib.exageo_set_nugget.restype = st
    lib.exageo_set_nugget.argtypes = [p, d]
    lib.exageo_set_verbose.restype = st
    lib.exageo_set_verbose.argtypes = [p, i32]
    lib.exageo_last_error.restype = ctypes.c_char_p
    lib.exageo_last_error.argtypes = [p]
    lib.exageo_matern_cov.restype = st
    lib.exageo_matern_cov.argtypes = [p, i64, p, p, pd, p, i64]
    lib.exageo_simulate.restype = st
    lib.exageo_simulate.argtypes = [p, i64, p, p, pd, p, p, pi64]
    lib.exageo_loglik.restype = st
    lib.exageo_loglik.argtypes = [p, i64, p, p, p, pd, i32, pd, pi64]
    lib.exageo_loglik_grad.restype = st
    lib.exageo_loglik_grad.argtypes = [p, i64, p, p, p, pd, i32, pd, pd, pi64]
    lib.exageo_loglik_grad_noalloc.restype = st
    lib.exageo_loglik_grad_noalloc.argtypes = [p, i64, p, p, p, pd, pd, pd, pi64]
    lib.exageo_predict.restype = st
    lib.exageo_predict.argtypes = [p, i64, p, p, p, pd, i64, p, p, p, p, pi64]
    lib.exageo_fisher.restype = st
    lib.exageo_fisher.argtypes = [p, i64, p, p, pd, pd, pi64]
    lib.exageo_mle.restype = st
    lib.exageo_mle.argtypes = [p, i64, p, p, p, pd, pd, pd, d, i32, i32, i32, pd, pd, ctypes.POINTER(MleStats)]
    lib.exageo_get_timings.restype = ctypes.c_int
    lib.exageo_get_timings.argtypes = [p, pd, ctypes.c_int]
    lib.exageo_set_profiling.restype = st
    lib.exageo_set_profiling.argtypes = [p, i32]
    _lib = lib
    return lib


def darr(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr
