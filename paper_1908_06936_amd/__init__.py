"""Exact Gaussian-process MLE with a Matern covariance on MI355X (gfx950).

Python face of ``libexageo.so`` (C ABI in ``include/exageo.h``).  Every step
of the computation runs in the library's HIP kernels; this module only
passes torch device pointers, the current torch stream and host scalars.

    ctx = Context(ts=768)
    ll = ctx.loglik(x, y, z, (1.0, 0.1, 1.0))            # eq. (2) of the paper
    ll, g = ctx.loglik_grad(x, y, z, (1.0, 0.1, 1.0))     # and dl/d(sigma2, beta, nu)
    theta, ll, stats = ctx.mle(x, y, z, lb, ub)           # bounded MLE

``x, y, z`` are 1-D float64 CUDA (HIP) tensors of equal length.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

import torch

from . import _lib
from ._lib import (DFO, EINVAL, ENOCONV, ENOMEM, ENOTPD, FP64, LBFGSB, LBFGSB_FP64_FINISH, MIXED, OK,
                   STATUS_NAMES)

__all__ = ["Context", "ExaGeoError", "NotPositiveDefinite", "ExaGeoLoglik", "FP64", "MIXED", "DFO", "LBFGSB",
           "LBFGSB_FP64_FINISH"]


class ExaGeoError(RuntimeError):
    def __init__(self, status: int, message: str, info: int = 0):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.info = info


class NotPositiveDefinite(ExaGeoError):
    pass


def _prec(precision) -> int:
    if precision in (FP64, "fp64", "f64", "double"):
        return FP64
    if precision in (MIXED, "mixed", "mp"):
        return MIXED
    raise ValueError(f"unknown precision {precision!r}")


def _method(method) -> int:
    if method in (DFO, "dfo", "nelder-mead", "nm"):
        return DFO
    if method in (LBFGSB, "lbfgsb", "l-bfgs-b"):
        return LBFGSB
    if method in (LBFGSB_FP64_FINISH, "lbfgsb_fp64_finish"):
        return LBFGSB_FP64_FINISH
    raise ValueError(f"unknown method {method!r}")


def _dev_f64(t: torch.Tensor, name: str, n: int | None = None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a float64 tensor on the GPU")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    t = t.contiguous().view(-1)
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t


class Context:
    """One library context: a device, a tile size and a stream.

    Device memory for the tiles comes from torch (a uint8 tensor handed to the
    library as its workspace) and is reused across calls.
    """

    def __init__(self, ts: int = 768, device: int | None = None, stream: torch.cuda.Stream | None = None,
                 band_factor: float | None = None, fp64_band: float | None = None):
        self._lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to torch")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.ts = int(ts)
        self._stream = stream
        h = ctypes.c_void_p()
        st = self._lib.exageo_create(ctypes.byref(h), self.device, self.ts, self._stream_handle())
        if st != OK:
            raise ExaGeoError(st, f"exageo_create(device={self.device}, ts={self.ts}) failed")
        self._h = h
        self._ws = None
        self._ws_key = None
        self._nugget = 0.0
        # mixed precision: the library's correlation map unless distance bands are asked for
        if band_factor is not None or fp64_band is not None:
            self.set_mixed_policy(3.0 if band_factor is None else band_factor,
                                  0.0 if fp64_band is None else fp64_band)

    # ------------------------------------------------------------ plumbing
    def _stream_handle(self):
        s = self._stream if self._stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    def _sync_stream(self):
        self._lib.exageo_set_stream(self._h, self._stream_handle())

    def _ensure_ws(self, n: int, precision: int, want_grad):
        # want_grad: False / True, or 2 / 3 for the Fisher information (see exageo_workspace_bytes)
        need = self._lib.exageo_workspace_bytes(n, self.ts, precision, int(want_grad))
        if need == 0:
            raise ExaGeoError(EINVAL, f"bad problem size n={n}, ts={self.ts}")
        if self._ws is None or self._ws.numel() < need:
            self._lib.exageo_set_workspace(self._h, None, 0)
            self._ws = None
            torch.cuda.synchronize(self.device)
            torch.cuda.empty_cache()  # return the old block before taking a larger one
            self._ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
            st = self._lib.exageo_set_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()), need)
            self._check(st, "set_workspace")

    def _check(self, st: int, what: str, info: int = 0):
        if st == OK:
            return
        msg = self._lib.exageo_last_error(self._h).decode(errors="replace")
        if st == ENOTPD:
            raise NotPositiveDefinite(st, f"{what}: {msg}", info)
        raise ExaGeoError(st, f"{what}: {msg}", info)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.exageo_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mixed_policy(self, band_factor: float, fp64_band: float | None = None):
        """Mixed precision: BF16 for tiles at least band_factor * beta apart,
        FP64 for tiles closer than fp64_band * beta (unchanged if None)."""
        self._check(self._lib.exageo_set_mixed_policy(self._h, float(band_factor)), "set_mixed_policy")
        if fp64_band is not None:
            self._check(self._lib.exageo_set_mixed_fp64_band(self._h, float(fp64_band)), "set_mixed_fp64_band")

    def set_mixed_correlation(self, fp64_at_or_above: float = 0.3, bf16_below: float = 1e-4):
        """Mixed precision by correlation (the library's default map): FP64
        tiles whose correlation bound is >= fp64_at_or_above, BF16 below
        bf16_below (with their updates), FP32 otherwise."""
        self._check(self._lib.exageo_set_mixed_correlation(self._h, float(fp64_at_or_above), float(bf16_below)),
                    "set_mixed_correlation")

    def set_mixed_refinement(self, steps: int = 1):
        """FP64 refinement steps of Sigma^-1 z through the mixed factor."""
        self._check(self._lib.exageo_set_mixed_refinement(self._h, int(steps)), "set_mixed_refinement")

    def set_mixed_bf16_block(self, edge: int = 256):
        """Output block edge (256 or 128) of the BF16 targets' update."""
        self._check(self._lib.exageo_set_mixed_bf16_block(self._h, int(edge)), "set_mixed_bf16_block")

    def set_distance(self, metric: str):
        """'euclidean' (default) or 'great_circle' (x = longitude, y = latitude
        in degrees, km on a sphere of radius 6371)."""
        m = {"euclidean": _lib.EUCLIDEAN, "great_circle": _lib.GREAT_CIRCLE}[metric]
        self._check(self._lib.exageo_set_distance(self._h, m), "set_distance")

    def set_verbose(self, on: bool = True):
        """MLE progress: one line per objective evaluation on stderr."""
        self._check(self._lib.exageo_set_verbose(self._h, int(on)), "set_verbose")

    def set_nugget(self, tau2: float):
        """Fixed nugget: tau2 added to the diagonal of Sigma in every later
        call (0 = none)."""
        self._check(self._lib.exageo_set_nugget(self._h, float(tau2)), "set_nugget")
        self._nugget = float(tau2)

    def set_dst_band(self, band: int):
        """DST approximation of the likelihood calls: tiles |I - J| >= band
        set to zero (0 = exact)."""
        self._check(self._lib.exageo_set_dst_band(self._h, int(band)), "set_dst_band")

    def set_profiling(self, on: bool = True):
        self._check(self._lib.exageo_set_profiling(self._h, int(on)), "set_profiling")

    def timings(self) -> dict:
        buf = (ctypes.c_double * 24)()
        m = self._lib.exageo_get_timings(self._h, buf, 24)
        keys = ["total_ms", "prep_ms", "gen_ms", "chol_ms", "update_kernel_ms", "update_flops", "solve_ms",
                "grad_ms", "chol_flops", "update_launches", "precision", "frac_bf16", "frac_fp32", "update_steps",
                "frac_fp64", "update_flops_fp32", "update_flops_bf16", "update_flops_fp64", "fisher_flops", "logdet",
                "quad_form", "refine_steps"]
        return {k: buf[i] for i, k in enumerate(keys[:m])}

    # ---------------------------------------------------------- operations
    def matern_cov(self, x: torch.Tensor, y: torch.Tensor, theta) -> torch.Tensor:
        """Dense Sigma(theta) (eq. 3) in the caller's order, n x n float64."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y = _dev_f64(y, "y", n)
        cov = torch.empty((n, n), dtype=torch.float64, device=x.device)
        self._sync_stream()
        self._ensure_ws(1, FP64, False)
        st = self._lib.exageo_matern_cov(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                         _lib.darr(theta), ctypes.c_void_p(cov.data_ptr()), n)
        self._check(st, "matern_cov")
        return cov.t()  # column-major fill -> transpose view gives [i, j]

    def simulate(self, x: torch.Tensor, y: torch.Tensor, theta, e: torch.Tensor) -> torch.Tensor:
        """z = L e with L the Cholesky factor of Sigma(theta) (Section 3, Example 1)."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y, e = _dev_f64(y, "y", n), _dev_f64(e, "e", n)
        z = torch.empty(n, dtype=torch.float64, device=x.device)
        self._sync_stream()
        self._ensure_ws(n, FP64, False)
        info = ctypes.c_int64(0)
        st = self._lib.exageo_simulate(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       _lib.darr(theta), ctypes.c_void_p(e.data_ptr()),
                                       ctypes.c_void_p(z.data_ptr()), ctypes.byref(info))
        self._check(st, "simulate", info.value)
        return z

    def loglik(self, x, y, z, theta, precision="fp64") -> float:
        """l(theta) of eq. (2); raises NotPositiveDefinite on a failed pivot."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y, z = _dev_f64(y, "y", n), _dev_f64(z, "z", n)
        prec = _prec(precision)
        self._sync_stream()
        self._ensure_ws(n, prec, False)
        ll = ctypes.c_double(0.0)
        info = ctypes.c_int64(0)
        st = self._lib.exageo_loglik(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     ctypes.c_void_p(z.data_ptr()), _lib.darr(theta), prec, ctypes.byref(ll),
                                     ctypes.byref(info))
        self._check(st, "loglik", info.value)
        return ll.value

    def loglik_status(self, x, y, z, theta, precision="fp64"):
        """(status, l, info) without raising (status codes of exageo.h)."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y, z = _dev_f64(y, "y", n), _dev_f64(z, "z", n)
        prec = _prec(precision)
        self._sync_stream()
        self._ensure_ws(n, prec, False)
        ll = ctypes.c_double(0.0)
        info = ctypes.c_int64(0)
        st = self._lib.exageo_loglik(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     ctypes.c_void_p(z.data_ptr()), _lib.darr(theta), prec, ctypes.byref(ll),
                                     ctypes.byref(info))
        return st, ll.value, info.value

    def loglik_grad(self, x, y, z, theta, precision="fp64"):
        """(l, grad) with grad = dl/d(sigma2, beta, nu) as a length-3 list."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y, z = _dev_f64(y, "y", n), _dev_f64(z, "z", n)
        prec = _prec(precision)
        self._sync_stream()
        self._ensure_ws(n, prec, True)
        ll = ctypes.c_double(0.0)
        g = (ctypes.c_double * 3)()
        info = ctypes.c_int64(0)
        st = self._lib.exageo_loglik_grad(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                          ctypes.c_void_p(z.data_ptr()), _lib.darr(theta), prec, ctypes.byref(ll), g,
                                          ctypes.byref(info))
        self._check(st, "loglik_grad", info.value)
        return ll.value, [g[0], g[1], g[2]]

    def loglik_grad_noalloc(self, x, y, z, theta, with_grad: bool = True):
        """(l, grad) like loglik_grad in FP64, on the library's fixed device
        scratch: no device memory is allocated by this call (grad is None
        when with_grad is False).  Returns (status, l, grad, info) without
        raising, ENOMEM when n is above the scratch's limit."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y, z = _dev_f64(y, "y", n), _dev_f64(z, "z", n)
        self._sync_stream()
        ll = ctypes.c_double(0.0)
        g = (ctypes.c_double * 3)()
        info = ctypes.c_int64(0)
        st = self._lib.exageo_loglik_grad_noalloc(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                                  ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                                  _lib.darr(theta), ctypes.byref(ll), g if with_grad else None,
                                                  ctypes.byref(info))
        return st, ll.value, ([g[0], g[1], g[2]] if with_grad else None), info.value

    def last_error(self) -> str:
        return self._lib.exageo_last_error(self._h).decode(errors="replace")

    def predict(self, x, y, z, theta, xnew, ynew, with_mse: bool = True):
        """Kriging at (xnew, ynew): (mean, mse) float64 tensors (mse None
        when with_mse is False)."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y, z = _dev_f64(y, "y", n), _dev_f64(z, "z", n)
        xnew = _dev_f64(xnew, "xnew")
        m = xnew.numel()
        ynew = _dev_f64(ynew, "ynew", m)
        mean = torch.empty(m, dtype=torch.float64, device=x.device)
        mse = torch.empty(m, dtype=torch.float64, device=x.device) if with_mse else None
        self._sync_stream()
        self._ensure_ws(n, FP64, True)  # the variance blocks use the gradient plan's staging buffer
        info = ctypes.c_int64(0)
        st = self._lib.exageo_predict(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      ctypes.c_void_p(z.data_ptr()), _lib.darr(theta), m,
                                      ctypes.c_void_p(xnew.data_ptr()), ctypes.c_void_p(ynew.data_ptr()),
                                      ctypes.c_void_p(mean.data_ptr()),
                                      ctypes.c_void_p(mse.data_ptr()) if mse is not None else None,
                                      ctypes.byref(info))
        self._check(st, "predict", info.value)
        return mean, mse

    def fisher(self, x, y, theta):
        """Fisher information of theta = (sigma^2, beta, nu) at the locations:
        a 3 x 3 float64 numpy array (FP64 whatever the precision policy)."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y = _dev_f64(y, "y", n)
        self._sync_stream()
        self._ensure_ws(n, FP64, 3 if self._nugget > 0 else 2)  # derivative matrices in the workspace
        out = (ctypes.c_double * 9)()
        info = ctypes.c_int64(0)
        st = self._lib.exageo_fisher(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                     _lib.darr(theta), out, ctypes.byref(info))
        self._check(st, "fisher", info.value)
        return np.array(out[:], dtype=np.float64).reshape(3, 3)

    def mle(self, x, y, z, lb, ub, theta0=None, tol: float = 1e-4, max_iters: int = 0, method="dfo",
            precision="fp64"):
        """Bounded MLE; returns (theta_hat, loglik_hat, stats dict).  Raises on
        errors other than ENOCONV (which is reported in stats['status'])."""
        x = _dev_f64(x, "x")
        n = x.numel()
        y, z = _dev_f64(y, "y", n), _dev_f64(z, "z", n)
        prec, meth = _prec(precision), _method(method)
        self._sync_stream()
        self._ensure_ws(n, prec, meth != DFO)
        if meth == LBFGSB_FP64_FINISH:
            self._ensure_ws(n, FP64, True)  # the finish runs the FP64 plan in the same workspace
        th = (ctypes.c_double * 3)()
        ll = ctypes.c_double(0.0)
        stats = _lib.MleStats()
        t0 = _lib.darr(theta0) if theta0 is not None else None
        st = self._lib.exageo_mle(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  ctypes.c_void_p(z.data_ptr()), _lib.darr(lb), _lib.darr(ub), t0, float(tol),
                                  int(max_iters), meth, prec, th, ctypes.byref(ll), ctypes.byref(stats))
        if st not in (OK, ENOCONV):
            self._check(st, "mle")
        out = {"n_evals": stats.n_evals, "n_grad_evals": stats.n_grad_evals, "iters": stats.iters,
               "total_s": stats.total_s, "per_eval_s": stats.per_eval_s,
               "status": STATUS_NAMES.get(stats.status, stats.status),
               "n_fp64_finish_evals": stats.n_fp64_finish_evals}
        return [th[0], th[1], th[2]], ll.value, out


class ExaGeoLoglik(torch.autograd.Function):
    """l(theta) as a differentiable function of theta (float64 CPU tensor of 3).

    The forward pass already computes the gradient when theta requires it
    (one factorisation for both); backward scales it by the incoming grad.
    """

    @staticmethod
    def forward(fctx, theta, x, y, z, context: Context, precision="fp64"):
        th = [float(v) for v in theta.detach().cpu().tolist()]
        if theta.requires_grad:
            ll, g = context.loglik_grad(x, y, z, th, precision)
        else:
            ll, g = context.loglik(x, y, z, th, precision), [math.nan] * 3
        fctx.save_for_backward(torch.tensor(g, dtype=torch.float64))
        return torch.tensor(ll, dtype=torch.float64)

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        return grad_out * g, None, None, None, None, None
