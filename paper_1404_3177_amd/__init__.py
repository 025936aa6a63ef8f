"""MI355X Newton-Raphson fitter of multinomial logit models.

Python face of libmnl.so: torch tensors on the GPU hold the data, the calls
go straight to the library's C ABI (include/mnl.h) on the current stream.

    import torch, paper_1404_3177_amd as mnl
    ctx = mnl.Context()
    prob = mnl.Problem(X, Y, Z, choice, w)        # device tensors
    theta, info = ctx.fit(prob, gtol=1e-8)

Letters: X [N,p] individual-specific data (alternative-specific coefficients
beta), Y [N,K,g] alternative-varying data with generic coefficients alpha,
Z [N,K,a] alternative-varying data with alternative-specific coefficients
gamma; theta = (beta_1..beta_{K-1}, gamma_0..gamma_{K-1}, alpha).
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import _lib
from ._lib import (MnlError, MnlFitInfo, MnlFitOpts, MnlProblem, PREC,  # noqa
                   STOP_FTOL, STOP_GTOL, STOP_LS_FAIL, STOP_MAXITER,
                   STOP_NONE, STOP_NONFINITE, STOP_NOT_PD)

__all__ = ["Context", "Problem", "num_params", "default_opts", "MnlError"]


def num_params(K: int, p: int, g: int, a: int) -> int:
    return int(_lib.load().mnl_num_params(K, p, g, a))


def default_opts() -> dict:
    o = MnlFitOpts()
    _lib.load().mnl_default_opts(ctypes.byref(o))
    return {f: getattr(o, f) for f, _ in MnlFitOpts._fields_}


def _stream_handle(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Problem:
    """Device-resident problem.  Tensors must be contiguous: X float64
    [N, p], Y float64 [N, K, g], Z float64 [N, K, a], choice int32 [N],
    w float64 [N] or None."""

    def __init__(self, X, Y, Z, choice, w=None):
        import torch
        N, p = X.shape
        K, g = Y.shape[1], Y.shape[2]
        a = Z.shape[2]
        for t, name in ((X, "X"), (Y, "Y"), (Z, "Z")):
            if t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous float64")
        if choice.dtype != torch.int32 or not choice.is_contiguous():
            raise ValueError("choice must be contiguous int32")
        if w is not None and (w.dtype != torch.float64 or not w.is_contiguous()):
            raise ValueError("w must be contiguous float64")
        if Y.shape[0] != N or Z.shape[0] != N or Z.shape[1] != K or \
                choice.shape[0] != N:
            raise ValueError("inconsistent shapes")
        self.N, self.K, self.p, self.g, self.a = N, K, p, g, a
        self.device = X.device
        self._refs = (X, Y, Z, choice, w)
        self.c = MnlProblem(
            N=N, K=K, p=p, g=g, a=a,
            X=X.data_ptr() if p else None, Y=Y.data_ptr() if g else None,
            Z=Z.data_ptr() if a else None, choice=choice.data_ptr(),
            w=w.data_ptr() if w is not None else None)

    @property
    def n_params(self) -> int:
        return (self.K - 1) * self.p + self.K * self.a + self.g

    @classmethod
    def from_numpy(cls, prob, device="cuda"):
        """Copy a synth.Problem (numpy arrays) to the device."""
        import torch

        def t(x, dt):
            return torch.from_numpy(x).to(device=device, dtype=dt).contiguous()
        w = None if prob.w is None else t(prob.w, torch.float64)
        return cls(t(prob.X, torch.float64), t(prob.Y, torch.float64),
                   t(prob.Z, torch.float64), t(prob.choice, torch.int32), w)


class Context:
    """One library context (device workspace) on a HIP device."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        rc = self.lib.mnl_create(ctypes.byref(h), device)
        if rc != 0:
            raise MnlError(rc, "mnl_create failed")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.lib.mnl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            msg = self.lib.mnl_last_error(self.h).decode()
            raise MnlError(rc, msg)

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.mnl_workspace_bytes(self.h))

    @staticmethod
    def _opts(**kw) -> MnlFitOpts:
        o = MnlFitOpts()
        _lib.load().mnl_default_opts(ctypes.byref(o))
        for k, v in kw.items():
            if k == "prec" and isinstance(v, str):
                v = PREC[v]
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        return o

    def loglik_grad(self, prob: Problem, theta, want_P: bool = False,
                    stream=None):
        """(l, g, P): device tensors; l has shape [1]."""
        import torch
        dev = prob.device
        l = torch.empty(1, dtype=torch.float64, device=dev)
        g = torch.empty(prob.n_params, dtype=torch.float64, device=dev)
        P = torch.empty(prob.N, prob.K, dtype=torch.float64, device=dev) \
            if want_P else None
        self._check(self.lib.mnl_loglik_grad(
            self.h, ctypes.byref(prob.c), theta.data_ptr(), l.data_ptr(),
            g.data_ptr(), P.data_ptr() if P is not None else None,
            _stream_handle(stream)))
        return l, g, P

    def hessian(self, prob: Problem, theta, prec="fp64", stream=None):
        import torch
        n = prob.n_params
        H = torch.empty(n, n, dtype=torch.float64, device=prob.device)
        pr = PREC[prec] if isinstance(prec, str) else int(prec)
        self._check(self.lib.mnl_hessian(
            self.h, ctypes.byref(prob.c), theta.data_ptr(), pr, H.data_ptr(),
            _stream_handle(stream)))
        return H

    def newton_step(self, prob: Problem, theta, stream=None, **opts) -> dict:
        """One NR iteration; theta (device tensor) is updated in place."""
        o = self._opts(**opts)
        info = MnlFitInfo()
        self._check(self.lib.mnl_newton_step(
            self.h, ctypes.byref(prob.c), theta.data_ptr(), ctypes.byref(o),
            ctypes.byref(info), _stream_handle(stream)))
        return info.as_dict()

    def fit(self, prob: Problem, theta0=None, stream=None, **opts):
        """Newton-Raphson fit; returns (theta tensor, info dict)."""
        import torch
        o = self._opts(**opts)
        info = MnlFitInfo()
        theta = torch.empty(prob.n_params, dtype=torch.float64,
                            device=prob.device)
        self._check(self.lib.mnl_fit(
            self.h, ctypes.byref(prob.c),
            theta0.data_ptr() if theta0 is not None else None,
            ctypes.byref(o), theta.data_ptr(), ctypes.byref(info),
            _stream_handle(stream)))
        return theta, info.as_dict()
