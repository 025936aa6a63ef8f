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
from ._lib import (METHOD, MnlError, MnlFitInfo, MnlFitOpts,  # noqa
                   MnlProblem, MnlServerOpts, MnlServerResult,
                   MnlServerStats, PREC,
                   STOP_FTOL, STOP_GTOL, STOP_LS_FAIL, STOP_MAXITER,
                   STOP_NONE, STOP_NONFINITE, STOP_NOT_PD)

__all__ = ["Context", "Problem", "HostProblem", "Server", "num_params",
           "batch_eligible", "default_opts", "fit_footprint", "chi2_sf", "lr_stat", "MnlError"]


def num_params(K: int, p: int, g: int, a: int) -> int:
    return int(_lib.load().mnl_num_params(K, p, g, a))


def chi2_sf(x: float, df: float) -> float:
    """Upper tail of the chi-square distribution (the library's)."""
    return float(_lib.load().mnl_chi2_sf(float(x), float(df)))


def lr_stat(loglik_full: float, loglik_restricted: float, df: int):
    """Likelihood-ratio statistic of nested fits and its chi-square
    p-value, (stat, p), from the library (mnl_lrtest)."""
    stat, p = ctypes.c_double(), ctypes.c_double()
    rc = _lib.load().mnl_lrtest(float(loglik_full), float(loglik_restricted),
                                int(df), ctypes.byref(stat), ctypes.byref(p))
    if rc != 0:
        raise MnlError(rc, "mnl_lrtest failed")
    return stat.value, p.value


def batch_eligible(N: int, K: int, p: int, g: int, a: int, **opts) -> bool:
    """Whether the server runs a fit of this shape with these options
    through the batched kernel (mnl_batch_eligible)."""
    o = Context._opts(**opts)
    shape = MnlProblem(N=N, K=K, p=p, g=g, a=a)
    return bool(_lib.load().mnl_batch_eligible(ctypes.byref(shape),
                                               ctypes.byref(o)))


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
    [N, p], Y float64 [N, K, g], Z float64 [N, K, a], choice int32 [N]
    (None for data that are only predicted or summarised), w float64 [N] or
    None."""

    def __init__(self, X, Y, Z, choice, w=None):
        import torch
        N, p = X.shape
        K, g = Y.shape[1], Y.shape[2]
        a = Z.shape[2]
        for t, name in ((X, "X"), (Y, "Y"), (Z, "Z")):
            if t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous float64")
        if choice is not None and (choice.dtype != torch.int32 or
                                   not choice.is_contiguous()):
            raise ValueError("choice must be contiguous int32")
        if w is not None and (w.dtype != torch.float64 or not w.is_contiguous()):
            raise ValueError("w must be contiguous float64")
        if Y.shape[0] != N or Z.shape[0] != N or Z.shape[1] != K or \
                (choice is not None and choice.shape[0] != N):
            raise ValueError("inconsistent shapes")
        self.N, self.K, self.p, self.g, self.a = N, K, p, g, a
        self.device = X.device
        self._refs = (X, Y, Z, choice, w)
        self.c = MnlProblem(
            N=N, K=K, p=p, g=g, a=a,
            X=X.data_ptr() if p else None, Y=Y.data_ptr() if g else None,
            Z=Z.data_ptr() if a else None,
            choice=choice.data_ptr() if choice is not None else None,
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
    """One library context (device workspace) on a HIP device;
    workspace_bytes caps the workspace (0: no cap)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        rc = self.lib.mnl_create(ctypes.byref(h), device, int(workspace_bytes))
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
            if k == "method" and isinstance(v, str):
                v = METHOD[v]
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

    def loglik_grad_noalloc(self, prob: Problem, theta, want_P: bool = False,
                            stream=None):
        """loglik_grad through mnl_loglik_grad_noalloc: no device
        allocation by the library (the outputs here are torch tensors)."""
        import torch
        dev = prob.device
        l = torch.empty(1, dtype=torch.float64, device=dev)
        g = torch.empty(prob.n_params, dtype=torch.float64, device=dev)
        P = torch.empty(prob.N, prob.K, dtype=torch.float64, device=dev) \
            if want_P else None
        self._check(self.lib.mnl_loglik_grad_noalloc(
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

    def fit_batch(self, probs, theta0s=None, opts=None, stream=None):
        """Many small fits in one persistent kernel (mnl_fit_batch); probs
        is a list of Problems, theta0s None or a list of tensors / None,
        opts None (defaults), one dict for all, or a list of dicts.
        Returns ([theta tensors], [info dicts])."""
        import torch
        n = len(probs)
        pa = (MnlProblem * max(n, 1))(*[pr.c for pr in probs])
        if opts is None or isinstance(opts, dict):
            one = self._opts(**(opts or {}))
            oa = (MnlFitOpts * max(n, 1))(*([one] * n))
        else:
            oa = (MnlFitOpts * max(n, 1))(*[self._opts(**o) for o in opts])
        thetas = [torch.empty(pr.n_params, dtype=torch.float64,
                              device=pr.device) for pr in probs]
        ta = (ctypes.c_void_p * max(n, 1))(*[t.data_ptr() for t in thetas])
        t0 = None
        if theta0s is not None:
            t0 = (ctypes.c_void_p * max(n, 1))(
                *[t.data_ptr() if t is not None else None for t in theta0s])
        infos = (MnlFitInfo * max(n, 1))()
        self._check(self.lib.mnl_fit_batch(
            self.h, n, pa, t0, oa, ta, infos, _stream_handle(stream)))
        return thetas, [infos[i].as_dict() for i in range(n)]

    def collinear(self, prob: Problem, tol: float = 1e-6, stream=None):
        """Keep masks (numpy bool) of the X, Y and Z variables."""
        import numpy as np
        ks = [np.zeros(n, dtype=np.int32) for n in (prob.p, prob.g, prob.a)]
        self._check(self.lib.mnl_collinear(
            self.h, ctypes.byref(prob.c), float(tol),
            *[k.ctypes.data if k.size else None for k in ks],
            _stream_handle(stream)))
        return tuple(k.astype(bool) for k in ks)

    def select_columns(self, prob: Problem, keep_x, keep_y, keep_z,
                       stream=None) -> "Problem":
        """A new device Problem holding only the kept columns (same
        choices and weights)."""
        import numpy as np
        import torch
        ks = [np.ascontiguousarray(k, dtype=np.int32)
              for k in (keep_x, keep_y, keep_z)]
        px, py, pz = (int(k.sum()) for k in ks)
        dev = prob.device
        N, K = prob.N, prob.K
        Xo = torch.empty(N, px, dtype=torch.float64, device=dev)
        Yo = torch.empty(N, K, py, dtype=torch.float64, device=dev)
        Zo = torch.empty(N, K, pz, dtype=torch.float64, device=dev)
        self._check(self.lib.mnl_select_columns(
            self.h, ctypes.byref(prob.c),
            *[k.ctypes.data if k.size else None for k in ks],
            Xo.data_ptr() if px else None, Yo.data_ptr() if py else None,
            Zo.data_ptr() if pz else None, _stream_handle(stream)))
        # the host masks are read before the call returns
        _, _, _, choice, w = prob._refs
        return Problem(Xo, Yo, Zo, choice, w)

    def covariance(self, prob: Problem, theta, idx=None, stream=None):
        """(-H)^{-1} at theta restricted to the coefficients idx (all if
        None): a device tensor [s, s]."""
        import numpy as np
        import torch
        n = prob.n_params
        sel = None if idx is None else np.ascontiguousarray(idx, np.int32)
        s = n if sel is None else sel.size
        V = torch.empty(s, s, dtype=torch.float64, device=prob.device)
        self._check(self.lib.mnl_covariance(
            self.h, ctypes.byref(prob.c), theta.data_ptr(),
            sel.ctypes.data if sel is not None else None,
            0 if sel is None else s, V.data_ptr(), _stream_handle(stream)))
        return V

    def quadform(self, A, x, B=None, x0=None, hessian_sign: bool = False,
                 stream=None) -> float:
        """d^T (A - B)^{-1} d with d = x - x0 (B, x0 optional) for a
        symmetric positive definite A - B on the device (d^T (B - A)^{-1} d
        when hessian_sign)."""
        out = ctypes.c_double()
        ts = [None if t is None else t.contiguous() for t in (A, B, x, x0)]
        self._check(self.lib.mnl_quadform(
            self.h, *[t.data_ptr() if t is not None else None for t in ts],
            int(x.numel()), 1 if hessian_sign else 0, ctypes.byref(out),
            _stream_handle(stream)))
        return out.value

    def hessvec(self, prob: Problem, theta, v, stream=None):
        """H(theta) v (device tensor, Hessian sign) without forming H."""
        import torch
        Hv = torch.empty(prob.n_params, dtype=torch.float64,
                         device=prob.device)
        self._check(self.lib.mnl_hessvec(
            self.h, ctypes.byref(prob.c), theta.data_ptr(), v.data_ptr(),
            Hv.data_ptr(), _stream_handle(stream)))
        return Hv

    def predict(self, prob: Problem, theta, stream=None):
        """Choice probabilities [N, K] (device tensor) on prob's data; its
        choices and weights are not read."""
        import torch
        P = torch.empty(prob.N, prob.K, dtype=torch.float64,
                        device=prob.device)
        self._check(self.lib.mnl_predict(
            self.h, ctypes.byref(prob.c), theta.data_ptr(), P.data_ptr(),
            _stream_handle(stream)))
        return P

    def summary(self, prob: Problem, theta, stream=None):
        """(se, z, p) device tensors: standard errors sqrt(diag((-H)^-1)),
        Wald statistics theta / se and two-sided normal p-values."""
        import torch
        n = prob.n_params
        out = [torch.empty(n, dtype=torch.float64, device=prob.device)
               for _ in range(3)]
        self._check(self.lib.mnl_stderr(
            self.h, ctypes.byref(prob.c), theta.data_ptr(),
            out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
            _stream_handle(stream)))
        return tuple(out)


def fit_footprint(N: int, K: int, p: int, g: int, a: int, prec="fp64",
                  weights: bool = False) -> int:
    """Device bytes a served fit of this shape holds (data + workspace)."""
    pr = PREC[prec] if isinstance(prec, str) else int(prec)
    shape = MnlProblem(N=N, K=K, p=p, g=g, a=a, X=None, Y=None, Z=None,
                       choice=None, w=1 if weights else None)
    return int(_lib.load().mnl_fit_footprint(ctypes.byref(shape), pr))


class HostProblem:
    """Problem whose arrays live in host memory (the server's input).
    Arrays are made contiguous float64 / int32; with pinned=True they are
    copied into page-locked torch tensors, which the device reads faster."""

    def __init__(self, X, Y, Z, choice, w=None, pinned: bool = False):
        import numpy as np
        N, p = X.shape
        K, g, a = Y.shape[1], Y.shape[2], Z.shape[2]
        if Y.shape[0] != N or Z.shape[0] != N or Z.shape[1] != K or \
                choice.shape[0] != N:
            raise ValueError("inconsistent shapes")

        def host(x, dt):
            x = np.ascontiguousarray(x, dtype=dt)
            if not pinned:
                return x, x.ctypes.data
            import torch
            t = torch.from_numpy(x).pin_memory()
            return t, t.data_ptr()
        self.N, self.K, self.p, self.g, self.a = N, K, p, g, a
        hx, px = host(X, np.float64)
        hy, py = host(Y, np.float64)
        hz, pz = host(Z, np.float64)
        hc, pc = host(choice, np.int32)
        hw, pw = host(w, np.float64) if w is not None else (None, None)
        self._refs = (hx, hy, hz, hc, hw)
        self.c = MnlProblem(N=N, K=K, p=p, g=g, a=a,
                            X=px if p else None, Y=py if g else None,
                            Z=pz if a else None, choice=pc, w=pw)

    @property
    def n_params(self) -> int:
        return (self.K - 1) * self.p + self.K * self.a + self.g

    @classmethod
    def from_numpy(cls, prob, pinned: bool = False):
        """From a synth.Problem."""
        return cls(prob.X, prob.Y, prob.Z, prob.choice, prob.w, pinned=pinned)


class Server:
    """Continuous-batching fit server (mnl_server_* in include/mnl.h).

    submit() queues a HostProblem and returns its id; wait() returns
    finished requests as dicts with the fitted theta (numpy), status, the
    fit report and the arrival / admission / completion times (ms on the
    server clock, now_ms())."""

    def __init__(self, slots: int = 8, hbm_budget: int = 0, device: int = 0,
                 host_only: bool = False, host_fit_ms: float = 0.0,
                 max_group: int = 0):
        self.lib = _lib.load()
        o = MnlServerOpts(device=device, slots=slots, hbm_budget=hbm_budget,
                          host_only=1 if host_only else 0,
                          max_group=int(max_group),
                          host_fit_ms=float(host_fit_ms))
        h = ctypes.c_void_p()
        rc = self.lib.mnl_server_create(ctypes.byref(h), ctypes.byref(o))
        if rc != 0:
            raise MnlError(rc, "mnl_server_create failed")
        self.h = h
        self._live = {}
        import threading
        # submit() and wait() may run on different threads: a result is
        # matched to its request only after submit() has recorded it
        self._lock = threading.Lock()

    def now_ms(self) -> float:
        return float(self.lib.mnl_server_now_ms())

    def submit(self, prob: HostProblem, theta0=None, t_arrival: float = -1.0,
               **opts) -> int:
        import numpy as np
        o = Context._opts(**opts)
        theta = np.empty(prob.n_params, dtype=np.float64)
        th0 = None
        if theta0 is not None:
            th0 = np.ascontiguousarray(theta0, dtype=np.float64)
        rid = ctypes.c_int64()
        with self._lock:
            rc = self.lib.mnl_server_submit(
                self.h, ctypes.byref(prob.c),
                th0.ctypes.data if th0 is not None else None,
                ctypes.byref(o), theta.ctypes.data, float(t_arrival),
                ctypes.byref(rid))
            if rc != 0:
                raise MnlError(rc, "mnl_server_submit refused the request")
            self._live[rid.value] = (prob, theta, th0)
        return rid.value

    def wait(self, max_results: int = 256, timeout_ms: float = -1.0) -> list:
        buf = (MnlServerResult * max_results)()
        n = ctypes.c_int32()
        rc = self.lib.mnl_server_wait(self.h, buf, max_results,
                                      float(timeout_ms), ctypes.byref(n))
        if rc != 0:
            raise MnlError(rc, "mnl_server_wait failed")
        out = []
        for r in buf[:n.value]:
            with self._lock:
                _, theta, _ = self._live.pop(r.id)
            out.append(dict(id=r.id, status=r.status, slot=r.slot,
                            t_arrival=r.t_arrival, t_admit=r.t_admit,
                            t_done=r.t_done, footprint=r.footprint,
                            info=r.info.as_dict(), theta=theta))
        return out

    def stats(self) -> dict:
        st = MnlServerStats()
        rc = self.lib.mnl_server_get_stats(self.h, ctypes.byref(st))
        if rc != 0:
            raise MnlError(rc, "mnl_server_get_stats failed")
        return st.as_dict()

    @property
    def pending(self) -> int:
        return len(self._live)

    def close(self):
        if self.h:
            self.lib.mnl_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
