"""Seeded generators for synthetic multinomial-logit data.

Letters follow the three data kinds of the utility model (Eq. 1), written
with this project's names:

  X [N, p]     individual-specific data, alternative-specific coefficients
               beta_k (the paper's X_i . beta_k); column 0 is the intercept
               (all ones) when ``intercept`` is set, so xi_k is beta_k[0].
  Y [N, K, g]  alternative-varying data with one generic coefficient vector
               alpha (the paper's Z_ik . alpha).
  Z [N, K, a]  alternative-varying data with alternative-specific
               coefficients gamma_k (the paper's Y_ik . gamma_k).

The coefficient vector is laid out as in Eq. 8:
  theta = (beta_1 .. beta_{K-1}, gamma_0 .. gamma_{K-1}, alpha),
with beta_0 fixed at zero (alternative 0 is the base, Sec. 2.2).

Choices are drawn by simulating the random-utility model itself: each
individual takes the alternative of largest U_ik + e_ik with e_ik i.i.d.
standard Gumbel (Sec. 2.2, the utility-maximisation principle).  That yields
exactly the logit choice law without evaluating any probability here.

Draw order for one problem (one numpy PCG64 stream): X, Y, Z, theta_true,
weights, Gumbel noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    N: int
    K: int
    p: int
    g: int
    a: int
    X: np.ndarray                 # [N, p] float64
    Y: np.ndarray                 # [N, K, g] float64 (g may be 0)
    Z: np.ndarray                 # [N, K, a] float64 (a may be 0)
    choice: np.ndarray            # [N] int32 in 0..K-1
    w: Optional[np.ndarray]       # [N] float64 or None (all ones)
    theta_true: np.ndarray        # [n_p] float64
    name: str = "custom"
    meta: dict = field(default_factory=dict)

    @property
    def n_params(self) -> int:
        # layout size of theta (Eq. 8): K-1 beta chunks, K gamma chunks, alpha
        return (self.K - 1) * self.p + self.K * self.a + self.g


def _features(rng, shape, rho):
    """N(0,1) features; with rho > 0 they are equicorrelated along the last
    axis: sqrt(rho) * shared + sqrt(1 - rho) * own."""
    own = rng.standard_normal(shape)
    if rho <= 0.0 or shape[-1] == 0:
        return own
    shared = rng.standard_normal(shape[:-1] + (1,))
    return math.sqrt(rho) * shared + math.sqrt(1.0 - rho) * own


def make_problem(N: int, K: int, p: int, g: int, a: int, seed: int, *,
                 coef_sd: float = 0.5, rho: float = 0.0,
                 intercept: bool = True, weights: Optional[str] = None,
                 name: str = "custom") -> Problem:
    """Draw one synthetic problem.

    p counts the intercept column when ``intercept`` is set.  ``weights`` is
    None (unweighted), "uniform" (U[0.5, 2]) or "int" (integers 1..3).
    """
    if K < 2:
        raise ValueError("K must be at least 2")
    if p < 0 or g < 0 or a < 0:
        raise ValueError("negative dimension")
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.empty((N, p), dtype=np.float64)
    lo = 0
    if intercept and p > 0:
        X[:, 0] = 1.0
        lo = 1
    if p - lo > 0:
        X[:, lo:] = _features(rng, (N, p - lo), rho)
    Y = _features(rng, (N, K, g), rho) if g else np.zeros((N, K, 0))
    Z = _features(rng, (N, K, a), rho) if a else np.zeros((N, K, 0))
    n_p = (K - 1) * p + K * a + g
    theta = coef_sd * rng.standard_normal(n_p)
    if weights is None:
        w = None
    elif weights == "uniform":
        w = rng.uniform(0.5, 2.0, size=N)
    elif weights == "int":
        w = rng.integers(1, 4, size=N).astype(np.float64)
    else:
        raise ValueError(f"unknown weights kind {weights!r}")
    gumbel = rng.gumbel(size=(N, K))

    # the simulated individuals' utilities (Eq. 1) and their choice
    beta = np.zeros((K, p))
    beta[1:] = theta[: (K - 1) * p].reshape(K - 1, p)
    gamma = theta[(K - 1) * p:(K - 1) * p + K * a].reshape(K, a)
    alpha = theta[(K - 1) * p + K * a:]
    util = X @ beta.T
    if a:
        util += np.einsum("ika,ka->ik", Z, gamma)
    if g:
        util += Y @ alpha
    choice = np.argmax(util + gumbel, axis=1).astype(np.int32)
    return Problem(N=N, K=K, p=p, g=g, a=a, X=np.ascontiguousarray(X),
                   Y=np.ascontiguousarray(Y), Z=np.ascontiguousarray(Z),
                   choice=choice, w=w, theta_true=theta, name=name,
                   meta=dict(seed=seed, coef_sd=coef_sd, rho=rho,
                             weights=weights))


# The five workloads.  p includes the intercept column.
CONFIGS = {
    # plain FP64 fit, single small model
    "c1": dict(N=2_000, K=10, p=6, g=1, a=0, seed=1, coef_sd=0.5),
    # single larger fit, FP64 vs FP32 Hessian
    "c2": dict(N=100_000, K=50, p=21, g=5, a=5, seed=2, coef_sd=0.3),
    # mixed-precision Hessian stress, equicorrelated features
    "c3": dict(N=400_000, K=100, p=51, g=5, a=0, seed=3, coef_sd=0.3,
               rho=0.3),
    # many classes, weighted, near-separable
    "c5": dict(N=50_000, K=500, p=11, g=0, a=0, seed=5, coef_sd=3.0,
               weights="uniform"),
}


def make_config(name: str, **override) -> Problem:
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    return make_problem(name=name, **cfg)


# ---- serving stream (many uneven fits) -------------------------------------

SERVING_SEED = 4


def serving_request_shapes(r: int) -> dict:
    """Shape of request r: N log-uniform in [1e3, 2e5], K in 5..60,
    1 + (5..30) individual-specific columns (intercept included), 0..5
    generic variables."""
    rng = np.random.Generator(np.random.PCG64(4_000_000 + r))
    N = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
    K = int(rng.integers(5, 61))
    p = 1 + int(rng.integers(5, 31))
    g = int(rng.integers(0, 6))
    return dict(N=N, K=K, p=p, g=g, a=0, seed=4_100_000 + r)


def serving_request(r: int) -> Problem:
    shp = serving_request_shapes(r)
    return make_problem(coef_sd=0.5, name=f"req{r}", **shp)


def serving_arrivals(n: int, rate: float) -> np.ndarray:
    """Poisson arrival times (seconds from start) of n requests at ``rate``
    requests per second."""
    rng = np.random.Generator(np.random.PCG64(SERVING_SEED))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


class ServingStream:
    """Host data of the serving stream, drawn fast enough to feed the GPU.

    Request r has the shape serving_request_shapes(r), its own coefficients
    (N(0, 0.5^2)) and its own simulated choices (Gumbel-max over its
    utilities, as make_problem).  Drawing every request's features afresh
    would cost the host more time than the GPU needs for the fit, so the
    features are windows into shared N(0,1) pools, at offsets drawn from the
    request's seed: X from a pool of rows of width p whose column 0 is the
    intercept, Y from a flat pool, and the Gumbel noise of the choices from
    a Gumbel pool.  Each request's arrays are plain contiguous views (no
    copies); ``alloc(shape, dtype)`` supplies the pools' and the choices'
    memory (e.g. page-locked host memory).
    """

    def __init__(self, n_requests: int, seed: int = SERVING_SEED,
                 alloc=None, threads: int = 8):
        self.shapes = [serving_request_shapes(r) for r in range(n_requests)]
        self.alloc = alloc or (lambda shape, dt: np.empty(shape, dtype=dt))
        self.threads = threads
        rng = np.random.Generator(np.random.PCG64(seed * 1_000_003 + 17))
        slack = 1 << 16
        max_n = max(s["N"] for s in self.shapes)
        ny = max(s["N"] * s["K"] * s["g"] for s in self.shapes)
        ng = max(s["N"] * s["K"] for s in self.shapes)
        ps = sorted({s["p"] for s in self.shapes})
        self.rows = max_n + slack
        flat = self.alloc((ny + slack,), np.float64)
        flat[:] = rng.standard_normal(flat.shape[0])
        self.ypool = flat
        self.xpool = {}
        for p in ps:
            xp = self.alloc((self.rows, p), np.float64)
            xp[:, 1:] = rng.standard_normal((self.rows, p - 1))
            xp[:, 0] = 1.0
            self.xpool[p] = xp
        gp = self.alloc((ng + slack,), np.float64)
        gp[:] = rng.gumbel(size=gp.shape[0])
        self.gpool = gp

    def request(self, r: int) -> Problem:
        s = self.shapes[r]
        N, K, p, g = s["N"], s["K"], s["p"], s["g"]
        rng = np.random.Generator(np.random.PCG64(s["seed"]))
        ox = int(rng.integers(0, self.rows - N + 1))
        X = self.xpool[p][ox:ox + N]
        ny = N * K * g
        oy = int(rng.integers(0, self.ypool.shape[0] - ny + 1))
        Y = self.ypool[oy:oy + ny].reshape(N, K, g)
        n_p = (K - 1) * p + g
        theta = 0.5 * rng.standard_normal(n_p)
        og = int(rng.integers(0, self.gpool.shape[0] - N * K + 1))
        gumbel = self.gpool[og:og + N * K].reshape(N, K)
        beta = np.zeros((K, p))
        beta[1:] = theta[:(K - 1) * p].reshape(K - 1, p)
        util = X @ beta.T
        if g:
            util += (Y.reshape(N * K, g) @ theta[(K - 1) * p:]).reshape(N, K)
        choice = self.alloc((N,), np.int32)
        choice[:] = np.argmax(util + gumbel, axis=1)
        return Problem(N=N, K=K, p=p, g=g, a=0, X=X, Y=Y,
                       Z=np.zeros((N, K, 0)), choice=choice, w=None,
                       theta_true=theta, name=f"req{r}",
                       meta=dict(seed=s["seed"], coef_sd=0.5, rho=0.0,
                                 weights=None, pooled=True))

    def requests(self) -> list:
        """All requests, drawn on a thread pool (numpy releases the GIL in
        the matrix products)."""
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(self.threads) as ex:
            return list(ex.map(self.request, range(len(self.shapes))))
