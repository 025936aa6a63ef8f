"""Plain FP64 CPU oracle of the Newton-Raphson multinomial-logit fit.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and is deliberately slow and literal: every quantity is computed the
way the paper writes it, block by block, with numpy/scipy primitives as the
only steps.

Paper: Hasan, Wang, Mahani, "Fast Estimation of Multinomial Logit Models:
R Package mnlogit" (arXiv:1404.3177).

Letter mapping (the paper's Y and Z are swapped in this project):

  role                                   paper      here   coefficients
  individual-specific data               X_i        X      beta_k  (K-1 chunks of p)
  alternative-varying, generic coef      Z_ik       Y      alpha   (g)
  alternative-varying, alt-specific coef Y_ik       Z      gamma_k (K chunks of a)

theta = (beta_1..beta_{K-1}, gamma_0..gamma_{K-1}, alpha)      (Eq. 8)

Readings taken where the paper is silent (all also used by the GPU path):
  * weights are frequency weights multiplying each individual's term of the
    log-likelihood, hence every gradient and Hessian term;
  * the gradient norm of the stopping rule is the Euclidean norm of the
    gradient of the summed log-likelihood;
  * the line search accepts a trial step when l(theta + t*delta) is not lower
    than l(theta) by more than tau = ls_tol_ulps * eps * |l(theta)| (the
    literal "not lower" rule stalls at the round-off floor of l); it halves t
    at most ls_max times, then reports a line-search failure; every trial
    evaluation counts as one line-search iteration;
  * the Newton system is solved by Cholesky of -H; a failed factorisation, or
    a pivot d_j <= n_p * eps * max_k(-H_kk), is reported as "Hessian not
    negative definite".
  * the summary's standard errors are the square roots of the diagonal of
    the inverse observed information (-H)^{-1} at the given theta, its
    p-values two-sided normal tails of z = theta / se; predict returns the
    probabilities of Eqs. 3-4 on data without choices.
  * the inexact Newton method (the paper's stated next step) takes its
    direction from truncated conjugate gradients on (-H) d = g from d = 0,
    with relative residual eta = min(1/2, sqrt(||g|| / ||g_0||)) (g_0 the
    gradient where the fit started), at most cg_maxiter
    Hessian-vector products, and d = g when the first search direction
    shows non-positive curvature; line search and stop rules are Newton's.
  * the collinearity check follows App. B's necessary conditions with a
    column-order QR at tolerance linDepTol (default 1e-6): X and every Z_k
    must have full column rank, the differenced generic data stacked over
    alternatives too; a dependent Z variable is dropped for every
    alternative (coefficient chunks have one length).
  * hypothesis tests are the textbook likelihood-ratio, Wald, Rao score and
    Hausman-McFadden statistics with chi-square p-values; the score test is
    taken at the restricted estimate embedded in the full model.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg

# stop reasons / status codes (same numeric values as the C library)
STOP_GTOL = 1
STOP_FTOL = 2
STOP_MAXITER = 3
STOP_LS_FAIL = 4
STOP_NOT_PD = 5
STOP_NONFINITE = 6


def num_params(K: int, p: int, g: int, a: int) -> int:
    """Number of coefficients: K-1 identified beta chunks (beta_0 = 0 after
    normalisation, Sec. 2.2), K gamma chunks and one alpha chunk (Eq. 8)."""
    return (K - 1) * p + K * a + g


def split_theta(theta, K, p, g, a):
    """Chunks of theta in Eq. 8 order: beta [K-1, p] for alternatives
    1..K-1, gamma [K, a] for 0..K-1, alpha [g]."""
    theta = np.asarray(theta, dtype=np.float64)
    nb = (K - 1) * p
    beta = theta[:nb].reshape(K - 1, p)
    gamma = theta[nb:nb + K * a].reshape(K, a)
    alpha = theta[nb + K * a:nb + K * a + g]
    return beta, gamma, alpha


def differenced_generic(Y):
    """Generic-coefficient data relative to the base alternative (Sec. 2.2,
    after Eq. 2): Ytil_k = Y_k - Y_0, so Ytil_0 = 0."""
    return Y - Y[:, :1, :]


def normalized_utility(theta, X, Y, Z):
    """V_ik of Eq. 2 for k = 1..K-1, with V_i0 = 0:
    V_ik = x_i.beta_k + z_ik.gamma_k - z_i0.gamma_0 + ytil_ik.alpha."""
    N, K = Y.shape[0], Y.shape[1]
    p, g, a = X.shape[1], Y.shape[2], Z.shape[2]
    beta, gamma, alpha = split_theta(theta, K, p, g, a)
    Yt = differenced_generic(Y)
    V = np.zeros((N, K))
    for k in range(1, K):
        v = X @ beta[k - 1]
        if a:
            v = v + Z[:, k, :] @ gamma[k] - Z[:, 0, :] @ gamma[0]
        if g:
            v = v + Yt[:, k, :] @ alpha
        V[:, k] = v
    return V


def probabilities(V):
    """P_ik = P_i0 exp(V_ik) with P_i0 = 1 / (1 + sum_{k>=1} exp(V_ik))
    (Eqs. 3-4).  Evaluated with the common factor exp(-m_i),
    m_i = max(0, max_k V_ik), which leaves the ratios unchanged and keeps
    exp() finite."""
    m = np.maximum(V[:, 1:].max(axis=1), 0.0) if V.shape[1] > 1 else \
        np.zeros(V.shape[0])
    e = np.exp(V - m[:, None])          # column 0: exp(0 - m_i)
    denom = e[:, 0] + e[:, 1:].sum(axis=1)
    return e / denom[:, None]


def log_denominator(V):
    """log(1 + sum_{k>=1} exp(V_ik)), evaluated with the same shift."""
    m = np.maximum(V[:, 1:].max(axis=1), 0.0) if V.shape[1] > 1 else \
        np.zeros(V.shape[0])
    return m + np.log(np.exp(-m) + np.exp(V[:, 1:] - m[:, None]).sum(axis=1))


def _weights(w, N):
    return np.ones(N) if w is None else np.asarray(w, dtype=np.float64)


def indicators(choice, K):
    """y_k of Sec. 3.3: y[i, k] = I(choice_i = k)."""
    N = choice.shape[0]
    ind = np.zeros((N, K))
    ind[np.arange(N), choice] = 1.0
    return ind


def loglik_terms(theta, X, Y, Z, choice):
    """Per-individual terms of Eq. 5:
    -log(1 + sum_{k>=1} exp V_ik) + sum_{k>=1} V_ik I(y_i = k)."""
    V = normalized_utility(theta, X, Y, Z)
    K = V.shape[1]
    ind = indicators(choice, K)
    return -log_denominator(V) + (V[:, 1:] * ind[:, 1:]).sum(axis=1)


def loglik(theta, X, Y, Z, choice, w=None):
    """Weighted log-likelihood (Eq. 5)."""
    terms = loglik_terms(theta, X, Y, Z, choice)
    return float(_weights(w, terms.shape[0]) @ terms)


def gradient(theta, X, Y, Z, choice, w=None):
    """Gradient by chunks (Eq. 9):
    beta_m  : X^T D(w) (y_m - P_m)              m = 1..K-1
    gamma_m : Z_m^T D(w) (y_m - P_m)            m = 0..K-1
    alpha   : sum_{k>=1} Ytil_k^T D(w) (y_k - P_k)."""
    N, K = Y.shape[0], Y.shape[1]
    p, g, a = X.shape[1], Y.shape[2], Z.shape[2]
    V = normalized_utility(theta, X, Y, Z)
    P = probabilities(V)
    ww = _weights(w, N)
    R = ww[:, None] * (indicators(choice, K) - P)    # D(w)(y - P)
    Yt = differenced_generic(Y)
    parts = []
    for m in range(1, K):
        parts.append(X.T @ R[:, m])
    for m in range(K):
        parts.append(Z[:, m, :].T @ R[:, m])
    ga = np.zeros(g)
    for k in range(1, K):
        ga = ga + Yt[:, k, :].T @ R[:, k]
    parts.append(ga)
    return np.concatenate(parts) if parts else np.zeros(0)


# ---- Hessian, Eq. 10 -------------------------------------------------------

def chunk_list(K, p, g, a):
    """Chunks theta_m of Eq. 8 as (kind, alternative, offset, size)."""
    out = []
    off = 0
    for k in range(1, K):
        out.append(("beta", k, off, p))
        off += p
    for k in range(K):
        out.append(("gamma", k, off, a))
        off += a
    out.append(("alpha", None, off, g))
    return out


def weight_diag(P, w, n, m):
    """Diagonal of W_nm: w_i P_in (delta_nm - P_im) (Eq. 10 and the
    probability derivative of App. A)."""
    d = 1.0 if n == m else 0.0
    return w * P[:, n] * (d - P[:, m])


def hessian_block(P, X, Y, Z, w, cn, cm, Yt=None):
    """Block H_nm of Eq. 10 for chunks cn, cm (tuples from chunk_list):
      both alternative-specific : -M_n^T W_nm M_m
      one is alpha              : -sum_{k=1}^{K-1} M_n^T W_nk Ytil_k
      both alpha                : -sum_{k,t=1}^{K-1} Ytil_k^T W_kt Ytil_t
    with M = X for beta chunks and M = Z_k for gamma_k.  ``Yt`` is the
    differenced generic data (computed here when not given)."""
    K = P.shape[1]
    if Yt is None:
        Yt = differenced_generic(Y)

    def M(c):
        return X if c[0] == "beta" else Z[:, c[1], :]

    kn, km = cn[0], cm[0]
    if kn != "alpha" and km != "alpha":
        Wd = weight_diag(P, w, cn[1], cm[1])
        return -M(cn).T @ (Wd[:, None] * M(cm))
    if kn != "alpha" and km == "alpha":
        acc = np.zeros((cn[3], cm[3]))
        for k in range(1, K):
            Wd = weight_diag(P, w, cn[1], k)
            acc -= M(cn).T @ (Wd[:, None] * Yt[:, k, :])
        return acc
    if kn == "alpha" and km != "alpha":
        return hessian_block(P, X, Y, Z, w, cm, cn, Yt).T
    acc = np.zeros((cn[3], cm[3]))
    for k in range(1, K):
        for t in range(1, K):
            Wd = weight_diag(P, w, k, t)
            acc -= Yt[:, k, :].T @ (Wd[:, None] * Yt[:, t, :])
    return acc


def hessian_from_P(P, X, Y, Z, w=None):
    """Full Hessian from the probabilities: the upper-triangular blocks of
    Eq. 10, the rest by the block symmetry H_mn = H_nm^T."""
    N, K = P.shape
    p, g, a = X.shape[1], Y.shape[2], Z.shape[2]
    ww = _weights(w, N)
    n_p = num_params(K, p, g, a)
    H = np.zeros((n_p, n_p))
    chunks = [c for c in chunk_list(K, p, g, a) if c[3] > 0]
    Yt = differenced_generic(Y)
    for i, cn in enumerate(chunks):
        for cm in chunks[i:]:
            B = hessian_block(P, X, Y, Z, ww, cn, cm, Yt)
            H[cn[2]:cn[2] + cn[3], cm[2]:cm[2] + cm[3]] = B
            H[cm[2]:cm[2] + cm[3], cn[2]:cn[2] + cn[3]] = B.T
    return H


def hessian(theta, X, Y, Z, choice=None, w=None):
    """Hessian of Eq. 5 at theta (Eq. 10)."""
    P = probabilities(normalized_utility(theta, X, Y, Z))
    return hessian_from_P(P, X, Y, Z, w)


# ---- Newton-Raphson ----------------------------------------------------------

class NotNegativeDefinite(Exception):
    pass


def newton_direction(H, grad):
    """Full Newton step delta = -H^{-1} dl/dtheta (Eq. 6), through the
    Cholesky factor L L^T = -H and two triangular solves."""
    A = -H
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError as exc:
        raise NotNegativeDefinite(str(exc)) from exc
    # a pivot at the round-off level of the largest diagonal entry means -H
    # is numerically singular (e.g. App. B's always-singular models)
    floor = A.shape[0] * np.finfo(np.float64).eps * float(np.max(np.diag(A)))
    if not np.all(np.diag(L) ** 2 > floor):
        raise NotNegativeDefinite("pivot below the round-off floor")
    y = scipy.linalg.solve_triangular(L, grad, lower=True)
    return scipy.linalg.solve_triangular(L.T, y, lower=False)


@dataclass
class FitOptions:
    maxiter: int = 50          # mnlogit() defaults (Sec. 2.4)
    ftol: float = 1e-6
    gtol: float = 1e-6
    ls_max: int = 30
    ls_tol_ulps: float = 64.0
    # "newton": the direction solves the Newton system exactly (Eq. 6);
    # "newton-cg": truncated conjugate gradients on Hessian-vector products
    # (the inexact Newton method of Sec. 5), at most cg_maxiter products
    method: str = "newton"
    cg_maxiter: int = 250


@dataclass
class FitResult:
    theta: np.ndarray
    loglik: float
    grad: np.ndarray
    grad_norm: float
    iters: int
    ls_iters: int
    ls_backtracks: int
    stop_reason: int
    loglik_diff: float
    history: List[dict] = field(default_factory=list)
    cg_iters: int = 0          # Hessian-vector products (newton-cg)


def line_search(theta, delta, l_old, X, Y, Z, choice, w, opts: FitOptions):
    """Step-halving line search (Sec. 3.1): try t = 1, 1/2, 1/4, ... and
    accept the first trial whose log-likelihood is not lower than l_old
    (within tau, see the module notes).  Returns (theta_new, l_new, trials,
    ok)."""
    tau = opts.ls_tol_ulps * np.finfo(np.float64).eps * abs(l_old)
    t = 1.0
    for trial in range(1, opts.ls_max + 2):
        cand = theta + t * delta
        l_new = loglik(cand, X, Y, Z, choice, w)
        if np.isfinite(l_new) and l_new >= l_old - tau:
            return cand, l_new, trial, True
        t *= 0.5
    return theta, l_old, opts.ls_max + 1, False


def fit(X, Y, Z, choice, w=None, theta0=None, opts: Optional[FitOptions] = None,
        record: bool = False) -> FitResult:
    """Newton-Raphson maximisation of Eq. 5 with the halving line search.

    Stopping (mnlogit's maxiter/ftol/gtol, first met): at the top of each
    iteration stop if ||g||_2 <= gtol, or if maxiter iterations were done;
    after a step stop if |l_new - l_old| < ftol."""
    opts = opts or FitOptions()
    N, K = Y.shape[0], Y.shape[1]
    p, g, a = X.shape[1], Y.shape[2], Z.shape[2]
    n_p = num_params(K, p, g, a)
    theta = np.zeros(n_p) if theta0 is None else np.array(theta0, dtype=np.float64)
    l = loglik(theta, X, Y, Z, choice, w)
    gr = gradient(theta, X, Y, Z, choice, w)
    iters = ls_iters = backtracks = cg_iters = 0
    gnorm0 = None
    dl = float("nan")
    hist = []
    reason = None
    while True:
        if not (np.isfinite(l) and np.all(np.isfinite(gr))):
            reason = STOP_NONFINITE
            break
        gnorm = float(np.linalg.norm(gr))
        if gnorm <= opts.gtol:
            reason = STOP_GTOL
            break
        if iters >= opts.maxiter:
            reason = STOP_MAXITER
            break
        H = hessian(theta, X, Y, Z, choice, w)
        if opts.method == "newton-cg":
            if gnorm0 is None:
                gnorm0 = gnorm
            delta, ncg = cg_direction(lambda v: H @ v, gr,
                                      forcing_term(gnorm, gnorm0),
                                      opts.cg_maxiter)
            cg_iters += ncg
        else:
            try:
                delta = newton_direction(H, gr)
            except NotNegativeDefinite:
                reason = STOP_NOT_PD
                break
        th_new, l_new, trials, ok = line_search(theta, delta, l, X, Y, Z,
                                                choice, w, opts)
        ls_iters += trials
        backtracks += trials - 1
        if record:
            hist.append(dict(theta=theta.copy(), loglik=l, grad=gr.copy(),
                             grad_norm=gnorm, delta=delta, trials=trials,
                             accepted=ok))
        if not ok:
            reason = STOP_LS_FAIL
            break
        iters += 1
        dl = l_new - l
        theta, l = th_new, l_new
        gr = gradient(theta, X, Y, Z, choice, w)
        if abs(dl) < opts.ftol:
            reason = STOP_FTOL
            break
    return FitResult(theta=theta, loglik=l, grad=gr,
                     grad_norm=float(np.linalg.norm(gr)), iters=iters,
                     ls_iters=ls_iters, ls_backtracks=backtracks,
                     stop_reason=reason, loglik_diff=dl, history=hist,
                     cg_iters=cg_iters)


def fit_problem(prob, theta0=None, opts=None, record=False) -> FitResult:
    return fit(prob.X, prob.Y, prob.Z, prob.choice, prob.w, theta0, opts,
               record)


# ---- inexact (truncated) Newton (Sec. 5) -------------------------------------

def hessian_vector(theta, X, Y, Z, v, w=None):
    """H(theta) v with H of Eq. 10: the product an inexact Newton method
    takes instead of forming and factoring H."""
    return hessian(theta, X, Y, Z, None, w) @ np.asarray(v, dtype=np.float64)


def forcing_term(gnorm, gnorm0):
    """Relative residual at which the inner solve stops:
    eta = min(1/2, sqrt(||g|| / ||g_0||)), g_0 the gradient where the fit
    started: the choice min(1/2, sqrt(||g||)) that keeps truncated Newton
    superlinearly convergent near the optimum, made independent of the
    scale of the summed log-likelihood."""
    return min(0.5, math.sqrt(gnorm / gnorm0))


def cg_direction(hv, grad, eta, maxcg):
    """Truncated conjugate gradients for (-H) d = g from d = 0, where hv(v)
    returns H v.  Stops when ||r|| <= eta ||g||, after maxcg products, or
    when a search direction p has p^T (-H) p <= 0 (then d = g if no step
    was taken yet).  Returns (d, number of Hessian-vector products)."""
    grad = np.asarray(grad, dtype=np.float64)
    d = np.zeros_like(grad)
    r = grad.copy()
    p = r.copy()
    rr = float(r @ r)
    gn = math.sqrt(rr)
    for j in range(maxcg):
        if math.sqrt(rr) <= eta * gn:
            return d, j
        Ap = -hv(p)
        pAp = float(p @ Ap)
        if not pAp > 0.0:
            return (grad.copy() if j == 0 else d), j + 1
        alpha = rr / pAp
        d = d + alpha * p
        r = r - alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return d, maxcg


# ---- fitted-model methods: predict and summary (Sec. 2.4) --------------------

def predict(theta, X, Y, Z):
    """Choice probabilities of the fitted model on (new) data: Eqs. 3-4 at
    the utilities of Eq. 2.  No choices are needed."""
    return probabilities(normalized_utility(theta, X, Y, Z))


def covariance(theta, X, Y, Z, w=None, H=None):
    """Asymptotic covariance of the maximum-likelihood estimate: the inverse
    of the observed information -H, with H of Eq. 10 at theta (computed
    unless given).  Raises NotNegativeDefinite when -H has no Cholesky
    factor."""
    A = -(hessian(theta, X, Y, Z, None, w) if H is None else H)
    try:
        np.linalg.cholesky(A)
    except np.linalg.LinAlgError as exc:
        raise NotNegativeDefinite(str(exc)) from exc
    return np.linalg.inv(A)


def summary(theta, X, Y, Z, w=None, H=None):
    """Coefficient table of the summary method (Sec. 2.4): standard errors
    sqrt(diag((-H)^{-1})), Wald statistics z = theta / se and two-sided
    normal p-values erfc(|z| / sqrt 2)."""
    import math
    theta = np.asarray(theta, dtype=np.float64)
    se = np.sqrt(np.diag(covariance(theta, X, Y, Z, w, H)))
    z = theta / se
    pval = np.array([math.erfc(abs(v) / math.sqrt(2.0)) for v in z])
    return se, z, pval


# ---- collinearity check (Sec. 2.4 linDepTol, App. B) -------------------------

def independent_columns(M, tol=1e-6):
    """Columns of M [rows, n] kept by a column-order QR with tolerance tol
    (R's qr as mnlogit calls it with linDepTol): column j is dropped when
    the norm of its part orthogonal to the kept columns before it is below
    tol times its own norm (a zero column is always dropped).  Gram-Schmidt
    with a second orthogonalisation pass.  Returns a boolean mask [n]."""
    M = np.asarray(M, dtype=np.float64)
    keep = np.zeros(M.shape[1], dtype=bool)
    Q = []
    for j in range(M.shape[1]):
        col = M[:, j]
        nrm = float(np.linalg.norm(col))
        r = col.copy()
        for _ in range(2):
            for q in Q:
                r = r - (q @ r) * q
        res = float(np.linalg.norm(r))
        if nrm > 0.0 and res >= tol * nrm:
            keep[j] = True
            Q.append(r / res)
    return keep


def collinearity_mask(X, Y, Z, tol=1e-6):
    """Variables kept so that App. B's necessary conditions for a
    non-singular Hessian hold: X and every Z_k of full column rank, and the
    differenced generic data Ytil_k (k >= 1) stacked over alternatives of
    full column rank.  A Z variable is dropped if it is dependent in any
    alternative (its coefficients gamma_kc go for every k).  Returns boolean
    masks (keep_x [p], keep_y [g], keep_z [a])."""
    N, K = Y.shape[0], Y.shape[1]
    g, a = Y.shape[2], Z.shape[2]
    keep_x = independent_columns(X, tol)
    keep_z = np.ones(a, dtype=bool)
    for k in range(K):
        keep_z &= independent_columns(Z[:, k, :], tol)
    Yt = differenced_generic(Y)[:, 1:, :].reshape(N * (K - 1), g)
    keep_y = independent_columns(Yt, tol)
    return keep_x, keep_y, keep_z


# ---- hypothesis tests (Sec. 2.4: lrtest, waldtest, scoretest, hmftest) -------

def chi2_sf(x, df):
    """Upper tail of the chi-square distribution with df degrees of
    freedom (scipy)."""
    import scipy.stats
    return float(scipy.stats.chi2.sf(x, df))


def lr_test(l_full, l_restricted, df):
    """Likelihood-ratio statistic 2 (l_full - l_restricted), df and its
    chi-square p-value."""
    stat = 2.0 * (l_full - l_restricted)
    return stat, df, chi2_sf(stat, df)


def wald_test(theta, V, idx):
    """Wald statistic of theta_S = 0 for the coefficients idx:
    theta_S^T (V_SS)^{-1} theta_S with V the estimate's covariance."""
    idx = np.asarray(idx)
    t = np.asarray(theta, dtype=np.float64)[idx]
    stat = float(t @ np.linalg.solve(V[np.ix_(idx, idx)], t))
    return stat, idx.size, chi2_sf(stat, idx.size)


def score_test(grad, H, df):
    """Rao score statistic g^T (-H)^{-1} g of the full model at the
    restricted estimate (restricted coefficients at zero)."""
    stat = float(grad @ np.linalg.solve(-H, grad))
    return stat, df, chi2_sf(stat, df)


def hm_test(theta_sub, V_sub, theta_full, V_full):
    """Hausman-McFadden statistic for IIA on the coefficients common to a
    fit on a subset of alternatives and the full fit:
    d^T (V_sub - V_full)^{-1} d, d = theta_sub - theta_full."""
    d = np.asarray(theta_sub) - np.asarray(theta_full)
    stat = float(d @ np.linalg.solve(V_sub - V_full, d))
    return stat, d.size, chi2_sf(stat, d.size)
