"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Every check here uses something other than the oracle's own formulas:
values the paper prints, closed forms, brute force in high precision,
independently written textbook algorithms (binary IRLS), finite differences,
two independent Hessian constructions (per-observation Jacobian form and the
dense design/weight form of App. B), and invariants of the model.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.special

import synth
from oracle import mnl_ref as R
from tests.conftest import read_golden


# ---------------------------------------------------------------------------
# independent helpers (NOT the oracle's code paths)

def unnormalized_jacobians(X, Y, Z):
    """J_i[k, :] = dU_ik/dtheta for the un-normalised utility of Eq. 1 with
    beta_0 = 0, in theta's Eq. 8 layout.  Returns J [N, K, n_p]."""
    N, K = Y.shape[:2]
    p, g, a = X.shape[1], Y.shape[2], Z.shape[2]
    n_p = (K - 1) * p + K * a + g
    J = np.zeros((N, K, n_p))
    for k in range(K):
        if k >= 1:
            J[:, k, (k - 1) * p:k * p] = X
        off = (K - 1) * p + k * a
        J[:, k, off:off + a] = Z[:, k, :]
        J[:, k, (K - 1) * p + K * a:] = Y[:, k, :]
    return J


def jform(theta, X, Y, Z, choice, w):
    """l, g, H from the per-observation Jacobian form with a library
    log-sum-exp: l = sum w (U_ic - lse U_i), g = sum w J^T (e - P),
    H = -sum w J^T (diag P - P P^T) J."""
    J = unnormalized_jacobians(X, Y, Z)
    U = J @ theta
    lse = scipy.special.logsumexp(U, axis=1)
    P = np.exp(U - lse[:, None])
    N, K = U.shape
    ww = np.ones(N) if w is None else w
    E = np.zeros((N, K))
    E[np.arange(N), choice] = 1.0
    l = float(ww @ (U[np.arange(N), choice] - lse))
    g = np.einsum("i,ikq,ik->q", ww, J, E - P)
    H = np.zeros((J.shape[2],) * 2)
    for i in range(N):
        S = np.diag(P[i]) - np.outer(P[i], P[i])
        H -= ww[i] * J[i].T @ S @ J[i]
    return l, g, H


def appendix_b_hessian(theta, X, Y, Z, w):
    """-Xtil^T Wtil Xtil with the design matrix of Eq. 14 and the weight
    matrix of Eq. 15 (sign as in Eq. 7), built densely."""
    N, K = Y.shape[:2]
    p, g, a = X.shape[1], Y.shape[2], Z.shape[2]
    ww = np.ones(N) if w is None else w
    J = unnormalized_jacobians(X, Y, Z)
    U = J @ theta
    P = np.exp(U - scipy.special.logsumexp(U, axis=1)[:, None])
    Ytil = Y - Y[:, :1, :]
    # row blocks: beta rows for alternatives 1..K-1, then gamma rows 0..K-1
    slots = list(range(1, K)) + list(range(K))
    nb, ng = (K - 1) * p, K * a
    n_p = nb + ng + g
    Xt = np.zeros((len(slots) * N, n_p))
    for s, k in enumerate(slots):
        rows = slice(s * N, (s + 1) * N)
        if s < K - 1:
            Xt[rows, (k - 1) * p:k * p] = X
            Xt[rows, nb + ng:] = Ytil[:, k, :] / 2
        else:
            Xt[rows, nb + k * a:nb + (k + 1) * a] = Z[:, k, :]
            if k >= 1:
                Xt[rows, nb + ng:] = Ytil[:, k, :] / 2

    def Wblk(k, t):
        return np.diag(ww * P[:, k] * ((1.0 if k == t else 0.0) - P[:, t]))

    Q = np.block([[Wblk(k, t) for t in range(1, K)] for k in range(1, K)])
    Q0 = np.vstack([Wblk(k, 0) for k in range(1, K)])
    W00 = Wblk(0, 0)
    Wt = np.block([[Q, Q0, Q], [Q0.T, W00, Q0.T], [Q, Q0, Q]])
    return -Xt.T @ Wt @ Xt


def irls_binary(X, y, w, iters=100):
    """Textbook IRLS for binary logistic regression."""
    b = np.zeros(X.shape[1])
    for _ in range(iters):
        eta = X @ b
        s = 1.0 / (1.0 + np.exp(-eta))
        Wd = w * s * (1 - s)
        step = np.linalg.solve(X.T @ (Wd[:, None] * X), X.T @ (w * (y - s)))
        b = b + step
        if np.max(np.abs(step)) < 1e-15:
            break
    return b


def tiny(seed, N=30, K=4, p=3, g=2, a=2, weights="uniform", sd=0.5):
    return synth.make_problem(N, K, p, g, a, seed=seed, weights=weights,
                              coef_sd=sd)


SHAPES = [  # (N, K, p, g, a)
    (30, 4, 3, 2, 2), (25, 2, 2, 1, 1), (40, 5, 1, 0, 2), (20, 3, 3, 2, 0),
    (35, 3, 0, 2, 1), (18, 6, 2, 1, 0),
]


# ---------------------------------------------------------------------------
# values printed in the paper

def test_num_params_matches_paper():
    for K, p, g, a, n_p, *src in read_golden("num_params.txt"):
        assert R.num_params(int(K), int(p), int(g), int(a)) == int(n_p), src


def test_initial_loglik_matches_printed_nnet_value():
    (N, K, val), = read_golden("nnet_initial_value.txt")
    N, K = int(N), int(K)
    pr = synth.make_problem(N, K, 50, 0, 0, seed=11, intercept=False)
    l0 = R.loglik(np.zeros(R.num_params(K, 50, 0, 0)), pr.X, pr.Y, pr.Z,
                  pr.choice)
    # printed with 6 decimals
    assert abs(-l0 - float(val)) < 5e-7


# ---------------------------------------------------------------------------
# closed forms

def test_loglik_at_zero_weighted():
    pr = tiny(3, N=50, K=7)
    th = np.zeros(pr.n_params)
    l0 = R.loglik(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    assert l0 == pytest.approx(-pr.w.sum() * math.log(7), rel=1e-14)


def test_hessian_at_zero_kronecker_closed_form():
    # X-only model at theta = 0: P = 1/K, so the beta-beta part is
    # -[(1/K)(I - 11^T/K)] (x) X^T D(w) X over alternatives 1..K-1
    K, p = 5, 3
    pr = synth.make_problem(40, K, p, 0, 0, seed=4, weights="uniform")
    H = R.hessian(np.zeros(pr.n_params), pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    S = (np.eye(K - 1) - np.ones((K - 1, K - 1)) / K) / K
    XtX = pr.X.T @ (pr.w[:, None] * pr.X)
    np.testing.assert_allclose(H, -np.kron(S, XtX), rtol=1e-13, atol=1e-12)


def test_intercept_only_closed_form():
    # X = column of ones: xi_k = log(n_k / n_0), l = sum n_k log(n_k / n)
    K = 5
    pr = synth.make_problem(600, K, 1, 0, 0, seed=8, weights="uniform",
                            coef_sd=0.7)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-10, ftol=0.0))
    assert res.stop_reason == R.STOP_GTOL
    n = np.array([pr.w[pr.choice == k].sum() for k in range(K)])
    np.testing.assert_allclose(res.theta, np.log(n[1:] / n[0]), rtol=0,
                               atol=1e-10)
    assert res.loglik == pytest.approx(float(n @ np.log(n / n.sum())),
                                       rel=1e-13)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_binary_logit_equals_irls(seed):
    # K = 2 is binary logistic regression (Sec. 2.2)
    pr = synth.make_problem(300, 2, 4, 0, 0, seed=seed, weights="uniform")
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-11, ftol=0.0))
    b = irls_binary(pr.X, (pr.choice == 1).astype(float), pr.w)
    np.testing.assert_allclose(res.theta, b, rtol=0, atol=1e-9)


def test_binary_logit_saturated_group_log_odds():
    # one-hot groups, K = 2: each coefficient is its group's log-odds
    rng = np.random.default_rng(5)
    G, N = 4, 800
    grp = rng.integers(0, G, N)
    X = np.zeros((N, G))
    X[np.arange(N), grp] = 1.0
    choice = (rng.random(N) < 0.3 + 0.1 * grp).astype(np.int32)
    Y = np.zeros((N, 2, 0))
    res = R.fit(X, Y, Y, choice, None, opts=R.FitOptions(gtol=1e-11, ftol=0))
    for j in range(G):
        c1 = np.sum((grp == j) & (choice == 1))
        c0 = np.sum((grp == j) & (choice == 0))
        assert res.theta[j] == pytest.approx(math.log(c1 / c0), abs=1e-10)


# ---------------------------------------------------------------------------
# brute force and independent forms on tiny inputs

@pytest.mark.parametrize("shape", SHAPES[:3])
def test_loglik_brute_force_high_precision(shape):
    N, K, p, g, a = shape
    pr = synth.make_problem(N, K, p, g, a, seed=21, weights="uniform")
    th = np.random.default_rng(1).normal(0, 0.7, pr.n_params)
    beta, gamma, alpha = R.split_theta(th, K, p, g, a)
    mpmath.mp.dps = 40
    total = mpmath.mpf(0)
    for i in range(N):
        U = []
        for k in range(K):
            u = mpmath.mpf(0)
            if k >= 1:
                u += mpmath.fsum(mpmath.mpf(pr.X[i, j]) * mpmath.mpf(beta[k - 1, j])
                                 for j in range(p))
            u += mpmath.fsum(mpmath.mpf(pr.Z[i, k, j]) * mpmath.mpf(gamma[k, j])
                             for j in range(a))
            u += mpmath.fsum(mpmath.mpf(pr.Y[i, k, j]) * mpmath.mpf(alpha[j])
                             for j in range(g))
            U.append(u)
        total += mpmath.mpf(pr.w[i]) * (U[pr.choice[i]] -
                                        mpmath.log(mpmath.fsum(mpmath.exp(u) for u in U)))
    l = R.loglik(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    assert l == pytest.approx(float(total), rel=1e-13)


@pytest.mark.parametrize("shape", SHAPES)
def test_gradient_central_differences(shape):
    N, K, p, g, a = shape
    pr = synth.make_problem(N, K, p, g, a, seed=31, weights="uniform")
    th = np.random.default_rng(2).normal(0, 0.5, pr.n_params)
    gr = R.gradient(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    h = 1e-5
    fd = np.empty_like(gr)
    for j in range(th.size):
        e = np.zeros_like(th)
        e[j] = h
        fd[j] = (R.loglik(th + e, pr.X, pr.Y, pr.Z, pr.choice, pr.w) -
                 R.loglik(th - e, pr.X, pr.Y, pr.Z, pr.choice, pr.w)) / (2 * h)
    np.testing.assert_allclose(gr, fd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("shape", SHAPES)
def test_hessian_central_differences_of_gradient(shape):
    N, K, p, g, a = shape
    pr = synth.make_problem(N, K, p, g, a, seed=41, weights="uniform")
    th = np.random.default_rng(3).normal(0, 0.5, pr.n_params)
    H = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    h = 1e-5
    fd = np.empty_like(H)
    for j in range(th.size):
        e = np.zeros_like(th)
        e[j] = h
        fd[:, j] = (R.gradient(th + e, pr.X, pr.Y, pr.Z, pr.choice, pr.w) -
                    R.gradient(th - e, pr.X, pr.Y, pr.Z, pr.choice, pr.w)) / (2 * h)
    np.testing.assert_allclose(H, fd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("shape", SHAPES)
def test_three_hessian_forms_agree(shape):
    N, K, p, g, a = shape
    pr = synth.make_problem(N, K, p, g, a, seed=51, weights="uniform")
    th = np.random.default_rng(4).normal(0, 0.6, pr.n_params)
    H = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    l_j, g_j, H_j = jform(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    H_b = appendix_b_hessian(th, pr.X, pr.Y, pr.Z, pr.w)
    scale = np.abs(H).max()
    np.testing.assert_allclose(H, H_j, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(H, H_b, rtol=0, atol=1e-13 * scale)
    assert R.loglik(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w) == \
        pytest.approx(l_j, rel=1e-13)
    np.testing.assert_allclose(R.gradient(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w),
                               g_j, rtol=0, atol=1e-13 * np.abs(g_j).max())


# ---------------------------------------------------------------------------
# invariants

def test_probabilities_rows_sum_to_one_and_in_open_interval():
    pr = tiny(61, N=200, K=9)
    th = np.random.default_rng(5).normal(0, 2.0, pr.n_params)
    P = R.probabilities(R.normalized_utility(th, pr.X, pr.Y, pr.Z))
    np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.all(P > 0) and np.all(P < 1)


def test_probabilities_no_overflow_at_large_utilities():
    V = np.array([[0.0, 800.0, 799.0], [0.0, -800.0, -801.0]])
    P = R.probabilities(V)
    assert np.all(np.isfinite(P))
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-15)
    assert P[0, 1] == pytest.approx(1 / (1 + math.exp(-1)), rel=1e-14)


@pytest.mark.parametrize("shape", SHAPES)
def test_hessian_symmetric_negative_semidefinite(shape):
    N, K, p, g, a = shape
    pr = synth.make_problem(N, K, p, g, a, seed=71, weights="uniform")
    th = np.random.default_rng(6).normal(0, 0.8, pr.n_params)
    H = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-14 * np.abs(H).max())
    ev = np.linalg.eigvalsh(H)
    assert ev.max() <= 1e-12 * np.abs(ev).max()


def test_generic_data_shift_invariance():
    pr = tiny(81, N=60, K=5)
    th = np.random.default_rng(7).normal(0, 0.5, pr.n_params)
    c = np.random.default_rng(8).normal(0, 3, (pr.N, 1, pr.g))
    Y2 = pr.Y + c
    args = (pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    args2 = (pr.X, Y2, pr.Z, pr.choice, pr.w)
    assert R.loglik(th, *args) == pytest.approx(R.loglik(th, *args2), rel=1e-13)
    np.testing.assert_allclose(R.gradient(th, *args), R.gradient(th, *args2),
                               rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(R.hessian(th, *args), R.hessian(th, *args2),
                               rtol=1e-11, atol=1e-11)


def test_observation_permutation_invariance():
    pr = tiny(91, N=60, K=4)
    th = np.random.default_rng(9).normal(0, 0.5, pr.n_params)
    perm = np.random.default_rng(10).permutation(pr.N)
    a1 = (pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    a2 = (pr.X[perm], pr.Y[perm], pr.Z[perm], pr.choice[perm], pr.w[perm])
    assert R.loglik(th, *a1) == pytest.approx(R.loglik(th, *a2), rel=1e-13)
    np.testing.assert_allclose(R.hessian(th, *a1), R.hessian(th, *a2),
                               rtol=1e-12, atol=1e-12)


def test_base_change_reparametrises_beta():
    K, p, g, a = 4, 3, 1, 1
    pr = synth.make_problem(400, K, p, g, a, seed=12, weights="uniform")
    opts = R.FitOptions(gtol=1e-10, ftol=0.0)
    r1 = R.fit_problem(pr, opts=opts)
    b = 2                                     # new base alternative
    order = [b] + [k for k in range(K) if k != b]
    inv = np.empty(K, dtype=np.int32)
    inv[order] = np.arange(K)
    r2 = R.fit(pr.X, pr.Y[:, order], pr.Z[:, order], inv[pr.choice], pr.w,
               opts=opts)
    assert r2.loglik == pytest.approx(r1.loglik, rel=1e-12)
    beta1, gam1, al1 = R.split_theta(r1.theta, K, p, g, a)
    beta1 = np.vstack([np.zeros(p), beta1])           # beta_0 = 0
    beta2, gam2, al2 = R.split_theta(r2.theta, K, p, g, a)
    for j in range(1, K):
        np.testing.assert_allclose(beta2[j - 1], beta1[order[j]] - beta1[b],
                                   atol=1e-8)
        np.testing.assert_allclose(gam2[j], gam1[order[j]], atol=1e-8)
    np.testing.assert_allclose(gam2[0], gam1[b], atol=1e-8)
    np.testing.assert_allclose(al2, al1, atol=1e-8)


def test_moment_matching_and_vanishing_gradient_at_optimum():
    pr = synth.make_problem(500, 5, 3, 2, 1, seed=13, weights="uniform")
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-9, ftol=0.0))
    assert res.stop_reason == R.STOP_GTOL and res.grad_norm <= 1e-9
    P = R.probabilities(R.normalized_utility(res.theta, pr.X, pr.Y, pr.Z))
    obs = np.array([pr.w[pr.choice == k].sum() for k in range(5)])
    np.testing.assert_allclose(pr.w @ P, obs, rtol=0, atol=1e-8)
    H = R.hessian(res.theta, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    assert np.linalg.eigvalsh(H).max() < 0


# ---------------------------------------------------------------------------
# weights

def test_integer_weights_equal_row_replication():
    pr = synth.make_problem(40, 4, 2, 1, 1, seed=14, weights="int")
    rep = np.repeat(np.arange(pr.N), pr.w.astype(int))
    th = np.random.default_rng(11).normal(0, 0.5, pr.n_params)
    a1 = (pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    a2 = (pr.X[rep], pr.Y[rep], pr.Z[rep], pr.choice[rep], None)
    assert R.loglik(th, *a1) == pytest.approx(R.loglik(th, *a2), rel=1e-13)
    np.testing.assert_allclose(R.gradient(th, *a1), R.gradient(th, *a2),
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(R.hessian(th, *a1), R.hessian(th, *a2),
                               rtol=1e-12, atol=1e-12)
    f1 = R.fit(*a1, opts=R.FitOptions(gtol=1e-10, ftol=0))
    f2 = R.fit(*a2, opts=R.FitOptions(gtol=1e-10, ftol=0))
    np.testing.assert_allclose(f1.theta, f2.theta, atol=1e-9)


def test_weight_scaling():
    pr = tiny(15)
    th = np.random.default_rng(12).normal(0, 0.5, pr.n_params)
    c = 3.5
    a1 = (pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    a2 = (pr.X, pr.Y, pr.Z, pr.choice, c * pr.w)
    assert R.loglik(th, *a2) == pytest.approx(c * R.loglik(th, *a1), rel=1e-13)
    np.testing.assert_allclose(R.hessian(th, *a2), c * R.hessian(th, *a1),
                               rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Newton-Raphson behaviour

def test_newton_direction_solves_system():
    pr = tiny(16, N=80)
    th = np.random.default_rng(13).normal(0, 0.3, pr.n_params)
    H = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    gr = R.gradient(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    d = R.newton_direction(H, gr)
    np.testing.assert_allclose(H @ d, -gr, rtol=0, atol=1e-10 * np.abs(gr).max())


def test_quadratic_convergence_and_monotone_loglik():
    pr = synth.make_problem(3000, 6, 4, 2, 1, seed=17)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-10, ftol=0.0),
                        record=True)
    assert res.stop_reason == R.STOP_GTOL
    ls = [h["loglik"] for h in res.history] + [res.loglik]
    assert all(b >= a - 1e-9 for a, b in zip(ls, ls[1:]))
    gn = [h["grad_norm"] for h in res.history] + [res.grad_norm]
    # near the optimum the gradient norm roughly squares per step
    pairs = [(a, b) for a, b in zip(gn, gn[1:]) if a < 1e-1 and b > 1e-13]
    assert pairs, gn
    for a, b in pairs:
        assert b <= 50 * a * a, gn


def test_singular_model_reports_not_pd():
    # App. B: generic data that do not vary over alternatives give an
    # identically zero alpha block
    pr = synth.make_problem(200, 4, 2, 1, 0, seed=18)
    Y = np.repeat(pr.Y[:, :1, :], 4, axis=1)
    res = R.fit(pr.X, Y, pr.Z, pr.choice, None,
                opts=R.FitOptions(gtol=1e-8, ftol=0))
    assert res.stop_reason == R.STOP_NOT_PD


def test_maxiter_and_ftol_stops():
    pr = tiny(19, N=300)
    r = R.fit_problem(pr, opts=R.FitOptions(maxiter=1, gtol=1e-12, ftol=0))
    assert r.stop_reason == R.STOP_MAXITER and r.iters == 1
    r = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-14, ftol=1e-3))
    assert r.stop_reason == R.STOP_FTOL and abs(r.loglik_diff) < 1e-3


def test_line_search_backtracks_from_far_start():
    # a far starting point makes the full Newton step overshoot
    pr = synth.make_problem(400, 3, 3, 0, 0, seed=20, coef_sd=2.0)
    th0 = np.full(pr.n_params, 6.0)
    res = R.fit_problem(pr, theta0=th0, opts=R.FitOptions(gtol=1e-8, ftol=0),
                        record=True)
    assert res.stop_reason == R.STOP_GTOL
    assert res.ls_backtracks > 0 and res.ls_iters == res.iters + res.ls_backtracks
    # the paper's rule: a step is taken only if the log-likelihood does not
    # drop; a halving happens only when the longer step did drop it
    # (checked with the independent Jacobian-form log-likelihood)
    eps = np.finfo(float).eps
    seq = [h["loglik"] for h in res.history] + [res.loglik]
    for h, l_next in zip(res.history, seq[1:]):
        tau = 64 * eps * abs(h["loglik"])
        assert l_next >= h["loglik"] - tau
        t = 1.0
        for _ in range(h["trials"] - 1):
            l_try = jform(h["theta"] + t * h["delta"], pr.X, pr.Y, pr.Z,
                          pr.choice, None)[0]
            assert l_try < h["loglik"] - tau
            t *= 0.5
        l_acc = jform(h["theta"] + t * h["delta"], pr.X, pr.Y, pr.Z,
                      pr.choice, None)[0]
        assert l_acc == pytest.approx(l_next, rel=1e-12)


def test_line_search_rule_at_optimum():
    # At the maximiser every direction lowers l, by about t^2/2 d^T(-H)d for
    # step t (strict concavity, Sec. 3.1); the halving search must keep
    # halving until that drop falls below the tolerance tau.
    pr = synth.make_problem(400, 4, 3, 1, 1, seed=22)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-10, ftol=0))
    th = res.theta
    d = np.random.default_rng(14).normal(0, 1.0, th.size)
    l_hat, _, H_j = jform(th, pr.X, pr.Y, pr.Z, pr.choice, None)
    q = float(d @ (-H_j) @ d)
    tau = 64 * np.finfo(float).eps * abs(l_hat)
    # smallest halving count with t^2 q / 2 <= tau (cubic terms negligible)
    want = next(j for j in range(80) if 0.5 * (0.5 ** j) ** 2 * q <= tau)
    opts = R.FitOptions(ls_max=60)
    _, l_new, trials, ok = R.line_search(th, d, l_hat, pr.X, pr.Y, pr.Z,
                                         pr.choice, None, opts)
    assert ok and l_new >= l_hat - tau
    assert abs(trials - (want + 1)) <= 1
    # a cap below that count is a line-search failure
    _, _, trials, ok = R.line_search(th, d, l_hat, pr.X, pr.Y, pr.Z,
                                     pr.choice, None, R.FitOptions(ls_max=3))
    assert not ok and trials == 4


# ---------------------------------------------------------------------------
# fitted-model methods (Sec. 2.4): predict and the summary's standard errors

def test_intercept_only_standard_errors_closed_form():
    # inverse information of the log-odds xi_k = log(n_k / n_0):
    # var = 1/n_k + 1/n_0 on the diagonal, cov = 1/n_0 off it
    K = 5
    pr = synth.make_problem(600, K, 1, 0, 0, seed=8, weights="uniform",
                            coef_sd=0.7)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-10, ftol=0.0))
    n = np.array([pr.w[pr.choice == k].sum() for k in range(K)])
    C = R.covariance(res.theta, pr.X, pr.Y, pr.Z, pr.w)
    ref = np.full((K - 1, K - 1), 1.0 / n[0]) + np.diag(1.0 / n[1:])
    np.testing.assert_allclose(C, ref, rtol=1e-9, atol=0)
    se, z, pval = R.summary(res.theta, pr.X, pr.Y, pr.Z, pr.w)
    np.testing.assert_allclose(se, np.sqrt(1.0 / n[1:] + 1.0 / n[0]),
                               rtol=1e-9)
    np.testing.assert_allclose(z, res.theta / se, rtol=1e-15)


def test_binary_logit_standard_errors_equal_irls():
    # K = 2: the textbook logistic-regression covariance (X^T W X)^{-1}
    pr = synth.make_problem(400, 2, 4, 0, 0, seed=6, weights="uniform")
    b = irls_binary(pr.X, (pr.choice == 1).astype(float), pr.w)
    s = 1.0 / (1.0 + np.exp(-(pr.X @ b)))
    info = pr.X.T @ ((pr.w * s * (1 - s))[:, None] * pr.X)
    se_ref = np.sqrt(np.diag(np.linalg.inv(info)))
    se, _, _ = R.summary(b, pr.X, pr.Y, pr.Z, pr.w)
    np.testing.assert_allclose(se, se_ref, rtol=1e-12)


def test_saturated_groups_standard_errors():
    # one-hot groups, K = 2: se of a group's log-odds is sqrt(1/c1 + 1/c0)
    rng = np.random.default_rng(9)
    G, N = 3, 900
    grp = rng.integers(0, G, N)
    X = np.zeros((N, G))
    X[np.arange(N), grp] = 1.0
    choice = (rng.random(N) < 0.25 + 0.15 * grp).astype(np.int32)
    Y = np.zeros((N, 2, 0))
    res = R.fit(X, Y, Y, choice, None, opts=R.FitOptions(gtol=1e-11, ftol=0))
    se, _, _ = R.summary(res.theta, X, Y, Y)
    for j in range(G):
        c1 = np.sum((grp == j) & (choice == 1))
        c0 = np.sum((grp == j) & (choice == 0))
        assert se[j] == pytest.approx(math.sqrt(1 / c1 + 1 / c0), rel=1e-9)


def test_standard_errors_weight_scaling_and_replication():
    pr = tiny(12, N=40, K=4, p=2, g=1, a=1, weights="int")
    th = pr.theta_true
    se, _, _ = R.summary(th, pr.X, pr.Y, pr.Z, pr.w)
    se3, _, _ = R.summary(th, pr.X, pr.Y, pr.Z, 3.0 * pr.w)
    np.testing.assert_allclose(se3, se / math.sqrt(3.0), rtol=1e-12)
    idx = np.repeat(np.arange(pr.N), pr.w.astype(int))
    se_rep, _, _ = R.summary(th, pr.X[idx], pr.Y[idx], pr.Z[idx])
    np.testing.assert_allclose(se_rep, se, rtol=1e-12)


def test_p_values_normal_tail():
    pr = tiny(13, N=200, K=3, p=2, g=1, a=1)
    se, z, pval = R.summary(pr.theta_true, pr.X, pr.Y, pr.Z, pr.w)
    import scipy.stats
    np.testing.assert_allclose(pval, 2.0 * scipy.stats.norm.sf(np.abs(z)),
                               rtol=1e-12)


def test_covariance_rejects_singular_model():
    # a duplicated column: -H is singular
    pr = tiny(14, N=60, K=3, p=2, g=0, a=0)
    X = np.concatenate([pr.X, pr.X[:, 1:2]], axis=1)
    th = np.zeros(R.num_params(3, 3, 0, 0))
    with pytest.raises(R.NotNegativeDefinite):
        R.covariance(th, X, pr.Y, pr.Z, pr.w)


def test_predict_binary_is_sigmoid():
    pr = synth.make_problem(50, 2, 3, 0, 0, seed=15)
    P = R.predict(pr.theta_true, pr.X, pr.Y, pr.Z)
    s = 1.0 / (1.0 + np.exp(-(pr.X @ pr.theta_true)))
    np.testing.assert_allclose(P[:, 1], s, rtol=1e-14)
    np.testing.assert_allclose(P[:, 0], 1.0 - s, rtol=1e-13, atol=1e-16)


def test_predict_at_zero_and_at_intercept_only_optimum():
    pr = tiny(16, N=30, K=6)
    P = R.predict(np.zeros(pr.n_params), pr.X, pr.Y, pr.Z)
    np.testing.assert_allclose(P, 1.0 / 6.0, rtol=1e-15)
    K = 4
    pr = synth.make_problem(500, K, 1, 0, 0, seed=17, coef_sd=0.6)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-10, ftol=0.0))
    n = np.bincount(pr.choice, minlength=K).astype(float)
    P = R.predict(res.theta, pr.X, pr.Y, pr.Z)
    np.testing.assert_allclose(P, np.tile(n / n.sum(), (pr.N, 1)), rtol=1e-10)


def test_predict_utility_by_hand():
    # Eq. 2 written out for one observation of a model with every chunk
    pr = tiny(18, N=5, K=3, p=2, g=2, a=1)
    beta, gamma, alpha = R.split_theta(pr.theta_true, 3, 2, 2, 1)
    i = 3
    u = np.array([(pr.X[i] @ beta[k - 1] if k else 0.0)
                  + pr.Z[i, k] @ gamma[k] + pr.Y[i, k] @ alpha
                  for k in range(3)])
    e = np.exp(u - u.max())
    np.testing.assert_allclose(R.predict(pr.theta_true, pr.X, pr.Y, pr.Z)[i],
                               e / e.sum(), rtol=1e-14)


# ---------------------------------------------------------------------------
# inexact Newton (Sec. 5): Hessian-vector products and truncated CG

@pytest.mark.parametrize("shape", SHAPES[:4])
def test_hessian_vector_central_differences(shape):
    N, K, p, g, a = shape
    pr = tiny(50 + K, N=N, K=K, p=p, g=g, a=a)
    th = pr.theta_true
    v = np.random.default_rng(3).normal(size=pr.n_params)
    hv = R.hessian_vector(th, pr.X, pr.Y, pr.Z, v, pr.w)
    h = 1e-5
    gp = R.gradient(th + h * v, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    gm = R.gradient(th - h * v, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    fd = (gp - gm) / (2 * h)
    assert np.abs(hv - fd).max() <= 1e-7 * np.abs(hv).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_hessian_vector_per_observation_form(shape):
    # -sum_i w_i J_i^T (P_i o u_i - P_i (P_i . u_i)), u_i = J_i v: no H formed
    N, K, p, g, a = shape
    pr = tiny(60 + K, N=N, K=K, p=p, g=g, a=a)
    th = pr.theta_true
    v = np.random.default_rng(4).normal(size=pr.n_params)
    J = unnormalized_jacobians(pr.X, pr.Y, pr.Z)
    U = J @ th
    P = np.exp(U - scipy.special.logsumexp(U, axis=1)[:, None])
    u = J @ v
    s = P * (u - (P * u).sum(axis=1, keepdims=True))
    ref = -np.einsum("i,ikq,ik->q", pr.w, J, s)
    hv = R.hessian_vector(th, pr.X, pr.Y, pr.Z, v, pr.w)
    np.testing.assert_allclose(hv, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_cg_distinct_eigenvalues_and_exact_solve():
    # CG on an SPD system ends in as many steps as distinct eigenvalues
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.normal(size=(12, 12)))
    lam = np.array([1.0] * 5 + [3.0] * 4 + [10.0] * 3)
    A = Q @ np.diag(lam) @ Q.T
    b = rng.normal(size=12)
    d, it = R.cg_direction(lambda v: -A @ v, b, 1e-12, 50)
    assert it == 3
    np.testing.assert_allclose(d, np.linalg.solve(A, b), rtol=1e-10)
    # a loose tolerance stops early with the residual below it
    d2, it2 = R.cg_direction(lambda v: -A @ v, b, 0.5, 50)
    assert it2 < 3 and np.linalg.norm(b - A @ d2) <= 0.5 * np.linalg.norm(b)
    # the iteration cap
    _, it3 = R.cg_direction(lambda v: -A @ v, b, 1e-12, 2)
    assert it3 == 2


def test_cg_non_positive_curvature_returns_gradient():
    A = np.diag([-1.0, 2.0])
    b = np.array([1.0, 0.0])
    d, it = R.cg_direction(lambda v: -A @ v, b, 1e-12, 10)
    assert it == 1 and np.array_equal(d, b)


def test_cg_matches_newton_direction_at_full_depth():
    pr = tiny(70, N=60, K=4, p=3, g=1, a=1)
    th = pr.theta_true
    H = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    gr = R.gradient(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    d, it = R.cg_direction(lambda v: H @ v, gr, 1e-13, 4 * pr.n_params)
    np.testing.assert_allclose(d, R.newton_direction(H, gr), rtol=1e-9,
                               atol=1e-11)


def test_forcing_term():
    assert R.forcing_term(1e4, 1e4) == 0.5
    assert R.forcing_term(1e-2, 1e4) == pytest.approx(1e-3, rel=1e-15)
    # independent of the log-likelihood's scale
    assert R.forcing_term(3e-3, 7.0) == pytest.approx(R.forcing_term(3e-2, 70.0),
                                                      rel=1e-15)


@pytest.mark.parametrize("seed", [1, 2])
def test_newton_cg_fit_reaches_newton_optimum(seed):
    pr = synth.make_problem(800, 5, 3, 1, 1, seed=80 + seed, weights="uniform")
    o_nr = R.FitOptions(gtol=1e-9, ftol=0.0)
    o_cg = R.FitOptions(gtol=1e-9, ftol=0.0, method="newton-cg")
    nr = R.fit_problem(pr, opts=o_nr)
    cg = R.fit_problem(pr, opts=o_cg)
    assert nr.stop_reason == cg.stop_reason == R.STOP_GTOL
    assert np.linalg.norm(cg.theta - nr.theta) <= 1e-9 * np.linalg.norm(nr.theta)
    assert cg.cg_iters >= cg.iters >= nr.iters


def test_newton_cg_binary_equals_irls():
    pr = synth.make_problem(300, 2, 4, 0, 0, seed=7, weights="uniform")
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-11, ftol=0.0,
                                              method="newton-cg"))
    b = irls_binary(pr.X, (pr.choice == 1).astype(float), pr.w)
    np.testing.assert_allclose(res.theta, b, rtol=0, atol=1e-9)


# ---------------------------------------------------------------------------
# collinearity check (linDepTol, App. B)

def test_independent_columns_exact_dependencies():
    rng = np.random.default_rng(21)
    M = rng.normal(size=(200, 6))
    assert R.independent_columns(M).all()
    M[:, 3] = 2.0 * M[:, 0] - M[:, 1]       # in the span of earlier columns
    M[:, 5] = 0.0                           # zero column
    np.testing.assert_array_equal(R.independent_columns(M),
                                  [1, 1, 1, 0, 1, 0])
    # a column spanned by later columns is kept; the first column that
    # closes the dependent set goes
    M2 = rng.normal(size=(100, 3))
    M2 = np.column_stack([M2[:, 0] + M2[:, 1], M2])
    np.testing.assert_array_equal(R.independent_columns(M2), [1, 1, 0, 1])


def test_independent_columns_rank_and_tolerance():
    rng = np.random.default_rng(22)
    B = rng.normal(size=(300, 4))
    M = np.column_stack([B, B @ rng.normal(size=(4, 3))])
    keep = R.independent_columns(M)
    assert keep.sum() == np.linalg.matrix_rank(M) == 4
    # a perturbation far above tol keeps the column, far below drops it
    for eps, kept in ((1e-3, True), (1e-9, False)):
        C = np.column_stack([B, B[:, 0] + eps * rng.normal(size=300)])
        assert R.independent_columns(C, 1e-6)[4] == kept


def test_collinearity_mask_app_b_generic_constant():
    # generic data equal over alternatives: Ytil = 0, every alpha dropped,
    # and the fit on the remaining data converges where it was singular
    pr = synth.make_problem(500, 4, 2, 2, 1, seed=18)
    pr.Y = np.ascontiguousarray(np.repeat(pr.Y[:, :1, :], 4, axis=1))
    kx, ky, kz = R.collinearity_mask(pr.X, pr.Y, pr.Z)
    assert kx.all() and kz.all() and not ky.any()
    bad = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-8, ftol=0))
    assert bad.stop_reason == R.STOP_NOT_PD
    ok = R.fit(pr.X[:, kx], pr.Y[:, :, ky], pr.Z[:, :, kz], pr.choice, pr.w,
               opts=R.FitOptions(gtol=1e-8, ftol=0))
    assert ok.stop_reason == R.STOP_GTOL


def test_collinearity_mask_z_dependent_in_one_alternative():
    pr = synth.make_problem(300, 3, 2, 0, 3, seed=23)
    pr.Z[:, 1, 2] = pr.Z[:, 1, 0] - 3.0 * pr.Z[:, 1, 1]
    kx, ky, kz = R.collinearity_mask(pr.X, pr.Y, pr.Z)
    np.testing.assert_array_equal(kz, [1, 1, 0])
    assert kx.all() and ky.size == 0


# ---------------------------------------------------------------------------
# hypothesis tests (Sec. 2.4)

def _two_by_two(seed):
    rng = np.random.default_rng(seed)
    N = 1200
    x = (rng.random(N) < 0.4).astype(float)
    y = (rng.random(N) < 0.25 + 0.15 * x).astype(np.int32)
    X1 = np.column_stack([np.ones(N), x])
    E = np.zeros((N, 2, 0))
    return X1, E, y, x


def test_score_and_lr_tests_in_a_two_by_two_table():
    # binary logit with one binary covariate against the intercept-only
    # model: the score statistic is Pearson's chi-square of the 2 x 2 table
    # and the likelihood ratio is the G statistic 2 sum O log(O / E)
    X1, E, y, x = _two_by_two(41)
    opts = R.FitOptions(gtol=1e-11, ftol=0.0)
    full = R.fit(X1, E, E, y, None, opts=opts)
    rest = R.fit(X1[:, :1], E, E, y, None, opts=opts)
    th0 = np.array([rest.theta[0], 0.0])
    g = R.gradient(th0, X1, E, E, y)
    H = R.hessian(th0, X1, E, E, y)
    O = np.array([[np.sum((x == a) & (y == b)) for b in (0, 1)]
                  for a in (0, 1)], dtype=float)
    Ex = O.sum(1, keepdims=True) * O.sum(0, keepdims=True) / O.sum()
    pearson = float(((O - Ex) ** 2 / Ex).sum())
    gstat = float(2.0 * (O * np.log(O / Ex)).sum())
    s, df, p = R.score_test(g, H, 1)
    assert s == pytest.approx(pearson, rel=1e-9) and df == 1
    lr, _, plr = R.lr_test(full.loglik, rest.loglik, 1)
    assert lr == pytest.approx(gstat, rel=1e-9)
    assert p == pytest.approx(math.erfc(math.sqrt(s / 2.0)), rel=1e-12)


def test_wald_single_coefficient_is_z_squared():
    pr = tiny(42, N=400, K=3, p=2, g=1, a=1)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-10, ftol=0.0))
    V = R.covariance(res.theta, pr.X, pr.Y, pr.Z, pr.w)
    se, z, pv = R.summary(res.theta, pr.X, pr.Y, pr.Z, pr.w)
    for j in (0, 3, pr.n_params - 1):
        w, df, p = R.wald_test(res.theta, V, [j])
        assert w == pytest.approx(z[j] ** 2, rel=1e-12) and df == 1
        assert p == pytest.approx(pv[j], rel=1e-9)


def test_score_test_vanishes_at_the_optimum_and_chi2_closed_form():
    pr = tiny(43, N=300, K=3, p=2, g=1, a=0)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-12, ftol=0.0))
    H = R.hessian(res.theta, pr.X, pr.Y, pr.Z, None, pr.w)
    s, _, p = R.score_test(res.grad, H, 2)
    assert s < 1e-20 and p == pytest.approx(1.0)
    for x in (0.1, 1.0, 7.5):
        assert R.chi2_sf(x, 2) == pytest.approx(math.exp(-x / 2), rel=1e-14)


def test_hm_test_identical_fits_and_definition():
    pr = tiny(44, N=400, K=4, p=2, g=0, a=0)
    res = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-10, ftol=0.0))
    V = R.covariance(res.theta, pr.X, pr.Y, pr.Z, pr.w)
    d = np.array([0.1, -0.2])
    Vd = np.array([[0.02, 0.005], [0.005, 0.03]])
    s, df, _ = R.hm_test(res.theta[:2] + d, V[:2, :2] + Vd, res.theta[:2],
                         V[:2, :2])
    assert s == pytest.approx(float(d @ np.linalg.inv(Vd) @ d), rel=1e-12)
    assert df == 2


def test_wald_test_two_by_two_is_woolf():
    # the log odds ratio of a 2 x 2 table has variance 1/a + 1/b + 1/c + 1/d
    # at the optimum (Woolf), so its Wald statistic is in closed form
    X1, E, y, x = _two_by_two(45)
    full = R.fit(X1, E, E, y, None, opts=R.FitOptions(gtol=1e-12, ftol=0.0))
    O = np.array([[np.sum((x == a) & (y == b)) for b in (0, 1)]
                  for a in (0, 1)], dtype=float)
    lor = math.log(O[1, 1] * O[0, 0] / (O[1, 0] * O[0, 1]))
    V = R.covariance(full.theta, X1, E, E)
    w, df, _ = R.wald_test(full.theta, V, [1])
    assert full.theta[1] == pytest.approx(lor, rel=1e-10)
    assert w == pytest.approx(lor ** 2 / (1.0 / O).sum(), rel=1e-9)


def _hm_pipeline(X, Y, Z, choice, alts):
    """Full fit, fit on the alternatives `alts` (base first), and the HM
    statistic over their common coefficients."""
    K, p, g, a = Y.shape[1], X.shape[1], Y.shape[2], Z.shape[2]
    o = R.FitOptions(gtol=1e-11, ftol=0.0)
    full = R.fit(X, Y, Z, choice, None, opts=o)
    m = np.isin(choice, alts)
    lut = -np.ones(K, int)
    lut[alts] = np.arange(len(alts))
    Xs, Ys, Zs = X[m], Y[m][:, alts], Z[m][:, alts]
    sub = R.fit(Xs, Ys, Zs, lut[choice[m]].astype(np.int32), None, opts=o)
    idx = [(j - 1) * p + c for j in alts[1:] for c in range(p)]
    idx += [(K - 1) * p + j * a + c for j in alts for c in range(a)]
    idx += [(K - 1) * p + K * a + c for c in range(g)]
    Vf = R.covariance(full.theta, X, Y, Z)[np.ix_(idx, idx)]
    Vs = R.covariance(sub.theta, Xs, Ys, Zs)
    return R.hm_test(sub.theta, Vs, full.theta[idx], Vf)


def test_hm_test_invariant_to_rescaling_a_variable():
    # rescaling a column of X rescales its coefficients and their
    # covariances; the HM statistic of the refits does not change
    pr = synth.make_problem(3000, 4, 3, 1, 0, seed=73)
    alts = [0, 1, 3]
    s1, df, _ = _hm_pipeline(pr.X, pr.Y, pr.Z, pr.choice, alts)
    X2 = pr.X.copy()
    X2[:, 2] *= 8.0
    Y2 = pr.Y * 0.25
    s2, _, _ = _hm_pipeline(X2, Y2, pr.Z, pr.choice, alts)
    assert df == 2 * 3 + 1
    assert s2 == pytest.approx(s1, rel=1e-7)



def _hm_parts(X, choice, alts, K):
    """Full and subset fits of an X-only model: the subset estimate, the
    matching full-model coefficients and both covariances."""
    N = X.shape[0]
    E = np.zeros((N, K, 0))
    o = R.FitOptions(gtol=1e-11, ftol=0.0)
    full = R.fit(X, E, E, choice, None, opts=o)
    m = np.isin(choice, alts)
    lut = -np.ones(K, int)
    lut[alts] = np.arange(len(alts))
    Xs = X[m]
    Es = np.zeros((Xs.shape[0], len(alts), 0))
    sub = R.fit(Xs, Es, Es, lut[choice[m]].astype(np.int32), None, opts=o)
    p = X.shape[1]
    idx = [(j - 1) * p + c for j in alts[1:] for c in range(p)]
    Vf = R.covariance(full.theta, X, E, E)[np.ix_(idx, idx)]
    Vs = R.covariance(sub.theta, Xs, Es, Es)
    return sub.theta, full.theta[idx], Vs, Vf


def test_hm_test_chi_square_law_under_iia():
    # Choices drawn from a logit with fixed coefficients satisfy IIA.  Then
    # d = theta_sub - theta_full is asymptotically normal with covariance
    # V_sub - V_full (the full fit is efficient, the subset fit only
    # consistent), so d^T (V_sub - V_full)^{-1} d is chi-square with df =
    # the number of common coefficients (Hausman and McFadden 1984).  With
    # the covariances averaged over the replications (the per-sample
    # difference is nearly singular at these sizes) the statistic's mean
    # must lie within 3 standard errors of df.  A swapped difference gives
    # -df, a sum a mean far below df.
    B = np.array([[0.0, 0.0], [0.8, -0.5], [-0.4, 0.9]])
    reps, N = 200, 3000
    TS, TF, VS, VF = [], [], [], []
    for r in range(reps):
        rng = np.random.default_rng(7000 + r)
        X = rng.normal(size=(N, 2))
        U = X @ B.T + rng.gumbel(size=(N, 3))
        ts, tf, Vs, Vf = _hm_parts(X, U.argmax(1).astype(np.int32), [0, 1], 3)
        TS.append(ts); TF.append(tf); VS.append(Vs); VF.append(Vf)
    TS, TF = np.array(TS), np.array(TF)
    Vs, Vf = np.mean(VS, axis=0), np.mean(VF, axis=0)
    # the covariance of d across replications is V_sub - V_full
    C = np.cov((TS - TF).T)
    np.testing.assert_allclose(np.diag(C), np.diag(Vs - Vf), rtol=0.3)
    stats = np.array([R.hm_test(TS[r], Vs, TF[r], Vf)[0] for r in range(reps)])
    df = R.hm_test(TS[0], Vs, TF[0], Vf)[1]
    assert df == 2
    se = math.sqrt(2.0 * df / reps)
    assert abs(stats.mean() - df) <= 3.0 * se, (stats.mean(), se)
    assert np.all(stats >= 0.0)
    # tail probabilities roughly uniform: about 10 % fall below 0.1
    pv = np.array([R.chi2_sf(x, df) for x in stats])
    assert 0.05 <= np.mean(pv < 0.1) <= 0.17
