"""Parity of the fitted-model methods (predict, summary's standard errors)
with the FP64 oracle."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem, hess_scale, theta_tensor

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EPS = np.finfo(np.float64).eps

PRED_SHAPES = [  # N, K, p, g, a
    (1, 3, 2, 1, 1), (37, 4, 3, 2, 2), (2049, 7, 5, 2, 1), (777, 19, 3, 1, 0),
    (300, 129, 3, 1, 1), (1000, 5, 0, 3, 0), (513, 2, 4, 0, 0),
]

# n_p from 2 to 2,144: one-panel, several-panel and outer-panel (n_p >= 2048)
# factorisations, with and without every data kind
SE_SHAPES = [  # N, K, p, g, a, weights
    (400, 2, 1, 0, 0, None),
    (600, 3, 2, 1, 1, "uniform"),
    (3000, 7, 5, 2, 1, None),
    (2000, 19, 3, 1, 0, "uniform"),
    (5000, 13, 12, 2, 2, "int"),
    (3000, 33, 2, 0, 2, None),
    (4000, 70, 2, 1, 1, "uniform"),   # more than 64 alternatives
    (3000, 43, 50, 1, 1, "uniform"),
]


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


def _no_choice(pr):
    import paper_1404_3177_amd as mnl
    dp = device_problem(pr)
    X, Y, Z, _, w = dp._refs
    return mnl.Problem(X, Y, Z, None, w)


@pytest.mark.parametrize("shape", PRED_SHAPES)
def test_predict_matches_oracle(ctx, shape):
    N, K, p, g, a = shape
    pr = synth.make_problem(N, K, p, g, a, seed=300 + K, coef_sd=1.0)
    P = ctx.predict(_no_choice(pr), theta_tensor(pr.theta_true)).cpu().numpy()
    P_ref = R.predict(pr.theta_true, pr.X, pr.Y, pr.Z)
    assert np.abs(P - P_ref).max() <= 1e-13
    np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-14)


def test_predict_equals_pass_probabilities(ctx):
    import torch
    pr = synth.make_problem(3001, 23, 6, 2, 2, seed=31, weights="uniform")
    dp = device_problem(pr)
    th = theta_tensor(pr.theta_true)
    _, _, P_pass = ctx.loglik_grad(dp, th, want_P=True)
    assert torch.equal(ctx.predict(dp, th), P_pass)
    assert torch.equal(ctx.predict(_no_choice(pr), th), P_pass)


def _se_tolerance(pr, H_ref):
    """Bound on the relative error of each standard error.  With -H
    perturbed by dA (the GPU Hessian's deviation, elementwise at most
    1e-12 sum_i |term_i|, plus the factorisation's backward error
    n eps ||A||), diag(Z) with Z = (-H)^{-1} moves by at most
    ||Z e_j||^2 ||dA||, and se by half that relative to Z_jj."""
    A = -H_ref
    Z = np.linalg.inv(A)
    n = A.shape[0]
    dA = 1e-12 * np.linalg.norm(hess_scale(pr)) + n * EPS * np.linalg.norm(A, 2)
    amp = (Z * Z).sum(axis=0) / np.diag(Z)
    return 10.0 * 0.5 * amp * dA


@pytest.mark.parametrize("shape", SE_SHAPES)
def test_standard_errors_match_oracle(ctx, shape):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=400 + K, weights=wk)
    th = 0.8 * pr.theta_true
    se, z, pv = (t.cpu().numpy() for t in
                 ctx.summary(_no_choice(pr), theta_tensor(th)))
    se_ref, z_ref, pv_ref = R.summary(th, pr.X, pr.Y, pr.Z, pr.w)
    tol = _se_tolerance(pr, R.hessian(th, pr.X, pr.Y, pr.Z, None, pr.w))
    rel = np.abs(se - se_ref) / se_ref
    assert np.all(rel <= tol), (shape, rel.max(), (rel / tol).max())
    np.testing.assert_allclose(z, th / se, rtol=1e-15, atol=0)
    # p = erfc(|z| / sqrt 2): relative error bounded by that of z times
    # |z| sqrt(2/pi) e^{-z^2/2} / p, plus a few ulps
    dz = np.abs(z_ref) * tol
    dp = dz * np.sqrt(2 / np.pi) * np.exp(-z_ref ** 2 / 2) + 4 * EPS * pv_ref
    assert np.all(np.abs(pv - pv_ref) <= 2 * dp + 1e-300), shape


def test_standard_errors_intercept_only_closed_form(ctx):
    # at the optimum of the intercept-only model se_k = sqrt(1/n_k + 1/n_0)
    K = 6
    pr = synth.make_problem(5000, K, 1, 0, 0, seed=44, weights="uniform",
                            coef_sd=0.7)
    dp = device_problem(pr)
    theta, info = ctx.fit(dp, gtol=1e-10, ftol=0.0)
    assert info["stop_reason"] == R.STOP_GTOL
    se, _, _ = ctx.summary(dp, theta)
    n = np.array([pr.w[pr.choice == k].sum() for k in range(K)])
    np.testing.assert_allclose(se.cpu().numpy(), np.sqrt(1 / n[1:] + 1 / n[0]),
                               rtol=1e-9)


def test_standard_errors_deterministic_and_weight_scaling(ctx):
    import torch
    import paper_1404_3177_amd as mnl
    pr = synth.make_problem(4000, 9, 4, 1, 1, seed=45, weights="uniform")
    dp = device_problem(pr)
    th = theta_tensor(pr.theta_true)
    s1 = ctx.summary(dp, th)[0]
    s2 = ctx.summary(dp, th)[0]
    assert torch.equal(s1, s2)
    X, Y, Z, c, w = dp._refs
    s4 = ctx.summary(mnl.Problem(X, Y, Z, c, 4.0 * w), th)[0]
    # scaling w by 4 scales H by 4 and se by 1/2 (a power of two: up to
    # the reciprocal estimates' last bits)
    assert torch.allclose(s4 * 2.0, s1, rtol=1e-14, atol=0)


def test_standard_errors_singular_model_not_pd(ctx):
    import paper_1404_3177_amd as mnl
    # generic data constant over alternatives: -H is singular (App. B)
    pr = synth.make_problem(500, 4, 2, 1, 0, seed=18)
    pr.Y = np.ascontiguousarray(np.repeat(pr.Y[:, :1, :], 4, axis=1))
    with pytest.raises(mnl.MnlError) as ei:
        ctx.summary(device_problem(pr), theta_tensor(np.zeros(pr.n_params)))
    assert ei.value.code == -3
    # the context stays usable
    ok = synth.make_problem(500, 4, 2, 1, 0, seed=19)
    se, _, _ = ctx.summary(device_problem(ok), theta_tensor(ok.theta_true))
    assert np.all(np.isfinite(se.cpu().numpy()))


def test_fit_after_summary_unchanged(ctx):
    # the summary grows the shared matrix buffer; a later fit is unaffected
    import torch
    pr = synth.make_problem(3000, 8, 4, 1, 1, seed=46)
    dp = device_problem(pr)
    t1, i1 = ctx.fit(dp, gtol=1e-8, ftol=0.0)
    ctx.summary(dp, t1)
    t2, i2 = ctx.fit(dp, gtol=1e-8, ftol=0.0)
    assert torch.equal(t1, t2) and i1["iters"] == i2["iters"]


@pytest.mark.parametrize("name", ["c2", "c5"])
def test_predict_config_full(ctx, name):
    # full workload sizes, every probability against the oracle
    pr = synth.make_config(name)
    th = 0.5 * pr.theta_true
    P = ctx.predict(_no_choice(pr), theta_tensor(th)).cpu().numpy()
    P_ref = R.predict(th, pr.X, pr.Y, pr.Z)
    assert np.abs(P - P_ref).max() <= 1e-13, name


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_standard_errors_config_golden(ctx, name):
    # the oracle's table at its own fitted optimum
    # (tests/golden/make_summary_golden.py)
    path = os.path.join(ROOT, "tests", "golden", f"summary_{name}.npz")
    gold = np.load(path)
    pr = synth.make_config(name)
    se, z, _ = (t.cpu().numpy() for t in
                ctx.summary(_no_choice(pr), theta_tensor(gold["theta"])))
    n = pr.n_params
    # ||dA||_2 <= n * 1e-11 max|H| (the elementwise Hessian bound of the
    # full-size Hessian test) + n eps ||A||_2; relative error of se_j is at
    # most 0.5 ||(-H)^{-1}||_2 ||dA||_2
    dA = n * 1e-11 * float(gold["hmax"]) + n * EPS * float(gold["lam_max"])
    tol = 10.0 * 0.5 * dA / float(gold["lam_min"])
    rel = np.abs(se - gold["se"]) / gold["se"]
    assert rel.max() <= tol, (name, rel.max(), tol)
    np.testing.assert_allclose(z, gold["theta"] / se, rtol=1e-15, atol=0)
