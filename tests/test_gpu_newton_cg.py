"""Parity of the inexact (truncated) Newton path: Hessian-vector products
and Newton-CG fits against the FP64 oracle."""
import os

import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem, hess_scale, theta_tensor

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GTOL = 1e-8

HV_SHAPES = [  # N, K, p, g, a, weights
    (37, 4, 3, 2, 2, "uniform"), (1, 3, 2, 1, 1, None),
    (2049, 7, 5, 2, 1, None), (513, 2, 4, 0, 0, "uniform"),
    (777, 19, 3, 1, 0, "uniform"), (1000, 5, 0, 3, 0, None),
    (1000, 6, 0, 0, 3, "int"), (1500, 13, 12, 2, 2, "uniform"),
    (300, 129, 3, 1, 1, "uniform"), (4000, 25, 4, 1, 5, None),
]


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("shape", HV_SHAPES)
def test_hessvec_matches_oracle(ctx, shape):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=500 + K, weights=wk)
    th = pr.theta_true
    v = np.random.default_rng(K).normal(size=pr.n_params)
    hv = ctx.hessvec(device_problem(pr), theta_tensor(th),
                     theta_tensor(v)).cpu().numpy()
    ref = R.hessian_vector(th, pr.X, pr.Y, pr.Z, v, pr.w)
    # every term of (H v)_j is bounded by w_i A_ij |s_i|, and
    # sum_k |s_ik| <= 2 max_k |u_ik| <= 2 sum_l A_il |v_l|
    bound = 2.0 * hess_scale(pr) @ np.abs(v)
    assert np.all(np.abs(hv - ref) <= 1e-12 * bound), shape


def test_newton_cg_step_matches_oracle_direction(ctx):
    pr = synth.make_problem(3000, 9, 5, 2, 1, seed=61, weights="uniform")
    th0 = np.zeros(pr.n_params)
    gr = R.gradient(th0, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    H = R.hessian(th0, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    gn = np.linalg.norm(gr)
    d_ref, n_ref = R.cg_direction(lambda v: H @ v, gr, R.forcing_term(gn, gn),
                                  250)
    th = theta_tensor(th0)
    info = ctx.newton_step(device_problem(pr), th, gtol=GTOL, ftol=0.0,
                           method="newton-cg")
    assert info["stop_reason"] == 0 and info["cg_iters"] == n_ref
    step_ref = 0.5 ** (info["ls_iters"] - 1) * d_ref
    assert rel(th.cpu().numpy() - th0, step_ref) <= 1e-10


@pytest.mark.parametrize("shape", [(2000, 10, 6, 1, 0, None),
                                   (5000, 13, 12, 2, 2, "uniform"),
                                   (600, 3, 2, 1, 1, "int"),
                                   (3000, 43, 8, 1, 1, "uniform")])
def test_newton_cg_fit_matches_oracle(ctx, shape):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=600 + K, weights=wk)
    nr = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0))
    cg = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0,
                                             method="newton-cg"))
    theta, info = ctx.fit(device_problem(pr), gtol=GTOL, ftol=0.0,
                          method="newton-cg")
    assert info["stop_reason"] == cg.stop_reason == R.STOP_GTOL
    # one fixed point: Newton's optimum
    assert rel(theta.cpu().numpy(), nr.theta) <= 1e-8
    # the same trajectory up to a product at a threshold crossing
    assert abs(info["iters"] - cg.iters) <= 1
    assert abs(info["cg_iters"] - cg.cg_iters) <= info["iters"]


def test_newton_cg_product_cap(ctx):
    # one product per iteration: d = (g.g / g.(-H)g) g, compared step by step
    pr = synth.make_problem(2500, 6, 4, 1, 1, seed=62)
    ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0, maxiter=5,
                                              method="newton-cg",
                                              cg_maxiter=1))
    theta, info = ctx.fit(device_problem(pr), gtol=GTOL, ftol=0.0, maxiter=5,
                          method="newton-cg", cg_maxiter=1)
    assert info["stop_reason"] == ref.stop_reason == R.STOP_MAXITER
    assert info["cg_iters"] == ref.cg_iters == 5
    assert info["ls_iters"] == ref.ls_iters
    assert rel(theta.cpu().numpy(), ref.theta) <= 1e-10


def test_newton_cg_options_rejected(ctx):
    import paper_1404_3177_amd as mnl
    pr = synth.make_problem(100, 4, 2, 1, 0, seed=3)
    with pytest.raises(mnl.MnlError) as ei:
        ctx.fit(device_problem(pr), method=2)
    assert ei.value.code == -1
    with pytest.raises(mnl.MnlError) as ei:
        ctx.fit(device_problem(pr), method="newton-cg", cg_maxiter=0)
    assert ei.value.code == -1


def test_newton_cg_deterministic(ctx):
    import torch
    pr = synth.make_problem(20000, 12, 6, 2, 1, seed=9, weights="uniform")
    dp = device_problem(pr)
    t1, i1 = ctx.fit(dp, gtol=GTOL, ftol=0.0, method="newton-cg")
    t2, i2 = ctx.fit(dp, gtol=GTOL, ftol=0.0, method="newton-cg")
    assert torch.equal(t1, t2) and i1["cg_iters"] == i2["cg_iters"]


def test_newton_cg_c2_reaches_oracle_optimum(ctx):
    # the 100,000-observation workload: the oracle's Newton optimum
    gold = np.load(os.path.join(ROOT, "tests", "golden", "fit_c2.npz"))
    pr = synth.make_config("c2")
    theta, info = ctx.fit(device_problem(pr), gtol=float(gold["gtol"]),
                          ftol=0.0, method="newton-cg")
    assert info["stop_reason"] == R.STOP_GTOL
    assert rel(theta.cpu().numpy(), gold["theta"]) <= 1e-8
    print(f"c2 newton-cg: iters={info['iters']} cg={info['cg_iters']} "
          f"t={info['t_total']:.1f} ms")
