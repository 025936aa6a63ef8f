"""Newton-Raphson on the GPU (Eq. 6 + halving line search) against the FP64
oracle: per-iteration steps, whole fits, mixed-precision Hessians, stops and
error paths."""
import os

import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.conftest import ROOT
from tests.gpu_util import device_problem, theta_tensor

pytestmark = pytest.mark.gpu

GTOL = 1e-8


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


FIT_SHAPES = [  # N, K, p, g, a, weights
    (400, 4, 3, 2, 2, "uniform"),
    (3000, 7, 5, 2, 1, None),
    (900, 2, 4, 0, 0, "uniform"),
    (2500, 19, 3, 1, 0, "uniform"),
    (1200, 5, 0, 3, 1, None),
    (5000, 66, 4, 1, 1, None),
]


@pytest.mark.parametrize("shape", FIT_SHAPES)
def test_fit_fp64_matches_oracle(ctx, shape):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=300 + N + K, weights=wk)
    ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0))
    theta, info = ctx.fit(device_problem(pr), gtol=GTOL, ftol=0.0)
    th = theta.cpu().numpy()
    assert info["stop_reason"] == ref.stop_reason == R.STOP_GTOL
    assert info["iters"] == ref.iters and info["ls_iters"] == ref.ls_iters
    assert info["grad_norm"] <= GTOL
    assert rel(th, ref.theta) <= 1e-8
    assert info["loglik"] == pytest.approx(ref.loglik, rel=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", FIT_SHAPES[:4])
def test_fit_mixed_matches_oracle(ctx, shape, prec):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=300 + N + K, weights=wk)
    ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0))
    theta, info = ctx.fit(device_problem(pr), gtol=GTOL, ftol=0.0, prec=prec)
    assert info["stop_reason"] == R.STOP_GTOL, info
    assert info["grad_norm"] <= GTOL
    assert rel(theta.cpu().numpy(), ref.theta) <= 1e-6
    # an inexact Hessian only slows convergence
    assert info["iters"] >= ref.iters


def test_newton_steps_follow_oracle_trajectory(ctx):
    pr = synth.make_problem(2000, 6, 4, 2, 1, seed=31, weights="uniform")
    ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0),
                        record=True)
    dp = device_problem(pr)
    seq = [h["theta"] for h in ref.history] + [ref.theta]
    for t, h in enumerate(ref.history):
        th = theta_tensor(h["theta"])
        info = ctx.newton_step(dp, th, gtol=GTOL, ftol=0.0)
        assert info["stop_reason"] == 0 and info["ls_iters"] == h["trials"]
        assert info["grad_norm"] == pytest.approx(h["grad_norm"], rel=1e-10)
        step_ref = seq[t + 1] - h["theta"]
        step = th.cpu().numpy() - h["theta"]
        # the gradient's own FP64 round-off (~1e-13 absolute here) bounds
        # how well the last, tiny steps can agree
        tol = 1e-9 * np.linalg.norm(step_ref) + 1e-11 * np.linalg.norm(seq[-1])
        assert np.linalg.norm(step - step_ref) <= tol, t
    info = ctx.newton_step(dp, theta_tensor(ref.theta), gtol=GTOL, ftol=0.0)
    assert info["stop_reason"] == R.STOP_GTOL and info["iters"] == 0


@pytest.mark.parametrize("shape", [(3000, 43, 50, 1, 1, "uniform"),
                                   (3000, 49, 48, 0, 0, None)])
def test_newton_step_large_system_matches_oracle(ctx, shape):
    # n_p >= 2048 (2,144 ragged, 2,304 a whole number of outer panels): the
    # factorisation runs by outer panels with FP64-MFMA trailing updates
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=77 + K, weights=wk)
    assert pr.n_params >= 2048
    th0 = np.zeros(pr.n_params)
    grad = R.gradient(th0, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    H = R.hessian(th0, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    d_ref = R.newton_direction(H, grad)
    dp = device_problem(pr)
    th = theta_tensor(th0)
    info = ctx.newton_step(dp, th, gtol=GTOL, ftol=0.0)
    assert info["stop_reason"] == 0, info
    step_ref = 0.5 ** (info["ls_iters"] - 1) * d_ref
    step = th.cpu().numpy() - th0
    assert np.linalg.norm(step - step_ref) <= 1e-9 * np.linalg.norm(step_ref)


def test_fit_is_deterministic(ctx):
    import torch
    pr = synth.make_problem(20000, 12, 6, 2, 1, seed=9, weights="uniform")
    dp = device_problem(pr)
    t1, i1 = ctx.fit(dp, gtol=GTOL, ftol=0.0)
    t2, i2 = ctx.fit(dp, gtol=GTOL, ftol=0.0)
    assert torch.equal(t1, t2) and i1["iters"] == i2["iters"]


def test_workspace_cap(ctx):
    # a context whose workspace cap is below what the fit needs refuses it
    # (OOM) without growing past the cap; a cap of exactly the need gives
    # the same fit bit for bit
    import torch
    import paper_1404_3177_amd as mnl
    pr = synth.make_problem(20000, 12, 6, 2, 1, seed=9, weights="uniform")
    dp = device_problem(pr)
    fresh = mnl.Context(0)
    t_ref, _ = fresh.fit(dp, gtol=GTOL, ftol=0.0)
    need = fresh.workspace_bytes
    small = mnl.Context(0, workspace_bytes=need // 2)
    with pytest.raises(mnl.MnlError) as err:
        small.fit(dp, gtol=GTOL, ftol=0.0)
    assert err.value.code == -2
    assert small.workspace_bytes <= need // 2
    exact = mnl.Context(0, workspace_bytes=need)
    t, _ = exact.fit(dp, gtol=GTOL, ftol=0.0)
    assert torch.equal(t, t_ref) and exact.workspace_bytes <= need


def test_fit_from_start_and_resume(ctx):
    pr = synth.make_problem(3000, 5, 3, 1, 1, seed=41)
    dp = device_problem(pr)
    t_full, i_full = ctx.fit(dp, gtol=GTOL, ftol=0.0)
    t_part, i_part = ctx.fit(dp, gtol=GTOL, ftol=0.0, maxiter=2)
    assert i_part["stop_reason"] == R.STOP_MAXITER and i_part["iters"] == 2
    t_res, i_res = ctx.fit(dp, theta0=t_part, gtol=GTOL, ftol=0.0)
    assert i_res["iters"] == i_full["iters"] - 2
    assert rel(t_res.cpu().numpy(), t_full.cpu().numpy()) <= 1e-12


def test_ftol_stop(ctx):
    pr = synth.make_problem(3000, 5, 3, 1, 1, seed=42)
    ref = R.fit_problem(pr, opts=R.FitOptions(gtol=1e-14, ftol=1e-3))
    _, info = ctx.fit(device_problem(pr), gtol=1e-14, ftol=1e-3)
    assert info["stop_reason"] == ref.stop_reason == R.STOP_FTOL
    assert info["iters"] == ref.iters


def test_singular_model_not_pd(ctx):
    # generic data constant over alternatives (App. B): singular Hessian
    pr = synth.make_problem(500, 4, 2, 1, 0, seed=18)
    pr.Y = np.ascontiguousarray(np.repeat(pr.Y[:, :1, :], 4, axis=1))
    ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0))
    _, info = ctx.fit(device_problem(pr), gtol=GTOL, ftol=0.0)
    assert ref.stop_reason == R.STOP_NOT_PD
    assert info["stop_reason"] == R.STOP_NOT_PD


def test_line_search_failure_reported(ctx):
    # at the optimum a huge start offset along a ray with ls_max = 0 fails
    pr = synth.make_problem(800, 3, 3, 0, 0, seed=20, coef_sd=2.0)
    th0 = np.full(pr.n_params, 6.0)
    ref = R.fit_problem(pr, theta0=th0,
                        opts=R.FitOptions(gtol=GTOL, ftol=0, ls_max=0))
    _, info = ctx.fit(device_problem(pr), theta0=theta_tensor(th0),
                      gtol=GTOL, ftol=0.0, ls_max=0)
    assert info["stop_reason"] == ref.stop_reason
    assert info["iters"] == ref.iters


def test_validation_errors(ctx):
    import paper_1404_3177_amd as mnl
    pr = synth.make_problem(100, 4, 2, 1, 0, seed=3)
    bad = synth.make_problem(100, 4, 2, 1, 0, seed=3)
    bad.choice[5] = 7
    with pytest.raises(mnl.MnlError) as ei:
        ctx.fit(device_problem(bad), validate=1)
    assert ei.value.code == -1
    nan = synth.make_problem(100, 4, 2, 1, 0, seed=3)
    nan.X[3, 1] = np.nan
    with pytest.raises(mnl.MnlError) as ei:
        ctx.fit(device_problem(nan), validate=1)
    assert ei.value.code == -4
    _, info = ctx.fit(device_problem(pr), validate=1, gtol=GTOL, ftol=0.0)
    assert info["stop_reason"] == R.STOP_GTOL


def _golden(name):
    path = os.path.join(ROOT, "tests", "golden", f"fit_{name}.npz")
    return np.load(path) if os.path.exists(path) else None


@pytest.mark.parametrize("name,prec,tol", [("c1", "fp64", 1e-8),
                                           ("c2", "fp64", 1e-8),
                                           ("c2", "fp32", 1e-6),
                                           ("c2", "bf16", 1e-6)])
def test_config_fit_matches_oracle_golden(ctx, name, prec, tol):
    gold = _golden(name)
    assert gold is not None, "run tests/golden/make_fit_golden.py"
    pr = synth.make_config(name)
    theta, info = ctx.fit(device_problem(pr), gtol=float(gold["gtol"]),
                          ftol=0.0, prec=prec)
    assert info["stop_reason"] == int(gold["stop_reason"]) == R.STOP_GTOL
    assert rel(theta.cpu().numpy(), gold["theta"]) <= tol
    if prec == "fp64":
        assert info["iters"] == int(gold["iters"])
        assert info["ls_iters"] == int(gold["ls_iters"])
