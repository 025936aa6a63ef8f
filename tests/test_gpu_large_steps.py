"""Newton steps at the largest workload sizes against the oracle's recorded
steps (tests/golden/make_step_golden.py: oracle and generator only).

* 400,000 observations, K = 100, p = 51, g = 5 (n_p = 5,054) at theta = 0:
  l, the gradient (Eq. 9) and the Newton direction of Eq. 6 solved against
  the full Eq. 10 Hessian, alpha-alpha block included.
* 50,000 observations, K = 500, p = 11, weighted, near separable
  (n_p = 5,489): the first two iterations of the fit from zero (theta, l,
  ||g||, line-search trials), and, when the oracle's whole fit is on
  record, where and why it stops.
"""
import os

import numpy as np
import pytest

import synth
from tests.conftest import golden_path
from tests.gpu_util import device_problem, grad_scale, theta_tensor

pytestmark = pytest.mark.gpu

GTOL = 1e-8


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


def _load(name):
    return np.load(golden_path(name))


def test_c3_gradient_and_newton_direction(ctx):
    gold = _load("step_c3.npz")
    pr = synth.make_config("c3")
    dp = device_problem(pr)
    th0 = theta_tensor(np.zeros(pr.n_params))
    l, g, _ = ctx.loglik_grad(dp, th0)
    l = float(l.cpu()[0])
    assert abs(l - float(gold["loglik"])) <= 1e-12 * abs(float(gold["loglik"]))
    err = np.abs(g.cpu().numpy() - gold["grad"]) / grad_scale(pr)
    assert err.max() <= 1e-12, err.max()
    # one Newton step from zero: theta_1 = t delta with t = 2^-(trials - 1)
    th = theta_tensor(np.zeros(pr.n_params))
    info = ctx.newton_step(dp, th, gtol=GTOL, ftol=0.0)
    t = 0.5 ** (info["ls_iters"] - 1)
    delta = th.cpu().numpy() / t
    ref = gold["delta"]
    rel = np.linalg.norm(delta - ref) / np.linalg.norm(ref)
    assert rel <= 1e-9, rel
    assert np.abs(delta - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.fixture(scope="module")
def c5():
    pr = synth.make_config("c5")
    return pr, device_problem(pr)


def test_c5_first_two_iterations(ctx, c5):
    gold = _load("traj_c5_it2.npz")
    pr, dp = c5
    hist = gold["hist_theta"]
    # each step from the oracle's own iterate
    for it in range(2):
        th = theta_tensor(hist[it])
        info = ctx.newton_step(dp, th, gtol=GTOL, ftol=0.0)
        assert info["ls_iters"] == int(gold["hist_trials"][it]), it
        assert abs(info["grad_norm"] - gold["hist_grad_norm"][it]) <= \
            1e-9 * gold["hist_grad_norm"][it]
        nxt = hist[it + 1] if it + 1 < len(hist) else gold["theta"]
        got = th.cpu().numpy()
        rel = np.linalg.norm(got - nxt) / np.linalg.norm(nxt)
        assert rel <= 1e-9, (it, rel)
    # and the fit itself, two iterations from zero
    theta, info = ctx.fit(dp, gtol=GTOL, ftol=0.0, maxiter=2)
    assert info["iters"] == int(gold["iters"]) == 2
    assert info["ls_iters"] == int(gold["ls_iters"])
    assert abs(info["loglik"] - float(gold["loglik"])) <= \
        1e-12 * abs(float(gold["loglik"]))
    rel = np.linalg.norm(theta.cpu().numpy() - gold["theta"]) / \
        np.linalg.norm(gold["theta"])
    assert rel <= 1e-9, rel


@pytest.mark.skipif(not os.path.exists(golden_path("traj_c5.npz")),
                    reason="the oracle's whole 500-alternative fit is not on "
                           "record")
def test_c5_fit_stops_where_the_oracle_stops(ctx, c5):
    gold = _load("traj_c5.npz")
    pr, dp = c5
    theta, info = ctx.fit(dp, gtol=GTOL, ftol=0.0)
    assert info["stop_reason"] == int(gold["stop_reason"])
    assert info["iters"] == int(gold["iters"])
    assert info["ls_iters"] == int(gold["ls_iters"])
    assert abs(info["loglik"] - float(gold["loglik"])) <= \
        1e-10 * abs(float(gold["loglik"]))
    # the per-iteration log-likelihoods of the recorded trajectory
    lls = gold["hist_loglik"]
    for it in range(min(len(lls), 5)):
        l, _, _ = ctx.loglik_grad(dp, theta_tensor(gold["hist_theta"][it]))
        assert abs(float(l.cpu()[0]) - lls[it]) <= 1e-12 * abs(lls[it])
