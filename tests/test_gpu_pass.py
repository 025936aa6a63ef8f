"""Parity of the fused GPU pass (P, l, g; Eqs. 3-5, 9) with the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem, grad_scale, theta_tensor

pytestmark = pytest.mark.gpu

# (N, K, p, g, a, weights): ragged tails, K beyond one wave, K = 2, empty
# data kinds, weights on and off
SHAPES = [
    (37, 4, 3, 2, 2, "uniform"),
    (1, 3, 2, 1, 1, None),
    (3001, 7, 5, 2, 1, None),
    (513, 2, 4, 0, 0, "uniform"),
    (777, 70, 3, 1, 0, "uniform"),
    (300, 130, 2, 0, 2, None),
    (1000, 5, 0, 3, 0, None),
    (1000, 6, 0, 0, 3, "int"),
    (4099, 33, 17, 3, 2, "uniform"),
]


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


def _check(ctx, pr, th, rtol_l=1e-12, grad_tol=1e-12, p_atol=1e-13):
    dp = device_problem(pr)
    l, g, P = ctx.loglik_grad(dp, theta_tensor(th), want_P=True)
    l = float(l.cpu()[0])
    g = g.cpu().numpy()
    P = P.cpu().numpy()
    l_ref = R.loglik(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    g_ref = R.gradient(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    P_ref = R.probabilities(R.normalized_utility(th, pr.X, pr.Y, pr.Z))
    assert abs(l - l_ref) <= rtol_l * abs(l_ref), (l, l_ref)
    err = np.abs(g - g_ref) / grad_scale(pr)
    assert err.max() <= grad_tol, (err.max(), int(err.argmax()))
    np.testing.assert_allclose(P, P_ref, rtol=0, atol=p_atol)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", SHAPES)
def test_pass_matches_oracle(ctx, shape):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=100 + N, weights=wk)
    for sd in (0.0, 0.7):
        th = np.random.default_rng(N).normal(0, sd, pr.n_params)
        _check(ctx, pr, th)


def test_pass_large_utilities(ctx):
    # near-separable regime: utilities far above exp()'s range
    pr = synth.make_problem(500, 9, 4, 1, 1, seed=7)
    th = np.random.default_rng(3).normal(0, 60.0, pr.n_params)
    _check(ctx, pr, th, p_atol=1e-12)


def test_pass_is_deterministic(ctx):
    import torch
    pr = synth.make_problem(20000, 12, 6, 2, 1, seed=9, weights="uniform")
    dp = device_problem(pr)
    th = theta_tensor(np.random.default_rng(1).normal(0, 0.4, pr.n_params))
    l1, g1, _ = ctx.loglik_grad(dp, th)
    l2, g2, _ = ctx.loglik_grad(dp, th)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5"])
def test_pass_config_sizes(ctx, name):
    pr = synth.make_config(name)
    th = pr.theta_true * 0.5
    _check(ctx, pr, th)


# Shapes whose kernels stage each observation's y rows through LDS one
# observation ahead (two workgroups per CU, eight value slots, K g even):
# several tiles per workgroup with a ragged last tile, K past one and past
# two waves, with and without Z; and one with K g odd, which reads y from
# global memory instead.
LDS_ROW_SHAPES = [
    (9001, 60, 40, 5, 0, "uniform"),
    (20011, 100, 51, 6, 0, None),
    (5000, 40, 60, 5, 3, "uniform"),
    (3000, 130, 20, 1, 5, None),
    (9003, 61, 40, 5, 2, None),
]


@pytest.mark.parametrize("shape", LDS_ROW_SHAPES)
def test_pass_staged_rows(ctx, shape):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=200 + K, weights=wk)
    th = np.random.default_rng(K).normal(0, 0.3, pr.n_params)
    _check(ctx, pr, th)


def test_pass_staged_rows_match_global_reads(ctx):
    # Y 8 bytes off a 16-byte boundary takes the kernel that reads the y
    # rows from global memory; the staged kernel does the same arithmetic
    # in the same order, so both give the same bits
    import torch
    import paper_1404_3177_amd as mnl
    pr = synth.make_problem(9001, 60, 40, 5, 0, seed=31, weights="uniform")
    dp = device_problem(pr)
    X, Y, Z, ch, w = dp._refs
    assert Y.data_ptr() % 16 == 0
    buf = torch.empty(Y.numel() + 1, dtype=torch.float64, device=Y.device)
    Ym = buf[1:].view(Y.shape)
    Ym.copy_(Y)
    assert Ym.is_contiguous() and Ym.data_ptr() % 16 == 8
    dm = mnl.Problem(X, Ym, Z, ch, w)
    th = theta_tensor(np.random.default_rng(5).normal(0, 0.3, pr.n_params))
    l1, g1, P1 = ctx.loglik_grad(dp, th, want_P=True)
    l2, g2, P2 = ctx.loglik_grad(dm, th, want_P=True)
    assert torch.equal(l1, l2) and torch.equal(g1, g2) and torch.equal(P1, P2)
