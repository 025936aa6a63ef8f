"""The entry point that allocates nothing, mnl_loglik_grad_noalloc, called
through the C ABI: the same results as mnl_loglik_grad, bitwise (same
kernels and partitions), on two calls in a row, the second with a smaller
input; the context's workspace does not grow; a shape whose scratch exceeds
the static buffer is refused before anything runs."""
import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem, grad_scale, theta_tensor

pytestmark = pytest.mark.gpu


def test_noalloc_pass_equals_the_allocating_pass():
    import torch
    import paper_1404_3177_amd as mnl
    ctx = mnl.Context(0)
    shapes = [(30000, 20, 9, 3, 2, "uniform", 71),
              (1200, 7, 4, 1, 1, None, 72)]   # the second call is smaller
    for N, K, p, g, a, wk, seed in shapes:
        pr = synth.make_problem(N, K, p, g, a, seed=seed, weights=wk)
        dp = device_problem(pr)
        th_np = np.random.default_rng(seed).normal(0, 0.5, pr.n_params)
        th = theta_tensor(th_np)
        ws0 = ctx.workspace_bytes
        l1, g1, P1 = ctx.loglik_grad_noalloc(dp, th, want_P=True)
        torch.cuda.synchronize()
        assert ctx.workspace_bytes == ws0   # nothing allocated in the context
        l0, g0, P0 = ctx.loglik_grad(dp, th, want_P=True)
        torch.cuda.synchronize()
        assert torch.equal(l0, l1) and torch.equal(g0, g1) and \
            torch.equal(P0, P1), (N, K)
        # and the oracle's values (Eqs. 3-5, 9)
        l_ref = R.loglik(th_np, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
        g_ref = R.gradient(th_np, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
        assert abs(float(l1.cpu()[0]) - l_ref) <= 1e-12 * abs(l_ref)
        err = np.abs(g1.cpu().numpy() - g_ref) / grad_scale(pr)
        assert err.max() <= 1e-12, err.max()


def test_noalloc_refuses_shapes_beyond_its_scratch():
    import paper_1404_3177_amd as mnl
    ctx = mnl.Context(0)
    # 699 x 13 = 9,087 coefficients: the pass's partial rows need more than
    # the 32 MiB static buffer
    pr = synth.make_problem(50000, 700, 13, 0, 0, seed=3)
    dp = device_problem(pr)
    th = theta_tensor(np.zeros(pr.n_params))
    with pytest.raises(mnl.MnlError) as ei:
        ctx.loglik_grad_noalloc(dp, th)
    assert ei.value.code == -7 and "scratch" in str(ei.value)
