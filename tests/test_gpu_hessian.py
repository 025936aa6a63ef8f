"""Parity of the GPU block Hessian (Eq. 10) with the FP64 oracle."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import HESS_TOL, device_problem, hess_scale, theta_tensor

pytestmark = pytest.mark.gpu

SHAPES = [  # N, K, p, g, a, weights
    (37, 4, 3, 2, 2, "uniform"),
    (1, 3, 2, 1, 1, None),
    (2049, 7, 5, 2, 1, None),
    (513, 2, 4, 0, 0, "uniform"),
    (777, 19, 3, 1, 0, "uniform"),
    (300, 30, 2, 0, 2, None),
    (1000, 5, 0, 3, 0, None),
    (1000, 6, 0, 0, 3, "int"),
    (1500, 13, 12, 2, 2, "uniform"),
    (600, 66, 1, 1, 1, None),
    (300, 129, 3, 1, 1, "uniform"),   # many alternatives: blocked pair rows
    (600, 100, 32, 1, 1, "uniform"),  # several beta-beta row and column tiles
    # 128-column tiles with one, two and several observation rounds per
    # tile and ragged last rounds
    (3001, 9, 21, 1, 3, "uniform"),
    (4000, 25, 4, 1, 5, None),
    (20, 9, 21, 1, 3, None),
    (45, 9, 21, 0, 2, "int"),
    # the x rows of the per-alternative sums in their own kernel (many
    # groups of alternatives against little alternative-varying data),
    # ragged rounds and observation ranges
    (2003, 30, 40, 1, 0, None),
    (1001, 30, 40, 1, 1, "uniform"),
    # three B fragments per wave: 128 staged alternatives in 8-wave tiles
    # (every wave's copy slots in use), 4-wave tiles, two row tiles
    (700, 129, 8, 1, 1, "uniform"),
    (1100, 12, 9, 0, 0, None),
    (900, 40, 8, 1, 0, None),
    # FP64 tiles of three A fragments per wave (384 pair rows) and six B
    # fragments: nine row tiles, the last one part padding; ragged rounds
    (3001, 80, 13, 1, 0, None),
    # three A fragments with 128 staged alternatives per row tile: twelve
    # FP32 B fragments would not fit LDS beside them (six are taken), BF16
    # takes twelve
    (300, 129, 19, 1, 1, "uniform"),
]


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


def _chunk_abs(pr, ch):
    """|dU_ik/dtheta| summed over k for one chunk's parameters, [N, size]."""
    kind, k, _, _ = ch
    if kind == "beta":
        return np.abs(pr.X)
    if kind == "gamma":
        return np.abs(pr.Z[:, k, :])
    return np.abs(pr.Y).sum(axis=1)


def _gpu_h(ctx, pr, th, prec):
    dp = device_problem(pr)
    return ctx.hessian(dp, theta_tensor(th), prec=prec).cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_hessian_matches_oracle(ctx, shape, prec):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=200 + N + K, weights=wk)
    th = np.random.default_rng(N + K).normal(0, 0.6, pr.n_params)
    H = _gpu_h(ctx, pr, th, prec)
    H_ref = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    assert np.array_equal(H, H.T)
    err = np.abs(H - H_ref) / hess_scale(pr)
    assert err.max() <= HESS_TOL[prec], (prec, err.max(),
                                         np.unravel_index(err.argmax(), H.shape))


def test_hessians_of_models_sharing_n_k_p_on_one_context(ctx):
    # the beta-beta plan is cached by (N, K, p) and serves models with other
    # generic / alternative-specific variables: each Hessian is laid out
    # with its own n_p
    base = synth.make_problem(4000, 6, 4, 2, 1, seed=71, weights="uniform")
    red = dataclasses.replace(base, g=0, Y=np.ascontiguousarray(
        base.Y[:, :, :0]), theta_true=base.theta_true[:-2])
    for pr in (base, red, base):
        th = np.random.default_rng(pr.n_params).normal(0, 0.5, pr.n_params)
        H = _gpu_h(ctx, pr, th, "fp64")
        H_ref = R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
        err = np.abs(H - H_ref) / hess_scale(pr)
        assert err.max() <= HESS_TOL["fp64"], (pr.n_params, err.max())


def test_hessian_deterministic(ctx):
    import torch
    pr = synth.make_problem(30000, 11, 7, 2, 2, seed=5, weights="uniform")
    dp = device_problem(pr)
    th = theta_tensor(np.random.default_rng(2).normal(0, 0.3, pr.n_params))
    h1 = ctx.hessian(dp, th)
    h2 = ctx.hessian(dp, th)
    assert torch.equal(h1, h2)


@pytest.fixture(scope="module")
def c2_ref():
    """The oracle's Eq. 10 Hessian of the 100,000-observation workload at
    half the true coefficients, and the per-entry bound of its terms."""
    pr = synth.make_config("c2")
    th = 0.5 * pr.theta_true
    return pr, th, R.hessian(th, pr.X, pr.Y, pr.Z, pr.choice, pr.w), \
        hess_scale(pr)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_hessian_c2_full(ctx, c2_ref, prec):
    pr, th, H_ref, S = c2_ref
    H = _gpu_h(ctx, pr, th, prec)
    assert np.array_equal(H, H.T)
    if prec == "fp64":
        scale = np.abs(H_ref).max()
        assert np.abs(H - H_ref).max() <= 1e-11 * scale
    err = np.abs(H - H_ref) / S
    assert err.max() <= HESS_TOL[prec], (prec, err.max())


@pytest.mark.parametrize("name,prec", [("c3", "fp64"), ("c5", "fp64"),
                                       ("c3", "fp32"), ("c3", "bf16"),
                                       ("c5", "fp32"), ("c5", "bf16")])
def test_hessian_config_sampled_blocks(ctx, name, prec):
    # full sizes: compare sampled blocks of Eq. 10 computed by the oracle
    # (several observation splits, row tiles closed by the staged
    # alternatives limit at 500 alternatives)
    pr = synth.make_config(name)
    th = 0.5 * pr.theta_true
    H = _gpu_h(ctx, pr, th, prec)
    assert np.array_equal(H, H.T)
    P = R.probabilities(R.normalized_utility(th, pr.X, pr.Y, pr.Z))
    w = np.ones(pr.N) if pr.w is None else pr.w
    chunks = [c for c in R.chunk_list(pr.K, pr.p, pr.g, pr.a) if c[3] > 0]
    rng = np.random.default_rng(0)
    picks = [(0, 0), (0, 1), (len(chunks) - 1, len(chunks) - 1),
             (len(chunks) - 2, len(chunks) - 1)]
    picks += [tuple(sorted(rng.integers(0, len(chunks), 2))) for _ in range(6)]
    last_is_alpha = pr.g > 0
    if last_is_alpha and pr.K > 50:
        # the literal alpha-alpha block of Eq. 10 sums K^2 products of N-row
        # matrices (minutes at this size); it is compared in full at the
        # c2 size and on the small shapes
        a_idx = len(chunks) - 1
        picks = [pk for pk in picks if pk != (a_idx, a_idx)]
    for i, j in picks:
        cn, cm = chunks[i], chunks[j]
        B = R.hessian_block(P, pr.X, pr.Y, pr.Z, w, cn, cm)
        G = H[cn[2]:cn[2] + cn[3], cm[2]:cm[2] + cm[3]]
        if prec == "fp64":
            scale = max(np.abs(B).max(), np.abs(np.diag(H)).max() * 1e-3)
            assert np.abs(G - B).max() <= 1e-11 * scale, (name, prec, cn, cm)
        else:
            # the block's part of the elementwise bound sum_i |term_i|
            S = _chunk_abs(pr, cn).T @ (w[:, None] * _chunk_abs(pr, cm))
            err = np.abs(G - B) / (S + 1e-300)
            assert err.max() <= HESS_TOL[prec], (name, prec, cn, cm, err.max())
