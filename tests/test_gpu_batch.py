"""Batched small fits (mnl_fit_batch, one workgroup per fit over a device
work list) against the FP64 oracle (Sec. 3.1 iteration: Eqs. 2-6, 9-10
and the halving line search): l and ||g|| at the start, the first Newton
step, whole fits, the degenerate stops, bitwise independence of each
result from the rest of the batch, and the entry point's errors."""
import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem, grad_scale

pytestmark = pytest.mark.gpu

GTOL = 1e-8

# N, K, p, g, a, weights: chunk tails (N not a multiple of the 16-, 32- or
# 64-observation chunks), N below one chunk, K = 2 (two lanes per
# observation) and K = 64 (one wave), wide p, p = 0, Z-only, g = 8, and the
# 2,000-observation, 10-alternative fit of 55 coefficients
CASES = [
    (2000, 10, 6, 1, 0, None), (37, 3, 2, 0, 0, None),
    (1000, 2, 5, 0, 0, None), (3001, 17, 3, 2, 1, "uniform"),
    (500, 64, 1, 1, 0, None), (800, 5, 31, 0, 0, None),
    (1200, 4, 0, 3, 2, None), (999, 9, 4, 0, 3, "int"),
    (1500, 3, 1, 0, 40, None), (1000, 8, 4, 8, 0, "uniform"),
]


def problems():
    return [synth.make_problem(N, K, p, g, a, seed=7100 + i, weights=wk)
            for i, (N, K, p, g, a, wk) in enumerate(CASES)]


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


@pytest.fixture(scope="module")
def probs():
    prs = problems()
    return prs, [device_problem(pr) for pr in prs]


def _fit(ctx, dps, **opts):
    thetas, infos = ctx.fit_batch(dps, opts=dict(gtol=GTOL, ftol=0.0, **opts))
    return [t.cpu().numpy() for t in thetas], infos


def test_every_case_is_within_the_batched_limits():
    import paper_1404_3177_amd as mnl
    for N, K, p, g, a, _ in CASES:
        assert mnl.batch_eligible(N, K, p, g, a, gtol=GTOL, ftol=0.0)


def test_start_values_match_the_oracle(ctx, probs):
    # maxiter = 0: theta stays at zero, l and ||g|| are those at theta = 0
    prs, dps = probs
    thetas, infos = _fit(ctx, dps, maxiter=0)
    for pr, th, info in zip(prs, thetas, infos):
        z = np.zeros(pr.n_params)
        l = R.loglik(z, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
        g = R.gradient(z, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
        assert info["stop_reason"] == R.STOP_MAXITER and info["iters"] == 0
        assert not th.any()
        assert abs(info["loglik"] - l) <= 1e-12 * abs(l), pr.name
        gn = np.linalg.norm(g)
        # entries of N-term sums, each within N eps of its term scale
        assert abs(info["grad_norm"] - gn) <= \
            1e-12 * np.linalg.norm(grad_scale(pr)), pr.name


def test_first_newton_step_matches_the_oracle(ctx, probs):
    prs, dps = probs
    thetas, infos = _fit(ctx, dps, maxiter=1)
    for pr, th, info in zip(prs, thetas, infos):
        ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0,
                                                  maxiter=1))
        assert info["iters"] == ref.iters == 1, pr.name
        assert info["ls_iters"] == ref.ls_iters, pr.name
        err = np.linalg.norm(th - ref.theta) / np.linalg.norm(ref.theta)
        assert err <= 1e-10, (pr.name, err)
        assert abs(info["loglik"] - ref.loglik) <= 1e-12 * abs(ref.loglik)
        assert abs(info["loglik_diff"] - ref.loglik_diff) <= \
            1e-9 * abs(ref.loglik_diff) + 1e-12 * abs(ref.loglik)


def test_fits_match_the_oracle(ctx, probs):
    prs, dps = probs
    thetas, infos = _fit(ctx, dps)
    for pr, th, info in zip(prs, thetas, infos):
        ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0))
        assert info["stop_reason"] == ref.stop_reason == R.STOP_GTOL, pr.name
        assert info["iters"] == ref.iters, pr.name
        assert info["n_hess"] == ref.iters
        assert info["n_pass"] == 1 + info["ls_iters"]
        err = np.linalg.norm(th - ref.theta) / np.linalg.norm(ref.theta)
        assert err <= 1e-8, (pr.name, err)
        assert abs(info["loglik"] - ref.loglik) <= 1e-12 * abs(ref.loglik)
        assert info["grad_norm"] <= GTOL


def test_fits_agree_with_the_multi_kernel_path(ctx, probs):
    import paper_1404_3177_amd as mnl
    prs, dps = probs
    thetas, infos = _fit(ctx, dps)
    for pr, dp, th, info in zip(prs, dps, thetas, infos):
        try:
            ref, rinfo = ctx.fit(dp, gtol=GTOL, ftol=0.0)
        except mnl.MnlError as e:
            # the fused pass takes a + g <= 16 per alternative; the batched
            # kernel stages whole observations and has no such cap
            assert e.code == -7 and pr.a + pr.g > 16, pr.name
            continue
        ref = ref.cpu().numpy()
        assert info["iters"] == rinfo["iters"], pr.name
        err = np.linalg.norm(th - ref) / np.linalg.norm(ref)
        assert err <= 1e-8, (pr.name, err)


def test_each_result_is_bitwise_independent_of_the_batch(ctx, probs):
    prs, dps = probs
    alone = [_fit(ctx, [dp]) for dp in dps]
    fwd = _fit(ctx, dps)
    rev = _fit(ctx, dps[::-1])
    # more fits than workgroups: replicas land on different workgroups
    # and in different orders of the work list
    idx = [i % len(dps) for i in range(7 * 97)]
    big = _fit(ctx, [dps[i] for i in idx])
    for i in range(len(dps)):
        th, info = alone[i][0][0], alone[i][1][0]
        j = len(dps) - 1 - i
        for t2, i2 in ((fwd[0][i], fwd[1][i]), (rev[0][j], rev[1][j])):
            assert np.array_equal(t2, th)
            for k in ("iters", "ls_iters", "stop_reason", "loglik",
                      "grad_norm"):
                assert i2[k] == info[k], k
    for r, i in enumerate(idx):
        assert np.array_equal(big[0][r], alone[i][0][0])


def test_warm_start_at_the_oracle_estimate_stops_at_once(ctx, probs):
    import torch
    prs, dps = probs
    refs = [R.fit_problem(pr, opts=R.FitOptions(gtol=1e-9, ftol=0.0))
            for pr in prs[:3]]
    th0 = [torch.from_numpy(r.theta).cuda() for r in refs]
    thetas, infos = ctx.fit_batch(dps[:3], theta0s=th0,
                                  opts=dict(gtol=1e-7, ftol=0.0))
    for r, t, info in zip(refs, thetas, infos):
        assert info["iters"] == 0 and info["stop_reason"] == R.STOP_GTOL
        assert np.array_equal(t.cpu().numpy(), r.theta)


def test_degenerate_stops_match_the_oracle(ctx):
    # a column of zeros makes -H singular (pivot exactly 0: NOT_PD at the
    # first factorisation); a NaN in the data makes l non-finite at once
    zero = synth.make_problem(400, 4, 3, 0, 0, seed=7201)
    zero.X = zero.X.copy()
    zero.X[:, 2] = 0.0
    nan = synth.make_problem(300, 3, 2, 1, 0, seed=7202)
    nan.Y = nan.Y.copy()
    nan.Y[17, 1, 0] = np.nan
    ok = synth.make_problem(350, 5, 2, 0, 0, seed=7203)
    prs = [zero, nan, ok]
    thetas, infos = _fit(ctx, [device_problem(pr) for pr in prs])
    for pr, th, info in zip(prs, thetas, infos):
        ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0))
        assert info["stop_reason"] == ref.stop_reason, pr.name
        assert info["iters"] == ref.iters
    assert infos[0]["stop_reason"] == R.STOP_NOT_PD and not thetas[0].any()
    assert infos[1]["stop_reason"] == R.STOP_NONFINITE
    assert infos[2]["stop_reason"] == R.STOP_GTOL


def test_ftol_and_maxiter_rules(ctx, probs):
    prs, dps = probs
    thetas, infos = _fit(ctx, dps[:4], maxiter=3)
    for pr, th, info in zip(prs, thetas, infos):
        ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0,
                                                  maxiter=3))
        assert info["stop_reason"] == ref.stop_reason
        assert info["iters"] == ref.iters
    thetas, infos = ctx.fit_batch(dps[:4], opts=dict(gtol=0.0, ftol=1e-3))
    for pr, info in zip(prs, infos):
        ref = R.fit_problem(pr, opts=R.FitOptions(gtol=0.0, ftol=1e-3))
        assert info["stop_reason"] == ref.stop_reason == R.STOP_FTOL
        assert info["iters"] == ref.iters


def test_errors(ctx, probs):
    import paper_1404_3177_amd as mnl
    _, dps = probs
    assert ctx.fit_batch([]) == ([], [])
    with pytest.raises(mnl.MnlError, match="UNSUPPORTED"):
        ctx.fit_batch(dps[:2], opts=dict(prec="bf16"))
    with pytest.raises(mnl.MnlError, match="UNSUPPORTED"):
        ctx.fit_batch(dps[:1], opts=dict(method="newton-cg"))
    wide = device_problem(synth.make_problem(50, 65, 1, 0, 0, seed=7301))
    with pytest.raises(mnl.MnlError, match="UNSUPPORTED"):
        ctx.fit_batch([dps[0], wide])
