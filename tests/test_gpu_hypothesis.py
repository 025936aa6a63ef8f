"""Parity of the hypothesis tests (covariance blocks, quadratic forms and
the four statistics) with the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem, hess_scale, theta_tensor

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


@pytest.mark.parametrize("shape", [(3000, 7, 5, 2, 1, None),
                                   (5000, 13, 12, 2, 2, "int"),
                                   (3000, 43, 50, 1, 1, "uniform")])
def test_covariance_matches_oracle(ctx, shape):
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=700 + K, weights=wk)
    th = 0.8 * pr.theta_true
    H = R.hessian(th, pr.X, pr.Y, pr.Z, None, pr.w)
    Zr = np.linalg.inv(-H)
    rng = np.random.default_rng(K)
    idx = np.sort(rng.choice(pr.n_params, size=min(40, pr.n_params),
                             replace=False))
    V = ctx.covariance(device_problem(pr), theta_tensor(th), idx).cpu().numpy()
    assert np.array_equal(V, V.T)
    # first order: |dZ_ab| <= ||Z e_a|| ||Z e_b|| ||dA||
    n = pr.n_params
    dA = 1e-12 * np.linalg.norm(hess_scale(pr)) + n * EPS * np.linalg.norm(-H, 2)
    cn = np.linalg.norm(Zr, axis=0)[idx]
    bound = 10.0 * np.outer(cn, cn) * dA
    assert np.all(np.abs(V - Zr[np.ix_(idx, idx)]) <= bound), shape
    if n <= 200:
        Vall = ctx.covariance(device_problem(pr), theta_tensor(th)).cpu().numpy()
        cn = np.linalg.norm(Zr, axis=0)
        assert np.all(np.abs(Vall - Zr) <= 10.0 * np.outer(cn, cn) * dA)


@pytest.mark.parametrize("n", [1, 7, 64, 333, 2100])
def test_quadform_matches_solve(ctx, n):
    import torch
    rng = np.random.default_rng(n)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = (Q * rng.uniform(1.0, 10.0, n)) @ Q.T
    B = 0.1 * np.eye(n)
    x, x0 = rng.normal(size=n), rng.normal(size=n)
    d = x - x0
    ref = d @ np.linalg.solve(A - B, d)
    t = lambda m: torch.from_numpy(np.ascontiguousarray(m)).cuda()
    q = ctx.quadform(t(A), t(x), B=t(B), x0=t(x0))
    assert q == pytest.approx(ref, rel=1e-11 * max(1.0, n / 100))
    # Hessian sign: x^T (-M)^{-1} x with M negative definite
    qh = ctx.quadform(t(-A), t(x), hessian_sign=True)
    assert qh == pytest.approx(x @ np.linalg.solve(A, x),
                               rel=1e-11 * max(1.0, n / 100))


def test_quadform_not_pd(ctx):
    import torch
    import paper_1404_3177_amd as mnl
    A = torch.tensor([[1.0, 2.0], [2.0, 1.0]], dtype=torch.float64).cuda()
    x = torch.ones(2, dtype=torch.float64).cuda()
    with pytest.raises(mnl.MnlError) as ei:
        ctx.quadform(A, x)
    assert ei.value.code == -3


def test_wald_and_score_tests_match_oracle(ctx):
    # every statistic at the oracle's estimates (the GPU fits themselves are
    # compared with those estimates)
    from paper_1404_3177_amd import Problem
    from paper_1404_3177_amd import hypothesis as hyp
    pr = synth.make_problem(4000, 6, 4, 2, 1, seed=71, weights="uniform")
    o = R.FitOptions(gtol=1e-10, ftol=0.0)
    full = R.fit_problem(pr, opts=o)
    rest = R.fit(pr.X, pr.Y[:, :, :0], pr.Z, pr.choice, pr.w, opts=o)
    dp = device_problem(pr)
    theta_g, info = ctx.fit(dp, gtol=1e-10, ftol=0.0)
    assert info["stop_reason"] == R.STOP_GTOL
    assert np.linalg.norm(theta_g.cpu().numpy() - full.theta) <= \
        1e-8 * np.linalg.norm(full.theta)
    th = full.theta
    theta = theta_tensor(th)
    V = R.covariance(th, pr.X, pr.Y, pr.Z, pr.w)
    idx = [1, 5, 9, pr.n_params - 1]
    w, df, p = hyp.waldtest(ctx, dp, theta, idx)
    wr, _, pr_ = R.wald_test(th, V, idx)
    assert df == 4 and w == pytest.approx(wr, rel=1e-9)
    assert p == pytest.approx(pr_, rel=1e-8)
    # single coefficient: z^2 of the summary
    se, z, _ = ctx.summary(dp, theta)
    w1, _, _ = hyp.waldtest(ctx, dp, theta, [3])
    assert w1 == pytest.approx(float(z[3]) ** 2, rel=1e-12)
    # the model without the generic variables, fitted on the same context
    # (its beta-beta plan is the full model's)
    X, Y, Z, c, wt = dp._refs
    red = Problem(X, Y[:, :, :0].contiguous(), Z, c, wt)
    th_r, info_r = ctx.fit(red, gtol=1e-10, ftol=0.0)
    assert info_r["stop_reason"] == R.STOP_GTOL
    assert np.linalg.norm(th_r.cpu().numpy() - rest.theta) <= \
        1e-8 * np.linalg.norm(rest.theta)
    # score test of the generic coefficients at the restricted estimate
    emb = np.concatenate([rest.theta, np.zeros(pr.g)])
    s, df, ps = hyp.scoretest(ctx, dp, theta_tensor(emb), pr.g)
    g = R.gradient(emb, pr.X, pr.Y, pr.Z, pr.choice, pr.w)
    Hr = R.hessian(emb, pr.X, pr.Y, pr.Z, None, pr.w)
    sr, _, psr = R.score_test(g, Hr, pr.g)
    assert s == pytest.approx(sr, rel=1e-8) and ps == pytest.approx(psr, rel=1e-7)
    # likelihood ratio of the same pair of models
    l_full, _, _ = ctx.loglik_grad(dp, theta)
    l_red, _, _ = ctx.loglik_grad(red, theta_tensor(rest.theta))
    lr, _, _ = hyp.lrtest(float(l_full.cpu()[0]), float(l_red.cpu()[0]), pr.g)
    lrr, _, _ = R.lr_test(full.loglik, rest.loglik, pr.g)
    assert lr == pytest.approx(lrr, abs=1e-7)


def test_score_test_two_by_two_is_pearson(ctx):
    import paper_1404_3177_amd as mnl
    from paper_1404_3177_amd import hypothesis as hyp
    rng = np.random.default_rng(41)
    N = 1200
    x = (rng.random(N) < 0.4).astype(float)
    y = (rng.random(N) < 0.25 + 0.15 * x).astype(np.int32)
    X1 = np.column_stack([np.ones(N), x])
    import torch
    E = torch.zeros(N, 2, 0, dtype=torch.float64).cuda()
    full = mnl.Problem(torch.from_numpy(X1).cuda(), E, E,
                       torch.from_numpy(y).cuda())
    rest = mnl.Problem(torch.from_numpy(X1[:, :1].copy()).cuda(), E, E,
                       torch.from_numpy(y).cuda())
    th_r, _ = ctx.fit(rest, gtol=1e-11, ftol=0.0)
    emb = theta_tensor([float(th_r.cpu()[0]), 0.0])
    s, _, _ = hyp.scoretest(ctx, full, emb, 1)
    O = np.array([[np.sum((x == a) & (y == b)) for b in (0, 1)]
                  for a in (0, 1)], dtype=float)
    Ex = O.sum(1, keepdims=True) * O.sum(0, keepdims=True) / O.sum()
    assert s == pytest.approx(float(((O - Ex) ** 2 / Ex).sum()), rel=1e-9)


def _oracle_hm(pr, alts):
    # the coefficients the subset model shares with the full one, in the
    # subset model's Eq. 8 order: beta of its non-base alternatives, gamma
    # of all its alternatives, then alpha
    o = R.FitOptions(gtol=1e-10, ftol=0.0)
    full = R.fit_problem(pr, opts=o)
    m = np.isin(pr.choice, alts)
    lut = -np.ones(pr.K, int)
    lut[alts] = np.arange(len(alts))
    Xs, Ys, Zs = pr.X[m], pr.Y[m][:, alts], pr.Z[m][:, alts]
    sub = R.fit(Xs, Ys, Zs, lut[pr.choice[m]].astype(np.int32), None, opts=o)
    idx = [(j - 1) * pr.p + c for j in alts[1:] for c in range(pr.p)]
    idx += [(pr.K - 1) * pr.p + j * pr.a + c for j in alts
            for c in range(pr.a)]
    idx += [(pr.K - 1) * pr.p + pr.K * pr.a + c for c in range(pr.g)]
    Vf = R.covariance(full.theta, pr.X, pr.Y, pr.Z)[np.ix_(idx, idx)]
    Vs = R.covariance(sub.theta, Xs, Ys, Zs)
    return R.hm_test(sub.theta, Vs, full.theta[idx], Vf)


def test_hmftest_matches_oracle(ctx):
    from paper_1404_3177_amd import hypothesis as hyp
    pr = synth.make_problem(4000, 5, 3, 1, 1, seed=73)
    dp = device_problem(pr)
    theta, _ = ctx.fit(dp, gtol=1e-10, ftol=0.0)
    s, df, p, _, info = hyp.hmftest(ctx, dp, theta, [0, 1, 3], gtol=1e-10,
                                    ftol=0.0)
    sr, dfr, pr_ = _oracle_hm(pr, [0, 1, 3])
    assert info["stop_reason"] == R.STOP_GTOL and df == dfr
    assert s == pytest.approx(sr, rel=1e-6) and p == pytest.approx(pr_, rel=1e-5)


def test_hmftest_indefinite_difference_reported(ctx):
    # V_sub - V_full is indefinite for this sample: NOT_PD, as in the oracle
    import paper_1404_3177_amd as mnl
    from paper_1404_3177_amd import hypothesis as hyp
    pr = synth.make_problem(4000, 5, 3, 1, 1, seed=70)
    dp = device_problem(pr)
    theta, _ = ctx.fit(dp, gtol=1e-10, ftol=0.0)
    with pytest.raises(mnl.MnlError) as ei:
        hyp.hmftest(ctx, dp, theta, [0, 1, 3], gtol=1e-10, ftol=0.0)
    assert ei.value.code == -3


def test_wald_test_two_by_two_is_woolf(ctx):
    # log odds ratio of a 2 x 2 table: (log OR)^2 / (1/a + 1/b + 1/c + 1/d)
    import torch
    import paper_1404_3177_amd as mnl
    from paper_1404_3177_amd import hypothesis as hyp
    rng = np.random.default_rng(45)
    N = 1200
    x = (rng.random(N) < 0.4).astype(float)
    y = (rng.random(N) < 0.25 + 0.15 * x).astype(np.int32)
    X1 = np.column_stack([np.ones(N), x])
    E = torch.zeros(N, 2, 0, dtype=torch.float64).cuda()
    prob = mnl.Problem(torch.from_numpy(X1).cuda(), E, E,
                       torch.from_numpy(y).cuda())
    theta, info = ctx.fit(prob, gtol=1e-12, ftol=0.0)
    O = np.array([[np.sum((x == a) & (y == b)) for b in (0, 1)]
                  for a in (0, 1)], dtype=float)
    lor = np.log(O[1, 1] * O[0, 0] / (O[1, 0] * O[0, 1]))
    w, df, _ = hyp.waldtest(ctx, prob, theta, [1])
    assert float(theta.cpu()[1]) == pytest.approx(lor, rel=1e-10)
    assert w == pytest.approx(lor ** 2 / (1.0 / O).sum(), rel=1e-9)
