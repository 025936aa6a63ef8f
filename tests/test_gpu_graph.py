"""Newton steps captured into HIP graphs (opts.graph): the same fits,
bitwise, as the eager path, on a non-default stream."""
import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem, theta_tensor

pytestmark = pytest.mark.gpu
GTOL = 1e-8


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


@pytest.fixture(scope="module")
def stream():
    import torch
    return torch.cuda.Stream()


@pytest.mark.parametrize("shape,prec", [
    ((2000, 10, 6, 1, 0, None), "fp64"),
    ((20000, 12, 6, 2, 1, "uniform"), "fp64"),
    ((5000, 13, 12, 2, 2, "int"), "bf16"),
    ((100000, 50, 21, 5, 5, None), "fp32"),
])
def test_graph_fit_equals_eager_fit(ctx, stream, shape, prec):
    import torch
    N, K, p, g, a, wk = shape
    pr = synth.make_problem(N, K, p, g, a, seed=900 + K, weights=wk)
    dp = device_problem(pr)
    t_e, i_e = ctx.fit(dp, gtol=GTOL, ftol=0.0, prec=prec, graph=0,
                       stream=stream)
    # two graph fits in a row: the graphs of one fit never serve the next
    for _ in range(2):
        t_g, i_g = ctx.fit(dp, gtol=GTOL, ftol=0.0, prec=prec, graph=1,
                           stream=stream)
        stream.synchronize()
        assert torch.equal(t_g, t_e)
        assert (i_g["iters"], i_g["ls_iters"], i_g["stop_reason"]) == \
            (i_e["iters"], i_e["ls_iters"], i_e["stop_reason"])
        # every step after the first was a replay
        assert i_g["graph_steps"] == i_g["iters"] - 1 and \
            i_e["graph_steps"] == 0


def test_default_captures_small_fits_only(ctx, stream):
    # MNL_GRAPH_AUTO (the default): graph steps for n_p <= 512 on a
    # non-default stream, eager steps above, bitwise the eager results
    import torch
    for shape, small in (((2000, 10, 6, 1, 0), True),
                         ((20000, 30, 20, 2, 1), False)):
        pr = synth.make_problem(*shape, seed=950 + shape[1])
        dp = device_problem(pr)
        assert (pr.n_params <= 512) == small
        t_e, i_e = ctx.fit(dp, gtol=GTOL, ftol=0.0, graph=0, stream=stream)
        t_a, i_a = ctx.fit(dp, gtol=GTOL, ftol=0.0, stream=stream)
        stream.synchronize()
        assert torch.equal(t_a, t_e)
        assert i_a["graph_steps"] == (i_a["iters"] - 1 if small else 0)


def test_graph_fit_with_backtracking_matches_oracle(ctx, stream):
    # a far start: line-search halvings run eagerly between replays
    pr = synth.make_problem(3000, 5, 3, 1, 1, seed=43, coef_sd=1.0)
    th0 = np.full(pr.n_params, 2.0)
    ref = R.fit_problem(pr, theta0=th0, opts=R.FitOptions(gtol=GTOL, ftol=0))
    theta, info = ctx.fit(device_problem(pr), theta0=theta_tensor(th0),
                          gtol=GTOL, ftol=0.0, graph=1, stream=stream)
    stream.synchronize()
    assert ref.ls_iters > ref.iters   # backtracking happened
    assert info["iters"] == ref.iters and info["ls_iters"] == ref.ls_iters
    th = theta.cpu().numpy()
    assert np.linalg.norm(th - ref.theta) <= 1e-8 * np.linalg.norm(ref.theta)


def test_graph_option_falls_back_where_it_cannot_capture(ctx, stream):
    import torch
    # the default stream, and a shape on the outer-panel factorisation
    pr = synth.make_problem(1500, 6, 4, 1, 1, seed=44)
    dp = device_problem(pr)
    t_e, _ = ctx.fit(dp, gtol=GTOL, ftol=0.0)
    t_g, i_g = ctx.fit(dp, gtol=GTOL, ftol=0.0, graph=1)
    assert torch.equal(t_e, t_g) and i_g["graph_steps"] == 0
    pr = synth.make_problem(3000, 43, 50, 1, 1, seed=120, weights="uniform")
    dp = device_problem(pr)
    t_e, i_e = ctx.fit(dp, gtol=GTOL, ftol=0.0, maxiter=2, graph=0,
                       stream=stream)
    t_g, i_g = ctx.fit(dp, gtol=GTOL, ftol=0.0, maxiter=2, graph=1,
                       stream=stream)
    stream.synchronize()
    assert torch.equal(t_e, t_g) and i_g["graph_steps"] == 0


def test_graph_fit_with_fp64_retries_equals_eager_fit(ctx, stream):
    # near-separable data: as the probabilities saturate the BF16 Hessian
    # stops being positive definite and the step is redone in FP64 between
    # replays; the retry's larger partials move the workspace, so the
    # captured steps are dropped and captured again
    import torch
    pr = synth.make_problem(20000, 100, 11, 0, 0, seed=5, coef_sd=3.0,
                            weights="int")
    dp = device_problem(pr)
    t_e, i_e = ctx.fit(dp, gtol=GTOL, ftol=0.0, prec="bf16", maxiter=12,
                       graph=0, stream=stream)
    t_g, i_g = ctx.fit(dp, gtol=GTOL, ftol=0.0, prec="bf16", maxiter=12,
                       graph=1, stream=stream)
    stream.synchronize()
    print("fallbacks", i_e["hess_fallbacks"], "graph steps", i_g["graph_steps"],
          "iters", i_e["iters"], flush=True)
    assert i_e["hess_fallbacks"] > 0 and i_g["graph_steps"] > 0
    assert torch.equal(t_g, t_e)
    for k in ("iters", "ls_iters", "stop_reason", "hess_fallbacks", "loglik"):
        assert i_g[k] == i_e[k], k


def test_served_graph_fits_equal_eager_served_fits():
    import paper_1404_3177_amd as mnl
    probs = [synth.make_problem(20000, 100, 11, 0, 0, seed=5, coef_sd=3.0,
                                weights="int"),
             synth.make_problem(1500, 6, 4, 1, 0, seed=45),
             synth.make_problem(4000, 12, 5, 2, 1, seed=46, weights="uniform")]
    hps = [mnl.HostProblem.from_numpy(pr) for pr in probs]
    out = []
    for graph in (0, 1):
        srv = mnl.Server(slots=2)
        try:
            ids = [srv.submit(h, gtol=GTOL, ftol=0.0, prec="bf16", maxiter=12,
                              graph=graph) for h in hps]
            res = {}
            while len(res) < len(ids):
                for r in srv.wait(timeout_ms=60_000):
                    res[r["id"]] = r
            out.append([res[i] for i in ids])
        finally:
            srv.close()
    for r0, r1 in zip(*out):
        assert r0["status"] == 0 and r1["status"] == 0
        assert np.array_equal(r0["theta"], r1["theta"])
        for k in ("iters", "ls_iters", "stop_reason", "hess_fallbacks"):
            assert r0["info"][k] == r1["info"][k], k
    assert out[1][0]["info"]["hess_fallbacks"] > 0
    assert out[1][0]["info"]["graph_steps"] > 0


def test_graph_option_is_ignored_by_newton_cg_and_single_steps(ctx, stream):
    import torch
    pr = synth.make_problem(3000, 8, 5, 1, 1, seed=47, weights="uniform")
    dp = device_problem(pr)
    t_e, i_e = ctx.fit(dp, gtol=GTOL, ftol=0.0, method="newton-cg", graph=0,
                       stream=stream)
    t_g, i_g = ctx.fit(dp, gtol=GTOL, ftol=0.0, method="newton-cg", graph=1,
                       stream=stream)
    stream.synchronize()
    assert torch.equal(t_e, t_g) and i_g["graph_steps"] == 0
    assert i_g["cg_iters"] == i_e["cg_iters"] > 0
    th_e = theta_tensor(np.zeros(pr.n_params))
    th_g = theta_tensor(np.zeros(pr.n_params))
    for _ in range(3):
        s_e = ctx.newton_step(dp, th_e, stream=stream)
        s_g = ctx.newton_step(dp, th_g, stream=stream, graph=1)
        stream.synchronize()
        assert torch.equal(th_e, th_g) and s_g["graph_steps"] == 0
        assert s_e["loglik"] == s_g["loglik"]
