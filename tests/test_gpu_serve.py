"""Continuous-batching server on the GPU: served fits against the FP64 oracle,
bitwise identity of each result alone and in a mix (with and without
grouped small fits), admission by device footprint, requests joining a
running mix, and error reports."""
import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem

pytestmark = pytest.mark.gpu

GTOL = 1e-8

# uneven shapes: N, K, p, g, a, weights
MIX = [
    (1500, 6, 4, 1, 0, None), (800, 3, 3, 0, 1, "uniform"),
    (4000, 12, 5, 2, 0, None), (600, 2, 6, 0, 0, None),
    (2500, 9, 3, 1, 2, "uniform"), (3000, 20, 4, 0, 0, None),
    (1200, 5, 2, 2, 1, None), (5000, 7, 7, 1, 0, "uniform"),
    (900, 15, 3, 1, 0, None), (2000, 4, 5, 0, 2, None),
    (3500, 30, 3, 2, 0, None), (700, 8, 4, 1, 1, "uniform"),
]


def problems():
    return [synth.make_problem(N, K, p, g, a, seed=5000 + i, weights=wk)
            for i, (N, K, p, g, a, wk) in enumerate(MIX)]


def serve(probs, slots, prec="fp64", budget=0, max_group=0, **opts):
    import paper_1404_3177_amd as mnl
    srv = mnl.Server(slots=slots, hbm_budget=budget, max_group=max_group)
    try:
        hps = [mnl.HostProblem.from_numpy(pr, pinned=(i % 2 == 0))
               for i, pr in enumerate(probs)]
        ids = [srv.submit(h, gtol=GTOL, ftol=0.0, prec=prec, **opts)
               for h in hps]
        res = {}
        while len(res) < len(ids):
            for r in srv.wait(timeout_ms=60_000):
                res[r["id"]] = r
        return [res[i] for i in ids], srv.stats()
    finally:
        srv.close()


@pytest.fixture(scope="module")
def alone():
    """Each problem fitted on its own (device data): through mnl_fit_batch
    when the server groups such fits, else through mnl_fit."""
    import paper_1404_3177_amd as mnl
    ctx = mnl.Context(0)
    out = []
    for pr in problems():
        dp = device_problem(pr)
        if mnl.batch_eligible(pr.N, pr.K, pr.p, pr.g, pr.a, gtol=GTOL,
                              ftol=0.0):
            th, info = ctx.fit_batch([dp], opts=dict(gtol=GTOL, ftol=0.0))
            theta, info = th[0], info[0]
        else:
            theta, info = ctx.fit(dp, gtol=GTOL, ftol=0.0)
        out.append((theta.cpu().numpy(), info))
    return out


def test_served_fits_match_the_oracle():
    probs = problems()
    res, st = serve(probs, slots=4)
    assert st["completed"] == len(probs) and st["in_use"] == 0
    for pr, r in zip(probs, res):
        ref = R.fit_problem(pr, opts=R.FitOptions(gtol=GTOL, ftol=0.0))
        assert r["status"] == 0
        assert r["info"]["stop_reason"] == ref.stop_reason == R.STOP_GTOL
        assert r["info"]["iters"] == ref.iters
        err = np.linalg.norm(r["theta"] - ref.theta) / np.linalg.norm(ref.theta)
        assert err <= 1e-8, (pr.name, err)


@pytest.mark.parametrize("slots,max_group", [(1, 0), (5, 0), (12, 1),
                                             (3, 4)])
def test_each_result_is_bitwise_the_same_alone_and_in_the_mix(alone, slots,
                                                              max_group):
    res, st = serve(problems(), slots=slots, max_group=max_group)
    if max_group == 1:
        assert st["max_running"] <= slots
    if slots > 1:
        assert st["max_running"] > 1  # the fits did overlap
    for (theta, info), r in zip(alone, res):
        assert r["status"] == 0
        assert np.array_equal(r["theta"], theta)
        for k in ("iters", "ls_iters", "stop_reason", "loglik", "grad_norm"):
            assert r["info"][k] == info[k], k


def test_mixed_precision_served_fits_converge_to_the_fp64_fixed_point(alone):
    res, _ = serve(problems(), slots=6, prec="bf16")
    res2, _ = serve(problems(), slots=2, prec="bf16")
    for (theta, _), r, r2 in zip(alone, res, res2):
        assert r["status"] == 0 and r["info"]["stop_reason"] == R.STOP_GTOL
        err = np.linalg.norm(r["theta"] - theta) / np.linalg.norm(theta)
        assert err <= 1e-6
        assert np.array_equal(r["theta"], r2["theta"])


def test_admission_respects_the_memory_budget():
    import paper_1404_3177_amd as mnl
    probs = problems()
    fps = [mnl.fit_footprint(pr.N, pr.K, pr.p, pr.g, pr.a, "fp64",
                             pr.w is not None) for pr in probs]
    budget = int(2.2 * max(fps))
    res, st = serve(probs, slots=8, budget=budget)
    assert all(r["status"] == 0 for r in res)
    assert st["peak_in_use"] <= budget
    assert [r["footprint"] for r in res] == fps
    # intervals of fits in flight never hold more than the budget
    ev = sorted([(r["t_admit"], r["footprint"]) for r in res] +
                [(r["t_done"], -r["footprint"]) for r in res],
                key=lambda e: (e[0], e[1]))
    cur = 0
    for _, df in ev:
        cur += df
        assert cur <= budget
    # a request larger than the whole budget is refused at submit
    srv = mnl.Server(slots=2, hbm_budget=max(fps) - 1)
    try:
        big = probs[int(np.argmax(fps))]
        with pytest.raises(mnl.MnlError, match="OOM"):
            srv.submit(mnl.HostProblem.from_numpy(big))
    finally:
        srv.close()


def test_requests_join_a_running_mix():
    import paper_1404_3177_amd as mnl
    probs = problems()
    srv = mnl.Server(slots=4, max_group=1)
    try:
        hps = [mnl.HostProblem.from_numpy(pr) for pr in probs]
        first = [srv.submit(h, gtol=GTOL, ftol=0.0) for h in hps[:8]]
        got = srv.wait(max_results=1, timeout_ms=60_000)
        assert len(got) == 1
        late = [srv.submit(h, gtol=GTOL, ftol=0.0) for h in hps[8:]]
        res = {r["id"]: r for r in got}
        while len(res) < len(probs):
            for r in srv.wait(timeout_ms=60_000):
                res[r["id"]] = r
    finally:
        srv.close()
    for r in res.values():
        assert r["status"] == 0
        assert r["t_arrival"] <= r["t_admit"] <= r["t_done"]
    # some late request started while an earlier one was still running
    assert any(res[i]["t_admit"] < res[j]["t_admit"] < res[i]["t_done"]
               for j in late for i in first)


def test_a_failing_request_is_reported_and_the_server_goes_on():
    import paper_1404_3177_amd as mnl
    bad = synth.make_problem(500, 4, 3, 0, 0, seed=77)
    bad.choice = bad.choice.copy()
    bad.choice[10] = 9  # out of range
    good = synth.make_problem(600, 4, 3, 0, 0, seed=78)
    srv = mnl.Server(slots=2)
    try:
        i_bad = srv.submit(mnl.HostProblem.from_numpy(bad), validate=1)
        i_good = srv.submit(mnl.HostProblem.from_numpy(good), gtol=GTOL,
                            ftol=0.0, validate=1)
        res = {}
        while len(res) < 2:
            for r in srv.wait(timeout_ms=60_000):
                res[r["id"]] = r
        assert srv.stats()["in_use"] == 0
    finally:
        srv.close()
    assert res[i_bad]["status"] == -1  # MNL_ERR_ARG
    assert res[i_good]["status"] == 0
    ref = R.fit_problem(good, opts=R.FitOptions(gtol=GTOL, ftol=0.0))
    assert np.linalg.norm(res[i_good]["theta"] - ref.theta) <= \
        1e-8 * np.linalg.norm(ref.theta)
