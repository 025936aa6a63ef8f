"""The serving scheduler without a device (host-only mode): admission in
arrival order by memory footprint, slot and budget accounting, requests
joining a running mix, refusal of requests larger than the budget, and the
grouping of small requests into one batched launch (a slot takes the
batch-eligible requests right behind an eligible head, never one further
back)."""
import time

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def mnl():
    import paper_1404_3177_amd as m
    m._lib.load()
    return m


def _requests(mnl, shapes):
    probs = [mnl.HostProblem.from_numpy(
        synth.make_problem(N, K, p, g, 0, seed=10 + i))
        for i, (N, K, p, g) in enumerate(shapes)]
    fps = [mnl.fit_footprint(N, K, p, g, 0) for (N, K, p, g) in shapes]
    return probs, fps


def _drain(srv, n):
    out = []
    while len(out) < n:
        out += srv.wait(max_results=64, timeout_ms=5000.0)
    return sorted(out, key=lambda r: r["id"])


def test_budget_and_slots_bound_the_mix(mnl):
    shapes = [(2000, 6, 4, 1)] * 12
    probs, fps = _requests(mnl, shapes)
    budget = int(2.5 * fps[0])          # two fits at a time by memory
    srv = mnl.Server(slots=4, hbm_budget=budget, host_only=True,
                     host_fit_ms=20.0, max_group=1)
    for pr in probs:
        srv.submit(pr)
    res = _drain(srv, len(probs))
    st = srv.stats()
    assert st["max_running"] == 2 and st["peak_in_use"] <= budget
    assert st["in_use"] == 0 and st["completed"] == len(probs)
    # never more than two admitted intervals overlap
    ev = sorted([(r["t_admit"], 1) for r in res] + [(r["t_done"], -1)
                                                     for r in res])
    cur = peak = 0
    for _, d in ev:
        cur += d
        peak = max(peak, cur)
    assert peak <= 2
    for r in res:
        assert r["status"] == 0 and not r["theta"].any()
        assert r["footprint"] == fps[0]
    srv.close()


def test_admission_is_first_come_first_served(mnl):
    # a large request at the head of the queue is not bypassed by the
    # small ones behind it
    shapes = [(2000, 6, 4, 1), (20000, 30, 12, 3)] + [(2000, 6, 4, 1)] * 5
    probs, fps = _requests(mnl, shapes)
    budget = fps[1] + fps[0] // 2       # the large one only runs alone
    srv = mnl.Server(slots=4, hbm_budget=budget, host_only=True,
                     host_fit_ms=15.0, max_group=1)
    for pr in probs:
        srv.submit(pr)
    res = _drain(srv, len(probs))
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)
    big = res[1]
    for r in res[2:]:
        assert r["t_admit"] >= big["t_done"] - 1e-6
    assert res[0]["t_done"] <= big["t_admit"] + 1e-6
    srv.close()


def test_all_slots_fill_when_memory_allows(mnl):
    shapes = [(1000, 5, 3, 0)] * 16
    probs, fps = _requests(mnl, shapes)
    srv = mnl.Server(slots=5, hbm_budget=100 * fps[0], host_only=True,
                     host_fit_ms=30.0, max_group=1)
    for pr in probs:
        srv.submit(pr)
    _drain(srv, len(probs))
    assert srv.stats()["max_running"] == 5
    srv.close()


def test_requests_join_a_running_mix(mnl):
    shapes = [(1000, 5, 3, 0)] * 4
    probs, fps = _requests(mnl, shapes)
    srv = mnl.Server(slots=2, hbm_budget=10 * fps[0], host_only=True,
                     host_fit_ms=60.0, max_group=1)
    srv.submit(probs[0])
    first = srv.wait(max_results=1, timeout_ms=20.0)
    assert first == []                  # still running
    t_late = srv.now_ms()
    srv.submit(probs[1], t_arrival=t_late)
    res = _drain(srv, 2)
    # the late request was admitted while the first one still ran
    assert res[1]["t_admit"] < res[0]["t_done"]
    assert res[1]["t_arrival"] == t_late
    srv.close()


def test_oversized_request_is_refused(mnl):
    probs, fps = _requests(mnl, [(5000, 8, 5, 1)])
    srv = mnl.Server(slots=2, hbm_budget=fps[0] - 1, host_only=True)
    with pytest.raises(mnl.MnlError) as ei:
        srv.submit(probs[0])
    assert ei.value.code == -2
    srv.close()


def test_host_only_needs_a_budget(mnl):
    with pytest.raises(mnl.MnlError):
        mnl.Server(slots=2, hbm_budget=0, host_only=True)


def test_batch_eligibility(mnl):
    # the 2,000-observation, 10-alternative fit of 55 coefficients
    assert mnl.batch_eligible(2000, 10, 6, 1, 0)
    assert mnl.batch_eligible(2000, 10, 6, 1, 0, gtol=1e-8, ftol=0.0)
    assert not mnl.batch_eligible(2000, 10, 6, 1, 0, prec="bf16")
    assert not mnl.batch_eligible(2000, 10, 6, 1, 0, method="newton-cg")
    assert not mnl.batch_eligible(2000, 10, 6, 1, 0, validate=1)
    assert not mnl.batch_eligible(2000, 65, 1, 0, 0)       # K > 64
    assert not mnl.batch_eligible(2000, 12, 12, 0, 0)      # n_p = 132
    assert mnl.batch_eligible(2000, 12, 10, 0, 1)          # n_p = 122
    assert not mnl.batch_eligible(2000, 12, 11, 0, 1)      # n_p = 133
    # work bound: N n_p^2 <= 2^26
    assert mnl.batch_eligible(2 ** 26 // 55 ** 2, 10, 6, 1, 0)
    assert not mnl.batch_eligible(2 ** 26 // 55 ** 2 + 1, 10, 6, 1, 0)
    assert not mnl.batch_eligible(0, 10, 6, 1, 0)          # invalid shape


def _blocked_queue(mnl, slots, budget_mult, n_small, max_group, fit_ms,
                   extra=()):
    """A slow ineligible request (FP32 Hessian) holds the only slot while
    the queue fills, so the groups that follow depend on the queue alone."""
    shapes = [(1000, 5, 3, 0)] * (1 + n_small)
    probs, fps = _requests(mnl, shapes)
    srv = mnl.Server(slots=slots, hbm_budget=int(budget_mult * fps[0]),
                     host_only=True, host_fit_ms=fit_ms, max_group=max_group)
    srv.submit(probs[0], prec="fp32")
    time.sleep(0.005)
    opts = list(extra) + [{}] * (n_small - len(extra))
    for pr, o in zip(probs[1:], opts):
        srv.submit(pr, **o)
    return srv, len(probs)


def _groups(res):
    g = {}
    for r in res:
        g.setdefault((r["slot"], r["t_admit"]), []).append(r["id"])
    return sorted(g.values())


def test_small_requests_run_in_groups(mnl):
    srv, n = _blocked_queue(mnl, 1, 100, 10, 4, 40.0)
    res = _drain(srv, n)
    # the blocker alone, then groups of consecutive ids of at most 4
    assert _groups(res) == [[0], [1, 2, 3, 4], [5, 6, 7, 8], [9, 10]]
    for r in res:
        assert r["status"] == 0
    # a group's requests finish together
    for grp in _groups(res):
        assert len({res[i]["t_done"] for i in grp}) == 1
    st = srv.stats()
    assert st["max_running"] == 4 and st["in_use"] == 0
    srv.close()


def test_a_group_stops_at_an_ineligible_request(mnl):
    # request 4 asks for a BF16 Hessian: the batched kernel does not take
    # it, so the group ends before it and nothing behind it jumps ahead
    srv, n = _blocked_queue(mnl, 1, 100, 7, 16, 30.0,
                            extra=[{}, {}, {}, {"prec": "bf16"}])
    res = _drain(srv, n)
    assert _groups(res) == [[0], [1, 2, 3], [4], [5, 6, 7]]
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)
    srv.close()


def test_a_group_is_bounded_by_the_budget(mnl):
    # room for three footprints at a time: groups of three, one slot
    srv, n = _blocked_queue(mnl, 1, 3.5, 7, 64, 30.0)
    res = _drain(srv, n)
    assert _groups(res) == [[0], [1, 2, 3], [4, 5, 6], [7]]
    assert srv.stats()["peak_in_use"] <= int(3.5 * res[1]["footprint"])
    srv.close()


def test_max_group_must_not_be_negative(mnl):
    with pytest.raises(mnl.MnlError):
        mnl.Server(slots=2, hbm_budget=1 << 30, host_only=True, max_group=-1)
