"""Serving scheduler against the fake executor (virtual clock, no GPU):
Poisson request stream, FIFO admission by HBM footprint, slot reuse,
percentile arithmetic, budget exhaustion and cancellation."""
import math

import numpy as np
import pytest

from paper_1401_4350_amd.inputs import Request, WORKLOADS, serving_requests
from paper_1401_4350_amd.serve import FakeExecutor, Report, Scheduler, percentile, summarize


def test_request_stream_is_seeded_and_shaped():
    a = serving_requests(3000, 50.0, seed=0)
    b = serving_requests(3000, 50.0, seed=0)
    c = serving_requests(3000, 50.0, seed=1)
    assert [(r.arrival, r.workload) for r in a] == [(r.arrival, r.workload) for r in b]
    assert [r.workload.n for r in a] != [r.workload.n for r in c]
    n = np.array([r.workload.n for r in a])
    assert n.min() >= 500 and n.max() <= 50000
    # log-uniform: the median sits near the geometric mean of the range
    assert abs(math.log(np.median(n)) - 0.5 * math.log(500 * 50000)) < 0.15
    patchy = np.array([r.workload.pot == "patchy" for r in a])
    assert abs(patchy.mean() - 0.3) < 0.03
    rho = np.array([r.workload.rho for r in a])
    assert rho[patchy].min() >= 0.3 and rho[patchy].max() <= 0.6
    assert rho[~patchy].min() >= 0.6 and rho[~patchy].max() <= 0.9
    t = np.array([r.arrival for r in a])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert (gaps > 0).all()
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0  # Poisson rate
    # exponential gaps: coefficient of variation 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.08
    assert [r.seed for r in a[:3]] == [1, 2, 3]
    assert all(r.workload.steps == 1000 for r in a)
    assert all(r.workload.box > 2 * r.workload.rv for r in a)


@pytest.mark.parametrize("q", [1, 25, 50, 90, 99, 100])
def test_percentile_is_nearest_rank(q):
    rng = np.random.default_rng(q)
    v = rng.exponential(size=137)
    assert percentile(v, q) == np.percentile(v, q, method="inverted_cdf")
    assert percentile([3.0], q) == 3.0
    assert math.isnan(percentile([], q))


def small_stream(count=40, rate=2000.0, steps=200, seed=0):
    reqs = serving_requests(count, rate, seed=seed, steps=steps, n_min=500, n_max=5000)
    return reqs


def foot(req):
    return 1000 + req.workload.n  # a stand-in footprint, bytes


class Watch(FakeExecutor):
    """Records admissions and checks the scheduler's footprint accounting."""

    def __init__(self, budget, **kw):
        super().__init__(footprint=foot, **kw)
        self.budget = budget
        self.in_use = 0
        self.order = []
        self.max_in_use = 0

    def admit(self, req):
        h = super().admit(req)
        if h is not None:
            self.in_use += foot(req)
            assert self.in_use <= self.budget
            self.max_in_use = max(self.max_in_use, self.in_use)
            self.order.append(req.rid)
        return h

    def retire(self, h, cancelled=False):
        self.in_use -= foot(self.req[h])
        return super().retire(h, cancelled)


def test_all_requests_complete_with_slot_reuse():
    reqs = small_stream()
    ex = Watch(budget=10 ** 9, max_systems=4, steps_per_launch=32)
    rep = Scheduler(ex, 10 ** 9, max_slots=4).run(reqs)
    s = summarize(rep)
    assert s["completed"] == len(reqs) and s["rejected"] == 0
    assert rep.peak_active <= 4
    assert ex.order == sorted(ex.order)  # FIFO
    for r in rep.records:
        assert r.arrival <= r.admitted <= r.done
        # each launch advances by at most 32 steps
        assert r.done - r.admitted >= 200 * ex.step_s
    assert 0 < s["p50_s"] <= s["p99_s"]
    lat = [r.done - r.arrival for r in rep.records]
    assert s["p99_s"] == percentile(lat, 99)
    assert s["pair_evals_per_s"] > 0


def test_footprint_budget_limits_concurrency_and_never_crashes():
    reqs = small_stream(count=30)
    budget = max(foot(r) for r in reqs) + 10  # room for about one request at a time
    ex = Watch(budget=budget, max_systems=16)
    rep = Scheduler(ex, budget, max_slots=16).run(reqs)
    s = summarize(rep)
    assert s["completed"] == 30
    assert ex.max_in_use <= budget
    assert rep.peak_bytes <= budget
    # with room for ~one system the runs barely overlap: queueing dominates
    ex2 = Watch(budget=10 ** 9, max_systems=16)
    rep2 = Scheduler(ex2, 10 ** 9, max_slots=16).run(reqs)
    assert summarize(rep2)["p99_s"] < s["p99_s"]
    assert rep2.peak_active > rep.peak_active


def test_request_larger_than_budget_is_rejected():
    reqs = small_stream(count=10)
    big = Request(rid=99, arrival=reqs[2].arrival, workload=WORKLOADS["lj_small"].with_(n=10 ** 6, steps=10),
                  seed=5)
    budget = 10 ** 5
    ex = Watch(budget=budget, max_systems=4)
    rep = Scheduler(ex, budget, max_slots=4).run(reqs + [big])
    by = {r.rid: r for r in rep.records}
    assert by[99].status == "rejected" and "budget" in by[99].error
    assert sum(r.status == "done" for r in rep.records) == 10


def test_cancellation_frees_the_slot():
    w = WORKLOADS["lj_small"].with_(n=1000)
    reqs = [Request(0, 0.0, w.with_(steps=10 ** 6), 1), Request(1, 0.001, w.with_(steps=100), 2)]
    ex = Watch(budget=10 ** 9, max_systems=1)
    rep = Scheduler(ex, 10 ** 9, max_slots=1).run(reqs, cancel={0: 0.01})
    by = {r.rid: r for r in rep.records}
    assert by[0].status == "failed" and by[0].error == "cancelled"
    assert by[1].status == "done" and by[1].admitted >= 0.01
    assert ex.in_use == 0 and not ex.left


def test_fake_launch_sizes_follow_the_batch_rule():
    ex = FakeExecutor(steps_per_launch=64, footprint=foot)
    w = WORKLOADS["lj_small"].with_(n=1000)
    h1 = ex.admit(Request(0, 0.0, w.with_(steps=100), 1))
    h2 = ex.admit(Request(1, 0.0, w.with_(steps=5), 2))
    ex.step()
    assert ex.left[h1] == 36 and ex.left[h2] == 0
    ex.retire(h2)
    ex.step()  # need 36 < 64: 64 rounded down to the power of two covering 36
    assert ex.left[h1] == 0 and ex.steps_run[h1] == 100
