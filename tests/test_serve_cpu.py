"""Admission rules of the serving scheduler (no GPU): budget, FIFO order,
folding of equal shapes, cancellation, a simulated run in which the bytes
in flight never exceed the budget, and the serving loop on the host clock."""
import random
import time

import pytest

from paper_2405_02603_amd.serve import Job, Scheduler, Server, percentile, request_bytes


def _job(rid, n=32, greens="vico_dct", nbytes=100, spot=False, t=0.0):
    return Job(rid=rid, t_arrival=t, n=n, greens=greens, nbytes=nbytes, spot_check=spot)


def test_request_bytes():
    assert request_bytes(32, "f32", 1000) == 2 * 32 ** 3 * 4 + 1000
    assert request_bytes(32, "f64", 0) == 2 * 32 ** 3 * 8


def test_rejects_job_larger_than_budget():
    s = Scheduler(budget_bytes=1000, slots=2)
    j = _job(1, nbytes=1001)
    assert not s.submit(j)
    assert j.status == "rejected" and "budget" in j.error
    assert s.admit(0.0) == []


def test_fifo_head_blocks_later_jobs():
    s = Scheduler(budget_bytes=1000, slots=4)
    s.submit(_job(1, nbytes=600))
    s.submit(_job(2, n=48, nbytes=600))   # does not fit beside job 1
    s.submit(_job(3, n=64, nbytes=100))   # would fit, but must not overtake job 2
    got = s.admit(0.0)
    assert [[j.rid for j in g] for _, g in got] == [[1]]
    assert s.in_use == 600
    s.complete(got[0][0], 1.0)
    got = s.admit(1.0)
    assert [[j.rid for j in g] for _, g in got] == [[2], [3]]


def test_folds_equal_shapes_into_one_launch():
    s = Scheduler(budget_bytes=10_000, slots=2, max_fold=3)
    for rid in range(5):
        s.submit(_job(rid, n=32, nbytes=100))
    s.submit(_job(9, n=64, nbytes=100))
    got = s.admit(0.0)
    assert [[j.rid for j in g] for _, g in got] == [[0, 1, 2], [3, 4]]
    assert [j.rid for j in s.queue] == [9]


def test_spot_checks_are_not_folded():
    s = Scheduler(budget_bytes=10_000, slots=4)
    s.submit(_job(0, spot=True))
    s.submit(_job(1))
    got = s.admit(0.0)
    assert [[j.rid for j in g] for _, g in got] == [[0], [1]]


def test_cancel_queued():
    s = Scheduler(budget_bytes=1000, slots=1)
    s.submit(_job(1, nbytes=900))
    s.submit(_job(2, nbytes=900))
    s.admit(0.0)
    assert s.cancel(2)
    assert not s.cancel(1)  # running jobs are not cancellable
    assert list(s.queue) == []


def test_simulated_run_respects_budget():
    rnd = random.Random(7)
    budget = 5000
    s = Scheduler(budget_bytes=budget, slots=3, max_fold=4)
    jobs = [_job(i, n=rnd.choice([32, 48, 64]), nbytes=rnd.randint(100, 2500), t=i * 0.01) for i in range(200)]
    for j in jobs:
        s.submit(j)
    t = 0.0
    running = []
    while s.queue or s.busy:
        for slot, g in s.admit(t):
            running.append((t + 0.05 * len(g), slot))
        assert s.in_use <= budget
        running.sort()
        t, slot = running.pop(0)
        s.complete(slot, t)
    assert all(j.status == "done" for j in jobs)
    assert s.peak_bytes <= budget
    assert s.in_use == 0


def test_failed_launch_frees_bytes():
    s = Scheduler(budget_bytes=1000, slots=1)
    s.submit(_job(1, nbytes=800))
    (slot, group), = s.admit(0.0)
    s.complete(slot, 0.5, failed="FSP_ERR_OUT_OF_MEMORY")
    assert group[0].status == "failed" and s.in_use == 0
    s.submit(_job(2, nbytes=800))
    assert len(s.admit(1.0)) == 1


def test_percentile():
    assert percentile([1, 2, 3, 4], 50) == pytest.approx(2.5)
    assert percentile([5], 99) == 5


class _HostExecutor:
    """Executor stand-in on the host clock: a launch finishes ``service`` seconds later."""

    def __init__(self, service=0.002):
        self.service = service
        self.inflight = {}
        self.t0 = None

    def size_job(self, job):
        job.nbytes = 1 << 20

    def start_clock(self):
        self.t0 = time.perf_counter()
        return self.t0

    def now(self):
        return time.perf_counter() - self.t0

    def launch(self, slot, group):
        self.inflight[slot] = self.now() + self.service

    def poll(self):
        now = self.now()
        out = [(s, t) for s, t in self.inflight.items() if t <= now]
        for s, _ in out:
            del self.inflight[s]
        return out


def test_server_loop_on_host_clock():
    """The serving loop end to end: every request completes no earlier than its arrival plus the
    service time, completions are seen after they happen, and the budget and slots hold."""
    ex = _HostExecutor(service=0.002)
    srv = Server(ex, budget_bytes=3 << 20, slots=2)
    jobs = [_job(i, n=32, t=0.004 * i + (0.001 if i % 3 else 0.0)) for i in range(40)]
    rep = srv.run(jobs)
    assert rep["done"] == 40 and rep["rejected"] == 0
    assert rep["peak_bytes"] <= 3 << 20
    for j in jobs:
        assert j.t_done - j.t_arrival >= 0.002 - 1e-9
        assert j.t_seen >= j.t_done
    assert rep["seen_lag_ms"]["min"] >= 0.0
    assert rep["p99_ms"] >= rep["p50_ms"] >= 2.0
