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


# ------------------------------------------------------------------ resident set
from paper_2405_02603_amd.serve import ResidentSet  # noqa: E402

SIZES = {"a": (100, 50, 400), "b": (200, 50, 400), "c": (300, 50, 400), "d": (100, 50, 900)}


def _res(log=None):
    return ResidentSet(lambda k: SIZES[k[0]], (lambda e, i: log.append((e.key, i))) if log is not None else None)


def test_resident_reserve_release_and_extra_slots():
    r = _res()
    assert r.peek(("a",)) == 550 and r.bytes() == 0
    t1 = r.reserve(("a",))
    assert t1.created and t1.index == 0
    assert r.bytes() == 100 + 50 + 400           # transform, home workspace, refresh transient
    assert r.peek(("a",)) == 50                  # the home plan is busy: one more workspace
    t2 = r.reserve(("a",))
    assert not t2.created and t2.index == 1 and r.bytes() == 100 + 2 * 50 + 400
    r.release(t1)
    assert r.bytes() == 100 + 2 * 50              # the transient ends with the job that carried it
    assert r.peek(("a",)) == 0
    r.release(t2)
    assert r.entries[("a",)].refs == 0 and r.hits == 1 and r.misses == 1


def test_resident_evicts_idle_workspaces_then_lru_entries():
    log = []
    r = _res(log)
    ta, tb, tc = (r.reserve((k,)) for k in "abc")
    ta2 = r.reserve(("a",))                       # an extra workspace for "a"
    for t in (ta, tb, tc, ta2):
        r.release(t)
    r.release(r.reserve(("a",)))                 # touch "a": now most recently used
    assert list(r.entries) == [("b",), ("c",), ("a",)]
    freed = r.evict(10)                          # the idle extra workspace is enough
    assert freed == 50 and log == [(("a",), 1)]
    freed = r.evict(201)                         # then "b" (250) as least recently used
    assert freed == 250 and log[-1] == (("b",), None) and ("b",) not in r.entries
    assert r.evictions == 1


def test_resident_never_evicts_what_a_ticket_uses():
    r = _res()
    t = r.reserve(("c",))
    assert r.evict(10_000) == 0 and ("c",) in r.entries
    r.release(t)
    assert r.evict(10_000) == 350 and not r.entries


def test_scheduler_counts_resident_bytes_in_the_budget():
    r = _res()
    s = Scheduler(budget_bytes=1200, slots=4, resident=r)
    jobs = [Job(rid=i, t_arrival=0.0, n=8, greens="x", nbytes=100, rkeys=((k,),)) for i, k in enumerate("abc")]
    for j in jobs:
        assert s.submit(j)
    got = s.admit(0.0)
    # a: 100 + 550 = 650; b would add 100 + 650 -> 1400 > 1200: it waits, c behind it
    assert [[j.rid for j in g] for _, g in got] == [[0]] and s.held() == 650
    s.complete(got[0][0], 1.0)
    assert s.held() == 150                       # a's transform and home workspace stay resident
    got = s.admit(1.0)
    assert [[j.rid for j in g] for _, g in got] == [[1]] and s.held() == 150 + 100 + 650
    s.complete(got[0][0], 2.0)
    got = s.admit(2.0)                           # c needs 850 beside 400 resident: a is evicted
    assert [[j.rid for j in g] for _, g in got] == [[2]]
    assert ("a",) not in r.entries and r.evictions == 1 and s.held() <= 1200


def test_scheduler_rejects_what_cannot_fit_alone():
    s = Scheduler(budget_bytes=1000, slots=1, resident=_res())
    j = Job(rid=0, t_arrival=0.0, n=8, greens="x", nbytes=100, rkeys=(("d",),))   # 100 + 1050
    assert not s.submit(j) and j.status == "rejected"


def test_simulated_run_with_resident_set_respects_budget():
    rnd = random.Random(11)
    sizes = {}

    def size(key):
        if key not in sizes:
            sizes[key] = (rnd.randint(50, 400), rnd.randint(20, 200), rnd.randint(100, 800))
        return sizes[key]

    r = ResidentSet(size)
    budget = 4000
    s = Scheduler(budget_bytes=budget, slots=3, max_fold=4, resident=r)
    jobs = []
    for i in range(300):
        n = rnd.choice([8, 16])
        box = rnd.randrange(6)                   # boxes change: six extents per grid
        keys = ((n, box, "f32"),) + (((n, box, "f64"),) if i % 17 == 0 else ())
        jobs.append(Job(rid=i, t_arrival=i * 0.01, n=n, greens="x", nbytes=rnd.randint(50, 500), rkeys=keys,
                        spot_check=len(keys) > 1))
    for j in jobs:
        s.submit(j)
    t, running = 0.0, []
    while s.queue or s.busy:
        for slot, g in s.admit(t):
            running.append((t + 0.05 * len(g), slot))
        assert s.held() <= budget
        running.sort()
        t, slot = running.pop(0)
        s.complete(slot, t)
        assert s.held() <= budget
    assert all(j.status == "done" for j in jobs)
    assert s.peak_bytes <= budget and s.in_use == 0 and r.transient == 0
    assert r.evictions > 0 and r.hits > 0
    assert all(e.refs == 0 for e in r.entries.values())


class _FailingExecutor(_HostExecutor):
    """Host stand-in whose second launch fails (as a launch whose plan cannot get its memory)."""

    def __init__(self):
        super().__init__(service=0.001)
        self.launches = 0
        self.errors = {}

    def launch(self, slot, group):
        self.launches += 1
        super().launch(slot, group)
        self.errors[slot] = "FspError: FSP_ERR_OUT_OF_MEMORY" if self.launches == 2 else None

    def poll(self):
        return [(s, t, self.errors.pop(s)) for s, t in super().poll()]


def test_server_keeps_serving_after_a_failed_launch():
    ex = _FailingExecutor()
    srv = Server(ex, budget_bytes=8 << 20, slots=1, max_fold=1)
    jobs = [_job(i, n=32, t=0.002 * i) for i in range(10)]
    rep = srv.run(jobs)
    assert rep["failed"] == 1 and rep["done"] == 9
    assert jobs[1].status == "failed" and "OUT_OF_MEMORY" in jobs[1].error
    assert srv.sched.in_use == 0
