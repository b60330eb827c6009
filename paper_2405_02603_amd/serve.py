"""Continuous-batching request loop for free-space Poisson solves.

Requests (grid size, Green's function, precision) arrive over time.  The
scheduler admits them in arrival order whenever a slot is free and the device
bytes they need (rho, phi and a solve workspace) fit the HBM budget; requests
that arrive while others run are admitted as slots and bytes free up, so their
work overlaps on the device (one HIP stream per slot).  Admitted requests of
the same shape that are waiting together are folded into one batched launch.
The precomputed Green's transforms and the solve plans stay resident between
requests (a cache keyed by kernel, grid, box, alpha and precision).

The scheduler (``Scheduler``) is plain Python and holds no device state, so its
admission rules are tested without a GPU; ``GpuExecutor`` runs admitted work
through the C ABI (``fsp_solve_batched`` per slot launch).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

__all__ = ["Job", "Scheduler", "GpuExecutor", "Server", "request_bytes", "percentile"]


def request_bytes(n: int, prec: str, work_bytes: int) -> int:
    """Device bytes one request holds while in flight: rho, phi and its workspace."""
    s = 8 if prec == "f64" else 4
    return 2 * n * n * n * s + int(work_bytes)


@dataclasses.dataclass
class Job:
    rid: int
    t_arrival: float
    n: int
    greens: str
    prec: str = "f32"
    spot_check: bool = False
    nbytes: int = 0              # filled by the executor's sizing callback
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    t_seen: Optional[float] = None   # host clock when the completion was observed
    status: str = "queued"       # queued | running | done | rejected | cancelled | failed
    error: Optional[str] = None
    spot_rel_l2: Optional[float] = None
    slot: Optional[int] = None

    @property
    def shape_key(self) -> Tuple[int, str, str]:
        return (self.n, self.greens, self.prec)


class Scheduler:
    """FIFO admission under a slot count and a device-byte budget.

    * a job whose own bytes exceed the budget is rejected at submission;
    * the head of the queue is admitted when a slot is free and its bytes fit;
      later jobs never overtake a head that does not fit (no starvation);
    * jobs admitted in one step that share a shape go to one slot together
      (up to ``max_fold``) and are launched as one batched call.
    """

    def __init__(self, budget_bytes: int, slots: int, max_fold: int = 8):
        if budget_bytes <= 0 or slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.max_fold = max(1, int(max_fold))
        self.queue: Deque[Job] = collections.deque()
        self.in_use = 0
        self.busy: Dict[int, List[Job]] = {}
        self.peak_bytes = 0

    def submit(self, job: Job) -> bool:
        if job.nbytes > self.budget:
            job.status = "rejected"
            job.error = f"needs {job.nbytes} bytes, budget {self.budget}"
            return False
        self.queue.append(job)
        return True

    def cancel(self, rid: int) -> bool:
        for j in list(self.queue):
            if j.rid == rid:
                self.queue.remove(j)
                j.status = "cancelled"
                return True
        return False

    def free_slots(self) -> List[int]:
        return [s for s in range(self.slots) if s not in self.busy]

    def admit(self, now: float) -> List[Tuple[int, List[Job]]]:
        """Jobs to launch now, grouped per slot."""
        out = []
        free = self.free_slots()
        while self.queue and free:
            head = self.queue[0]
            if self.in_use + head.nbytes > self.budget:
                break
            slot = free.pop(0)
            group = [self.queue.popleft()]
            self.in_use += head.nbytes
            # fold waiting jobs of the same shape into this launch
            for j in list(self.queue):
                if len(group) >= self.max_fold:
                    break
                if j.shape_key == head.shape_key and not j.spot_check and not head.spot_check \
                        and self.in_use + j.nbytes <= self.budget:
                    self.queue.remove(j)
                    group.append(j)
                    self.in_use += j.nbytes
            for j in group:
                j.status = "running"
                j.t_admit = now
                j.slot = slot
            self.busy[slot] = group
            self.peak_bytes = max(self.peak_bytes, self.in_use)
            out.append((slot, group))
        return out

    def complete(self, slot: int, t_done: float, failed: Optional[str] = None) -> List[Job]:
        group = self.busy.pop(slot)
        for j in group:
            self.in_use -= j.nbytes
            j.t_done = t_done
            j.status = "failed" if failed else "done"
            j.error = failed
        return group


def percentile(values: Sequence[float], q: float) -> float:
    if not values:
        return float("nan")
    v = sorted(values)
    k = (len(v) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


class GpuExecutor:
    """Runs admitted jobs on the GPU: one stream per slot, resident Green's cache.

    ``source_for(job, dtype)`` returns the job's rho as a host tensor of the
    job's shape (pinned memory recommended); it is copied to the device on the
    slot's stream as part of the request.
    """

    def __init__(self, slots: int, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), alpha: float = 1.1,
                 source_for: Optional[Callable] = None, device=None, keep_results: bool = False):
        import torch

        from . import Plan

        self.torch = torch
        self.Plan = Plan
        self.device = torch.device(device if device is not None else "cuda")
        self.lo, self.hi, self.alpha = tuple(lo), tuple(hi), float(alpha)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        # Green's transforms are computed on a stream of their own; every solve that
        # reads one waits for its event first (on the solving slot's stream)
        self.pre_stream = torch.cuda.Stream(device=self.device)
        self.greens_cache: Dict[Tuple, object] = {}
        self.greens_ready: Dict[Tuple, object] = {}
        self.idle_plans: Dict[Tuple, List[object]] = collections.defaultdict(list)
        self.source_for = source_for
        self.keep_results = keep_results
        self.results: Dict[int, object] = {}
        self.inflight: Dict[int, Tuple[object, List[Job], List[object]]] = {}
        self.t0_wall = None
        self.t0_event = None
        self._work_bytes: Dict[Tuple, int] = {}

    # -------------------------------------------------------------- sizing
    def work_bytes(self, n: int, greens: str, prec: str) -> int:
        key = (n, greens, prec)
        if key not in self._work_bytes:
            p = self.Plan(n=n, lo=self.lo, hi=self.hi, greens=greens, prec=prec, alpha=self.alpha, bind=False)
            self._work_bytes[key] = p.work_bytes
            p.close()
        return self._work_bytes[key]

    def size_job(self, job: Job) -> None:
        job.nbytes = request_bytes(job.n, job.prec, self.work_bytes(job.n, job.greens, job.prec))
        if job.spot_check:
            job.nbytes += request_bytes(job.n, "f64", self.work_bytes(job.n, job.greens, "f64"))

    # -------------------------------------------------------------- plans
    def _source_key(self, n, greens, prec):
        return (greens, n, self.lo, self.hi, self.alpha, prec)

    def _source_plan(self, n, greens, prec):
        """The cached plan holding the Green's transform of this shape; on a miss it is
        precomputed on the executor's precompute stream and an event marks its end."""
        torch = self.torch
        key = self._source_key(n, greens, prec)
        p = self.greens_cache.get(key)
        if p is None:
            with torch.cuda.stream(self.pre_stream):
                p = self.Plan(n=n, lo=self.lo, hi=self.hi, greens=greens, prec=prec, alpha=self.alpha,
                              device=self.device, stream=self.pre_stream)
                ev = torch.cuda.Event()
                ev.record(self.pre_stream)
            self.greens_cache[key] = p
            self.greens_ready[key] = ev
        return p

    def _await_greens(self, n, greens, prec, stream) -> None:
        """Make `stream` wait until the Green's transform of this shape is computed."""
        self._source_plan(n, greens, prec)
        stream.wait_event(self.greens_ready[self._source_key(n, greens, prec)])

    def warm(self, shapes: Sequence[Tuple[int, str, str]]) -> None:
        """Precompute the Green's transforms of the given (n, greens, prec) shapes."""
        for n, g, pr in shapes:
            self._source_plan(n, g, pr)
        self.torch.cuda.synchronize(self.device)

    def _plan_for(self, n, greens, prec):
        key = (n, greens, prec)
        if self.idle_plans[key]:
            return self.idle_plans[key].pop()
        src = self._source_plan(n, greens, prec)
        p = self.Plan(n=n, lo=self.lo, hi=self.hi, greens=greens, prec=prec, alpha=self.alpha,
                      device=self.device, precompute=False)
        p.share_ghat(src)
        return p

    # -------------------------------------------------------------- clock
    def start_clock(self) -> float:
        """Zero of both clocks.  An event recorded on an idle stream may carry the
        time stamp of that stream's last finished command, so a tiny kernel runs
        right before the start event to give it the current time."""
        torch = self.torch
        torch.cuda.synchronize(self.device)
        stream = torch.cuda.current_stream(self.device)
        self.t0_event = torch.cuda.Event(enable_timing=True)
        tick = torch.zeros(1, device=self.device)
        tick.add_(1.0)
        self.t0_event.record(stream)
        torch.cuda.synchronize(self.device)
        self.t0_wall = time.perf_counter()
        return self.t0_wall

    def now(self) -> float:
        return time.perf_counter() - self.t0_wall

    # -------------------------------------------------------------- launches
    def launch(self, slot: int, group: List[Job]) -> None:
        from . import solve_batched

        torch = self.torch
        st = self.streams[slot]
        prec = group[0].prec
        dt = torch.float64 if prec == "f64" else torch.float32
        plans, rhos, outs, held = [], [], [], []
        with torch.cuda.stream(st):
            for j in group:
                plan = self._plan_for(j.n, j.greens, prec)
                self._await_greens(j.n, j.greens, prec, st)
                host = self.source_for(j, dt)
                rho = host.to(self.device, non_blocking=True)
                plans.append(plan)
                rhos.append(rho)
                outs.append(torch.empty_like(rho))
            solve_batched(plans, rhos, outs, stream=st)
            held = [plans, rhos, outs]
            if group[0].spot_check:
                j = group[0]
                p64 = self._plan_for(j.n, j.greens, "f64")
                self._await_greens(j.n, j.greens, "f64", st)
                r64 = rhos[0].double()
                o64 = p64.solve(r64, stream=st)
                diff = torch.linalg.vector_norm((outs[0].double() - o64).flatten())
                den = torch.linalg.vector_norm(o64.flatten())
                held += [[p64], r64, o64, diff, den]
            done = torch.cuda.Event(enable_timing=True)
            done.record(st)
        self.inflight[slot] = (done, group, held)

    def poll(self) -> List[Tuple[int, float]]:
        """(slot, completion time in seconds since start) of launches that finished."""
        out = []
        for slot, (ev, group, held) in list(self.inflight.items()):
            if ev.query():
                t = self.t0_event.elapsed_time(ev) / 1e3  # GPU clock, seconds since start
                plans, rhos, outs = held[0], held[1], held[2]
                if group[0].spot_check and len(held) > 3:
                    diff, den = held[-2], held[-1]
                    group[0].spot_rel_l2 = float(diff / den)
                    self.idle_plans[(group[0].n, group[0].greens, "f64")].append(held[3][0])
                for j, p, o in zip(group, plans, outs):
                    self.idle_plans[(j.n, j.greens, j.prec)].append(p)
                    if self.keep_results:
                        self.results[j.rid] = o
                del self.inflight[slot]
                out.append((slot, t))
        return out

    def idle(self) -> bool:
        return not self.inflight


class Server:
    """Drive a Scheduler and an executor over a timed stream of requests."""

    def __init__(self, executor, budget_bytes: int, slots: int, max_fold: int = 8):
        self.ex = executor
        self.sched = Scheduler(budget_bytes, slots, max_fold)
        self.jobs: List[Job] = []

    def run(self, jobs: Sequence[Job], time_scale: float = 1.0, max_wall: float = 600.0) -> Dict:
        """Serve ``jobs`` (sorted by t_arrival); arrival times are scaled by time_scale."""
        for j in jobs:
            self.ex.size_job(j)
        pending = collections.deque(sorted(jobs, key=lambda j: j.t_arrival))
        self.jobs = list(pending)
        self.ex.start_clock()
        launches = 0
        while pending or self.sched.queue or self.sched.busy:
            now = self.ex.now()
            if now > max_wall:
                break
            while pending and pending[0].t_arrival * time_scale <= now:
                j = pending.popleft()
                j.t_arrival *= time_scale
                self.sched.submit(j)
            for slot, t in self.ex.poll():
                seen = self.ex.now()
                for j in self.sched.complete(slot, t):
                    j.t_seen = seen
            for slot, group in self.sched.admit(now):
                self.ex.launch(slot, group)
                launches += 1
            if not self.sched.busy and not self.sched.queue and pending:
                wait = pending[0].t_arrival * time_scale - self.ex.now()
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif self.sched.busy:
                time.sleep(0.0001)
        return self.report(launches)

    def report(self, launches: int) -> Dict:
        done = [j for j in self.jobs if j.status == "done"]
        lat = [(j.t_done - j.t_arrival) * 1e3 for j in done]
        span = (max(j.t_done for j in done) - min(j.t_arrival for j in done)) if done else float("nan")
        spots = [j.spot_rel_l2 for j in done if j.spot_rel_l2 is not None]
        # host time at which a completion was seen minus its device time: small and
        # non-negative when the two clocks share their zero
        seen_lag = [(j.t_seen - j.t_done) * 1e3 for j in done if j.t_seen is not None]
        return {
            "requests": len(self.jobs),
            "done": len(done),
            "rejected": sum(j.status == "rejected" for j in self.jobs),
            "launches": launches,
            "p50_ms": percentile(lat, 50),
            "p99_ms": percentile(lat, 99),
            "mean_ms": sum(lat) / len(lat) if lat else float("nan"),
            "solves_per_s": len(done) / span if done else 0.0,
            "peak_bytes": self.sched.peak_bytes,
            "budget_bytes": self.sched.budget,
            "spot_checks": len(spots),
            "spot_rel_l2_max": max(spots) if spots else None,
            "seen_lag_ms": {"min": min(seen_lag), "p50": percentile(seen_lag, 50),
                            "max": max(seen_lag)} if seen_lag else None,
        }
