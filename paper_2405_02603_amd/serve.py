"""Continuous-batching request loop for free-space Poisson solves.

Requests (grid size, box, Green's function, precision) arrive over time.  The
scheduler admits them in arrival order whenever a slot is free and the device
bytes they need fit the HBM budget; requests that arrive while others run are
admitted as slots and bytes free up, so their work overlaps on the device (one
HIP stream per slot).  Admitted requests of the same grid, kernel and precision
that are waiting together are folded into one batched launch, whatever their
boxes.

Between requests the device keeps a resident set (``ResidentSet``): one Green's
transform per (kernel, grid, box, alpha, precision), with the plan that
computed it, plus extra plans (workspaces) that share it.  The transform
depends on the grid and on the domain's extents (Section 2.3), so a request
whose box changed (a domain fitted to the particles, Section 1) needs a new
one.  A request whose transform is missing has it computed on a stream of its
own, which its solve waits for; that refresh is timed and reported.  The budget
covers everything held: requests in flight, the resident set, and the float64
transients of refreshes in progress.  When the head of the queue does not fit,
idle workspaces and then transforms that no request is using are evicted,
least recently used first.

``Scheduler`` and ``ResidentSet`` are plain Python and hold no device state, so
their rules are tested without a GPU; ``GpuExecutor`` runs admitted work
through the C ABI (``fsp_solve_batched`` per slot launch).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

__all__ = ["Job", "Scheduler", "ResidentSet", "Ticket", "GpuExecutor", "Server", "request_bytes",
           "field_bytes", "percentile"]


def field_bytes(n: int, prec: str) -> int:
    """Device bytes of one request's rho and phi."""
    s = 8 if prec == "f64" else 4
    return 2 * n * n * n * s


def request_bytes(n: int, prec: str, work_bytes: int) -> int:
    """Device bytes of a request's rho, phi and one solve workspace."""
    return field_bytes(n, prec) + int(work_bytes)


@dataclasses.dataclass
class Job:
    rid: int
    t_arrival: float
    n: int
    greens: str
    prec: str = "f32"
    spot_check: bool = False
    lo: Optional[Tuple[float, float, float]] = None   # box; None: the executor's default
    hi: Optional[Tuple[float, float, float]] = None
    nbytes: int = 0              # bytes the job itself holds (filled by the executor's sizing)
    rkeys: Tuple = ()            # resident-set keys the job reads (filled by the executor)
    tickets: List = dataclasses.field(default_factory=list)
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    t_seen: Optional[float] = None   # host clock when the completion was observed
    status: str = "queued"       # queued | running | done | rejected | cancelled | failed
    error: Optional[str] = None
    spot_rel_l2: Optional[float] = None
    slot: Optional[int] = None
    refreshed: bool = False      # its solve waited for a Green's transform being computed

    @property
    def shape_key(self) -> Tuple[int, str, str]:
        return (self.n, self.greens, self.prec)


# ------------------------------------------------------------------ resident set
@dataclasses.dataclass
class _Entry:
    key: Tuple
    ghat_bytes: int
    work_bytes: int
    pre_bytes: int
    plans: List[Optional[object]] = dataclasses.field(default_factory=list)  # device objects, [0] = home plan
    busy: List[bool] = dataclasses.field(default_factory=list)               # per plan slot
    refs: int = 0                # tickets not yet released
    pending_pre: bool = True     # the transform may still be being computed
    handle: object = None        # executor state: the event that ends the computation

    @property
    def bytes(self) -> int:
        return self.ghat_bytes + self.work_bytes * len(self.busy)


@dataclasses.dataclass
class Ticket:
    """One job's claim on a resident entry: the plan slot it solves with, whether
    its admission created the entry, and the refresh transient it carries
    (counted until the job completes)."""
    entry: _Entry
    index: int
    transient: int
    created: bool


class ResidentSet:
    """Accounting of the device bytes held between requests, with LRU eviction.

    ``sizes(key) -> (ghat_bytes, work_bytes, precompute_bytes)`` sizes an entry;
    ``free(entry, index)`` releases device objects (index None: the whole entry).
    An entry holds the Green's transform and its home plan's workspace; extra
    plan slots (one more workspace each) are added when launches of one key
    overlap, and kept idle for later launches.  Nothing a ticket uses is evicted.
    """

    def __init__(self, sizes: Callable[[Tuple], Tuple[int, int, int]],
                 free: Optional[Callable[[_Entry, Optional[int]], None]] = None):
        self.sizes = sizes
        self.free = free or (lambda entry, index: None)
        self.entries: "collections.OrderedDict[Tuple, _Entry]" = collections.OrderedDict()
        self.transient = 0
        self.reset_counters()

    def reset_counters(self) -> None:
        self.evictions = 0
        self.misses = 0
        self.hits = 0

    def bytes(self) -> int:
        return sum(e.bytes for e in self.entries.values()) + self.transient

    def alone(self, key) -> int:
        """Bytes the key needs with nothing else resident."""
        g, w, p = self.sizes(key)
        return g + w + p

    def peek(self, key) -> int:
        """Bytes ``reserve(key)`` would add now."""
        e = self.entries.get(key)
        if e is None:
            return self.alone(key)
        return 0 if not all(e.busy) else e.work_bytes

    def reserve(self, key) -> Ticket:
        e = self.entries.get(key)
        created = e is None
        transient = 0
        if created:
            g, w, p = self.sizes(key)
            e = _Entry(key=key, ghat_bytes=g, work_bytes=w, pre_bytes=p, plans=[None], busy=[False])
            self.entries[key] = e
            transient = p
            self.transient += p
            self.misses += 1
        else:
            self.hits += 1
            self.entries.move_to_end(key)
        idx = next((i for i, b in enumerate(e.busy) if not b), None)
        if idx is None:
            e.plans.append(None)
            e.busy.append(False)
            idx = len(e.busy) - 1
        e.busy[idx] = True
        e.refs += 1
        return Ticket(entry=e, index=idx, transient=transient, created=created)

    def release(self, t: Ticket) -> None:
        e = t.entry
        e.busy[t.index] = False
        e.refs -= 1
        self.transient -= t.transient
        t.transient = 0

    def evictable(self) -> int:
        """Bytes evict() could free now."""
        total = 0
        for e in self.entries.values():
            if e.refs == 0:
                total += e.bytes
            else:
                k = len(e.busy)
                while k > 1 and not e.busy[k - 1]:
                    k -= 1
                total += (len(e.busy) - k) * e.work_bytes
        return total

    def evict(self, need: int) -> int:
        """Free at least ``need`` bytes if possible: idle extra workspaces first, then
        whole entries that no ticket uses, each in least-recently-used order.
        Returns the bytes freed."""
        freed = 0
        for e in self.entries.values():
            # extra slots go from the end while idle (slot 0 is the home plan)
            while freed < need and len(e.busy) > 1 and not e.busy[-1]:
                self.free(e, len(e.busy) - 1)
                e.busy.pop()
                e.plans.pop()
                freed += e.work_bytes
            if freed >= need:
                return freed
        for key, e in list(self.entries.items()):
            if freed >= need:
                break
            if e.refs == 0:
                self.free(e, None)
                freed += e.bytes
                del self.entries[key]
                self.evictions += 1
        return freed


class Scheduler:
    """FIFO admission under a slot count and a device-byte budget.

    * a job that cannot fit even with nothing else held is rejected at submission;
    * the head of the queue is admitted when a slot is free and its bytes fit,
      after evicting idle resident bytes if needed; later jobs never overtake a
      head that does not fit (no starvation);
    * jobs admitted in one step that share a shape go to one slot together
      (up to ``max_fold``) and are launched as one batched call, when they fit
      without evicting anything.

    ``resident`` (a ResidentSet, optional): bytes held between requests, counted
    in the budget; jobs then carry ``rkeys``, and ``nbytes`` counts their own
    fields only.  Without it ``nbytes`` is everything a job holds.
    """

    def __init__(self, budget_bytes: int, slots: int, max_fold: int = 8, resident: Optional[ResidentSet] = None):
        if budget_bytes <= 0 or slots <= 0:
            raise ValueError("budget and slots must be positive")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.max_fold = max(1, int(max_fold))
        self.resident = resident
        self.queue: Deque[Job] = collections.deque()
        self.in_use = 0
        self.busy: Dict[int, List[Job]] = {}
        self.peak_bytes = 0

    def held(self) -> int:
        """Bytes held now: jobs in flight plus the resident set."""
        return self.in_use + (self.resident.bytes() if self.resident is not None else 0)

    def _alone(self, job: Job) -> int:
        if self.resident is None:
            return job.nbytes
        return job.nbytes + sum(self.resident.alone(k) for k in job.rkeys)

    def _extra(self, job: Job) -> int:
        # keys that repeat within one job (never the case for a job's f32 and f64 keys) would
        # be under-counted here; reserve() takes one slot per key
        return 0 if self.resident is None else sum(self.resident.peek(k) for k in job.rkeys)

    def submit(self, job: Job) -> bool:
        need = self._alone(job)
        if need > self.budget:
            job.status = "rejected"
            job.error = f"needs {need} bytes, budget {self.budget}"
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

    def _fits(self, job: Job, evict: bool) -> bool:
        over = self.held() + job.nbytes + self._extra(job) - self.budget
        # evict only when that makes the job fit (else it waits and the cache stays)
        if over > 0 and evict and self.resident is not None and self.resident.evictable() >= over:
            self.resident.evict(over)
            over = self.held() + job.nbytes + self._extra(job) - self.budget
        return over <= 0

    def _take(self, job: Job) -> None:
        if self.resident is not None:
            job.tickets = [self.resident.reserve(k) for k in job.rkeys]
        self.in_use += job.nbytes

    def admit(self, now: float) -> List[Tuple[int, List[Job]]]:
        """Jobs to launch now, grouped per slot."""
        out = []
        free = self.free_slots()
        while self.queue and free:
            head = self.queue[0]
            if not self._fits(head, evict=True):
                break
            slot = free.pop(0)
            group = [self.queue.popleft()]
            self._take(head)
            # fold waiting jobs of the same shape into this launch
            for j in list(self.queue):
                if len(group) >= self.max_fold:
                    break
                if j.shape_key == head.shape_key and not j.spot_check and not head.spot_check \
                        and self._fits(j, evict=False):
                    self.queue.remove(j)
                    group.append(j)
                    self._take(j)
            for j in group:
                j.status = "running"
                j.t_admit = now
                j.slot = slot
            self.busy[slot] = group
            self.peak_bytes = max(self.peak_bytes, self.held())
            out.append((slot, group))
        return out

    def complete(self, slot: int, t_done: float, failed: Optional[str] = None) -> List[Job]:
        group = self.busy.pop(slot)
        for j in group:
            self.in_use -= j.nbytes
            if self.resident is not None:
                for t in j.tickets:
                    self.resident.release(t)
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


# ------------------------------------------------------------------ device side
class GpuExecutor:
    """Runs admitted jobs on the GPU: one stream per slot, and the device objects of
    the resident set (``self.resident``, which a Server attaches to its scheduler).

    ``source_for(job, dtype)`` returns the job's rho of the job's shape, either a
    device tensor or a host tensor (pinned memory recommended), which is then
    copied to the device on the slot's stream as part of the request.
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
        self.resident = ResidentSet(self._sizes, self._free)
        self.source_for = source_for
        self.keep_results = keep_results
        self.results: Dict[int, object] = {}
        self.inflight: Dict[int, Tuple[object, List[Job], List[object]]] = {}
        self.t0_wall = None
        self.t0_event = None
        self._sized: Dict[Tuple, Tuple[int, int, int]] = {}
        self.refresh_events: List[Tuple[object, object]] = []

    # -------------------------------------------------------------- sizing
    def key_for(self, n, greens, prec, lo=None, hi=None) -> Tuple:
        lo = tuple(float(x) for x in (lo if lo is not None else self.lo))
        hi = tuple(float(x) for x in (hi if hi is not None else self.hi))
        return (greens, int(n), lo, hi, self.alpha, prec)

    def _sizes(self, key) -> Tuple[int, int, int]:
        if key not in self._sized:
            greens, n, lo, hi, alpha, prec = key
            p = self.Plan(n=n, lo=lo, hi=hi, greens=greens, prec=prec, alpha=alpha, bind=False)
            self._sized[key] = (p.ghat_bytes, p.work_bytes, p.precompute_bytes)
            p.close()
        return self._sized[key]

    def work_bytes(self, n: int, greens: str, prec: str) -> int:
        return self._sizes(self.key_for(n, greens, prec))[1]

    def size_job(self, job: Job) -> None:
        job.rkeys = (self.key_for(job.n, job.greens, job.prec, job.lo, job.hi),)
        job.nbytes = field_bytes(job.n, job.prec)
        if job.spot_check:
            job.rkeys += (self.key_for(job.n, job.greens, "f64", job.lo, job.hi),)
            job.nbytes += field_bytes(job.n, "f64")

    def attach(self, sched: Scheduler) -> None:
        sched.resident = self.resident

    # -------------------------------------------------------------- plans
    def _free(self, entry: _Entry, index: Optional[int]) -> None:
        """Drop the device objects of an entry (index None) or of one extra plan slot.
        Only called for slots no ticket holds, so no launch still reads them."""
        for i in (range(len(entry.plans)) if index is None else [index]):
            p = entry.plans[i]
            if p is not None:
                p.close()
                entry.plans[i] = None
        if index is None:
            entry.handle = None

    def _plan(self, ticket: Ticket):
        """The plan a ticket solves with.  An entry's first use computes its transform
        on the precompute stream, between two timing events."""
        torch = self.torch
        e = ticket.entry
        greens, n, lo, hi, alpha, prec = e.key
        if e.handle is None:
            start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(self.pre_stream):
                home = self.Plan(n=n, lo=lo, hi=hi, greens=greens, prec=prec, alpha=alpha,
                                 device=self.device, precompute=False)
                start.record(self.pre_stream)
                try:
                    home.precompute(self.pre_stream)
                except Exception:
                    # part of it may be enqueued: let it end before the buffers go
                    self.pre_stream.synchronize()
                    raise
                end.record(self.pre_stream)
            e.plans[0] = home
            e.handle = end
            e.pending_pre = True
            self.refresh_events.append((start, end))
        p = e.plans[ticket.index]
        if p is None:
            p = self.Plan(n=n, lo=lo, hi=hi, greens=greens, prec=prec, alpha=alpha, device=self.device,
                          precompute=False)
            p.share_ghat(e.plans[0])
            e.plans[ticket.index] = p
        return p

    def _await(self, ticket: Ticket, stream) -> bool:
        """Order `stream` after the ticket's transform; True if that transform was still
        being computed (the solve waits for a refresh)."""
        e = ticket.entry
        if e.pending_pre:
            if e.handle.query():
                e.pending_pre = False
            else:
                stream.wait_event(e.handle)
                return True
        return False

    def warm(self, shapes: Sequence[Tuple]) -> None:
        """Compute the Green's transforms of the given (n, greens, prec[, lo, hi]) shapes
        ahead of the requests; they enter the resident set like any other."""
        for s in shapes:
            n, g, pr = s[:3]
            lo, hi = (s[3], s[4]) if len(s) > 3 else (None, None)
            t = self.resident.reserve(self.key_for(n, g, pr, lo, hi))
            self._plan(t)
            self.resident.release(t)
        self.torch.cuda.synchronize(self.device)
        for e in self.resident.entries.values():
            e.pending_pre = False

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
        self.refresh_events = []
        self.resident.reset_counters()
        return self.t0_wall

    def now(self) -> float:
        return time.perf_counter() - self.t0_wall

    # -------------------------------------------------------------- launches
    def launch(self, slot: int, group: List[Job]) -> None:
        """Enqueue one slot launch.  A launch that cannot get its device memory (a
        plan's buffers, a result) fails alone: whatever it enqueued before the
        failure still completes before its tensors are released, and the loop goes
        on serving."""
        from . import FspError, solve_batched

        torch = self.torch
        st = self.streams[slot]
        prec = group[0].prec
        dt = torch.float64 if prec == "f64" else torch.float32
        plans, rhos, outs = [], [], []
        held = [rhos, outs]
        err = None
        with torch.cuda.stream(st):
            try:
                for j in group:
                    t = j.tickets[0]
                    plans.append(self._plan(t))
                    j.refreshed = self._await(t, st)
                    src = self.source_for(j, dt)
                    rho = src if src.device == self.device else src.to(self.device, non_blocking=True)
                    rhos.append(rho)
                    outs.append(torch.empty_like(rho))
                solve_batched(plans, rhos, outs, stream=st)
                if group[0].spot_check:
                    j = group[0]
                    t64 = j.tickets[1]
                    p64 = self._plan(t64)
                    j.refreshed = self._await(t64, st) or j.refreshed
                    r64 = rhos[0].double()
                    held.append(r64)
                    o64 = p64.solve(r64, stream=st)
                    held.append(o64)
                    diff = torch.linalg.vector_norm((outs[0].double() - o64).flatten())
                    den = torch.linalg.vector_norm(o64.flatten())
                    held += [diff, den]
            except (FspError, torch.cuda.OutOfMemoryError) as e:
                err = f"{type(e).__name__}: {e}"
            done = torch.cuda.Event(enable_timing=True)
            done.record(st)
        self.inflight[slot] = (done, group, held, err)

    def poll(self) -> List[Tuple[int, float, Optional[str]]]:
        """(slot, completion time in seconds since start, error or None) of launches that finished."""
        out = []
        for slot, (ev, group, held, err) in list(self.inflight.items()):
            if ev.query():
                t = self.t0_event.elapsed_time(ev) / 1e3  # GPU clock, seconds since start
                if err is None and group[0].spot_check:
                    diff, den = held[-2], held[-1]
                    group[0].spot_rel_l2 = float(diff / den)
                for j in group:
                    for tk in j.tickets:   # the launch waited for these transforms
                        if tk.entry.handle is not None and tk.entry.handle.query():
                            tk.entry.pending_pre = False
                if self.keep_results and err is None:
                    for j, o in zip(group, held[1]):
                        self.results[j.rid] = o
                del self.inflight[slot]
                out.append((slot, t, err))
        return out

    def refresh_stats(self) -> Dict:
        """Device time of the Green's transforms computed since the clock started
        (call once the device is idle)."""
        ms = [s.elapsed_time(e) for s, e in self.refresh_events]
        return {"refreshes": len(ms), "refresh_ms_total": sum(ms),
                "refresh_ms_mean": (sum(ms) / len(ms)) if ms else 0.0}

    def idle(self) -> bool:
        return not self.inflight


class Server:
    """Drive a Scheduler and an executor over a timed stream of requests."""

    def __init__(self, executor, budget_bytes: int, slots: int, max_fold: int = 8):
        self.ex = executor
        self.sched = Scheduler(budget_bytes, slots, max_fold)
        if hasattr(executor, "attach"):
            executor.attach(self.sched)
        self.jobs: List[Job] = []
        self.peak_held = 0

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
            for done in self.ex.poll():
                slot, t = done[0], done[1]
                seen = self.ex.now()
                for j in self.sched.complete(slot, t, failed=done[2] if len(done) > 2 else None):
                    j.t_seen = seen
            for slot, group in self.sched.admit(now):
                self.ex.launch(slot, group)
                launches += 1
            self.peak_held = max(self.peak_held, self.sched.held())
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
        out = {
            "requests": len(self.jobs),
            "done": len(done),
            "rejected": sum(j.status == "rejected" for j in self.jobs),
            "failed": sum(j.status == "failed" for j in self.jobs),
            "launches": launches,
            "p50_ms": percentile(lat, 50),
            "p99_ms": percentile(lat, 99),
            "mean_ms": sum(lat) / len(lat) if lat else float("nan"),
            "solves_per_s": len(done) / span if done else 0.0,
            "peak_bytes": max(self.sched.peak_bytes, self.peak_held),
            "budget_bytes": self.sched.budget,
            "spot_checks": len(spots),
            "spot_rel_l2_max": max(spots) if spots else None,
            "seen_lag_ms": {"min": min(seen_lag), "p50": percentile(seen_lag, 50),
                            "max": max(seen_lag)} if seen_lag else None,
        }
        res = self.sched.resident
        if res is not None:
            out["resident"] = {"entries": len(res.entries), "bytes": res.bytes(), "hits": res.hits,
                               "misses": res.misses, "evictions": res.evictions}
        if hasattr(self.ex, "refresh_stats"):
            rs = self.ex.refresh_stats()
            waited = [(j.t_done - j.t_arrival) * 1e3 for j in done if j.refreshed]
            cached = [(j.t_done - j.t_arrival) * 1e3 for j in done if not j.refreshed]
            # share of the run's span the device spent computing Green's transforms
            rs["refresh_share"] = (rs["refresh_ms_total"] / (span * 1e3)) if done and span > 0 else 0.0
            rs["requests_refreshed"] = len(waited)
            # None where no request falls in the class (JSON has no NaN)
            rs["p50_ms_refreshed"] = percentile(waited, 50) if waited else None
            rs["p99_ms_refreshed"] = percentile(waited, 99) if waited else None
            rs["p50_ms_cached"] = percentile(cached, 50) if cached else None
            rs["p99_ms_cached"] = percentile(cached, 99) if cached else None
            out["refresh"] = rs
        return out
