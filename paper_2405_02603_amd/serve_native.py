"""Serving: continuous batching of free-space Poisson solve requests on one GPU.

The engine is native (``serve_engine.hip``, C ABI in ``include/fsp_serve.h``):
one host thread inside ``fsp_server_run`` releases requests at their arrival
times, admits them in arrival order while a launch slot is free and the device
bytes the engine holds (cached Green's transforms, pooled workspaces, refresh
transients) fit its budget, folds queued requests of the head's grid and
precision into one launch, computes a missing Green's transform on its refresh
stream, and records per-request times.  This module only marshals arguments.

    srv = Server(budget_bytes=16 << 30, slots=8)
    results = srv.run(requests)          # requests: list of Request (device rho / phi)
    report = summarize(requests, results, srv.stats())
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Dict, List, Optional, Sequence

from . import _lib
from ._lib import GREENS, PREC, check

__all__ = ["Request", "Server", "summarize", "percentile"]


@dataclasses.dataclass
class Request:
    """One solve: rho / phi are device tensors of the grid's shape (phi may be rho)."""
    t_arrival: float
    n: tuple
    greens: str
    rho: object
    phi: object
    prec: str = "f32"
    lo: tuple = (-1.0, -1.0, -1.0)
    hi: tuple = (1.0, 1.0, 1.0)
    alpha: float = 1.1


class Server:
    """A native serving engine (fsp_server_*) on the current device."""

    def __init__(self, budget_bytes: int, slots: int = 8, max_fold: int = 16):
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        check(self._lib.fsp_server_create(ctypes.c_size_t(int(budget_bytes)), int(slots), int(max_fold),
                                          ctypes.byref(h)), "fsp_server_create")
        self._h = h
        self.budget = int(budget_bytes)

    def run(self, requests: Sequence[Request], time_scale: float = 1.0, max_wall_s: float = 600.0) -> List[Dict]:
        """Serve the requests (released at t_arrival * time_scale seconds; 0 = all at once) and
        return one result dict per request, in order."""
        import torch

        count = len(requests)
        reqs = (_lib.Request * max(count, 1))()
        for i, r in enumerate(requests):
            n = tuple(int(x) for x in (r.n if isinstance(r.n, (tuple, list)) else (r.n,) * 3))
            dt = torch.float64 if r.prec == "f64" else torch.float32
            for t, name in ((r.rho, "rho"), (r.phi, "phi")):
                if t.dtype != dt or tuple(t.shape) != n or not t.is_contiguous() or t.device.type != "cuda":
                    raise ValueError(f"request {i}: {name} must be a contiguous {dt} CUDA tensor of shape {n}")
            q = reqs[i]
            q.t_arrival = float(r.t_arrival)
            q.n[:] = list(n)
            q.greens = GREENS[r.greens]
            q.prec = PREC[r.prec]
            q.lo[:] = [float(x) for x in r.lo]
            q.hi[:] = [float(x) for x in r.hi]
            q.alpha = float(r.alpha)
            q.rho = r.rho.data_ptr()
            q.phi = r.phi.data_ptr()
        res = (_lib.RequestResult * max(count, 1))()
        torch.cuda.synchronize()   # the requests' inputs are ready before the engine's streams read them
        check(self._lib.fsp_server_run(self._h, count, reqs, res, float(time_scale), float(max_wall_s)),
              "fsp_server_run")
        return [{"t_arrival": x.t_arrival, "t_admit": x.t_admit, "t_done": x.t_done, "t_seen": x.t_seen,
                 "refresh_ms": x.refresh_ms, "status": x.status, "slot": x.slot, "launch_size": x.launch_size}
                for x in res[:count]]

    def stats(self) -> Dict:
        st = _lib.ServerStats()
        check(self._lib.fsp_server_get_stats(self._h, ctypes.byref(st)), "fsp_server_get_stats")
        return {f: getattr(st, f) for f, _ in _lib.ServerStats._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fsp_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def percentile(values: Sequence[float], q: float) -> float:
    if not values:
        return float("nan")
    v = sorted(values)
    k = (len(v) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def summarize(results: Sequence[Dict], stats: Optional[Dict] = None) -> Dict:
    """Latency (arrival -> device completion) percentiles, throughput and the share of
    latency spent waiting for Green's refreshes."""
    done = [r for r in results if r["status"] == _lib.FSP_OK]
    lat = [(r["t_done"] - r["t_arrival"]) * 1e3 for r in done]
    span = (max(r["t_done"] for r in done) - min(r["t_arrival"] for r in done)) if done else float("nan")
    refreshed = [r for r in done if r["refresh_ms"] > 0]
    lag = [(r["t_seen"] - r["t_done"]) * 1e3 for r in done]
    out = {
        "requests": len(results),
        "done": len(done),
        "rejected": sum(r["status"] == _lib.FSP_ERR_OUT_OF_MEMORY for r in results),
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "mean_ms": sum(lat) / len(lat) if lat else float("nan"),
        "solves_per_s": len(done) / span if done and span > 0 else 0.0,
        "mean_launch_size": (sum(r["launch_size"] for r in done) / len(done)) if done else 0.0,
        "refreshed_requests": len(refreshed),
        # latency share of the refreshes the requests waited for
        "refresh_share": (sum(r["refresh_ms"] for r in refreshed) / sum(lat)) if lat and sum(lat) > 0 else 0.0,
        "seen_lag_ms": {"min": min(lag), "p50": percentile(lag, 50), "max": max(lag)} if lag else None,
    }
    if stats:
        out.update({k: stats[k] for k in ("budget_bytes", "peak_held_bytes", "held_bytes", "launches", "refreshes",
                                          "evictions", "refresh_ms_total")})
    return out
