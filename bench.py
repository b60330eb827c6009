"""Benchmark: Vico-Greengard free-space Poisson solves of a 256^3 grid on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--greens vico_dct]
                    [--no-cpu-baseline] [--cpu-seconds 20] [--skip-f64] [--skip-extras]
                    [--workload single|batch|serve|serve_boxes|shard|grad]

A step is one full solve (all five passes: axis-2 real transform with the zero
padding fused, axis-1 forward, axis-0 forward + Green's multiply + inverse,
axis-1 inverse, axis-2 inverse real transform with the crop fused) of one
256^3 float32 right-hand side already resident in HBM, on the box [-1,1]^3
with an 8-Gaussian source (centres U[-0.5,0.5]^3, sigma U[0.02,0.08], weights
U[0.5,1.5], seed 3).  The Green's transform is precomputed (float64) outside
the timed region, as the paper excludes solver set-up from its solve time.

Printed: one JSON line.  ``value`` is float32 solves/s; the float64 solve of
the same input is reported under ``fp64``; ``rel_l2`` gives both against the
float64 CPU oracle.  ``roofline`` is the dominant kernel's algorithmic bytes per
launch over its average launch time (HIP events around that kernel inside a
timed loop, on the stream it runs on) against the 8 TB/s HBM peak.
``cpu_baseline`` times the oracle (float64 FFT route, scipy) on the host.
``grad`` times phi with its gradient (fsp_solve_grad) and ``precompute_ms`` the
float64 Green's-table refresh of each kernel (outside the headline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PASS_NAMES = ["P1_row_r2c", "P2_col_fwd", "P3_col_conv", "P4_col_inv", "P5_row_c2r"]


def pass_bytes(n, rb):
    """Algorithmic HBM bytes of each pass (reads + writes) for one solve."""
    n0, n1, n2 = n
    real = n0 * n1 * n2 * rb
    half1 = n0 * n1 * (n2 + 1) * 2 * rb
    half2 = n0 * 2 * n1 * (n2 + 1) * 2 * rb
    octant = (n0 + 1) * (n1 + 1) * (n2 + 1) * rb
    return [real + half1, half1 + half2, 2 * half2 + octant, half2 + half1, half1 + real]


def grad_bytes(n, rb):
    """Algorithmic HBM bytes of phi and grad phi in one call: the forward passes
    once, one axis-0 pass that reads the spectrum once and writes four (with four
    tables), and the two inverse passes for each of the four outputs."""
    pb = pass_bytes(n, rb)
    n0, n1, n2 = n
    half2 = n0 * 2 * n1 * (n2 + 1) * 2 * rb
    octant = (n0 + 1) * (n1 + 1) * (n2 + 1) * rb
    return pb[0] + pb[1] + half2 + 4 * (half2 + octant) + 4 * (pb[3] + pb[4])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_vico_dct_256.txt")


def source_digest():
    """Digest of the HIP sources (file names and contents); a counter summary
    taken from other sources no longer describes these kernels."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2405_02603_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(greens, n, prec, pass_idx, variant):
    """HBM bytes per launch (reads + writes, counter readings scaled by the copy
    calibration) of one pass kernel, from the committed rocprofv3 summary; None
    when the summary has no such entry or was taken from other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    except OSError:
        return None
    src = [ln[1] for ln in lines if ln[0] == "source"]
    if not src or src[0] != source_digest():
        return None
    key = [greens, str(n), prec, f"P{pass_idx + 1}", f"v{variant}"]
    for ln in lines:
        if ln[0] == "traffic" and ln[1:6] == key:
            return int(ln[6])
    return None


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--greens", default="vico_dct", choices=["vico_dct", "vico", "hockney"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="kept for older command lines: the 1 GiB device copy (counter calibration for "
                         "rocprofv3 --pmc) now always runs")
    ap.add_argument("--skip-f64", action="store_true")
    ap.add_argument("--skip-extras", action="store_true", help="skip the gradient and precompute timings")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default schedule")
    ap.add_argument("--workload", default="single", choices=["single", "batch", "serve", "serve_boxes", "shard", "grad"],
                    help="single: the 256^3 headline; batch: 64 uneven right-hand sides per graph launch; "
                         "serve: Poisson-arrival serving loop; serve_boxes: the same with a box fitted to "
                         "each request (Green's transforms computed on misses); shard: one GPU's share of an 8-way "
                         "slab-decomposed solve, at its real shapes; grad: phi and its gradient in one call")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    return ap.parse_args(argv)


def time_solves(torch, plan, rho, phi, steps, warmup):
    for _ in range(warmup):
        plan.solve(rho, phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(rho, phi)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def solve_percentiles(torch, plan, rho, phi, reps):
    """p10 / p50 / p90 of single-solve times (HIP events around each solve), ms."""
    import numpy as np

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        plan.solve(rho, phi, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"p10_ms": round(float(np.percentile(t, 10)), 5), "p50_ms": round(float(np.percentile(t, 50)), 5),
            "p90_ms": round(float(np.percentile(t, 90)), 5), "reps": reps}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_passes(torch, plan, rho, phi, steps):
    """Per-pass average milliseconds: events between passes, on the solve's stream."""
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    torch.cuda.synchronize()
    for s in range(steps):
        ev[s][0].record(stream)
        for p in range(5):
            plan.solve_passes(rho if p == 0 else None, phi if p == 4 else None, p, p, stream)
            ev[s][p + 1].record(stream)
    torch.cuda.synchronize()
    return [sum(ev[s][p].elapsed_time(ev[s][p + 1]) for s in range(steps)) / steps for p in range(5)]


def copy_calibration(torch):
    """Plain device copy of a known size (1 GiB read + 1 GiB write), for counter scaling."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"bytes": 2 * a.numel() * 4, "ms": ms, "GBs": 2 * a.numel() * 4 / ms / 1e6}


def cpu_threads():
    """Host threads for the CPU baseline: every core of this process's affinity set, within the
    host's CPU share when the environment states one (OMP_NUM_THREADS)."""
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(affinity, int(share)) if share.isdigit() and int(share) > 0 else affinity
    return max(1, threads), affinity


def cpu_baseline(rho64, lo, hi, greens_kind, seconds):
    """The oracle (FFT route, scipy) timed on the host on a bounded sample: float64 (the oracle as
    it stands, about two thirds of the time) and float32 (the same steps in single precision)."""
    import numpy as np

    from oracle import fftroute, greens

    n = rho64.shape
    if greens_kind == "hockney":
        k = greens.hockney_octant(n, lo, hi)
    else:
        k = greens.vico_octant(n, lo, hi)
    h = greens.spacing(n, lo, hi)
    cores, affinity = cpu_threads()

    def leg(dtype, budget_s):
        ref, count = None, 0
        t0 = time.perf_counter()
        while True:
            phi = fftroute.solve(rho64, k, h, workers=cores, dtype=dtype)
            if ref is None:
                ref = phi
            count += 1
            el = time.perf_counter() - t0
            if el >= budget_s or count >= 50:
                return ref, count, el

    ref, count, el = leg(np.float64, seconds * 2.0 / 3.0)
    ref32, count32, el32 = leg(np.float32, seconds / 3.0)
    out = {"value": count / el, "unit": "solves/s", "cores": cores, "kind": "oracle",
           "sample": f"{count} float64 FFT-route solves of the same {n[0]}^3 workload "
                     f"(scipy.fft, workers={cores}), {el:.1f} s; kernel table excluded",
           "cpu": cpu_model(), "affinity_cores": affinity,
           "f32": {"value": count32 / el32, "unit": "solves/s",
                   "sample": f"{count32} float32 FFT-route solves, {el32:.1f} s",
                   "rel_l2_vs_f64": float(np.linalg.norm((ref32 - ref).ravel()) / np.linalg.norm(ref.ravel()))}}
    out["direct_sum_32"] = direct_sum_timing()
    return ref, out


def direct_sum_timing():
    """The oracle's literal O(N^6) sum at 32^3 on one thread (informational)."""
    import workloads as W
    from oracle import direct, greens

    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        return None
    n, lo, hi = (32, 32, 32), (-0.5,) * 3, (0.5,) * 3
    rho = W.source_density(n, lo, hi, W.centred_gaussian(0.05))
    k = greens.hockney_octant(n, lo, hi)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        direct.convolve(rho, k, greens.spacing(n, lo, hi))
        el = time.perf_counter() - t0
    return {"seconds": round(el, 3), "threads": 1, "grid": "32^3 Hockney-Eastwood"}


def time_calls(torch, fn, steps, warmup):
    """Mean milliseconds of fn() on the current stream (HIP events around the loop)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def bench_grad(torch, W, n, lo, hi, src, args):
    """phi and grad phi in one call (fsp_solve_grad), both precisions, same input as the headline."""
    from paper_2405_02603_amd import Plan

    out = {}
    rho64 = W.source_density(n, lo, hi, src)
    for prec in ("f32", "f64"):
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = Plan(n=n, lo=lo, hi=hi, greens=args.greens, prec=prec, grad=True)
        rho = torch.from_numpy(rho64).to(device="cuda", dtype=dt)
        phi = torch.empty_like(rho)
        grad = torch.empty((3,) + rho.shape, dtype=dt, device="cuda")
        plan.autotune(rho, phi, reps=4)
        ms = time_calls(torch, lambda: plan.solve_grad(rho, grad=grad, phi=phi), max(10, args.steps // 4), 5)
        model = grad_bytes((n, n, n), 4 if prec == "f32" else 8)
        out[prec] = {"ms": round(ms, 5), "model_bytes": model,
                     "hbm_frac_model": round(model / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
        del plan, rho, phi, grad
        torch.cuda.empty_cache()
    return out


def bench_grad_line(args):
    """phi and grad phi of the 256^3 8-Gaussian workload in one call, both precisions, as its own line."""
    import torch

    import workloads as W

    n = args.n
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    r = bench_grad(torch, W, n, lo, hi, W.multiblob(seed=3, count=8), args)
    out = {"metric": f"phi and grad phi solves/s, {n}^3 {args.greens}", "value": round(1e3 / r["f32"]["ms"], 2),
           "unit": "solves/s", "n_gpus": 1, "steps": max(10, args.steps // 4), "warmup": 5,
           "ms_per_step": r["f32"]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{args.greens} potential and gradient, {n}^3 on [-1,1]^3, 8 Gaussians (seed 3)"},
           "grad": r}
    print(json.dumps(out), flush=True)
    return 0


def bench_large(torch, W, n, lo, hi, args):
    """The 512^3 single solve (same box and 8-Gaussian source), both precisions, autotuned."""
    from paper_2405_02603_amd import Plan

    rho64 = W.source_density(n, lo, hi, W.multiblob(seed=3, count=8))
    out = {}
    for prec in ("f32", "f64"):
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = Plan(n=n, lo=lo, hi=hi, greens=args.greens, prec=prec)
        rho = torch.from_numpy(rho64).to(device="cuda", dtype=dt)
        phi = torch.empty_like(rho)
        plan.autotune(rho, phi, reps=2)
        ms = time_calls(torch, lambda: plan.solve(rho, phi), 20, 3)
        out[prec] = {"ms": round(ms, 4), "solves_per_s": round(1e3 / ms, 2),
                     "hbm_frac_model": round(plan.model_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                     "schedule": plan.schedule}
        del plan, rho, phi
        torch.cuda.empty_cache()
    return out


def bench_precompute(torch, n, lo, hi):
    """Milliseconds of fsp_precompute (float64 Green's tables) per kernel and precision."""
    from paper_2405_02603_amd import Plan

    out = {}
    for greens in ("hockney", "vico_dct", "vico"):
        for prec in ("f32",):
            plan = Plan(n=n, lo=lo, hi=hi, greens=greens, prec=prec)
            torch.cuda.synchronize()
            out[greens] = round(time_calls(torch, plan.precompute, 3, 1), 3)
            del plan
            torch.cuda.empty_cache()
    return out


def run_batch(args, count=None, steps=None, warmup=None):
    """64 right-hand sides, n from {32,48,64,96,128} (seed 4), Vico-Greengard float32, one graph
    launch per step (device table of the items' buffers).  Returns the measurement as a dict."""
    import torch

    import workloads as W
    from paper_2405_02603_amd import Batch, Plan, autotune_batch

    count = count or args.batch_count
    steps = steps or args.steps
    warmup = args.warmup if warmup is None else warmup
    items = W.batch_mix(seed=4, count=count)
    src = {}
    plans, rhos, host = [], [], []
    tuned = {}
    for it in items:
        p = Plan(n=it.n, lo=it.lo, hi=it.hi, greens="vico_dct", prec="f32", precompute=False)
        if it.n not in src:
            p.precompute()
            src[it.n] = p
            if not args.no_autotune:   # later plans of this grid start with the tuned schedule
                r0 = torch.from_numpy(W.source_density(it.n, it.lo, it.hi, it.source)).to("cuda", torch.float32)
                p.autotune(r0, torch.empty_like(r0), reps=4)
                tuned[it.n] = p.schedule
        else:
            p.share_ghat(src[it.n])
        r = W.source_density(it.n, it.lo, it.hi, it.source)
        host.append(r)
        plans.append(p)
        rhos.append(torch.from_numpy(r).to("cuda", torch.float32))
    if not args.no_autotune:   # schedules of the equal-shape groups with their solves timed together
        autotune_batch(plans, rhos, reps=4)
    batch = Batch(plans, rhos)
    for _ in range(warmup):
        batch.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.launch()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    model = sum(p.model_bytes for p in plans)   # the bytes of each plan's schedule
    five_pass = sum(sum(pass_bytes(W._as3(it.n, int), 4)) for it in items)
    # the same right-hand sides as plain float64 single solves, one at a time
    p64 = {}
    r64 = [torch.from_numpy(h).to("cuda") for h in host]
    for it in items:
        if it.n not in p64:
            p64[it.n] = Plan(n=it.n, lo=it.lo, hi=it.hi, greens="vico_dct", prec="f64")
    outs64 = [p64[it.n].solve(r) for it, r in zip(items, r64)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, steps // 4)
    for _ in range(reps):
        for it, r, o in zip(items, r64, outs64):
            p64[it.n].solve(r, o)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3 / reps
    err = max(float(torch.linalg.vector_norm((o32.double() - o64).flatten()) / torch.linalg.vector_norm(o64.flatten()))
              for o32, o64 in zip(batch.outs, outs64))
    sizes = sorted({it.n for it in items})
    out = {"solves_per_s": round(len(items) * 1e3 / ms, 1), "ms_per_step": round(ms, 4), "count": len(items),
           "sizes": sizes, "steps": steps, "hbm_frac_model": round(model / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
           "model_bytes_per_step": model,
           "five_pass_model_bytes_per_step": five_pass,
           "hbm_frac_five_pass_model": round(five_pass / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
           "fp64_single_solves": {"solves_per_s": round(len(items) * 1e3 / ms64, 1), "ms_per_batch": round(ms64, 4)},
           "max_rel_l2_f32_vs_gpu_f64": err,
           "schedules": {str(k): v for k, v in sorted(tuned.items())},
           "batch_schedules": {str(it.n): p.schedule for it, p in sorted(zip(items, plans), key=lambda x: x[0].n)}}
    batch.close()
    return out


def bench_batch(args):
    r = run_batch(args)
    out = {
        "metric": "batched Vico-Greengard solves/s (64 uneven right-hand sides per graph launch)",
        "value": r["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{r['count']} right-hand sides, n in {r['sizes']} (seed 4), [-1,1]^3, 8 Gaussians "
                               "each, vico_dct float32, one captured graph per step"},
    }
    out.update({k: v for k, v in r.items() if k not in ("solves_per_s", "ms_per_step")})
    print(json.dumps(out), flush=True)
    return 0


def run_serve(args, seconds=None, rate=None, sweep=True):
    """Poisson arrivals (seed 5), n in {32..256}, 50/50 Hockney/Vico, float32 with 1% float64 spot
    checks, each request its own 8-Gaussian source (generated on the device before the run),
    through the serving loop of paper_2405_02603_amd.serve.  Returns the report as a dict."""
    import torch

    import workloads as W
    from paper_2405_02603_amd.serve import GpuExecutor, Job, Server

    seconds = args.serve_seconds if seconds is None else seconds
    rate = args.serve_rate if rate is None else rate
    sizes = (32, 48, 64, 96, 128, 192, 256)
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    arrivals = W.poisson_arrivals(rate=rate, duration=seconds, seed=5, sizes=sizes, spot_fraction=0.01, blobs=8)
    own = {a.rid: W.source_density_device((a.n,) * 3, lo, hi, a.source, dtype=torch.float32) for a in arrivals}
    torch.cuda.synchronize()
    ex = GpuExecutor(slots=args.serve_slots, source_for=lambda j, dt: own[j.rid] if dt == torch.float32
                     else own[j.rid].to(dt))
    ex.warm([(n, g, p) for n in sizes for g in ("hockney", "vico_dct") for p in ("f32", "f64")])
    budget = int(args.serve_budget_gb * (1 << 30))

    def run(scale):
        jobs = [Job(rid=a.rid, t_arrival=a.t_arrival, n=a.n, greens="hockney" if a.greens == "hockney" else "vico_dct",
                    spot_check=a.spot_check) for a in arrivals]
        return Server(ex, budget_bytes=budget, slots=args.serve_slots).run(jobs, time_scale=scale)

    rep = run(1.0)
    out = {"rate": rate, "seconds": seconds, "budget_bytes": budget, **rep}
    if sweep:
        sat = []
        for scale in (0.2, 0.05, 0.0):   # offered 5x, 20x the rate, then everything at once
            r = run(scale)
            sat.append({"offered_rate": (rate / scale) if scale else "all-at-once",
                        "solves_per_s": round(r["solves_per_s"], 1), "p50_ms": round(r["p50_ms"], 3),
                        "p99_ms": round(r["p99_ms"], 3), "launches": r["launches"]})
        out["saturation_sweep"] = sat
    del own, ex
    torch.cuda.empty_cache()
    return out


def _rounded(d):
    """Floats to 5 significant digits, through nested dicts."""
    if isinstance(d, dict):
        return {k: _rounded(v) for k, v in d.items()}
    return float(f"{d:.5g}") if isinstance(d, float) else d


def run_serve_boxes(args, seconds=10.0, rate=200.0, budget_gb=2.0):
    """Serving with a box per request: the domain fitted to each request's own 8 Gaussians
    (centres +- 4 sigma, edges at least 1.25, faces on a 0.25 lattice), n in {32..128},
    50/50 Hockney/Vico, float32.  Every new (kernel, grid, box) computes its Green's
    transform on the precompute stream (nothing is warmed); a 2 GB budget over everything
    held forces evictions.  Returns the report (refresh share and latencies with and
    without a refresh)."""
    import torch

    import workloads as W
    from paper_2405_02603_amd.serve import GpuExecutor, Job, Server

    sizes = (32, 48, 64, 96, 128)
    arrivals = W.poisson_arrivals(rate=rate, duration=seconds, seed=6, sizes=sizes, spot_fraction=0.0, blobs=8)
    boxes = {a.rid: W.fitted_box(a.source) for a in arrivals}
    own = {a.rid: W.source_density_device((a.n,) * 3, boxes[a.rid][0], boxes[a.rid][1], a.source,
                                          dtype=torch.float32) for a in arrivals}
    torch.cuda.synchronize()
    ex = GpuExecutor(slots=args.serve_slots, source_for=lambda j, dt: own[j.rid])
    jobs = [Job(rid=a.rid, t_arrival=a.t_arrival, n=a.n, greens="hockney" if a.greens == "hockney" else "vico_dct",
                lo=boxes[a.rid][0], hi=boxes[a.rid][1]) for a in arrivals]
    rep = Server(ex, budget_bytes=int(budget_gb * (1 << 30)), slots=args.serve_slots).run(jobs)
    out = {"rate": rate, "seconds": seconds, "distinct_boxes": len(set(boxes.values())), **rep}
    del own, ex
    torch.cuda.empty_cache()
    return out


def bench_serve(args):
    r = run_serve(args)
    out = {
        "metric": "served solves/s and p50/p99 latency (Poisson arrivals, mixed sizes and kernels)",
        "value": round(r["solves_per_s"], 1), "unit": "solves/s", "n_gpus": 1, "steps": r["done"],
        "warmup": 0, "ms_per_step": round(1e3 / max(r["solves_per_s"], 1e-9), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals {args.serve_rate}/s for {args.serve_seconds} s, n in "
                               "[32..256], 50/50 hockney/vico_dct, float32, 1% float64 spot checks, each request "
                               f"its own 8-Gaussian source, budget {args.serve_budget_gb} GB, "
                               f"{args.serve_slots} slots"},
    }
    out.update(r)
    print(json.dumps(out), flush=True)
    return 0


def bench_serve_boxes(args):
    r = run_serve_boxes(args, seconds=args.serve_seconds, rate=args.serve_rate)
    out = {
        "metric": "served solves/s and p50/p99 latency, a box fitted to each request",
        "value": round(r["solves_per_s"], 1), "unit": "solves/s", "n_gpus": 1, "steps": r["done"],
        "warmup": 0, "ms_per_step": round(1e3 / max(r["solves_per_s"], 1e-9), 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals {args.serve_rate}/s for {args.serve_seconds} s, n in [32..128], "
                               "50/50 hockney/vico_dct, float32, each request its own 8 Gaussians and the box "
                               "fitted to them, budget 2 GB, "
                               f"{args.serve_slots} slots"},
    }
    out.update(_rounded(r))
    print(json.dumps(out), flush=True)
    return 0


def bench_shard(args):
    """One GPU's share of a 256^3 solve slab-decomposed over G = 8 GPUs, at the
    share's real shapes: P1, P2, P4 and P5 on an n0 / G slab (a (n/G, n, n)
    plan), P3 on about (n2 + 1) / G of the axis-2 frequencies (a (n, n, n/G)
    plan: 2 n1 (n/G + 1) pencils of 2 n0 points).  The two all-to-all exchanges
    between them are not run (one GPU); their ideal time over xGMI is given
    from the bytes that leave each GPU, as a model."""
    import torch

    import workloads as W
    from paper_2405_02603_amd import Plan

    n, G = args.n, 8
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    out = {}
    for prec in (["f32"] if args.skip_f64 else ["f32", "f64"]):
        dt = torch.float32 if prec == "f32" else torch.float64
        rb = 4 if prec == "f32" else 8
        ms = {}
        for name, shape, keep in (("slab", (n // G, n, n), (0, 1, 3, 4)), ("columns", (n, n, n // G), (2,))):
            plan = Plan(n=shape, lo=lo, hi=hi, greens=args.greens, prec=prec)
            rho = torch.from_numpy(W.random_field(shape, 7)).to(device="cuda", dtype=dt)
            phi = torch.empty_like(rho)
            if not args.no_autotune:
                plan.autotune(rho, phi, reps=4)
            for _ in range(args.warmup):
                plan.solve(rho, phi)
            pm = time_passes(torch, plan, rho, phi, args.steps)
            pb = pass_bytes(shape, rb)
            for i in keep:
                ms[PASS_NAMES[i]] = {"ms": round(pm[i], 5), "bytes": pb[i], "shape": list(shape),
                                     "GBs": round(pb[i] / (pm[i] * 1e-3) / 1e9, 1)}
            del plan, rho, phi
            torch.cuda.empty_cache()
        total = sum(v["ms"] for v in ms.values())
        nbytes = sum(v["bytes"] for v in ms.values())
        # each exchange: this GPU's share of the half spectrum, (G - 1) / G of it leaving, one xGMI link per peer
        half2 = n * 2 * n * (n + 1) * 2 * rb
        per_peer = half2 / G / G
        xgmi = 153e9
        out[prec] = {"kernel_ms": round(total, 5), "passes": ms, "model_bytes": nbytes,
                     "hbm_frac_model": round(nbytes / (total * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                     "exchange_model": {"per_peer_bytes": int(per_peer), "links": G - 1, "link_GBs": 153.0,
                                        "ms_each": round(per_peer / xgmi * 1e3, 5), "count": 2}}
    r32 = out["f32"]
    line = {"metric": f"one GPU's share of a {n}^3 solve slab-decomposed over {G} GPUs (pass kernels at the share shapes)",
            "value": r32["kernel_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r32["kernel_ms"], "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{args.greens} {n}^3 on [-1,1]^3 split over {G} GPUs: P1/P2/P4/P5 on a "
                                   f"({n // G},{n},{n}) slab, P3 on a ({n},{n},{n // G}) column share; random field "
                                   f"(seed 7); the two all-to-alls are modelled, not run"},
            "shares": out}
    print(json.dumps(line))
    return 0


def main(argv=None):
    args = parse(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not "
                                   "implemented (batched and served solves shard by request)",
                          "n_gpus": args.gpus}))
        return 2
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "shard":
        return bench_shard(args)
    if args.workload == "grad":
        return bench_grad_line(args)
    if args.workload == "serve_boxes":
        return bench_serve_boxes(args)

    import numpy as np
    import torch

    import workloads as W
    from paper_2405_02603_amd import Plan

    n = args.n
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    src = W.multiblob(seed=3, count=8)
    rho64 = W.source_density(n, lo, hi, src)
    results = {}
    extra = {}
    for prec in (["f32"] if args.skip_f64 else ["f32", "f64"]):
        dt = torch.float32 if prec == "f32" else torch.float64
        plan = Plan(n=n, lo=lo, hi=hi, greens=args.greens, prec=prec)
        rho = torch.from_numpy(rho64).to(device="cuda", dtype=dt)
        phi = torch.empty_like(rho)
        tune = None
        if not args.no_autotune:
            tune = plan.autotune(rho, phi, reps=8)   # outside the timed region
        torch.cuda.synchronize()
        ms = time_solves(torch, plan, rho, phi, args.steps, args.warmup)
        pct = solve_percentiles(torch, plan, rho, phi, args.steps)
        pass_ms = time_passes(torch, plan, rho, phi, args.steps)
        plan.solve(rho, phi)
        torch.cuda.synchronize()
        results[prec] = {
            "ms": ms,
            "solves_per_s": 1e3 / ms,
            "model_bytes": plan.model_bytes,
            "hbm_frac_model": plan.model_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
            "pass_ms": pass_ms,
            "percentiles": pct,
            "phi": phi.double().cpu().numpy(),
            "rb": 4 if prec == "f32" else 8,
            "schedule": plan.schedule,
            "tune_ms": None if tune is None else {str(k): ([round(x, 5) for x in v] if isinstance(v, list) else round(v, 5))
                                                  for k, v in tune.items()},
        }
        del plan, rho, phi
        torch.cuda.empty_cache()

    # the gradient solve (phi and its three derivatives) and the Green's-table precompute
    if not args.skip_extras:
        extra["grad"] = bench_grad(torch, W, n, lo, hi, src, args)
        for prec, r in extra["grad"].items():    # time of phi + grad over the time of phi alone
            if prec in results:
                r["vs_potential_only"] = round(r["ms"] / results[prec]["ms"], 3)
        extra["precompute_ms"] = bench_precompute(torch, n, lo, hi)
        if n == 256:
            extra["n512"] = bench_large(torch, W, 512, lo, hi, args)
    # a plain device copy of 1 GiB: the bandwidth a streaming kernel reaches on this GPU
    extra["copy_calibration"] = copy_calibration(torch)
    # compact summaries of the batched (64 uneven right-hand sides per graph launch) and served
    # (Poisson arrivals at 200/s for 30 s; then 10 s with a box fitted to each request) workloads
    if not args.skip_extras and n == 256:
        b = run_batch(args, steps=50, warmup=10)
        extra["batch_64"] = {k: b[k] for k in ("solves_per_s", "ms_per_step", "hbm_frac_model",
                                                "max_rel_l2_f32_vs_gpu_f64", "sizes")}
        extra["batch_64"]["fp64_single_solves_per_s"] = b["fp64_single_solves"]["solves_per_s"]
        sv = run_serve(args, seconds=30.0, rate=200.0)
        extra["serve_200"] = {k: (float(f"{sv[k]:.5g}") if isinstance(sv[k], float) else sv[k])
                              for k in ("requests", "done", "rejected", "launches", "p50_ms", "p99_ms",
                                        "solves_per_s", "budget_bytes", "peak_bytes", "spot_checks",
                                        "spot_rel_l2_max", "saturation_sweep", "resident")}
        sb = run_serve_boxes(args)
        extra["serve_boxes"] = _rounded({k: sb[k] for k in ("requests", "done", "rejected", "distinct_boxes",
                                                            "launches", "p50_ms", "p99_ms", "solves_per_s",
                                                            "budget_bytes", "peak_bytes", "resident", "refresh")})

    r32 = results["f32"]
    pb = pass_bytes((n, n, n), r32["rb"])
    dom = int(np.argmax(r32["pass_ms"]))
    achieved = pb[dom] / (r32["pass_ms"][dom] * 1e-3) / 1e9
    traffic = measured_traffic(args.greens, n, "f32", dom, r32["schedule"][dom])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": PASS_NAMES[dom], "bytes_per_launch": pb[dom],
                "avg_launch_ms": round(r32["pass_ms"][dom], 5)}

    out = {
        "metric": "Vico 256^3 solves/s + %HBM peak, FP32 vs FP64 at stated rel-L2 error",
        "value": round(r32["solves_per_s"], 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.greens} free-space Poisson solve, {n}^3 grid on [-1,1]^3, "
                               "8-Gaussian source (seed 3), float32 passes, float64 precompute",
                   "n": n, "greens": args.greens, "box": [list(lo), list(hi)], "parallelism": "single GPU"},
        "hbm_frac_model": round(r32["hbm_frac_model"], 4),
        "model_bytes_per_solve": r32["model_bytes"],
        "passes": [{"kernel": PASS_NAMES[i], "ms": round(r32["pass_ms"][i], 5),
                    "GBs": round(pb[i] / (r32["pass_ms"][i] * 1e-3) / 1e9, 1)} for i in range(5)],
        "roofline": roofline,
        "schedule": r32["schedule"],
        "autotune_ms": r32["tune_ms"],
        "solve_time_percentiles": r32["percentiles"],
    }
    if "f64" in results:
        r64 = results["f64"]
        pb64 = pass_bytes((n, n, n), 8)
        out["fp64"] = {"solves_per_s": round(r64["solves_per_s"], 2), "ms_per_step": round(r64["ms"], 5),
                       "solve_time_percentiles": r64["percentiles"],
                       "schedule": r64["schedule"], "autotune_ms": r64["tune_ms"],
                       "hbm_frac_model": round(r64["hbm_frac_model"], 4),
                       "passes": [{"kernel": PASS_NAMES[i], "ms": round(r64["pass_ms"][i], 5),
                                   "GBs": round(pb64[i] / (r64["pass_ms"][i] * 1e-3) / 1e9, 1)}
                                  for i in range(5)]}
    out.update(extra)
    if not args.no_cpu_baseline:
        ref, cb = cpu_baseline(rho64, lo, hi, args.greens, args.cpu_seconds)
        out["cpu_baseline"] = cb
        den = float(np.linalg.norm(ref))
        out["rel_l2"] = {p: float(np.linalg.norm(results[p]["phi"] - ref) / den) for p in results}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
