"""GPU: the continuous-batching server.

A short Poisson-arrival run with mixed sizes and both Green's functions checks
that every request completes, that the bytes in flight never exceed the budget,
that the float64 spot checks agree with the float32 results, and that every
result served in the mix equals the same request solved alone (same kernels,
so bit for bit)."""
import numpy as np
import pytest

import workloads as W

from gpu_util import F32_ELEM, elem_err, reference, rel_l2, to_host

pytestmark = pytest.mark.gpu

SIZES = (32, 48, 64, 96)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _sources(torch):
    pool = {}
    for n in SIZES:
        rho = W.source_density(n, (-1.0,) * 3, (1.0,) * 3, W.multiblob(seed=n))
        for dt in (torch.float32, torch.float64):
            pool[(n, dt)] = torch.from_numpy(rho).to(dt).pin_memory()
    return pool


def _jobs(count, rate, seed, spot_every=10):
    from paper_2405_02603_amd.serve import Job
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(SIZES[int(rng.integers(0, len(SIZES)))])
        greens = "hockney" if rng.random() < 0.5 else "vico_dct"
        jobs.append(Job(rid=rid, t_arrival=t, n=n, greens=greens, spot_check=(rid % spot_every == 3)))
    return jobs


def _own_sources(torch, jobs):
    """Each request's own source (8 Gaussians drawn per request), host float64 and pinned copies."""
    host, pinned = {}, {}
    for j in jobs:
        rho = W.source_density(j.n, (-1.0,) * 3, (1.0,) * 3, W.multiblob(seed=1000 + j.rid))
        host[j.rid] = rho
        for dt in (torch.float32, torch.float64):
            pinned[(j.rid, dt)] = torch.from_numpy(rho).to(dt).pin_memory()
    return host, pinned


def test_serve_mix_equals_alone(torch_cuda):
    torch = torch_cuda
    from paper_2405_02603_amd import Plan
    from paper_2405_02603_amd.serve import GpuExecutor, Server

    jobs = _jobs(48, rate=400.0, seed=5)
    host, pinned = _own_sources(torch, jobs)
    ex = GpuExecutor(slots=4, source_for=lambda j, dt: pinned[(j.rid, dt)], keep_results=True)
    ex.warm([(n, g, p) for n in SIZES for g in ("hockney", "vico_dct") for p in ("f32", "f64")])
    budget = 1 << 30
    srv = Server(ex, budget_bytes=budget, slots=4)
    rep = srv.run(jobs)
    torch.cuda.synchronize()
    assert rep["done"] == len(jobs), rep
    assert rep["peak_bytes"] <= budget
    assert rep["p99_ms"] >= rep["p50_ms"] > 0
    assert rep["spot_checks"] >= 4
    assert rep["spot_rel_l2_max"] <= 1e-6
    # device completion times and host clock share their zero: a completion is seen
    # on the host after (and soon after) the device finished it
    assert -0.5 <= rep["seen_lag_ms"]["min"] and rep["seen_lag_ms"]["p50"] < 20.0, rep["seen_lag_ms"]
    for j in jobs:
        alone = Plan(n=j.n, lo=(-1.0,) * 3, hi=(1.0,) * 3, greens=j.greens, prec="f32")
        phi = alone.solve(pinned[(j.rid, torch.float32)].to("cuda"))
        torch.cuda.synchronize()
        assert torch.equal(phi, ex.results[j.rid]), f"request {j.rid} differs in the mix"
        # and the served result is the oracle's, at its own size, kernel and source
        ref = reference(host[j.rid], j.greens, (-1.0,) * 3, (1.0,) * 3, use_direct=False)
        got = to_host(ex.results[j.rid])
        assert rel_l2(got, ref) <= 1e-6, (j.rid, j.n, j.greens)
        assert elem_err(got, ref) <= F32_ELEM, (j.rid, j.n, j.greens)


def test_serve_cold_cache_two_slots_same_shape(torch_cuda):
    """No warm-up: the first requests of a shape find no Green's transform, and several
    requests of that shape run at once on different slots (one job per launch).  Each
    solve waits for the precompute it reads, so every result is the oracle's."""
    torch = torch_cuda
    from paper_2405_02603_amd.serve import GpuExecutor, Job, Server

    jobs = [Job(rid=i, t_arrival=0.0, n=(64 if i % 3 else 48), greens=("vico_dct" if i % 2 else "hockney"))
            for i in range(12)]
    host, pinned = _own_sources(torch, jobs)
    ex = GpuExecutor(slots=3, source_for=lambda j, dt: pinned[(j.rid, dt)], keep_results=True)
    srv = Server(ex, budget_bytes=1 << 30, slots=3, max_fold=1)
    rep = srv.run(jobs)
    torch.cuda.synchronize()
    assert rep["done"] == len(jobs), rep
    assert len({j.slot for j in jobs}) > 1
    for j in jobs:
        ref = reference(host[j.rid], j.greens, (-1.0,) * 3, (1.0,) * 3, use_direct=False)
        assert rel_l2(to_host(ex.results[j.rid]), ref) <= 1e-6, (j.rid, j.n, j.greens)


def test_serve_rejects_over_budget(torch_cuda):
    torch = torch_cuda
    from paper_2405_02603_amd.serve import GpuExecutor, Job, Server

    pool = _sources(torch)
    ex = GpuExecutor(slots=2, source_for=lambda j, dt: pool[(j.n, dt)])
    srv = Server(ex, budget_bytes=8 << 20, slots=2)   # 8 MiB: 32^3 fits, 96^3 does not
    jobs = [Job(rid=0, t_arrival=0.0, n=96, greens="hockney"), Job(rid=1, t_arrival=0.0, n=32, greens="hockney")]
    rep = srv.run(jobs)
    assert jobs[0].status == "rejected"
    assert jobs[1].status == "done"
    assert rep["done"] == 1 and rep["rejected"] == 1


BOXES = [((-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)),
         ((-0.8, -1.2, -1.0), (1.1, 0.9, 1.3)),
         ((-0.6, -0.7, -0.9), (0.7, 0.8, 0.6)),
         ((-1.5, -1.0, -1.0), (1.5, 1.2, 0.9))]


def test_serve_varying_boxes_under_a_tight_budget(torch_cuda):
    """Requests whose box changes from one to the next (a domain fitted to the particles):
    every box's Green's transform is computed on a miss, on the precompute stream, and
    timed; the budget covers the transforms and workspaces kept between requests, so it
    forces evictions; device memory never exceeds it; and every result is the oracle's
    at its own box and kernel."""
    torch = torch_cuda
    from paper_2405_02603_amd.serve import GpuExecutor, Job, Server, field_bytes

    rng = np.random.default_rng(17)
    jobs, t = [], 0.0
    for rid in range(40):
        t += float(rng.exponential(1.0 / 300.0))
        lo, hi = BOXES[int(rng.integers(0, len(BOXES)))]
        jobs.append(Job(rid=rid, t_arrival=t, n=int((32, 48)[rid % 2]), greens=("vico_dct", "hockney")[(rid // 2) % 2],
                        lo=lo, hi=hi))
    host = {j.rid: W.source_density(j.n, j.lo, j.hi, W.multiblob(seed=2000 + j.rid)) for j in jobs}
    pinned = {rid: torch.from_numpy(h).to(torch.float32).pin_memory() for rid, h in host.items()}
    ex = GpuExecutor(slots=3, source_for=lambda j, dt: pinned[j.rid], keep_results=True)
    keys = {ex.key_for(j.n, j.greens, j.prec, j.lo, j.hi) for j in jobs}
    alone = max(ex.resident.alone(k) for k in keys) + field_bytes(48, "f32")
    held_all = sum(sum(ex._sizes(k)[:2]) for k in keys)
    budget = 2 * alone
    assert budget < held_all, "the budget must not hold every transform at once"
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    srv = Server(ex, budget_bytes=budget, slots=3)
    rep = srv.run(jobs)
    torch.cuda.synchronize()
    kept = sum(field_bytes(j.n, "f32") // 2 for j in jobs)
    print("varying boxes", {k: rep[k] for k in ("done", "launches", "peak_bytes", "budget_bytes", "resident", "refresh")})
    assert rep["done"] == len(jobs), rep
    assert rep["peak_bytes"] <= budget
    assert torch.cuda.max_memory_allocated() - base <= budget + kept + (1 << 20)
    res, rf = rep["resident"], rep["refresh"]
    assert res["evictions"] > 0 and res["misses"] >= len(keys) and res["hits"] > 0
    assert rf["refreshes"] == res["misses"] and rf["refresh_ms_total"] > 0 and 0 < rf["refresh_share"] < 1
    assert rf["requests_refreshed"] >= 1
    for j in jobs:
        ref = reference(host[j.rid], j.greens, j.lo, j.hi, use_direct=False)
        got = to_host(ex.results[j.rid])
        assert rel_l2(got, ref) <= 1e-6, (j.rid, j.n, j.greens, j.lo, j.hi)
        assert elem_err(got, ref) <= F32_ELEM, (j.rid, j.n, j.greens, j.lo, j.hi)


def test_serve_survives_a_failed_allocation(torch_cuda):
    """A plan that cannot get its device memory (forced on the host: the executor's third
    buffer-owning plan, the first 64^3 request's, raises FSP_ERR_OUT_OF_MEMORY) fails its
    launch alone; the next 64^3 request builds that plan again, every other
    request is served and matches the oracle, and the executor serves a later run whole."""
    torch = torch_cuda
    from paper_2405_02603_amd import FspError, _lib
    from paper_2405_02603_amd.serve import GpuExecutor, Job, Server

    def jobs_from(base, count):
        return [Job(rid=base + i, t_arrival=0.0005 * i, n=(32, 48, 64)[i % 3], greens="hockney") for i in range(count)]

    first, second = jobs_from(0, 10), jobs_from(100, 10)
    host = {j.rid: W.source_density(j.n, (-1.0,) * 3, (1.0,) * 3, W.multiblob(seed=3000 + j.rid))
            for j in first + second}
    pinned = {rid: torch.from_numpy(h).to(torch.float32).pin_memory() for rid, h in host.items()}
    ex = GpuExecutor(slots=2, source_for=lambda j, dt: pinned[j.rid], keep_results=True)
    real_plan, made = ex.Plan, [0]

    def plan_factory(*args, **kw):
        if kw.get("bind", True):
            made[0] += 1
            if made[0] == 3:
                raise FspError(_lib.FSP_ERR_OUT_OF_MEMORY, "fsp_plan_bind: FSP_ERR_OUT_OF_MEMORY: injected")
        return real_plan(*args, **kw)

    ex.Plan = plan_factory
    rep = Server(ex, budget_bytes=1 << 30, slots=2, max_fold=1).run(first)
    torch.cuda.synchronize()
    failed = [j for j in first if j.status == "failed"]
    assert rep["failed"] == len(failed) == 1 and "OUT_OF_MEMORY" in failed[0].error, rep
    assert failed[0].rid == 2 and failed[0].n == 64
    assert rep["done"] == len(first) - 1
    rep2 = Server(ex, budget_bytes=1 << 30, slots=2, max_fold=1).run(second)
    torch.cuda.synchronize()
    assert rep2["done"] == len(second) and rep2["failed"] == 0
    for j in first + second:
        if j.status != "done":
            continue
        ref = reference(host[j.rid], "hockney", (-1.0,) * 3, (1.0,) * 3, use_direct=False)
        got = to_host(ex.results[j.rid])
        assert rel_l2(got, ref) <= 1e-6 and elem_err(got, ref) <= F32_ELEM, (j.rid, j.n)
