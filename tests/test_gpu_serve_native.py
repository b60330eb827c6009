"""GPU: the native serving engine (include/fsp_serve.h) through its binding.

Every served result is checked against the oracle at its own size, Green's
function, box and source, and against the same request solved alone (the same
kernels, so bit for bit).  The budget covers everything the engine holds
(cached Green's transforms, pooled workspaces, refresh transients); a run with
a budget too small for all of it must evict and still stay under the budget.
Requests whose box changes from call to call (a grid fitted to a moving bunch)
each need a new Green's transform, which the engine computes on a miss."""
import numpy as np
import pytest

import workloads as W

from gpu_util import F32_ELEM, elem_err, reference, rel_l2, to_host

# Skipped: a run of these tests left the GPU faulted, and a second run after the fix of the
# cause found (a workspace chosen for reuse could be freed while making room) faulted again.
# No second cause is shown; the engine is switched off in the device build (fsp_server_run
# returns FSP_ERR_DEVICE) and its logic is tested on the CPU against a stand-in device
# (tests/test_serve_engine_host.py).  These tests stay, skipped, until a cause is shown.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="native serving engine switched off: its GPU runs faulted twice, "
                                      "second cause not found (CPU tests cover its logic)")]

TOL = {"f32": 1e-6, "f64": 1e-12}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _requests(torch, specs):
    """specs: (t_arrival, n, greens, prec, lo, hi, seed) -> Requests with their own device
    sources (phi separate) and the matching host float64 sources."""
    from paper_2405_02603_amd.serve_native import Request
    reqs, host = [], []
    for t, n, greens, prec, lo, hi, seed in specs:
        src = W.multiblob(seed=seed)
        dt = torch.float64 if prec == "f64" else torch.float32
        rho = W.source_density_device((n,) * 3, lo, hi, src, dtype=dt)
        reqs.append(Request(t_arrival=t, n=(n,) * 3, greens=greens, prec=prec, lo=lo, hi=hi, rho=rho,
                            phi=torch.full_like(rho, float("nan"))))
        host.append(W.source_density((n,) * 3, lo, hi, src))
    return reqs, host


def _check(torch, reqs, host, results, solo=True):
    from paper_2405_02603_amd import Plan
    for i, (r, h, res) in enumerate(zip(reqs, host, results)):
        assert res["status"] == 0, (i, res)
        ref = reference(h, r.greens, r.lo, r.hi, use_direct=False)
        got = to_host(r.phi)
        assert rel_l2(got, ref) <= TOL[r.prec], (i, r.n, r.greens, r.prec)
        assert elem_err(got, ref) <= 6 * TOL[r.prec], (i, r.n, r.greens, r.prec)
        if solo:
            alone = Plan(n=r.n, lo=r.lo, hi=r.hi, greens=r.greens, prec=r.prec)
            phi = alone.solve(r.rho)
            torch.cuda.synchronize()
            assert torch.equal(phi, r.phi), f"request {i} differs from its solo solve"


def test_serve_mix_against_oracle_and_solo(torch_cuda):
    """Poisson arrivals, sizes 32-96, both Green's functions, float32 with some float64, each
    request its own 8-Gaussian source: every result is the oracle's and its solo solve's."""
    torch = torch_cuda
    from paper_2405_02603_amd.serve_native import Server, summarize
    rng = np.random.default_rng(5)
    t, specs = 0.0, []
    for i in range(40):
        t += float(rng.exponential(1.0 / 400.0))
        n = int((32, 48, 64, 96)[int(rng.integers(0, 4))])
        specs.append((t, n, "hockney" if rng.random() < 0.5 else "vico_dct", "f64" if i % 8 == 3 else "f32",
                      (-1.0,) * 3, (1.0,) * 3, 1000 + i))
    reqs, host = _requests(torch, specs)
    srv = Server(budget_bytes=1 << 30, slots=4, max_fold=8)
    res = srv.run(reqs)
    rep = summarize(res, srv.stats())
    print("serve mix", {k: rep[k] for k in ("p50_ms", "p99_ms", "mean_launch_size", "refreshes", "peak_held_bytes")})
    assert rep["done"] == len(reqs)
    assert rep["peak_held_bytes"] <= rep["budget_bytes"]
    assert rep["p99_ms"] >= rep["p50_ms"] > 0
    # device completion times and the host clock share their zero
    assert -0.5 <= rep["seen_lag_ms"]["min"] and rep["seen_lag_ms"]["p50"] < 20.0, rep["seen_lag_ms"]
    _check(torch, reqs, host, res)
    srv.close()


def test_serve_cold_cache_same_shape_all_at_once(torch_cuda):
    """No warm-up, every request arrives at once, one request per launch on three slots: the
    first solves of each shape read a Green's transform still being computed on the refresh
    stream; each waits for it on the device, so every result is right."""
    torch = torch_cuda
    from paper_2405_02603_amd.serve_native import Server
    specs = [(0.0, 64 if i % 3 else 48, "vico_dct" if i % 2 else "hockney", "f32", (-1.0,) * 3, (1.0,) * 3, 2000 + i)
             for i in range(12)]
    reqs, host = _requests(torch, specs)
    srv = Server(budget_bytes=1 << 30, slots=3, max_fold=1)
    res = srv.run(reqs, time_scale=0.0)
    assert len({r["slot"] for r in res}) > 1
    assert all(r["launch_size"] == 1 for r in res)
    assert sum(r["refresh_ms"] > 0 for r in res) >= 4   # the first of each of the 4 shapes waited
    _check(torch, reqs, host, res, solo=False)
    srv.close()


def test_serve_budget_evicts_and_never_exceeds(torch_cuda):
    """A budget that holds one 96^3 request's Green's buffer, transients and workspace but not
    the cache of every shape and box: the engine frees idle buffers (least recently used
    first) and the bytes it holds never exceed the budget."""
    torch = torch_cuda
    from paper_2405_02603_amd import Plan
    from paper_2405_02603_amd.serve_native import Server, summarize
    p = Plan(n=96, lo=(-1.0,) * 3, hi=(1.0,) * 3, greens="vico_dct", prec="f32", bind=False)
    one = p.ghat_bytes + p.precompute_bytes + p.work_bytes
    budget = int(one * 1.05)   # one 96^3 admission with a refresh, and little beside it
    boxes = [((-1.0,) * 3, (1.0,) * 3), ((-0.8,) * 3, (0.8,) * 3), ((-1.0, -1.0, -1.5), (1.0, 1.0, 1.5))]
    specs = []
    for i in range(12):
        lo, hi = boxes[i % 3]
        specs.append((0.002 * i, 96 if i % 2 == 0 else 48, "vico_dct", "f32", lo, hi, 3000 + i))
    reqs, host = _requests(torch, specs)
    srv = Server(budget_bytes=budget, slots=1, max_fold=2)
    res = srv.run(reqs)
    st = srv.stats()
    rep = summarize(res, st)
    print("serve budget", {k: rep[k] for k in ("peak_held_bytes", "budget_bytes", "evictions", "refreshes")})
    assert st["peak_held_bytes"] <= budget
    assert st["evictions"] > 0
    _check(torch, reqs, host, res, solo=False)
    srv.close()


def test_serve_box_changes_every_call(torch_cuda):
    """A bunch-fitted grid: each request's box differs (it shrinks step by step), so each needs
    its own Green's transform; the engine computes it on a miss, the request waits for it, the
    refresh time is reported with the request, and every result is the oracle's for its box."""
    torch = torch_cuda
    from paper_2405_02603_amd.serve_native import Server, summarize
    specs = []
    for i in range(8):
        a = 1.0 - 0.05 * i
        lo, hi = (-a, -a, -1.2 * a), (a, a, 1.2 * a)
        specs.append((0.003 * i, 48, "vico_dct" if i % 2 == 0 else "hockney", "f32", lo, hi, 4000 + i))
    reqs, host = _requests(torch, specs)
    srv = Server(budget_bytes=1 << 30, slots=2, max_fold=4)
    res = srv.run(reqs)
    rep = summarize(res, srv.stats())
    print("serve boxes", {k: rep[k] for k in ("refreshes", "refreshed_requests", "refresh_share", "p50_ms")})
    assert rep["refreshes"] == len(reqs)
    assert rep["refreshed_requests"] == len(reqs)
    assert all(r["refresh_ms"] > 0 for r in res)
    assert 0.0 < rep["refresh_share"] < 1.0
    _check(torch, reqs, host, res, solo=False)
    srv.close()


def test_serve_rejects_over_budget(torch_cuda):
    torch = torch_cuda
    from paper_2405_02603_amd import _lib
    from paper_2405_02603_amd.serve_native import Server
    specs = [(0.0, 96, "hockney", "f32", (-1.0,) * 3, (1.0,) * 3, 5000), (0.0, 32, "hockney", "f32", (-1.0,) * 3,
                                                                          (1.0,) * 3, 5001)]
    reqs, host = _requests(torch, specs)
    srv = Server(budget_bytes=8 << 20, slots=2)   # 8 MiB: a 32^3 request fits, a 96^3 one does not
    res = srv.run(reqs)
    assert res[0]["status"] == _lib.FSP_ERR_OUT_OF_MEMORY
    assert res[1]["status"] == 0
    assert srv.stats()["rejected"] == 1
    _check(torch, reqs[1:], host[1:], res[1:], solo=False)
    srv.close()
