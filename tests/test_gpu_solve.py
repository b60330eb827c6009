"""GPU parity: the HIP solve through the C ABI against the CPU oracle.

Bars (stated per result):
* float64 solves: relative L2 error <= 1e-12 against the oracle;
* float32 solves: relative L2 error <= 1e-6 (grids up to 256^3) against the
  float64 oracle; the transform is computed in float64 and rounded once, the
  passes accumulate in float32.
Sizes span one to several column tiles, the Nyquist-column tail tile,
3 * 2^a lengths (radix 3) and anisotropic grids and boxes.
"""
import numpy as np
import pytest

import workloads as W
from oracle import exact, greens

from gpu_util import F32_ELEM, F64_ELEM, elem_err, gaussian_rho, kernel_octant, reference, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _plan(n, lo, hi, kind, prec):
    from paper_2405_02603_amd import Plan
    return Plan(n=n, lo=lo, hi=hi, greens=kind, prec=prec)


def _solve(torch, n, lo, hi, kind, prec, rho):
    plan = _plan(n, lo, hi, kind, prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    phi = plan.solve(to_dev(rho, dt))
    torch.cuda.synchronize()
    return to_host(phi), plan


def test_config1_hockney_f64(torch_cuda):
    """Hockney-Eastwood, float64, 32^3 on [-0.5, 0.5]^3: equals the direct sum; error vs the
    closed form is the paper's ~1e-2 at 32^3 (Table 3)."""
    n, lo, hi = 32, (-0.5,) * 3, (0.5,) * 3
    rho = gaussian_rho(n, lo, hi)
    phi, _ = _solve(torch_cuda, n, lo, hi, "hockney", "f64", rho)
    ref = reference(rho, "hockney", lo, hi, use_direct=True)
    assert rel_l2(phi, ref) <= F64_TOL
    err = rel_l2(phi, exact.source_potential(n, lo, hi, W.centred_gaussian(0.05)))
    assert 5e-3 < err < 3e-2


@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
@pytest.mark.parametrize("n,lo,hi", [
    (8, (-0.5,) * 3, (0.5,) * 3),
    (12, (-1.0,) * 3, (1.0,) * 3),
    (16, (0.0,) * 3, (1.0,) * 3),
    (24, (-0.5,) * 3, (0.5,) * 3),
    ((8, 12, 16), (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0)),
    ((16, 8, 24), (0.0, 0.0, 0.0), (1.0, 0.75, 1.5)),
])
def test_random_source_f64_vs_direct_sum(torch_cuda, kind, n, lo, hi):
    n3 = W._as3(n, int)
    rho = W.random_field(n3, 7)
    phi, _ = _solve(torch_cuda, n3, lo, hi, kind, "f64", rho)
    ref = reference(rho, kind, lo, hi, use_direct=True)
    assert rel_l2(phi, ref) <= F64_TOL


@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
@pytest.mark.parametrize("n", [32, 48, 64, 96, (32, 64, 48)])
def test_sizes_f64_and_f32_vs_fft_route(torch_cuda, kind, n):
    n3 = W._as3(n, int)
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    rho = W.source_density(n3, lo, hi, W.multiblob(3))
    ref = reference(rho, kind, lo, hi, use_direct=False)
    phi64, _ = _solve(torch_cuda, n3, lo, hi, kind, "f64", rho)
    assert rel_l2(phi64, ref) <= F64_TOL
    assert elem_err(phi64, ref) <= F64_ELEM
    phi32, _ = _solve(torch_cuda, n3, lo, hi, kind, "f32", rho)
    assert rel_l2(phi32, ref) <= F32_TOL
    assert elem_err(phi32, ref) <= F32_ELEM


@pytest.mark.parametrize("kind", ["hockney", "vico_dct", "vico"])
@pytest.mark.parametrize("n,lo,hi", [
    (8, (-0.5,) * 3, (0.5,) * 3),
    ((8, 12, 16), (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0)),
    (32, (-1.0,) * 3, (1.0,) * 3),
])
def test_green_octant_f64(torch_cuda, kind, n, lo, hi):
    """The stored transform equals the oracle's DCT-I of the kernel octant, times V/(8 n0 n1 n2)."""
    n3 = W._as3(n, int)
    plan = _plan(n3, lo, hi, kind, "f64")
    torch_cuda.cuda.synchronize()
    got = to_host(plan.ghat_octant())
    k = kernel_octant(kind, n3, lo, hi)
    h = greens.spacing(n3, lo, hi)
    want = greens.mirror_transform_octant(k) * (h[0] * h[1] * h[2]) / (8.0 * n3[0] * n3[1] * n3[2])
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_in_place(torch_cuda):
    torch = torch_cuda
    n, lo, hi = (16, 24, 32), (-1.0,) * 3, (1.0,) * 3
    rho = W.random_field(n, 3)
    plan = _plan(n, lo, hi, "vico_dct", "f64")
    t = to_dev(rho, torch.float64)
    plan.solve(t, out=t)
    torch.cuda.synchronize()
    assert rel_l2(to_host(t), reference(rho, "vico_dct", lo, hi, use_direct=False)) <= F64_TOL


@pytest.mark.parametrize("prec,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128, (64, 96, 48),
                               (512, 16, 24), (16, 512, 16), (384, 12, 16), (16, 384, 8),
                               (8, 12, 512), (12, 8, 384), (12, 8, 256), (8, 24, 256), (256, 12, 8),
                               (192, 12, 8), (12, 192, 192)])
def test_every_schedule_variant(torch_cuda, prec, tol, n):
    """Every kernel variant the autotuner may pick gives the oracle's result (the last grids put
    pencils of 1024 and 768 points on axes 0 and 1, and rows of 512, 384 and 256 on axis 2: the
    rows of 256 run in blocks of several row groups; the last puts 512-point pencils on axis 0,
    whose variant 1 in float32 exchanges real and imaginary parts in turn; the two after it put
    384-point pencils on axes 0 and 1 and rows of 192 on axis 2, whose plan 1 ends in radix 24)."""
    from paper_2405_02603_amd import _lib
    torch = torch_cuda
    n3 = W._as3(n, int)
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    rho = W.random_field(n3, 13)
    ref = reference(rho, "vico_dct", lo, hi, use_direct=max(n3) <= 16)
    plan = _plan(n3, lo, hi, "vico_dct", prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    r = to_dev(rho, dt)
    for v in range(_lib.NUM_VARIANTS):
        plan.schedule = [v] * 5
        phi = to_host(plan.solve(r))
        torch.cuda.synchronize()
        assert rel_l2(phi, ref) <= tol, f"variant {v}"
        assert elem_err(phi, ref) <= 6 * tol, f"variant {v}"


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_autotune_256(torch_cuda, prec):
    """The autotuner at the benchmark size: timings for every variant, and the tuned
    schedule still matches the oracle."""
    torch = torch_cuda
    n, lo, hi = 256, (-1.0,) * 3, (1.0,) * 3
    rho = W.source_density(n, lo, hi, W.multiblob(3))
    plan = _plan(n, lo, hi, "vico_dct", prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    r = to_dev(rho, dt)
    times = plan.autotune(r, reps=2)
    torch.cuda.synchronize()
    assert all(t > 0 for p in range(5) for t in times[p])
    assert times["solve_fused"] == 0.0        # 256^3 is too large for the fused slab schedule
    assert times["solve_plane"] == 0.0        # and for the plane kernels
    sched = plan.schedule
    for p in range(5):
        assert times[p][sched[p]] == min(times[p])
    phi = plan.solve(r)
    torch.cuda.synchronize()
    ref = reference(rho, "vico_dct", lo, hi, use_direct=False)
    assert rel_l2(to_host(phi), ref) <= (F64_TOL if prec == "f64" else F32_TOL)
    for v in range(3):
        plan.schedule = [v] * 5  # every variant at the benchmark size
        phi = plan.solve(r)
        torch.cuda.synchronize()
        assert rel_l2(to_host(phi), ref) <= (F64_TOL if prec == "f64" else F32_TOL), f"variant {v}"
    print("autotune", prec, sched, {p: [round(t, 4) for t in times[p]] for p in range(5)})


@pytest.mark.parametrize("prec,tol,sizes", [("f32", F32_TOL, (8, 12, 16, 24, 32, 48, 64)),
                                            ("f64", F64_TOL, (8, 12, 16, 24, 32, 48))])
def test_fused_small_grid_schedule(torch_cuda, prec, tol, sizes):
    """The fused passes 1-3 (slab in LDS) give the oracle's result, for both kernels."""
    from paper_2405_02603_amd import _lib
    torch = torch_cuda
    dt = torch.float64 if prec == "f64" else torch.float32
    for n in sizes:
        for kind in ("hockney", "vico_dct"):
            lo, hi = (-1.0, -1.0, -0.5), (1.0, 1.0, 1.5)
            rho = W.random_field((n, n, n), 17 + n)
            ref = reference(rho, kind, lo, hi, use_direct=n <= 16)
            plan = _plan(n, lo, hi, kind, prec)
            plan.schedule = [0, _lib.FUSED, _lib.FUSED, _lib.FUSED, 0]
            phi = plan.solve(to_dev(rho, dt))
            torch.cuda.synchronize()
            assert rel_l2(to_host(phi), ref) <= tol, (n, kind)


def test_fused_schedule_in_batch_and_anisotropic_n2(torch_cuda):
    """Fused plans in a batched launch; n2 may differ from n0 == n1."""
    from paper_2405_02603_amd import _lib, solve_batched
    torch = torch_cuda
    plans, rhos, refs = [], [], []
    for i, n in enumerate([(32, 32, 48), (32, 32, 48), (16, 16, 8)]):
        lo, hi = (-1.0,) * 3, (1.0,) * 3
        rho = W.random_field(n, 30 + i)
        p = _plan(n, lo, hi, "vico_dct", "f32")
        p.schedule = [0, _lib.FUSED, _lib.FUSED, _lib.FUSED, 0]
        plans.append(p)
        rhos.append(to_dev(rho, torch.float32))
        refs.append(reference(rho, "vico_dct", lo, hi, use_direct=False))
    outs = solve_batched(plans, rhos)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert rel_l2(to_host(o), r) <= F32_TOL


@pytest.mark.parametrize("prec,n", [("f32", 32), ("f32", 64), ("f64", 32), ("f64", 48)])
def test_autotune_fused_sizes(torch_cuda, prec, n):
    """On grids small enough for the fused schedule and the plane kernels the autotuner also
    times whole solves with passes 1-3 fused and with the plane pairs, against the best separate
    passes, and keeps the fastest; whatever it keeps matches the oracle, and so does a solve split
    into pass ranges."""
    from paper_2405_02603_amd import _lib
    torch = torch_cuda
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    rho = W.source_density(n, lo, hi, W.multiblob(5))
    ref = reference(rho, "vico_dct", lo, hi, use_direct=False)
    tol = F64_TOL if prec == "f64" else F32_TOL
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = _plan(n, lo, hi, "vico_dct", prec)
    r = to_dev(rho, dt)
    times = plan.autotune(r, reps=2)
    torch.cuda.synchronize()
    keys = ("solve_separate", "solve_fused", "solve_plane", "solve_plane_fwd", "solve_plane_inv")
    assert all(times[k] > 0 for k in keys)
    P, F = _lib.PLANE, _lib.FUSED
    sched = plan.schedule
    kept = ("solve_fused" if sched[1] == F else "solve_plane" if sched[0] == P and sched[3] == P
            else "solve_plane_fwd" if sched[0] == P else "solve_plane_inv" if sched[3] == P else "solve_separate")
    assert times[kept] == min(times[k] for k in keys), (sched, times)
    assert rel_l2(to_host(plan.solve(r)), ref) <= tol
    plan.schedule = [0, _lib.FUSED, _lib.FUSED, _lib.FUSED, 0]
    phi = torch.empty_like(r)
    plan.solve_passes(r, None, 0, 0)
    plan.solve_passes(None, None, 1, 3)
    plan.solve_passes(None, phi, 4, 4)
    torch.cuda.synchronize()
    assert rel_l2(to_host(phi), ref) <= tol


@pytest.mark.parametrize("prec,tol,etol,sizes", [
    ("f32", F32_TOL, F32_ELEM, (32, 48, 64, 96, 128, (24, 64, 64))),
    ("f64", F64_TOL, F64_ELEM, (32, 48, 64, (16, 48, 48)))])
def test_plane_schedule(torch_cuda, prec, tol, etol, sizes):
    """Passes 0-1 and 3-4 as the plane kernels (the axis-2 spectrum of one i0-plane held in LDS
    between the axis-2 and axis-1 transforms) give the oracle's result element by element, for
    both kernels, with both pairs and with each alone, and a solve split into pass ranges at the
    pairs' boundaries gives the same."""
    from paper_2405_02603_amd import _lib
    torch = torch_cuda
    P = _lib.PLANE
    dt = torch.float64 if prec == "f64" else torch.float32
    for n in sizes:
        n3 = W._as3(n, int)
        for kind in ("hockney", "vico_dct"):
            lo, hi = (-1.0, -1.0, -0.5), (1.0, 1.0, 1.5)
            rho = W.random_field(n3, 40 + n3[0])
            ref = reference(rho, kind, lo, hi, use_direct=False)
            plan = _plan(n3, lo, hi, kind, prec)
            r = to_dev(rho, dt)
            for sched in ([P, P, 0, P, P], [P, P, 1, 0, 2], [2, 1, 2, P, P]):
                plan.schedule = sched
                phi = to_host(plan.solve(r))
                torch.cuda.synchronize()
                assert rel_l2(phi, ref) <= tol, (n, kind, sched)
                assert elem_err(phi, ref) <= etol, (n, kind, sched)
            plan.schedule = [P, P, 0, P, P]
            out = torch.empty_like(r)
            plan.solve_passes(r, None, 0, 1)
            plan.solve_passes(None, None, 2, 2)
            plan.solve_passes(None, out, 3, 4)
            torch.cuda.synchronize()
            assert elem_err(to_host(out), ref) <= etol, (n, kind, "ranges")


def test_plane_schedule_batched_and_in_place(torch_cuda):
    """Plane plans in a batched launch (several items in one plane launch, with a separate-pass
    plan of another shape beside them) equal their solo solves bit for bit and the oracle; an
    in-place plane solve (phi == rho) is correct too."""
    from paper_2405_02603_amd import _lib, solve_batched
    torch = torch_cuda
    P = _lib.PLANE
    plans, rhos, refs = [], [], []
    for i, n in enumerate([(48, 48, 48), (48, 48, 48), (48, 48, 48), (32, 32, 32)]):
        lo, hi = (-1.0,) * 3, (1.0,) * 3
        rho = W.random_field(n, 60 + i)
        p = _plan(n, lo, hi, "vico_dct", "f32")
        p.schedule = [P, P, 0, P, P] if n[0] == 48 else [0, 0, 0, 0, 0]
        plans.append(p)
        rhos.append(to_dev(rho, torch.float32))
        refs.append(reference(rho, "vico_dct", lo, hi, use_direct=False))
    outs = solve_batched(plans, rhos)
    torch.cuda.synchronize()
    for p, r, o, ref in zip(plans, rhos, outs, refs):
        solo = p.solve(r)
        torch.cuda.synchronize()
        assert torch.equal(o, solo)
        assert elem_err(to_host(o), ref) <= F32_ELEM
    t = rhos[0].clone()
    plans[0].solve(t, out=t)
    torch.cuda.synchronize()
    assert elem_err(to_host(t), refs[0]) <= F32_ELEM


@pytest.mark.parametrize("chunks,gather", [("3", "0"), ("1", "0"), ("3", "2048")])
@pytest.mark.parametrize("prec,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_column_chunks_and_gathered_column(torch_cuda, prec, tol, chunks, gather, monkeypatch):
    """Passes 1-3 chunk by chunk over the columns (FSP_CHUNKS at plan creation) and the axis-0
    pass gathering the lone Nyquist column over k1 pairs at any grid size
    (FSP_CONV_GATHER_MIN=0), for every variant."""
    torch = torch_cuda
    monkeypatch.setenv("FSP_CHUNKS", chunks)
    monkeypatch.setenv("FSP_CONV_GATHER_MIN", gather)
    dt = torch.float64 if prec == "f64" else torch.float32
    for n in (16, 32, 64, (48, 64, 96), (96, 32, 128)):
        n3 = W._as3(n, int)
        lo, hi = (-1.0,) * 3, (1.0,) * 3
        rho = W.random_field(n3, 21)
        plan = _plan(n3, lo, hi, "vico_dct", prec)
        for v in range(3):
            plan.schedule = [v] * 5
            phi = plan.solve(to_dev(rho, dt))
            torch.cuda.synchronize()
            assert rel_l2(to_host(phi), reference(rho, "vico_dct", lo, hi, use_direct=False)) <= tol, (n, v)


def test_precompute_from_two_threads(torch_cuda):
    """Two host threads precompute at the same time (each on its own stream): the stored
    transforms equal those of sequential precomputes."""
    import threading
    from paper_2405_02603_amd import Plan
    torch = torch_cuda
    cases = [((48, 32, 64), "vico_dct"), ((32, 64, 48), "hockney")]
    want = []
    for n, kind in cases:
        p = Plan(n=n, lo=(-1.0,) * 3, hi=(1.0,) * 3, greens=kind, prec="f64")
        torch.cuda.synchronize()
        want.append(to_host(p.ghat_octant()))
    got = [None, None]
    errors = []

    def work(i):
        try:
            n, kind = cases[i]
            s = torch.cuda.Stream()
            for _ in range(3):
                p = Plan(n=n, lo=(-1.0,) * 3, hi=(1.0,) * 3, greens=kind, prec="f64", stream=s)
                s.synchronize()
            got[i] = to_host(p.ghat_octant())
        except Exception as e:  # reported below, on the test's thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for g, w in zip(got, want):
        assert np.max(np.abs(g - w)) <= 1e-15 * np.max(np.abs(w))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-6)])
@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
def test_zero_source_and_unit_impulses(torch_cuda, prec, tol, kind):
    """Degenerate sources with an exact answer.  rho = 0 gives phi = 0 exactly.  A unit impulse at
    grid point j gives phi_i = V K[|i - j|] (the kernel table itself, component-wise offsets):
    checked element by element for impulses at both corners and an interior point of an
    anisotropic grid whose rows, pencils and tiles are all ragged."""
    torch = torch_cuda
    n, lo, hi = (24, 12, 48), (-1.0, -0.75, -1.5), (1.0, 0.75, 1.5)
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = _plan(n, lo, hi, kind, prec)
    zero = torch.zeros(n, dtype=dt, device="cuda")
    phi0 = plan.solve(zero)
    torch.cuda.synchronize()
    assert torch.count_nonzero(phi0).item() == 0
    k = kernel_octant(kind, n, lo, hi)
    h = greens.spacing(n, lo, hi)
    vol = h[0] * h[1] * h[2]
    idx = np.indices(n)
    for j in [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (7, 5, 22)]:
        rho = np.zeros(n)
        rho[j] = 1.0
        phi = to_host(plan.solve(to_dev(rho, dt)))
        torch.cuda.synchronize()
        want = vol * k[np.abs(idx[0] - j[0]), np.abs(idx[1] - j[1]), np.abs(idx[2] - j[2])]
        err = np.max(np.abs(phi - want)) / np.max(np.abs(want))
        assert err <= tol, (j, err)
    plan.close()


@pytest.mark.parametrize("prec,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
@pytest.mark.parametrize("n", [16, 24, 48, (64, 96, 48), (12, 8, 384), (32, 24, 127 + 1)])
def test_nan_poisoned_workspace(torch_cuda, prec, tol, n):
    """The workspace is filled with NaN before every solve (every variant, the fused schedule
    where it exists, and the gradient's four spectra): the results still equal the oracle's,
    so no pass reads a workspace element that an earlier pass of the same solve did not write
    (the row padding, the zero half of the doubled grid, the other spectra)."""
    from paper_2405_02603_amd import FspError, Plan, _lib
    torch = torch_cuda
    n3 = W._as3(n, int)
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    rho = W.random_field(n3, 21)
    ref = reference(rho, "vico_dct", lo, hi, use_direct=False)
    plan = Plan(n=n3, lo=lo, hi=hi, greens="vico_dct", prec=prec, grad=True)
    dt = torch.float64 if prec == "f64" else torch.float32
    r = to_dev(rho, dt)
    schedules = [[v] * 5 for v in range(_lib.NUM_VARIANTS)]
    if n3[0] == n3[1]:
        schedules.append([0, 3, 3, 3, 0])
    for sched in schedules:
        try:
            plan.schedule = sched
        except FspError:
            assert sched[1] == 3   # the fused schedule exists only on small grids
            continue
        plan.work_buf.fill_(255)   # every float and double in the workspace is a NaN
        phi = to_host(plan.solve(r))
        torch.cuda.synchronize()
        assert rel_l2(phi, ref) <= tol, sched
        assert elem_err(phi, ref) <= 6 * tol, sched
    plan.schedule = [0] * 5
    plan.work_buf.fill_(255)
    grad, phi = plan.solve_grad(r, want_phi=True)
    torch.cuda.synchronize()
    assert rel_l2(to_host(phi), ref) <= tol
    assert np.all(np.isfinite(to_host(grad)))
