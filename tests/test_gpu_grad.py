"""GPU parity of the gradient solve (fsp_solve_grad) against the float64 oracle.

The oracle's derivative convolution (``oracle.gradient``) is pinned on the CPU
against the closed-form gradient and independent routes; parity with the
paper itself is not available (the paper gives no method for the field), so
these tests hold the GPU to the oracle: float64 <= 1e-12 and float32 <= 1e-6
relative L2 per component, and to the closed form's convergence orders.
"""
import numpy as np
import pytest

import workloads as W
from oracle import exact, greens
from oracle import gradient as G

from gpu_util import reference, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _dtable(kind, n, lo, hi, a):
    if kind == "hockney":
        return G.hockney_grad_octant(n, lo, hi, a)
    return G.vico_grad_octant(n, lo, hi, a)


def _grad_ref(rho, kind, lo, hi, direct=False):
    n = rho.shape
    h = greens.spacing(n, lo, hi)
    out = []
    for a in range(3):
        d = _dtable(kind, n, lo, hi, a)
        out.append(G.convolve_odd(rho, d, h, a) if direct else G.fftroute_grad(rho, d, h, a))
    return out


def _plan(n, lo, hi, kind, prec):
    from paper_2405_02603_amd import Plan
    return Plan(n=n, lo=lo, hi=hi, greens=kind, prec=prec, grad=True)


@pytest.mark.parametrize("kind", ["hockney", "vico_dct", "vico"])
@pytest.mark.parametrize("n,lo,hi", [
    (8, (-0.5,) * 3, (0.5,) * 3),
    ((8, 12, 16), (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0)),
    (32, (-1.0,) * 3, (1.0,) * 3),
])
def test_derivative_octants_f64(torch_cuda, kind, n, lo, hi):
    """Stored derivative tables: the sine/cosine transform of the oracle's table, times V/(8 n0 n1 n2)."""
    n3 = W._as3(n, int)
    plan = _plan(n3, lo, hi, kind, "f64")
    torch_cuda.cuda.synchronize()
    h = greens.spacing(n3, lo, hi)
    scale = h[0] * h[1] * h[2] / (8.0 * n3[0] * n3[1] * n3[2])
    for a in range(3):
        got = to_host(plan.ghat_octant(1 + a))
        want = G.odd_transform_octant(_dtable(kind, n3, lo, hi, a), a) * scale
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), (kind, a)


@pytest.mark.parametrize("prec,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
def test_gradient_vs_oracle_every_schedule(torch_cuda, kind, prec, tol):
    """Components and the potential from one call, for every kernel variant; small grids against
    the direct odd sum, larger ones against the FFT route (the axis-0 pencils of 96, 192 and 384
    points take plans ending in radix 12 and 24 in variant 1)."""
    from paper_2405_02603_amd import _lib
    torch = torch_cuda
    dt = torch.float64 if prec == "f64" else torch.float32
    cases = [(8, (-0.5,) * 3, (0.5,) * 3), ((8, 12, 16), (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0)),
             (24, (0.0,) * 3, (1.0,) * 3), (48, (-1.0,) * 3, (1.0,) * 3), ((32, 64, 48), (-1.0,) * 3, (1.0,) * 3),
             (64, (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0)),
             ((96, 16, 24), (-1.0,) * 3, (1.0,) * 3), ((192, 8, 12), (-1.0,) * 3, (1.0,) * 3)]
    for n, lo, hi in cases:
        n3 = W._as3(n, int)
        rho = W.random_field(n3, 41)
        small = max(n3) <= 16
        refs = _grad_ref(rho, kind, lo, hi, direct=small)
        phi_ref = reference(rho, kind, lo, hi, use_direct=small)
        plan = _plan(n3, lo, hi, kind, prec)
        r = to_dev(rho, dt)
        scheds = [[v] * 5 for v in range(_lib.NUM_VARIANTS)]
        if n3[0] == n3[1] and n3[0] <= 48:
            scheds.append([0, _lib.FUSED, _lib.FUSED, _lib.FUSED, 0])   # passes 1-3 run separately here
        if n3[1] == n3[2] and n3[2] in ((32, 48, 64, 96, 128) if prec == "f32" else (32, 48, 64)):
            P = _lib.PLANE   # the plane kernels: passes 3-4 take the four outputs as items
            scheds += [[P, P, 0, P, P], [P, P, 1, 0, 0], [0, 0, 2, P, P]]
        for sched in scheds:
            plan.schedule = sched
            grad, phi = plan.solve_grad(r, want_phi=True)
            torch.cuda.synchronize()
            g = to_host(grad)
            for a in range(3):
                assert rel_l2(g[a], refs[a]) <= tol, (n, sched, a, rel_l2(g[a], refs[a]))
            assert rel_l2(to_host(phi), phi_ref) <= tol, (n, sched)


def test_gradient_in_place_phi_and_no_phi(torch_cuda):
    """phi may be rho; without phi only the gradient is written."""
    torch = torch_cuda
    n, lo, hi = (16, 24, 32), (-1.0,) * 3, (1.0,) * 3
    rho = W.random_field(n, 5)
    refs = _grad_ref(rho, "vico_dct", lo, hi)
    phi_ref = reference(rho, "vico_dct", lo, hi, use_direct=False)
    plan = _plan(n, lo, hi, "vico_dct", "f64")
    t = to_dev(rho, torch.float64)
    grad, phi = plan.solve_grad(t, phi=t)
    torch.cuda.synchronize()
    assert rel_l2(to_host(t), phi_ref) <= F64_TOL
    g = to_host(grad)
    assert max(rel_l2(g[a], refs[a]) for a in range(3)) <= F64_TOL
    grad2, none = plan.solve_grad(to_dev(rho, torch.float64))
    torch.cuda.synchronize()
    assert none is None and np.array_equal(to_host(grad2), g)


def test_gradient_convergence_to_closed_form(torch_cuda):
    """Centred sigma = 0.05 Gaussian on the unit cube: Hockney-Eastwood second order,
    Vico-Greengard spectral, as the oracle."""
    torch = torch_cuda
    lo, hi = (-0.5,) * 3, (0.5,) * 3
    src = W.centred_gaussian(0.05)
    err = {}
    for kind in ("hockney", "vico_dct"):
        for n in (16, 32, 64, 128):
            rho = W.source_density(n, lo, hi, src)
            ex = exact.source_gradient(n, lo, hi, src)
            plan = _plan(n, lo, hi, kind, "f64")
            grad, _ = plan.solve_grad(to_dev(rho, torch.float64))
            torch.cuda.synchronize()
            g = to_host(grad)
            err[(kind, n)] = max(rel_l2(g[a], ex[a]) for a in range(3))
            plan.close()
    for n in (16, 32, 64):
        order = np.log2(err[("hockney", n)] / err[("hockney", 2 * n)])
        assert 1.8 <= order <= 2.2, (n, order)
    assert 1e-8 < err[("vico_dct", 32)] < 1e-5 and err[("vico_dct", 64)] < 1e-13 and err[("vico_dct", 128)] < 1e-13
    print("grad convergence", {f"{k}_{n}": f"{e:.3e}" for (k, n), e in sorted(err.items())})


@pytest.mark.parametrize("kind", ["vico_dct", "hockney"])
def test_gradient_full_size_256(torch_cuda, kind):
    """256^3 on [-1,1]^3 with the 8-Gaussian source (seed 3), autotuned schedule: every
    component against the float64 oracle, both precisions."""
    torch = torch_cuda
    n, lo, hi = 256, (-1.0,) * 3, (1.0,) * 3
    rho = W.source_density(n, lo, hi, W.multiblob(seed=3, count=8))
    refs = _grad_ref(rho, kind, lo, hi)
    for prec, tol in (("f64", F64_TOL), ("f32", F32_TOL)):
        dt = torch.float64 if prec == "f64" else torch.float32
        plan = _plan(n, lo, hi, kind, prec)
        r = to_dev(rho, dt)
        plan.autotune(r, reps=2)
        grad, _ = plan.solve_grad(r)
        torch.cuda.synchronize()
        g = to_host(grad)
        errs = [rel_l2(g[a], refs[a]) for a in range(3)]
        print("grad 256", kind, prec, [f"{e:.3e}" for e in errs])
        assert max(errs) <= tol
        plan.close()
        del r, grad
        torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_gradient_long_axis0_pencils_every_variant(torch_cuda, prec, tol):
    """Axis-0 pencils of 256 to 1024 points (the gradient's own tile shapes, several tiles and a
    ragged last column along axis 2), every variant of that pass, against the oracle."""
    torch = torch_cuda
    dt = torch.float64 if prec == "f64" else torch.float32
    lo, hi = (-1.0, -0.5, -0.75), (1.0, 0.5, 0.75)
    for n in [(128, 12, 24), (256, 8, 48), (384, 8, 12), (512, 8, 24)]:
        rho = W.random_field(n, 17)
        refs = _grad_ref(rho, "vico_dct", lo, hi)
        phi_ref = reference(rho, "vico_dct", lo, hi, use_direct=False)
        plan = _plan(n, lo, hi, "vico_dct", prec)
        r = to_dev(rho, dt)
        for v in (0, 1, 2):
            plan.schedule = [0, 0, v, 0, 0]
            grad, phi = plan.solve_grad(r, want_phi=True)
            torch.cuda.synchronize()
            g = to_host(grad)
            errs = [rel_l2(g[a], refs[a]) for a in range(3)]
            assert max(errs) <= tol, (n, v, errs)
            assert rel_l2(to_host(phi), phi_ref) <= tol, (n, v)
        plan.close()


@pytest.mark.parametrize("prec,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
def test_gradient_of_unit_impulses(torch_cuda, prec, tol, kind):
    """A unit impulse at grid point j: component a is V D_a at the offset i - j, where the table
    D_a is odd along axis a (its octant value, negated where i_a < j_a); every variant of the
    axis-0 pass, element by element."""
    torch = torch_cuda
    n, lo, hi = (24, 12, 48), (-1.0, -0.75, -1.5), (1.0, 0.75, 1.5)
    dt = torch.float64 if prec == "f64" else torch.float32
    h = greens.spacing(n, lo, hi)
    vol = h[0] * h[1] * h[2]
    d = [_dtable(kind, n, lo, hi, a) for a in range(3)]
    idx = np.indices(n)
    plan = _plan(n, lo, hi, kind, prec)
    for v in range(3):
        plan.schedule = [0, 0, v, 0, 0]
        for j in [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (7, 5, 22)]:
            rho = np.zeros(n)
            rho[j] = 1.0
            grad, _ = plan.solve_grad(to_dev(rho, dt))
            torch.cuda.synchronize()
            g = to_host(grad)
            off = [idx[a] - j[a] for a in range(3)]
            for a in range(3):
                want = vol * np.sign(off[a]) * d[a][np.abs(off[0]), np.abs(off[1]), np.abs(off[2])]
                err = np.max(np.abs(g[a] - want)) / np.max(np.abs(want))
                assert err <= tol, (v, j, a, err)
    plan.close()


@pytest.mark.parametrize("lo,hi", [((-1.0,) * 3, (1.0,) * 3), ((-1.0, -1.0, -2.0), (1.0, 1.0, 2.0))],
                         ids=["cube", "slab"])
def test_gradient_full_size_512_sampled(torch_cuda, lo, hi):
    """512^3 on [-1,1]^3 and on [-1,1]^2 x [-2,2] (h2 = 2 h0) with the 8-Gaussian source (seed 3),
    Hockney-Eastwood (closed-form derivative tables), autotuned: every component against the
    literal odd sum at sampled outputs, corners included, in both precisions."""
    torch = torch_cuda
    n = 512
    rho = W.source_density(n, lo, hi, W.multiblob(seed=3, count=8))
    h = greens.spacing((n,) * 3, lo, hi)
    rng = np.random.default_rng(12)
    pts = [tuple(int(v) for v in rng.integers(0, n, size=3)) for _ in range(4)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, n // 3, n - 1)]
    want = []
    for a in range(3):
        d = G.hockney_grad_octant((n,) * 3, lo, hi, a)
        want.append(G.convolve_odd_at(rho, d, h, a, pts))
        del d
    for prec, tol in (("f64", 1e-12), ("f32", 1e-6)):
        dt = torch.float64 if prec == "f64" else torch.float32
        plan = _plan(n, lo, hi, "hockney", prec)
        r = to_dev(rho, dt)
        plan.autotune(r, reps=1)
        grad, _ = plan.solve_grad(r)
        torch.cuda.synchronize()
        for a in range(3):
            got = np.array([grad[a][p].item() for p in pts])
            scale = np.max(np.abs(want[a]))
            assert np.max(np.abs(got - want[a])) <= tol * scale, (prec, a, got, want[a])
        plan.close()
        del r, grad
        torch.cuda.empty_cache()


@pytest.mark.parametrize("prec,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_gradient_with_column_chunks(torch_cuda, prec, tol, monkeypatch):
    """Passes 1-3 chunk by chunk over the axis-2 columns (FSP_CHUNKS at plan creation): each chunk
    runs the gradient's axis-0 pass (all outputs at once, or one launch per output with phi in
    place last), every variant, against the oracle.  193 columns: in float32 (chunk step 64,
    the axis-1 tile of 48-point pencils) the chunks are [0, 128) and [128, 193), in float64
    (step 32) [0, 96), [96, 192) and [192, 193); both last chunks hold one column past a whole
    axis-0 tile, which is gathered over k1 pairs (FSP_CONV_GATHER_MIN=0)."""
    torch = torch_cuda
    monkeypatch.setenv("FSP_CHUNKS", "3")
    monkeypatch.setenv("FSP_CONV_GATHER_MIN", "0")
    n, lo, hi = (32, 24, 192), (-1.0, -1.0, -1.5), (1.0, 1.0, 1.5)
    rho = W.random_field(n, 23)
    refs = _grad_ref(rho, "vico_dct", lo, hi)
    phi_ref = reference(rho, "vico_dct", lo, hi, use_direct=False)
    plan = _plan(n, lo, hi, "vico_dct", prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    r = to_dev(rho, dt)
    for v in range(3):
        plan.schedule = [v] * 5
        grad, phi = plan.solve_grad(r, want_phi=True)
        torch.cuda.synchronize()
        g = to_host(grad)
        for a in range(3):
            assert rel_l2(g[a], refs[a]) <= tol, (v, a)
        assert rel_l2(to_host(phi), phi_ref) <= tol, v
    plan.close()
