"""Pins of the gradient oracle (no GPU).

The paper names the field E = -grad(phi) (Appendix B) but gives no method;
the oracle differentiates the kernel (see ``oracle.gradient``).  What pins it:
the closed-form gradient of the Gaussian potential (checked itself against a
finite difference of the closed-form potential), the convergence of both
kernels to it (second order for Hockney-Eastwood, spectral for
Vico-Greengard), two independent routes to the Vico-Greengard derivative table,
the FFT route against the direct odd sum, and the transform of the odd
extension against a library FFT of it.
"""
import numpy as np
import pytest

import workloads as W
from oracle import exact, greens
from oracle import gradient as G

UNIT = ((-0.5,) * 3, (0.5,) * 3)


def test_closed_form_gradient_is_the_derivative_of_the_closed_form_potential():
    n, lo, hi = (20, 24, 28), (-0.5, -0.6, -0.7), (0.5, 0.6, 0.7)
    src = W.Source(blobs=(W.Blob((0.05, -0.1, 0.02), 0.1, 1.3), W.Blob((-0.2, 0.15, 0.1), 0.06, 0.7)))
    g = exact.source_gradient(n, lo, hi, src)
    eps = 1e-5
    for a in range(3):
        lp, hp, lm, hm = list(lo), list(hi), list(lo), list(hi)
        lp[a] += eps
        hp[a] += eps
        lm[a] -= eps
        hm[a] -= eps
        fd = (exact.source_potential(n, tuple(lp), tuple(hp), src)
              - exact.source_potential(n, tuple(lm), tuple(hm), src)) / (2 * eps)
        assert np.max(np.abs(fd - g[a])) <= 1e-7 * np.max(np.abs(g[a]))


def test_closed_form_gradient_near_the_centre():
    """The series branch (u < 1e-2) joins the direct formula smoothly, and the gradient is 0 at r = 0."""
    sigma = 0.05
    n, lo, hi = (8, 8, 8), (-4e-4,) * 3, (4e-4,) * 3            # r / sigma up to ~1.4e-2
    g = exact.gaussian_gradient(n, lo, hi, (0.0, 0.0, 0.0), sigma)
    x = W.axis_centres(n, lo, hi)[0]
    r = np.sqrt(3) * np.abs(x[0])
    # small r: dphi/dr ~ -r / (6 sqrt(2 pi) pi sigma^3) ... times x_a / r
    want = -x[0] / (3.0 * (2 * np.pi) ** 1.5 * sigma ** 3)
    assert g[0][0, 0, 0] == pytest.approx(want, rel=1e-3)
    assert r > 0
    g0 = exact.gaussian_gradient((3, 3, 3), (-1.5,) * 3, (1.5,) * 3, (0.0, 0.0, 0.0), 0.5)
    assert np.all(g0[:, 1, 1, 1] == 0.0)


def test_direct_odd_sum_equals_loops():
    n, lo, hi = (3, 4, 5), (0.0, 0.0, 0.0), (1.0, 1.2, 1.5)
    rho = W.random_field(n, 1)
    h = greens.spacing(n, lo, hi)
    for a in range(3):
        d = G.hockney_grad_octant(n, lo, hi, a)
        assert np.max(np.abs(G.convolve_odd(rho, d, h, a) - G.convolve_odd_loops(rho, d, h, a))) < 1e-15


def test_odd_sum_at_points_equals_the_whole_grid_sum():
    """The sampled sum (used at sizes where the whole-grid sum is out of reach) against the
    whole-grid sum, which is itself pinned to six plain loops."""
    n, lo, hi = (6, 8, 10), (-1.0, -1.0, -1.0), (1.0, 1.5, 2.0)
    rho = W.random_field(n, 4)
    h = greens.spacing(n, lo, hi)
    pts = [(0, 0, 0), (5, 7, 9), (2, 3, 4), (5, 0, 9), (0, 7, 0)]
    for a in range(3):
        for d in (G.hockney_grad_octant(n, lo, hi, a), G.vico_grad_octant(n, lo, hi, a)):
            whole = G.convolve_odd(rho, d, h, a)
            got = G.convolve_odd_at(rho, d, h, a, pts)
            want = np.array([whole[p] for p in pts])
            assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(whole))


@pytest.mark.parametrize("kind", ["hockney", "vico"])
def test_fft_route_equals_direct_odd_sum(kind):
    n, lo, hi = (6, 8, 10), (-1.0, -1.0, -1.0), (1.0, 1.5, 2.0)
    rho = W.random_field(n, 2)
    h = greens.spacing(n, lo, hi)
    for a in range(3):
        d = G.hockney_grad_octant(n, lo, hi, a) if kind == "hockney" else G.vico_grad_octant(n, lo, hi, a)
        x = G.convolve_odd(rho, d, h, a)
        y = G.fftroute_grad(rho, d, h, a)
        assert np.max(np.abs(x - y)) <= 1e-13 * np.max(np.abs(x))


def test_vico_derivative_table_two_routes():
    """Sine sums over the (2n+1) non-negative frequencies vs a full (4n)^3 inverse FFT of i k_a Ghat_L."""
    n, lo, hi = (8, 12, 16), (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0)
    for a in range(3):
        k1 = G.vico_grad_octant(n, lo, hi, a)
        k2 = G.vico_grad_octant_4n(n, lo, hi, a)
        assert np.max(np.abs(k1 - k2)) <= 1e-14 * np.max(np.abs(k1))


def test_hockney_derivative_table_is_odd_and_matches_the_kernel_derivative():
    n, lo, hi = (8, 10, 12), (0.0, 0.0, 0.0), (1.0, 1.25, 1.5)
    h = greens.spacing(n, lo, hi)
    k = greens.hockney_octant(n, lo, hi)
    for a in range(3):
        d = G.hockney_grad_octant(n, lo, hi, a)
        assert d[0, 0, 0] == 0.0
        sl = [slice(None)] * 3
        sl[a] = 0
        assert np.all(d[tuple(sl)] == 0.0)            # x_a = 0: the derivative of an even function
        # d/dx_a of 1/(4 pi r) is -x_a / r^2 times the kernel
        m = np.indices(d.shape).astype(float)
        x = [m[e] * h[e] for e in range(3)]
        r2 = x[0] ** 2 + x[1] ** 2 + x[2] ** 2
        r2[0, 0, 0] = 1.0
        want = -x[a] / r2 * k
        want[0, 0, 0] = 0.0
        assert np.allclose(d, want, rtol=1e-14, atol=0)


def test_odd_transform_equals_fft_of_the_odd_extension():
    n, lo, hi = (6, 8, 10), (-1.0, -1.0, -1.0), (1.0, 1.5, 2.0)
    for a in range(3):
        d = G.vico_grad_octant(n, lo, hi, a)
        t = G.odd_transform_octant(d, a)
        f = np.fft.fftn(G.odd_extend(d, a))
        assert np.max(np.abs(f[: n[0] + 1, : n[1] + 1, : n[2] + 1] - (-1j * t))) <= 1e-13 * np.max(np.abs(t))
        # T is odd along a: its k_a = 0 and k_a = n_a planes vanish
        sl = [slice(None)] * 3
        sl[a] = 0
        assert np.max(np.abs(t[tuple(sl)])) <= 1e-15 * np.max(np.abs(t))


def _grad_errors(kind, n):
    src = W.centred_gaussian(0.05)
    rho = W.source_density(n, *UNIT, src)
    h = greens.spacing((n,) * 3, *UNIT)
    ex = exact.source_gradient(n, *UNIT, src)
    errs = []
    for a in range(3):
        d = G.hockney_grad_octant(n, *UNIT, a) if kind == "hockney" else G.vico_grad_octant(n, *UNIT, a)
        y = G.fftroute_grad(rho, d, h, a)
        errs.append(np.linalg.norm(y - ex[a]) / np.linalg.norm(ex[a]))
    return errs


def test_gradient_convergence_to_the_closed_form():
    """Hockney-Eastwood: second order (1.1e-1, 2.7e-2, 6.9e-3 at 16, 32, 64); Vico-Greengard:
    spectral (1.8e-2, 5.5e-7, ~1e-15)."""
    he = [max(_grad_errors("hockney", n)) for n in (16, 32, 64)]
    for e0, e1 in zip(he, he[1:]):
        assert 1.8 <= np.log2(e0 / e1) <= 2.2
    vg = [max(_grad_errors("vico", n)) for n in (16, 32, 64)]
    assert 1e-3 < vg[0] < 1e-1 and 1e-8 < vg[1] < 1e-5 and vg[2] < 1e-13
