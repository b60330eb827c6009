"""Pins of the mixed open/periodic oracle (oracle/mixed.py, Section 2.2 step 1).

* With every axis open it is the aperiodic sum already pinned (direct.convolve).
* It equals six plain loops on tiny grids, every mask of periodic axes.
* The FFT route that doubles only the open axes (the paper's step 1 taken
  literally) equals the sum, every mask, anisotropic grids, both kernels.
* A cyclic shift of rho along a periodic axis shifts phi the same way, exactly
  (fails if the nearest image is not taken); along an open axis it does not.
* A source confined to fewer than half the points of a periodic axis gives,
  at outputs inside its support, the all-open result (nearest image = the
  offset itself there).
* The table identity the device uses: the aperiodic sum with the table folded
  on the periodic axes equals the mixed sum.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import direct, greens, mixed

MASKS = list(itertools.product([False, True], repeat=3))


def _kernel(kind, n, lo, hi):
    return greens.hockney_octant(n, lo, hi) if kind == "hockney" else greens.vico_octant(n, lo, hi)


def test_all_open_is_the_aperiodic_sum():
    n, lo, hi = (6, 5, 7), (-1.0, -0.5, -1.0), (1.0, 0.5, 2.0)
    rho = W.random_field(n, 1)
    k = _kernel("hockney", n, lo, hi)
    h = greens.spacing(n, lo, hi)
    np.testing.assert_allclose(mixed.convolve_mixed(rho, k, h, (False,) * 3), direct.convolve(rho, k, h),
                               rtol=1e-13, atol=0)


@pytest.mark.parametrize("mask", MASKS)
def test_sum_equals_six_loops(mask):
    n, lo, hi = (4, 3, 5), (-1.0, -1.0, -1.0), (1.0, 0.5, 1.5)
    rho = W.random_field(n, 2)
    k = _kernel("hockney", n, lo, hi)
    h = greens.spacing(n, lo, hi)
    np.testing.assert_allclose(mixed.convolve_mixed(rho, k, h, mask), mixed.convolve_mixed_loops(rho, k, h, mask),
                               rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
@pytest.mark.parametrize("mask", MASKS)
def test_fft_route_with_only_open_axes_doubled(kind, mask):
    n, lo, hi = (8, 6, 10), (-1.0, -0.75, -1.0), (1.0, 0.75, 1.5)
    rho = W.random_field(n, 3)
    k = _kernel(kind, n, lo, hi)
    h = greens.spacing(n, lo, hi)
    want = mixed.convolve_mixed(rho, k, h, mask)
    got = mixed.solve_mixed_fft(rho, k, h, mask)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cyclic_shift_along_a_periodic_axis(axis):
    n, lo, hi = (6, 8, 10), (-1.0,) * 3, (1.0,) * 3
    rho = W.random_field(n, 4)
    k = _kernel("hockney", n, lo, hi)
    h = greens.spacing(n, lo, hi)
    mask = tuple(a == axis for a in range(3))
    phi = mixed.convolve_mixed(rho, k, h, mask)
    shifted = mixed.convolve_mixed(np.roll(rho, 3, axis=axis), k, h, mask)
    np.testing.assert_allclose(shifted, np.roll(phi, 3, axis=axis), rtol=1e-12, atol=1e-14)
    # an open axis is not cyclic
    open_phi = mixed.convolve_mixed(rho, k, h, (False,) * 3)
    open_shifted = mixed.convolve_mixed(np.roll(rho, 3, axis=axis), k, h, (False,) * 3)
    assert np.max(np.abs(open_shifted - np.roll(open_phi, 3, axis=axis))) > 1e-6 * np.max(np.abs(open_phi))


def test_confined_source_sees_no_image():
    """rho nonzero only in 5 of 12 points of periodic axis 1: every offset between outputs
    in that window and the source is at most 4 < 12 / 2, so the nearest image is the offset."""
    n, lo, hi = (6, 12, 7), (-1.0,) * 3, (1.0,) * 3
    rho = np.zeros(n)
    rho[:, 4:9, :] = W.random_field((6, 5, 7), 5)
    k = _kernel("hockney", n, lo, hi)
    h = greens.spacing(n, lo, hi)
    per = mixed.convolve_mixed(rho, k, h, (False, True, False))
    opn = mixed.convolve_mixed(rho, k, h, (False, False, False))
    np.testing.assert_allclose(per[:, 4:9, :], opn[:, 4:9, :], rtol=1e-13, atol=0)
    assert np.max(np.abs(per[:, 0, :] - opn[:, 0, :])) > 1e-6 * np.max(np.abs(opn))


@pytest.mark.parametrize("mask", MASKS)
def test_folded_table_gives_the_mixed_sum(mask):
    n, lo, hi = (6, 8, 5), (-1.0, -1.0, -0.5), (1.0, 1.0, 1.0)
    rho = W.random_field(n, 6)
    k = _kernel("vico_dct", n, lo, hi)
    h = greens.spacing(n, lo, hi)
    t = mixed.periodic_table(k, n, mask)
    np.testing.assert_allclose(direct.convolve(rho, t, h), mixed.convolve_mixed(rho, k, h, mask), rtol=1e-12,
                               atol=1e-15)
