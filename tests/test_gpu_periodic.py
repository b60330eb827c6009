"""GPU: mixed open / periodic axes (Section 2.2 step 1; FSP_PERIODIC_* plan flags)
against the oracle of oracle/mixed.py: the plain nearest-image sum on small
grids, the FFT route that doubles only the open axes on larger ones.  Every
mask of periodic axes, both Green's functions, both precisions; a cyclic shift
of rho along a periodic axis shifts phi the same way."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import greens, mixed

from gpu_util import elem_err, kernel_octant, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

MASKS = list(itertools.product([False, True], repeat=3))
TOL = {"f64": 1e-12, "f32": 1e-6}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _solve(torch, n, lo, hi, kind, prec, mask, rho):
    from paper_2405_02603_amd import Plan
    plan = Plan(n=n, lo=lo, hi=hi, greens=kind, prec=prec, periodic=mask)
    dt = torch.float64 if prec == "f64" else torch.float32
    phi = plan.solve(to_dev(rho, dt))
    torch.cuda.synchronize()
    return to_host(phi)


@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
@pytest.mark.parametrize("mask", MASKS, ids=["".join("p" if m else "o" for m in k) for k in MASKS])
def test_small_grid_against_the_sum(torch_cuda, kind, mask):
    n, lo, hi = (8, 12, 16), (-1.0, -1.0, -1.0), (1.0, 1.5, 1.5)
    rho = W.random_field(n, 31)
    k = kernel_octant(kind, n, lo, hi)
    ref = mixed.convolve_mixed(rho, k, greens.spacing(n, lo, hi), mask)
    for prec in ("f64", "f32"):
        got = _solve(torch_cuda, n, lo, hi, kind, prec, mask, rho)
        assert rel_l2(got, ref) <= TOL[prec], (prec, mask)
        assert elem_err(got, ref) <= 6 * TOL[prec], (prec, mask)


@pytest.mark.parametrize("kind", ["hockney", "vico_dct"])
@pytest.mark.parametrize("mask", [(True, False, False), (False, True, True), (True, True, True)])
@pytest.mark.parametrize("n", [(32, 48, 64), (64, 64, 64), (96, 32, 128)])
def test_larger_grids_against_the_fft_route(torch_cuda, kind, mask, n):
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.5)
    rho = W.source_density(n, lo, hi, W.multiblob(seed=32))
    k = kernel_octant(kind, n, lo, hi)
    ref = mixed.solve_mixed_fft(rho, k, greens.spacing(n, lo, hi), mask)
    for prec in ("f64", "f32"):
        got = _solve(torch_cuda, n, lo, hi, kind, prec, mask, rho)
        assert rel_l2(got, ref) <= TOL[prec], (prec, mask, n)
        assert elem_err(got, ref) <= 6 * TOL[prec], (prec, mask, n)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cyclic_shift_along_a_periodic_axis(torch_cuda, axis):
    n, lo, hi = (16, 24, 32), (-1.0,) * 3, (1.0,) * 3
    rho = W.random_field(n, 33)
    mask = tuple(a == axis for a in range(3))
    phi = _solve(torch_cuda, n, lo, hi, "hockney", "f64", mask, rho)
    shifted = _solve(torch_cuda, n, lo, hi, "hockney", "f64", mask, np.ascontiguousarray(np.roll(rho, 5, axis=axis)))
    assert rel_l2(shifted, np.roll(phi, 5, axis=axis)) <= 1e-12
