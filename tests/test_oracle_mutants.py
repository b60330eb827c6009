"""The oracle's pins catch plausible mistakes in the oracle (CPU only).

Each case plants one mistake in the oracle -- a dropped factor, a wrong sign,
an index off by one, a transposed spacing, a wrong weight -- by replacing one
of its functions for the duration of the test, then runs the pins of
``test_oracle.py`` (the paper's accuracy table and convergence orders, the
closed forms, the cyclic-embedding identity, the three Vico-Greengard routes,
the invariants).  At least one pin must fail for every planted mistake; the
unmodified oracle passes them all.
"""
import math

import numpy as np
import pytest

import test_oracle as T
from oracle import direct, exact, fftroute, greens

FFT_CASES = [(kind, n, lo, hi) for kind in ("hockney", "vico_dct") for n, lo, hi in (
    (8, (-0.5,) * 3, (0.5,) * 3),
    ((6, 10, 12), (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0)),
    ((16, 8, 12), (0.0, 0.0, 0.0), (1.0, 0.5, 0.75)),
)]
VICO_CASES = [(8, (-0.5,) * 3, (0.5,) * 3), ((8, 12, 16), (-1.0, -1.0, -2.0), (1.0, 1.0, 2.0))]


def _pins(golden_dir):
    return {
        "direct == six loops": T.test_direct_matches_six_loops,
        "fft route == direct": lambda: [T.test_fft_route_equals_direct_sum(*c) for c in FFT_CASES],
        "mirror value irrelevant": T.test_mirror_value_is_irrelevant,
        "three VG routes": lambda: [T.test_vico_three_routes_agree(*c) for c in VICO_CASES],
        "VG spectrum form": T.test_vico_spectrum_limit_and_form,
        "HE kernel values": T.test_hockney_kernel_values,
        "mirror transform": lambda: [T.test_mirror_transform_is_real_even_dct(k) for k in ("hockney", "vico_dct")],
        "Table 3": lambda: T.test_paper_accuracy_table(golden_dir),
        "HE second order": T.test_hockney_second_order,
        "anisotropic grids": T.test_anisotropic_grids_reach_the_closed_form,
        "VG spectral": T.test_vico_spectral_convergence,
        "closed forms": T.test_closed_forms_satisfy_poisson,
        "invariants": T.test_linearity_translation_symmetry,
    }


def _failing(golden_dir):
    failed = []
    for name, pin in _pins(golden_dir).items():
        try:
            pin()
        except Exception:  # an assertion, or a mistake that breaks a shape
            failed.append(name)
    return failed


# ------------------------------------------------------------ planted mistakes
_orig_hockney = greens.hockney_octant
_orig_ghat = greens._ghat_L
_orig_length = greens.vico_length
_orig_dct1 = greens._dct1_matrix
_orig_solve = fftroute.solve
_orig_gauss = exact.gaussian_potential


def _hockney_origin_sign(n, lo, hi, g0=None):
    return _orig_hockney(n, lo, hi, g0=-1.0 / (4.0 * math.pi) if g0 is None else g0)


def _hockney_spacing_transposed(n, lo, hi, g0=None):
    n = greens._as3(n, int)
    h = greens.spacing(n, lo, hi)[::-1]
    m = [np.arange(n[d] + 1, dtype=np.float64) * h[d] for d in range(3)]
    r = np.sqrt(m[0][:, None, None] ** 2 + m[1][None, :, None] ** 2 + m[2][None, None, :] ** 2)
    with np.errstate(divide="ignore"):
        k = 1.0 / (4.0 * np.pi * r)
    k[0, 0, 0] = 1.0 / (4.0 * np.pi) if g0 is None else g0
    return k


def _ghat_half(kabs, L):
    return 0.5 * _orig_ghat(kabs, L)


def _length_without_alpha(lo, hi, alpha=1.1):
    return _orig_length(lo, hi, 1.0)


def _dct1_endpoint_weight(n_out, n_in, period):
    m = _orig_dct1(n_out, n_in, period).copy()
    m[:, -1] *= 2.0
    return m


def _solve_crop_shifted(rho, k_oct, h, workers=None, dtype=np.float64):
    n = rho.shape
    big = np.zeros(tuple(2 * s for s in n), dtype=np.float64)
    big[: n[0], : n[1], : n[2]] = rho
    m = tuple(2 * s for s in n)
    g2 = greens.mirror_extend(np.asarray(k_oct, dtype=np.float64))
    f = np.fft.rfftn(big) * np.fft.rfftn(g2)
    phi2 = np.fft.irfftn(f, s=m, axes=(0, 1, 2))
    return (h[0] * h[1] * h[2] * phi2[1: n[0] + 1, : n[1], : n[2]]).astype(dtype, copy=False)


def _fold_off_by_one(m, n):
    m = np.asarray(m)
    return np.where(m <= n, m, np.maximum(2 * n - m - 1, 0))


def _gauss_erf_argument(n, lo, hi, centre, sigma, weight=1.0):
    return _orig_gauss(n, lo, hi, centre, sigma / math.sqrt(2.0), weight)


def _vol_dropped(h):
    return 1.0


MUTANTS = {
    "HE value at the origin negated": (greens, "hockney_octant", _hockney_origin_sign),
    "HE spacing axes transposed": (greens, "hockney_octant", _hockney_spacing_transposed),
    "eq. (3) missing its factor 2": (greens, "_ghat_L", _ghat_half),
    "VG window without alpha": (greens, "vico_length", _length_without_alpha),
    "DCT-I endpoint weighted 2": (greens, "_dct1_matrix", _dct1_endpoint_weight),
    "restriction shifted by one row": (fftroute, "solve", _solve_crop_shifted),
    "mirror fold off by one": (greens, "fold", _fold_off_by_one),
    "closed form erf argument": (exact, "gaussian_potential", _gauss_erf_argument),
    "cell volume dropped from the sum": (direct, "_vol", _vol_dropped),
}


def test_unmodified_oracle_passes_every_pin(golden_dir):
    assert _failing(golden_dir) == []


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_fails_a_pin(name, golden_dir, monkeypatch):
    module, attr, fn = MUTANTS[name]
    monkeypatch.setattr(module, attr, fn)
    failed = _failing(golden_dir)
    print(f"{name}: caught by {failed}")
    assert failed, f"no pin catches: {name}"


# ------------------------------------------------- the gradient and mixed-axis oracles
import itertools  # noqa: E402

import test_oracle_grad as TG  # noqa: E402
import test_oracle_mixed as TM  # noqa: E402
from oracle import gradient, mixed  # noqa: E402

MASKS = list(itertools.product([False, True], repeat=3))


def _grad_pins():
    return {
        "closed-form gradient = FD of potential": TG.test_closed_form_gradient_is_the_derivative_of_the_closed_form_potential,
        "gradient near the centre": TG.test_closed_form_gradient_near_the_centre,
        "odd sum == loops": TG.test_direct_odd_sum_equals_loops,
        "odd sum at points": TG.test_odd_sum_at_points_equals_the_whole_grid_sum,
        "odd FFT route == odd sum": lambda: [TG.test_fft_route_equals_direct_odd_sum(k) for k in ("hockney", "vico")],
        "VG derivative two routes": TG.test_vico_derivative_table_two_routes,
        "HE derivative table": TG.test_hockney_derivative_table_is_odd_and_matches_the_kernel_derivative,
        "odd transform == FFT": TG.test_odd_transform_equals_fft_of_the_odd_extension,
        "gradient convergence": TG.test_gradient_convergence_to_the_closed_form,
    }


def _mixed_pins():
    return {
        "all open == aperiodic": TM.test_all_open_is_the_aperiodic_sum,
        "mixed == loops": lambda: [TM.test_sum_equals_six_loops(m) for m in MASKS],
        "mixed FFT route": lambda: [TM.test_fft_route_with_only_open_axes_doubled(k, m)
                                    for k in ("hockney", "vico_dct") for m in MASKS],
        "cyclic shift": lambda: [TM.test_cyclic_shift_along_a_periodic_axis(a) for a in range(3)],
        "confined source": TM.test_confined_source_sees_no_image,
        "folded table": lambda: [TM.test_folded_table_gives_the_mixed_sum(m) for m in MASKS],
    }


def _failing_of(pins):
    failed = []
    for name, pin in pins.items():
        try:
            pin()
        except Exception:
            failed.append(name)
    return failed


_orig_hgrad = gradient.hockney_grad_octant
_orig_sine = gradient._sine_k_matrix
_orig_signed = gradient.signed_extend
_orig_dist = mixed.axis_distance
_orig_table = mixed.periodic_table


def _hgrad_sign(n, lo, hi, axis):
    return -_orig_hgrad(n, lo, hi, axis)


def _hgrad_wrong_axis(n, lo, hi, axis):
    return _orig_hgrad(n, lo, hi, (axis + 1) % 3)


def _sine_without_2(n_out, period, kfac):
    return 0.5 * _orig_sine(n_out, period, kfac)


def _signed_flipped(d_oct, n, axis):
    return -_orig_signed(d_oct, n, axis)


def _dist_off_by_one(n, periodic):
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    return np.minimum(d, np.maximum(n - d - 1, 0)) if periodic else d


def _dist_ignores_periodic(n, periodic):
    return _orig_dist(n, False)


def _solve_mixed_all_doubled(rho, k_oct, h, periodic):
    return fftroute.solve(rho, k_oct, h)  # every axis doubled: the periodic ones treated as open


def _table_off_by_one(k_oct, n, periodic):
    f = [np.minimum(np.arange(n[a] + 1), np.maximum(n[a] - np.arange(n[a] + 1) - 1, 0)) if periodic[a]
         else np.arange(n[a] + 1) for a in range(3)]
    return k_oct[f[0][:, None, None], f[1][None, :, None], f[2][None, None, :]]


GRAD_MUTANTS = {
    "HE derivative table sign flipped": (gradient, "hockney_grad_octant", _hgrad_sign),
    "HE derivative along the wrong axis": (gradient, "hockney_grad_octant", _hgrad_wrong_axis),
    "sine sums without their factor 2": (gradient, "_sine_k_matrix", _sine_without_2),
    "odd extension with the opposite sign": (gradient, "signed_extend", _signed_flipped),
}

MIXED_MUTANTS = {
    "nearest image off by one": (mixed, "axis_distance", _dist_off_by_one),
    "periodic axes summed as open": (mixed, "axis_distance", _dist_ignores_periodic),
    "FFT route doubling every axis": (mixed, "solve_mixed_fft", _solve_mixed_all_doubled),
    "folded table off by one": (mixed, "periodic_table", _table_off_by_one),
}


def test_unmodified_gradient_and_mixed_oracles_pass():
    assert _failing_of(_grad_pins()) == []
    assert _failing_of(_mixed_pins()) == []


@pytest.mark.parametrize("name", list(GRAD_MUTANTS))
def test_planted_gradient_mistake_fails_a_pin(name, monkeypatch):
    module, attr, fn = GRAD_MUTANTS[name]
    monkeypatch.setattr(module, attr, fn)
    failed = _failing_of(_grad_pins())
    print(f"{name}: caught by {failed}")
    assert failed, f"no pin catches: {name}"


@pytest.mark.parametrize("name", list(MIXED_MUTANTS))
def test_planted_mixed_mistake_fails_a_pin(name, monkeypatch):
    module, attr, fn = MIXED_MUTANTS[name]
    monkeypatch.setattr(module, attr, fn)
    failed = _failing_of(_mixed_pins())
    print(f"{name}: caught by {failed}")
    assert failed, f"no pin catches: {name}"
