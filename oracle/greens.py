"""Discrete Green's-function kernels of the free-space solve (oracle, float64).

Notation: a grid of n = (n0, n1, n2) cells over the box [lo, hi], spacing
h_d = (hi_d - lo_d) / n_d, cell volume V = h0 h1 h2.  A kernel is stored as
its octant K[m0, m1, m2], m_d in [0, n_d]; the solve uses K[|i - j|] for the
offset between two grid points.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

__all__ = [
    "spacing",
    "hockney_octant",
    "vico_length",
    "vico_spectrum",
    "vico_octant",
    "vico_octant_dct",
    "vico_octant_4n",
    "fold",
    "mirror_extend",
    "mirror_transform_octant",
    "apply_axes",
]


def _as3(v, t=float):
    if np.isscalar(v):
        return (t(v),) * 3
    return tuple(t(x) for x in v)


def spacing(n, lo, hi):
    n, lo, hi = _as3(n, int), _as3(lo), _as3(hi)
    return tuple((hi[d] - lo[d]) / n[d] for d in range(3))


def apply_axes(a: np.ndarray, mats) -> np.ndarray:
    """Contract axis d of ``a`` with matrix mats[d] (out_d x in_d), d = 0, 1, 2.

    Each step contracts the leading axis and appends the new axis at the end, so
    after three steps the axes are back in order (one matrix product per step).
    """
    for d in range(3):
        a = np.tensordot(a, mats[d], axes=([0], [1]))
    return a


# ---------------------------------------------------------------------------
# Hockney-Eastwood kernel (Section 2.2, step 3)
# ---------------------------------------------------------------------------
def hockney_octant(n, lo, hi, g0: float | None = None) -> np.ndarray:
    """K[m] = 1/(4 pi |m * h|) on the octant, with the singular value replaced.

    Section 2.2 (step 3) replaces the singularity at the origin by a constant
    of magnitude 1/(4 pi); with G = +1/(4 pi r) (so that -Laplace(phi) = rho)
    that constant is +1/(4 pi).  ``g0`` overrides it.
    """
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    m = [np.arange(n[d] + 1, dtype=np.float64) * h[d] for d in range(3)]
    r = np.sqrt(m[0][:, None, None] ** 2 + m[1][None, :, None] ** 2 + m[2][None, None, :] ** 2)
    with np.errstate(divide="ignore"):
        k = 1.0 / (4.0 * np.pi * r)
    k[0, 0, 0] = (1.0 / (4.0 * np.pi)) if g0 is None else float(g0)
    return k


# ---------------------------------------------------------------------------
# Vico-Greengard truncated spectral kernel (Sections 2.3 and 2.4, eq. (3))
# ---------------------------------------------------------------------------
def vico_length(lo, hi, alpha: float = 1.1) -> float:
    """Truncation window L = alpha * sqrt(Lx^2 + Ly^2 + Lz^2) (Section 2.3)."""
    lo, hi = _as3(lo), _as3(hi)
    return float(alpha) * math.sqrt(sum((hi[d] - lo[d]) ** 2 for d in range(3)))


def _ghat_L(kabs: np.ndarray, L: float) -> np.ndarray:
    """eq. (3): 2 (sin(L|k|/2) / |k|)^2, with its limit L^2/2 at k = 0."""
    out = np.empty_like(kabs)
    nz = kabs > 0
    out[nz] = 2.0 * (np.sin(0.5 * L * kabs[nz]) / kabs[nz]) ** 2
    out[~nz] = 0.5 * L * L
    return out


def vico_spectrum(n, lo, hi, alpha: float = 1.1) -> np.ndarray:
    """Samples of eq. (3) at the (2n+1)^3 non-negative frequencies of the 4n grid.

    The precompute grid has 4 n_d points of spacing h_d per axis (Section 2.3),
    so its frequencies are k_d = 2 pi l_d / (4 n_d h_d), l_d in [-2n_d, 2n_d).
    The kernel is even, so l_d in [0, 2 n_d] holds every distinct value
    (Section 2.4).
    """
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    L = vico_length(lo, hi, alpha)
    k = [np.pi * np.arange(2 * n[d] + 1, dtype=np.float64) / (2.0 * n[d] * h[d]) for d in range(3)]
    kabs = np.sqrt(k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2)
    return _ghat_L(kabs, L)


def _cos_pi_ratio(num: np.ndarray, den: int) -> np.ndarray:
    """cos(pi * num / den) for integer num, with the argument reduced exactly mod 2 den."""
    r = np.mod(num, 2 * den).astype(np.float64)
    return np.cos(np.pi * r / den)


def _dct1_matrix(n_out: int, n_in: int, period: int) -> np.ndarray:
    """Rows m < n_out of the DCT-I on n_in = period + 1 samples:

        y[m] = x[0] + (-1)^m x[period] + 2 sum_{0<l<period} x[l] cos(pi l m / period)

    which is the DFT of the even extension of x to length 2 * period.
    """
    assert n_in == period + 1
    m = np.arange(n_out)[:, None]
    l = np.arange(n_in)[None, :]
    c = np.full(n_in, 2.0)
    c[0] = 1.0
    c[-1] = 1.0
    return _cos_pi_ratio(m * l, period) * c[None, :]


def vico_octant(n, lo, hi, alpha: float = 1.1) -> np.ndarray:
    """Real-space Vico-Greengard kernel on the octant m in [0, n], modified route.

    K[m] = (1 / prod_d 4 n_d h_d) * sum_{l in [-2n, 2n)} Ghat_L(k_l) exp(i k_l . m h)

    is the inverse transform on the 4n grid (Section 2.3) restricted to the
    octant; because Ghat_L is real and even it equals a DCT-I over the
    (2n+1)^3 unique samples (Section 2.4), written here as three dense cosine
    matrices.  The prefactor 1/prod(4 n_d h_d) = 1/(64 n0 n1 n2 V).
    """
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    g = vico_spectrum(n, lo, hi, alpha)
    mats = [_dct1_matrix(n[d] + 1, 2 * n[d] + 1, 2 * n[d]) for d in range(3)]
    vol4 = 64.0 * n[0] * n[1] * n[2] * h[0] * h[1] * h[2]
    return apply_axes(g, mats) / vol4


def vico_octant_dct(n, lo, hi, alpha: float = 1.1) -> np.ndarray:
    """Same kernel via scipy's DCT-I (cross-check route)."""
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    g = vico_spectrum(n, lo, hi, alpha)
    y = scipy.fft.dctn(g, type=1, norm=None)
    vol4 = 64.0 * n[0] * n[1] * n[2] * h[0] * h[1] * h[2]
    return y[: n[0] + 1, : n[1] + 1, : n[2] + 1] / vol4


def vico_octant_4n(n, lo, hi, alpha: float = 1.1) -> np.ndarray:
    """Same kernel by the original route: a full (4n)^3 inverse FFT, then restriction.

    The frequency grid is laid out in FFT order (l = 0..2n-1, then -2n..-1).
    """
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    L = vico_length(lo, hi, alpha)
    k = []
    for d in range(3):
        l = np.fft.fftfreq(4 * n[d], d=1.0 / (4 * n[d]))  # integers in FFT order
        k.append(2.0 * np.pi * l / (4.0 * n[d] * h[d]))
    kabs = np.sqrt(k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2)
    g = _ghat_L(kabs, L)
    # ifftn divides by prod(4 n_d); the kernel wants 1/prod(4 n_d h_d).
    x = np.fft.ifftn(g) / (h[0] * h[1] * h[2])
    return np.real(x[: n[0] + 1, : n[1] + 1, : n[2] + 1]).copy()


# ---------------------------------------------------------------------------
# Mirror extension to the doubled grid and its transform (Section 2.2, steps 3-4)
# ---------------------------------------------------------------------------
def fold(m: np.ndarray, n: int) -> np.ndarray:
    """Index into the octant for position m in [0, 2n) of the doubled grid."""
    m = np.asarray(m)
    return np.where(m <= n, m, 2 * n - m)


def mirror_extend(k_oct: np.ndarray) -> np.ndarray:
    """G2 on the doubled grid: G2(x) = G(2L - x) on each axis's upper half (step 3)."""
    n = [s - 1 for s in k_oct.shape]
    idx = [fold(np.arange(2 * n[d]), n[d]) for d in range(3)]
    return k_oct[np.ix_(idx[0], idx[1], idx[2])]


def mirror_transform_octant(k_oct: np.ndarray) -> np.ndarray:
    """DFT of the mirror-extended kernel on the octant k in [0, n].

    The extension is real and even, so its DFT is real and even and equals a
    DCT-I of length n_d + 1 on each axis:
        Ghat2[k] = K[0] + (-1)^k K[n] + 2 sum_{0<m<n} K[m] cos(pi k m / n).
    """
    n = [s - 1 for s in k_oct.shape]
    mats = [_dct1_matrix(n[d] + 1, n[d] + 1, n[d]) for d in range(3)]
    return apply_axes(k_oct, mats)
