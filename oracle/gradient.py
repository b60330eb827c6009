"""Gradient of the potential along one axis (oracle, float64; test infrastructure).

The solve's potential is phi_i = V sum_j K[|i-j|] rho_j with an even kernel
table.  Its derivative along axis a is the same discrete convolution with the
derivative of the kernel, which is odd along a and even along the other axes:

    (d_a phi)_i = V sum_j sign(i_a - j_a) D_a[|i - j|] rho_j ,

with the octant table D_a[m], m in [0, n]:

* Hockney-Eastwood (Section 2.2): D_a[m] = -m_a h_a / (4 pi |m h|^3), the
  derivative of G = 1/(4 pi r); at m = 0 the table holds 0, the value of an
  odd function at the origin (the potential's own regularisation, step 3,
  has no such choice to make).
* Vico-Greengard (Sections 2.3-2.4): the inverse transform on the 4n grid of
  i k_a Ghat_L(k), eq. (3), restricted to the octant.  Ghat_L is even in every
  k_e, so only the sine part along a and the cosine parts along the other axes
  survive: a sine sum over the (2n+1) non-negative frequencies of axis a.

The paper asks for E = -grad(phi) without giving a method.  This reading
differentiates the kernel; differentiating the doubled-grid potential
spectrally would see its mirrored half, which is not smooth.

The FFT route embeds the odd table in the doubled grid by odd extension along
a (value 0 at offset n_a, which no physical output uses) and even extension
along the other axes; its DFT is -i times a real table (a sine transform along
a, DCT-I along the others).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from .greens import _as3, _dct1_matrix, _ghat_L, apply_axes, fold, spacing, vico_length, vico_spectrum

__all__ = [
    "hockney_grad_octant",
    "vico_grad_octant",
    "vico_grad_octant_4n",
    "signed_extend",
    "convolve_odd",
    "convolve_odd_loops",
    "odd_extend",
    "odd_transform_octant",
    "fftroute_grad",
]


def hockney_grad_octant(n, lo, hi, axis: int) -> np.ndarray:
    """D_a[m] = -m_a h_a / (4 pi |m h|^3) on the octant, 0 at m = 0."""
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    x = [np.arange(n[d] + 1, dtype=np.float64) * h[d] for d in range(3)]
    r = np.sqrt(x[0][:, None, None] ** 2 + x[1][None, :, None] ** 2 + x[2][None, None, :] ** 2)
    xa = [x[0][:, None, None], x[1][None, :, None], x[2][None, None, :]][axis]
    with np.errstate(divide="ignore", invalid="ignore"):
        d = -xa / (4.0 * np.pi * r ** 3)
    d[0, 0, 0] = 0.0
    return np.broadcast_to(d, r.shape).copy()


def _sine_k_matrix(n_out: int, period: int, kfac: float) -> np.ndarray:
    """Rows m < n_out of y[m] = 2 sum_{0<l<period} (-kfac l) sin(pi l m / period) x[l] over the
    period + 1 samples l in [0, period] (the end samples carry sin = 0)."""
    m = np.arange(n_out)[:, None]
    l = np.arange(period + 1)[None, :]
    r = np.mod(m * l, 2 * period).astype(np.float64)
    return 2.0 * (-kfac * l) * np.sin(np.pi * r / period)


def vico_grad_octant(n, lo, hi, axis: int, alpha: float = 1.1) -> np.ndarray:
    """D_a[m] = (1/(64 n0 n1 n2 V)) sum_{l in [0,2n]^3} w_l Ghat_L(k_l) (-k_{l_a}) sin(k_{l_a} m_a h_a)
    prod_{e != a} cos(k_{l_e} m_e h_e), with k_{l_d} = pi l_d / (2 n_d h_d) and the weights of the
    pairs +-l of the 4n grid (2 inside, 1 at the ends; the sine vanishes at the ends)."""
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    g = vico_spectrum(n, lo, hi, alpha)
    mats = []
    for d in range(3):
        if d == axis:
            mats.append(_sine_k_matrix(n[d] + 1, 2 * n[d], np.pi / (2.0 * n[d] * h[d])))
        else:
            mats.append(_dct1_matrix(n[d] + 1, 2 * n[d] + 1, 2 * n[d]))
    vol4 = 64.0 * n[0] * n[1] * n[2] * h[0] * h[1] * h[2]
    return apply_axes(g, mats) / vol4


def vico_grad_octant_4n(n, lo, hi, axis: int, alpha: float = 1.1) -> np.ndarray:
    """Same table by a full (4n)^3 inverse FFT of i k_a Ghat_L (FFT order), real part, restricted."""
    n = _as3(n, int)
    h = spacing(n, lo, hi)
    L = vico_length(lo, hi, alpha)
    k = []
    for d in range(3):
        l = np.fft.fftfreq(4 * n[d], d=1.0 / (4 * n[d]))
        k.append(2.0 * np.pi * l / (4.0 * n[d] * h[d]))
    kk = [k[0][:, None, None], k[1][None, :, None], k[2][None, None, :]]
    kabs = np.sqrt(kk[0] ** 2 + kk[1] ** 2 + kk[2] ** 2)
    spec = 1j * kk[axis] * _ghat_L(kabs, L)
    x = np.fft.ifftn(spec) / (h[0] * h[1] * h[2])
    return np.real(x[: n[0] + 1, : n[1] + 1, : n[2] + 1]).copy()


def signed_extend(d_oct: np.ndarray, n, axis: int) -> np.ndarray:
    """The table on all offsets o in (-n, n): sign(o_a) D_a[|o|], indexed by o + n - 1."""
    n = _as3(n, int)
    o = [np.arange(-(n[d] - 1), n[d]) for d in range(3)]
    t = d_oct[np.ix_(np.abs(o[0]), np.abs(o[1]), np.abs(o[2]))]
    s = np.sign(o[axis]).astype(np.float64)
    shape = [1, 1, 1]
    shape[axis] = -1
    return t * s.reshape(shape)


def convolve_odd(rho: np.ndarray, d_oct: np.ndarray, h, axis: int) -> np.ndarray:
    """(d_a phi)_i = V sum_j sign(i_a - j_a) D_a[|i-j|] rho_j for a whole grid (O(n^6)).

    As in ``direct.convolve``: for each axis-0 offset o, the (axis-1, axis-2)
    part is a matrix over the in-plane index pairs."""
    rho = np.asarray(rho, dtype=np.float64)
    n0, n1, n2 = rho.shape
    t = signed_extend(d_oct, (n0, n1, n2), axis)
    o1 = np.arange(n1)[:, None] - np.arange(n1)[None, :] + n1 - 1
    o2 = np.arange(n2)[:, None] - np.arange(n2)[None, :] + n2 - 1
    r = rho.reshape(n0, n1 * n2)
    out = np.zeros((n0, n1 * n2))
    for o in range(-(n0 - 1), n0):
        m = t[o + n0 - 1][o1[:, None, :, None], o2[None, :, None, :]].reshape(n1 * n2, n1 * n2)
        if o >= 0:
            out[o:] += r[: n0 - o] @ m.T         # i0 = j0 + o
        else:
            out[: n0 + o] += r[-o:] @ m.T        # i0 = j0 + o, o < 0
    return float(h[0]) * float(h[1]) * float(h[2]) * out.reshape(n0, n1, n2)


def convolve_odd_at(rho: np.ndarray, d_oct: np.ndarray, h, axis: int, points) -> np.ndarray:
    """The same sum at selected output points only (any grid size; O(n^3) per point)."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    ar = [np.arange(n[e]) for e in range(3)]
    v = float(h[0]) * float(h[1]) * float(h[2])
    out = np.empty(len(points))
    for p, i in enumerate(points):
        off = [i[e] - ar[e] for e in range(3)]
        dd = d_oct[np.abs(off[0])[:, None, None], np.abs(off[1])[None, :, None], np.abs(off[2])[None, None, :]]
        sgn = np.sign(off[axis]).reshape([-1 if e == axis else 1 for e in range(3)])
        out[p] = v * float(np.sum(sgn * dd * rho))
    return out


def convolve_odd_loops(rho: np.ndarray, d_oct: np.ndarray, h, axis: int) -> np.ndarray:
    """The same sum as six plain loops (tiny grids only; pins ``convolve_odd``)."""
    n0, n1, n2 = rho.shape
    v = float(h[0]) * float(h[1]) * float(h[2])
    out = np.zeros((n0, n1, n2))
    for i0 in range(n0):
        for i1 in range(n1):
            for i2 in range(n2):
                s = 0.0
                for j0 in range(n0):
                    for j1 in range(n1):
                        for j2 in range(n2):
                            o = (i0 - j0, i1 - j1, i2 - j2)
                            sg = (o[axis] > 0) - (o[axis] < 0)
                            s += sg * d_oct[abs(o[0]), abs(o[1]), abs(o[2])] * rho[j0, j1, j2]
                out[i0, i1, i2] = v * s
    return out


def odd_extend(d_oct: np.ndarray, axis: int) -> np.ndarray:
    """The table on the doubled grid: odd along ``axis`` (0 at offset n), even along the others."""
    n = [s - 1 for s in d_oct.shape]
    idx = [fold(np.arange(2 * n[d]), n[d]) for d in range(3)]
    t = d_oct[np.ix_(idx[0], idx[1], idx[2])].copy()
    m = np.arange(2 * n[axis])
    s = np.where(m < n[axis], 1.0, -1.0)
    s[n[axis]] = 0.0
    shape = [1, 1, 1]
    shape[axis] = -1
    return t * s.reshape(shape)


def odd_transform_octant(d_oct: np.ndarray, axis: int) -> np.ndarray:
    """T on the octant k in [0, n] with DFT(odd_extend(D)) = -i T (T odd in k_a, even elsewhere):

        along a:      T[k] = 2 sum_{0<m<n} D[m] sin(pi k m / n)
        along others: the DCT-I of ``greens.mirror_transform_octant``.
    """
    n = [s - 1 for s in d_oct.shape]
    mats = []
    for d in range(3):
        if d == axis:
            k = np.arange(n[d] + 1)[:, None]
            m = np.arange(n[d] + 1)[None, :]
            r = np.mod(k * m, 2 * n[d]).astype(np.float64)
            s = 2.0 * np.sin(np.pi * r / n[d])
            s[:, 0] = 0.0
            s[:, n[d]] = 0.0
            mats.append(s)
        else:
            mats.append(_dct1_matrix(n[d] + 1, n[d] + 1, n[d]))
    return apply_axes(d_oct, mats)


def fftroute_grad(rho: np.ndarray, d_oct: np.ndarray, h, axis: int, workers: int | None = None) -> np.ndarray:
    """The FFT route of Section 2.2 (steps 1-5) with the odd embedding of the derivative table."""
    if workers is None:
        workers = os.cpu_count() or 1
    n = rho.shape
    m = tuple(2 * s for s in n)
    rho2 = np.zeros(m)
    rho2[: n[0], : n[1], : n[2]] = rho
    g2 = odd_extend(np.asarray(d_oct, dtype=np.float64), axis)
    f = scipy.fft.rfftn(rho2, workers=workers)
    f *= scipy.fft.rfftn(g2, workers=workers)
    out2 = scipy.fft.irfftn(f, s=m, workers=workers)
    return float(h[0]) * float(h[1]) * float(h[2]) * out2[: n[0], : n[1], : n[2]]
