"""Mixed open / periodic axes (Section 2.2, step 1: the grid is doubled only
along the axes with open boundaries), float64, test infrastructure only.

Reading taken (the paper states the doubling rule, nothing more): along a
periodic axis of n points the convolution is cyclic with period n, and the
Green's function on that axis is the one circularly shifted over the n-point
period -- the value at offset m is G at the nearest image, m or n - m -- as
step 3 circularly shifts G over the doubled period of an open axis.  The
discrete result is then

    phi_i = V * sum_j K[d0, d1, d2] * rho_j ,
    d_a = |i_a - j_a|                           on an open axis,
    d_a = min(|i_a - j_a|, n_a - |i_a - j_a|)   on a periodic axis,

with K the octant table of ``oracle.greens`` (``convolve_mixed``, the plain
definition).  ``solve_mixed_fft`` takes the paper's steps literally: double
only the open axes, zero-pad rho there, extend the kernel by the circular
shift of each axis's own period, multiply the transforms, invert, restrict.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

__all__ = ["axis_distance", "convolve_mixed", "convolve_mixed_loops", "solve_mixed_fft", "periodic_table"]


def axis_distance(n: int, periodic: bool) -> np.ndarray:
    """The n x n matrix of offsets d(i, j) along one axis."""
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    return np.minimum(d, n - d) if periodic else d


def _vol(h) -> float:
    return float(h[0]) * float(h[1]) * float(h[2])


def convolve_mixed(rho: np.ndarray, k_oct: np.ndarray, h, periodic) -> np.ndarray:
    """The definition above for a whole grid: for every pair of axis-0 indices
    the (axis-1, axis-2) part is the matrix K[d0(i0,j0), d1, d2].  O(n^6)."""
    rho = np.asarray(rho, dtype=np.float64)
    n0, n1, n2 = rho.shape
    d0 = axis_distance(n0, bool(periodic[0]))
    d1 = axis_distance(n1, bool(periodic[1]))
    d2 = axis_distance(n2, bool(periodic[2]))
    r = rho.reshape(n0, n1 * n2)
    phi = np.zeros((n0, n1 * n2))
    for i0 in range(n0):
        for j0 in range(n0):
            m = k_oct[d0[i0, j0]][d1[:, None, :, None], d2[None, :, None, :]].reshape(n1 * n2, n1 * n2)
            phi[i0] += m @ r[j0]
    return _vol(h) * phi.reshape(n0, n1, n2)


def convolve_mixed_loops(rho: np.ndarray, k_oct: np.ndarray, h, periodic) -> np.ndarray:
    """The same sum as six plain loops (tiny grids only)."""
    n = rho.shape
    v = _vol(h)
    out = np.zeros(n)

    def dist(a, i, j):
        d = abs(i - j)
        return min(d, n[a] - d) if periodic[a] else d

    for i0 in range(n[0]):
        for i1 in range(n[1]):
            for i2 in range(n[2]):
                s = 0.0
                for j0 in range(n[0]):
                    for j1 in range(n[1]):
                        for j2 in range(n[2]):
                            s += k_oct[dist(0, i0, j0), dist(1, i1, j1), dist(2, i2, j2)] * rho[j0, j1, j2]
                out[i0, i1, i2] = v * s
    return out


def solve_mixed_fft(rho: np.ndarray, k_oct: np.ndarray, h, periodic) -> np.ndarray:
    """Section 2.2 steps 1-5 with only the open axes doubled (library FFTs).

    Step 1: M_a = 2 n_a on an open axis, n_a on a periodic one.  Step 2: rho
    zero-padded to the M grid.  Step 3: the kernel on the M grid, circularly
    shifted over each axis's period: index m takes the octant entry
    min(m, M_a - m).  Steps 4-5: multiply the transforms, invert, restrict."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    m = tuple(n[a] if periodic[a] else 2 * n[a] for a in range(3))
    rho2 = np.zeros(m)
    rho2[: n[0], : n[1], : n[2]] = rho
    idx = [np.minimum(np.arange(m[a]), m[a] - np.arange(m[a])) for a in range(3)]
    g = k_oct[idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]
    f = scipy.fft.rfftn(rho2) * scipy.fft.rfftn(g)
    phi2 = scipy.fft.irfftn(f, s=m)
    return _vol(h) * phi2[: n[0], : n[1], : n[2]]


def periodic_table(k_oct: np.ndarray, n, periodic) -> np.ndarray:
    """The octant table T[m] = K[f0(m0), f1(m1), f2(m2)] with f_a(m) = min(m, n_a - m)
    on the periodic axes (m on the open ones): the aperiodic sum with T over offsets
    |i - j| < n equals the mixed sum with K (the offsets n_a - |d| and |d| take the
    same value).  Test of the table the device precompute builds for periodic axes."""
    f = [np.minimum(np.arange(n[a] + 1), n[a] - np.arange(n[a] + 1)) if periodic[a] else np.arange(n[a] + 1)
         for a in range(3)]
    return k_oct[f[0][:, None, None], f[1][None, :, None], f[2][None, None, :]]
