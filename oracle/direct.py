"""The plain definition of the solve: a discrete aperiodic convolution (float64).

With the grid's cell volume V = h0 h1 h2, the sum of eq. (2) over the grid
points (Section 1: discretise G and rho and sum, O(N_g^2) work) is

    phi_i = V * sum_{j in grid} K[|i0-j0|, |i1-j1|, |i2-j2|] * rho_j .

K is an octant table from ``oracle.greens``.  Both methods of the paper compute
exactly this sum; they differ only in K.
"""
from __future__ import annotations

import numpy as np

__all__ = ["convolve", "convolve_loops", "convolve_at"]


def _vol(h) -> float:
    return float(h[0]) * float(h[1]) * float(h[2])


def convolve(rho: np.ndarray, k_oct: np.ndarray, h) -> np.ndarray:
    """The sum above for a whole grid.

    For each axis-0 offset d, the (axis-1, axis-2) part of the sum is a matrix
    M_d[(i1,i2), (j1,j2)] = K[d, |i1-j1|, |i2-j2|]; then
    phi[i0] = V sum_{j0} M_{|i0-j0|} rho[j0].  O(n^6) work: small grids only.
    """
    rho = np.asarray(rho, dtype=np.float64)
    n0, n1, n2 = rho.shape
    assert k_oct.shape[0] > n0 - 1 and k_oct.shape[1] > n1 - 1 and k_oct.shape[2] > n2 - 1
    d1 = np.abs(np.arange(n1)[:, None] - np.arange(n1)[None, :])
    d2 = np.abs(np.arange(n2)[:, None] - np.arange(n2)[None, :])
    r = rho.reshape(n0, n1 * n2)
    phi = np.zeros((n0, n1 * n2))
    for d in range(n0):
        m = k_oct[d][d1[:, None, :, None], d2[None, :, None, :]].reshape(n1 * n2, n1 * n2)
        phi[d:] += r[: n0 - d] @ m.T          # pairs with i0 = j0 + d
        if d:
            phi[: n0 - d] += r[d:] @ m.T      # pairs with i0 = j0 - d
    return _vol(h) * phi.reshape(n0, n1, n2)


def convolve_loops(rho: np.ndarray, k_oct: np.ndarray, h) -> np.ndarray:
    """The same sum as six plain loops (tiny grids only; pins ``convolve``)."""
    n0, n1, n2 = rho.shape
    v = _vol(h)
    out = np.zeros((n0, n1, n2))
    for i0 in range(n0):
        for i1 in range(n1):
            for i2 in range(n2):
                s = 0.0
                for j0 in range(n0):
                    for j1 in range(n1):
                        for j2 in range(n2):
                            s += k_oct[abs(i0 - j0), abs(i1 - j1), abs(i2 - j2)] * rho[j0, j1, j2]
                out[i0, i1, i2] = v * s
    return out


def convolve_at(rho: np.ndarray, k_oct: np.ndarray, h, points) -> np.ndarray:
    """The sum at selected output points only (any grid size; O(n^3) per point)."""
    rho = np.asarray(rho, dtype=np.float64)
    n0, n1, n2 = rho.shape
    a0, a1, a2 = np.arange(n0), np.arange(n1), np.arange(n2)
    out = np.empty(len(points))
    for p, (i0, i1, i2) in enumerate(points):
        kk = k_oct[np.abs(i0 - a0)[:, None, None], np.abs(i1 - a1)[None, :, None], np.abs(i2 - a2)[None, None, :]]
        out[p] = _vol(h) * float(np.sum(kk * rho))
    return out
