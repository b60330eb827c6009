"""Closed-form potentials of the test sources of Section 3.1 (float64).

Sign convention: -Laplace(phi) = rho with G = +1/(4 pi r), so a positive
source gives a positive potential.  (The paper's eq. (1) has this form; its
test section writes the source with a minus sign and the sphere potential with
a minus sign, which is the same physics under the opposite convention.)
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

from workloads import axis_centres, Source

__all__ = ["gaussian_potential", "sphere_potential", "source_potential", "gaussian_gradient",
           "source_gradient"]


def _r(n, lo, hi, centre) -> np.ndarray:
    x0, x1, x2 = axis_centres(n, lo, hi)
    c = [float(v) for v in centre]
    return np.sqrt((x0 - c[0])[:, None, None] ** 2 + (x1 - c[1])[None, :, None] ** 2
                   + (x2 - c[2])[None, None, :] ** 2)


def gaussian_potential(n, lo, hi, centre, sigma: float, weight: float = 1.0) -> np.ndarray:
    """weight * erf(r / (sqrt(2) sigma)) / (4 pi r); at r = 0 its limit weight / ((2 pi)^{3/2} sigma)."""
    r = _r(n, lo, hi, centre)
    out = np.empty_like(r)
    nz = r > 1e-300
    out[nz] = erf(r[nz] / (np.sqrt(2.0) * sigma)) / (4.0 * np.pi * r[nz])
    out[~nz] = 1.0 / ((2.0 * np.pi) ** 1.5 * sigma)
    return weight * out


def sphere_potential(n, lo, hi, centre, radius: float, density: float) -> np.ndarray:
    """Uniform ball (eq. (5)): density (3 R^2 - r^2)/6 inside, density R^3 / (3 r) outside."""
    r = _r(n, lo, hi, centre)
    inside = density * (3.0 * radius ** 2 - r ** 2) / 6.0
    with np.errstate(divide="ignore"):
        outside = density * radius ** 3 / (3.0 * r)
    return np.where(r <= radius, inside, outside)


def source_potential(n, lo, hi, src: Source) -> np.ndarray:
    phi = 0.0
    for b in src.blobs:
        phi = phi + gaussian_potential(n, lo, hi, b.centre, b.sigma, b.weight)
    for (c, rad, dens) in src.balls:
        phi = phi + sphere_potential(n, lo, hi, c, rad, dens)
    return np.asarray(phi, dtype=np.float64)


def gaussian_gradient(n, lo, hi, centre, sigma: float, weight: float = 1.0) -> np.ndarray:
    """grad of weight * erf(r / (sqrt(2) sigma)) / (4 pi r), shape (3, n0, n1, n2):

        dphi/dr = weight / (4 pi r^2) * ((2/sqrt(pi)) u exp(-u^2) - erf(u)),  u = r / (sqrt(2) sigma),

    times (x - centre) / r; the bracket is evaluated by its series
    (2/sqrt(pi)) (-2 u^3 / 3 + 2 u^5 / 5 - u^7 / 7) for u < 1e-2 (the two terms cancel there),
    and the gradient is 0 at r = 0.
    """
    x0, x1, x2 = axis_centres(n, lo, hi)
    c = [float(v) for v in centre]
    dx = [(x0 - c[0])[:, None, None], (x1 - c[1])[None, :, None], (x2 - c[2])[None, None, :]]
    r = np.sqrt(dx[0] ** 2 + dx[1] ** 2 + dx[2] ** 2)
    u = r / (np.sqrt(2.0) * sigma)
    two_over_sqrt_pi = 2.0 / np.sqrt(np.pi)
    small = u < 1e-2
    bracket = np.where(small, two_over_sqrt_pi * (-2.0 * u ** 3 / 3.0 + 2.0 * u ** 5 / 5.0 - u ** 7 / 7.0),
                       two_over_sqrt_pi * u * np.exp(-u * u) - erf(u))
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(r > 0, weight * bracket / (4.0 * np.pi * r ** 3), 0.0)   # (dphi/dr) / r
    return np.stack([np.broadcast_to(f * dx[a], r.shape) for a in range(3)])


def source_gradient(n, lo, hi, src: Source) -> np.ndarray:
    """grad phi of a sum of Gaussians (shape (3, n0, n1, n2))."""
    g = 0.0
    for b in src.blobs:
        g = g + gaussian_gradient(n, lo, hi, b.centre, b.sigma, b.weight)
    assert not src.balls, "closed-form gradients are given for Gaussian sources"
    return np.asarray(g, dtype=np.float64)
