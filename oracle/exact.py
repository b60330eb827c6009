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

__all__ = ["gaussian_potential", "sphere_potential", "source_potential"]


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
