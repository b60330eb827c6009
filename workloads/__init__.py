"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *draws and samples inputs*: grid geometry (cell-centre
coordinates), Gaussian and uniform-sphere source densities on those
coordinates, the random parameters of multi-blob sources, batch size mixes and
request arrival times.  It holds none of the solver's arithmetic (no Green's
function, no transform, no convolution), so the oracle and the GPU path can
both consume it without sharing any of the method.

Conventions
-----------
* A grid is ``n = (n0, n1, n2)`` points over the box ``[lo_d, hi_d]`` on each
  axis, stored C-order with axis 2 contiguous.
* Points are cell centres ``x_i = lo + (i + 1/2) h`` with ``h = (hi - lo)/n``
  (the paper states the spacing h = L/N of Section 2.2 but not where the
  points sit inside a cell; cell centres are the reading taken here).
* A Gaussian blob of weight ``w``, width ``sigma`` and centre ``c`` has unit
  mass times ``w``: ``w exp(-|x-c|^2 / 2 sigma^2) / ((2 pi)^{3/2} sigma^3)``
  (the correctness test of Section 3.1, eq. (4), with the ``sigma^-3`` of a
  normalised Gaussian and a positive sign).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "Blob",
    "Source",
    "axis_centres",
    "grid_spacing",
    "gaussian_density",
    "sphere_density",
    "source_density",
    "random_field",
    "source_density_device",
    "centred_gaussian",
    "offcentre_gaussian",
    "multiblob",
    "BatchItem",
    "batch_mix",
    "Request",
    "poisson_arrivals",
    "SUPPORTED_EDGE_SIZES",
]

# Edge lengths a plan accepts: 2^a or 3*2^a with 8 <= N <= 512.
SUPPORTED_EDGE_SIZES: Tuple[int, ...] = tuple(
    sorted({2 ** a for a in range(3, 10)} | {3 * 2 ** a for a in range(2, 8)})
)


def _as3(v, dtype=float) -> Tuple:
    if np.isscalar(v):
        return (dtype(v),) * 3
    v = tuple(dtype(x) for x in v)
    if len(v) != 3:
        raise ValueError("expected a scalar or a 3-sequence")
    return v


def grid_spacing(n, lo, hi) -> Tuple[float, float, float]:
    n, lo, hi = _as3(n, int), _as3(lo), _as3(hi)
    return tuple((hi[d] - lo[d]) / n[d] for d in range(3))


def axis_centres(n, lo, hi) -> List[np.ndarray]:
    """Cell-centre coordinates on each axis (float64)."""
    n, lo, hi = _as3(n, int), _as3(lo), _as3(hi)
    h = grid_spacing(n, lo, hi)
    return [lo[d] + (np.arange(n[d], dtype=np.float64) + 0.5) * h[d] for d in range(3)]


@dataclass(frozen=True)
class Blob:
    centre: Tuple[float, float, float]
    sigma: float
    weight: float = 1.0


@dataclass(frozen=True)
class Source:
    """A sum of Gaussian blobs and/or uniform balls."""

    blobs: Tuple[Blob, ...] = ()
    # (centre, radius, density) uniform balls
    balls: Tuple[Tuple[Tuple[float, float, float], float, float], ...] = ()


def _r2(n, lo, hi, centre) -> np.ndarray:
    x0, x1, x2 = axis_centres(n, lo, hi)
    c = _as3(centre)
    return ((x0 - c[0])[:, None, None] ** 2 + (x1 - c[1])[None, :, None] ** 2
            + (x2 - c[2])[None, None, :] ** 2)


def gaussian_density(n, lo, hi, blobs: Sequence[Blob], dtype=np.float64) -> np.ndarray:
    """Sum of unit-mass Gaussians (times weight) sampled at cell centres."""
    n = _as3(n, int)
    rho = np.zeros(n, dtype=np.float64)
    for b in blobs:
        s = float(b.sigma)
        rho += (b.weight / ((2.0 * np.pi) ** 1.5 * s ** 3)) * np.exp(-_r2(n, lo, hi, b.centre) / (2.0 * s * s))
    return rho.astype(dtype, copy=False)


def sphere_density(n, lo, hi, centre, radius: float, density: float, dtype=np.float64) -> np.ndarray:
    """Uniform ball of the given density (the non-smooth source of Section 3.1, eq. (5))."""
    rho = np.where(_r2(n, lo, hi, centre) <= radius * radius, float(density), 0.0)
    return rho.astype(dtype, copy=False)


def source_density(n, lo, hi, src: Source, dtype=np.float64) -> np.ndarray:
    rho = gaussian_density(n, lo, hi, src.blobs)
    for (c, r, dens) in src.balls:
        rho = rho + sphere_density(n, lo, hi, c, r, dens)
    return rho.astype(dtype, copy=False)


def source_density_device(n, lo, hi, src: Source, dtype=None, device="cuda"):
    """source_density evaluated with torch on the device (the same cell centres and
    blob formula, in float64, then cast): a per-request source for serving runs
    without a host round trip.  Gaussian blobs only."""
    import torch

    if src.balls:
        raise ValueError("device sources hold Gaussian blobs only")
    n = _as3(n, int)
    x0, x1, x2 = (torch.as_tensor(a, dtype=torch.float64, device=device) for a in axis_centres(n, lo, hi))
    rho = torch.zeros(n, dtype=torch.float64, device=device)
    for b in src.blobs:
        s = float(b.sigma)
        c = _as3(b.centre)
        r2 = ((x0 - c[0])[:, None, None] ** 2 + (x1 - c[1])[None, :, None] ** 2 + (x2 - c[2])[None, None, :] ** 2)
        rho += (b.weight / ((2.0 * np.pi) ** 1.5 * s ** 3)) * torch.exp(-r2 / (2.0 * s * s))
    return rho if dtype is None else rho.to(dtype)


def random_field(n, seed: int, dtype=np.float64) -> np.ndarray:
    """Uniform(-1, 1) field: a source with no structure at all."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=_as3(n, int)).astype(dtype)


def centred_gaussian(sigma: float = 0.05) -> Source:
    return Source(blobs=(Blob((0.0, 0.0, 0.0), sigma, 1.0),))


def offcentre_gaussian() -> Source:
    """sigma = 0.03 Gaussian at (0.1, -0.2, 0.15)."""
    return Source(blobs=(Blob((0.1, -0.2, 0.15), 0.03, 1.0),))


def multiblob(seed: int = 3, count: int = 8, rng: np.random.Generator | None = None) -> Source:
    """``count`` Gaussians: centres U[-0.5,0.5]^3, sigma U[0.02,0.08], weight U[0.5,1.5].

    Draw order is centres (count x 3), then sigmas, then weights.
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.5, 0.5, size=(count, 3))
    sigmas = rng.uniform(0.02, 0.08, size=count)
    weights = rng.uniform(0.5, 1.5, size=count)
    return Source(blobs=tuple(Blob(tuple(map(float, centres[i])), float(sigmas[i]), float(weights[i]))
                              for i in range(count)))


@dataclass(frozen=True)
class BatchItem:
    n: int
    source: Source
    lo: Tuple[float, float, float] = (-1.0, -1.0, -1.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)


def batch_mix(seed: int = 4, count: int = 64,
              sizes: Sequence[int] = (32, 48, 64, 96, 128)) -> List[BatchItem]:
    """Right-hand sides of uneven grid sizes, each an 8-blob source.

    For each item the edge size is drawn first, then its blobs, from one stream.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        out.append(BatchItem(n=n, source=multiblob(count=8, rng=rng)))
    return out


@dataclass(frozen=True)
class Request:
    rid: int
    t_arrival: float          # seconds since the start of the run
    n: int
    greens: str               # "hockney" or "vico"
    spot_check: bool          # also solve in FP64 on the device
    source: Source = field(compare=False, default=Source())


def poisson_arrivals(rate: float = 200.0, duration: float = 30.0, seed: int = 5,
                     sizes: Sequence[int] = (32, 48, 64, 96, 128, 192, 256),
                     spot_fraction: float = 0.01, blobs: int = 8) -> List[Request]:
    """Poisson request stream: exponential gaps, uniform sizes, 50/50 kernel choice."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out: List[Request] = []
    rid = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        greens = "hockney" if rng.random() < 0.5 else "vico"
        spot = bool(rng.random() < spot_fraction)
        src = multiblob(count=blobs, rng=rng)
        out.append(Request(rid, t, n, greens, spot, src))
        rid += 1
    return out


def fitted_box(src: Source, margin_sigmas: float = 4.0, quantum: float = 0.25, min_edge: float = 1.25):
    """A domain fitted to a source: the bounding box of its blobs' centres widened by
    ``margin_sigmas`` sigma, each edge widened about its middle to at least
    ``min_edge``, each face then moved outward to a multiple of ``quantum`` (so that
    nearby fits share a box).  Returns (lo, hi)."""
    c = np.array([b.centre for b in src.blobs], dtype=np.float64)
    s = np.array([b.sigma for b in src.blobs], dtype=np.float64)[:, None]
    lo = (c - margin_sigmas * s).min(axis=0)
    hi = (c + margin_sigmas * s).max(axis=0)
    short = np.maximum(min_edge - (hi - lo), 0.0) / 2
    lo = np.floor((lo - short) / quantum) * quantum
    hi = np.ceil((hi + short) / quantum) * quantum
    return tuple(float(x) for x in lo), tuple(float(x) for x in hi)
