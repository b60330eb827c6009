"""Helpers shared by the GPU tests: device round trips and oracle references."""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W
from oracle import direct, fftroute, greens


def kernel_octant(kind: str, n, lo, hi, alpha: float = 1.1):
    if kind == "hockney":
        return greens.hockney_octant(n, lo, hi)
    if kind == "vico":
        return greens.vico_octant_4n(n, lo, hi, alpha)
    return greens.vico_octant(n, lo, hi, alpha)


def reference(rho: np.ndarray, kind: str, lo, hi, use_direct: bool | None = None) -> np.ndarray:
    """Oracle phi for rho: the direct sum for small grids, else the float64 FFT route."""
    n = rho.shape
    k = kernel_octant(kind if kind != "vico" else "vico_dct", n, lo, hi)
    h = greens.spacing(n, lo, hi)
    if use_direct is None:
        use_direct = max(n) <= 24
    if use_direct:
        return direct.convolve(rho, k, h)
    return fftroute.solve(rho, k, h)


def to_dev(a: np.ndarray, dtype, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)


def to_host(t) -> np.ndarray:
    return t.detach().to("cpu").double().numpy()


def rel_l2(a, b) -> float:
    return oracle.rel_l2(a, b)


def gaussian_rho(n, lo, hi, src=None):
    return W.source_density(n, lo, hi, src if src is not None else W.centred_gaussian(0.05))
