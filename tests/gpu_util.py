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


def elem_err(got, ref) -> float:
    """Largest element error over the RMS of the reference: max|got - ref| / rms(ref).

    Beside the relative L2 error this catches an error confined to a few
    outputs (one pencil, one column), which the whole-grid norm dilutes."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(ref * ref)))
    return float(np.max(np.abs(got - ref))) / rms


# Per-element bars, derived from the relative L2 bars (1e-12 float64, 1e-6 float32):
# an error spread over the grid at that L2 level has a largest element below about
# 6 times its RMS (a normally distributed error exceeds 6 sigma with probability
# 2e-9 per element, so over 1.7e7 elements of a 256^3 grid about 0.03 times), so
# max|d| <= 6 * rel_l2_bar * rms(ref).  An error of 1e-4 |phi| in a single pencil
# passes the L2 bar at 256^3 but fails this one.
ELEM_FACTOR = 6.0
F64_ELEM = ELEM_FACTOR * 1e-12
F32_ELEM = ELEM_FACTOR * 1e-6
F64_TOL = 1e-12
F32_TOL = 1e-6
