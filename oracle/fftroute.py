"""Hockney-Eastwood cyclic embedding with library FFTs (Section 2.2, steps 1-5).

    1. double the grid on every (open) axis: M = 2n;
    2. zero-pad rho to rho2 on the doubled grid;
    3. extend the kernel to G2 by mirroring (``greens.mirror_extend``);
    4. phi2 = V * IFFT{ FFT{rho2} * FFT{G2} };
    5. restrict phi2 to the physical grid.

The same steps serve both kernels (Section 2.3: Vico-Greengard differs only in
the kernel).  Pinned to ``direct.convolve`` on small grids.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft

from .greens import mirror_extend

__all__ = ["solve"]


def solve(rho: np.ndarray, k_oct: np.ndarray, h, workers: int | None = None,
          dtype=np.float64) -> np.ndarray:
    """phi on the physical grid; ``dtype`` float32 runs the same steps in single precision."""
    if workers is None:
        workers = os.cpu_count() or 1
    n = rho.shape
    m = tuple(2 * s for s in n)                                   # step 1
    rho2 = np.zeros(m, dtype=dtype)                               # step 2
    rho2[: n[0], : n[1], : n[2]] = rho
    g2 = mirror_extend(np.asarray(k_oct, dtype=np.float64)).astype(dtype, copy=False)   # step 3
    f = scipy.fft.rfftn(rho2, workers=workers)                    # step 4
    f *= scipy.fft.rfftn(g2, workers=workers)
    phi2 = scipy.fft.irfftn(f, s=m, workers=workers)
    vol = dtype(h[0]) * dtype(h[1]) * dtype(h[2])
    return (vol * phi2[: n[0], : n[1], : n[2]]).astype(dtype, copy=False)   # step 5
