"""CPU oracle for the free-space Poisson solve (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never imports, links or calls it, and it never
imports the GPU library: the two share no code.  The seeded source generators
in ``workloads`` are the only module both sides use, and it holds none of the
method's arithmetic.

Everything here is plain float64 numpy/scipy, written for a reader to check
against the paper by eye:

``greens``    the two discrete kernels the method convolves with, on the
              octant m in [0, N] of offsets:
              * Hockney-Eastwood: the sampled 1/(4 pi r) with G(0) fixed
                (Section 2.2, step 3);
              * Vico-Greengard: the inverse transform of the truncated
                spectral kernel of eq. (3), computed three ways: dense
                cosine matrices on the (2N+1)^3 grid (the modified method of
                Section 2.4), scipy's DCT-I, and numpy's inverse FFT on the
                (4N)^3 grid (the original method of Section 2.3);
              and the transform of the mirror-extended kernel (step 3/4) as a
              DCT-I of length N+1 written with cosine matrices.
``direct``    the plain definition of the result, the discrete aperiodic
              convolution  phi_i = h0 h1 h2 sum_j K[|i - j|] rho_j  (the sum
              of eq. (2) discretised, Section 1), for small grids and for
              single sampled points of large grids.
``fftroute``  the Hockney-Eastwood steps 1-5 of Section 2.2 with library FFTs
              (double the grid, zero-pad, mirror-extend, transform, multiply,
              invert, restrict); pinned to ``direct``.
``exact``     closed-form potentials of the Section 3.1 test sources.
``memory``    the field-memory formulas of Section 3.3.
``mixed``     mixed open / periodic axes (Section 2.2, step 1: only the open
              axes are doubled): the plain sum with nearest-image offsets on
              the periodic axes, and the FFT route with only open axes doubled.

Parity pins (tests/test_oracle_*.py): ``fftroute`` equals ``direct`` to
rounding; ``direct`` equals a pure-Python six-loop sum on tiny grids; the three
Vico-Greengard routes agree; the transformed mirror kernel is real and even;
errors against the closed forms reproduce the orders of magnitude of the
paper's accuracy table (Table 3) and the second-order / spectral convergence
of Section 3.1; linearity, translation and symmetry hold; the memory formulas
reproduce Table 2.  No function in this package is "parity unpinned".
"""

from . import greens, direct, fftroute, exact, memory, mixed  # noqa: F401

__all__ = ["greens", "direct", "fftroute", "exact", "memory", "mixed", "rel_l2"]


def rel_l2(a, b) -> float:
    """Relative L2 error ||a - b|| / ||b|| over all grid points (Section 3.1)."""
    import numpy as np

    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
