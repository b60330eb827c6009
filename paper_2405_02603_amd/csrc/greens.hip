// greens.hip -- float64 precompute of the Green's-function transform (gfx950).
//
// Every route ends in the same object: the transform of the mirror-extended
// real-space kernel on the octant k in [0, n] (real and even, so the octant
// holds all of it), scaled by V / (8 n0 n1 n2) and rounded once to the solve
// precision.
//
//   Hockney-Eastwood (Section 2.2): K[m] = 1/(4 pi |m h|), K[0] = g0, then a
//     DCT-I of length n_d + 1 on each axis.
//   Vico-Greengard, modified (Section 2.4): the kernel of eq. (3) sampled at the
//     (2n+1)^3 non-negative frequencies of the 4n grid, a DCT-I of length
//     2 n_d + 1 on each axis keeping only outputs m_d <= n_d (that is the
//     restriction to the doubled grid), then as Hockney-Eastwood.
//   Vico-Greengard, original (Section 2.3): eq. (3) sampled on the full
//     (4n)^3 frequency grid, the inverse transform on that grid evaluated at
//     the octant outputs m_d <= n_d only (a real cosine sum, since the grid
//     data are real and even), then as Hockney-Eastwood.
//
// Derivative tables (the kernel's derivative along axis a, odd along a): the
// same steps with sine forms along a -- -k_a-weighted sine sums from the
// spectrum, and a sine transform of the odd extension on the doubled grid,
// whose transform is -i times the stored real octant.
//
// Each one-axis transform is a dense contraction of one axis with a small
// cosine (or sine) matrix, C[m][l] applied along that axis with the other axes
// in place -- a float64 GEMM, done by rocBLAS.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <map>

namespace fsp {

__global__ __launch_bounds__(256) void k_he_kernel(double* K, int n0, int n1, int n2, double h0, double h1,
                                                   double h2, double g0) {
  const long long total = (long long)(n0 + 1) * (n1 + 1) * (n2 + 1);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int m2 = (int)(i % (n2 + 1));
  const long long t = i / (n2 + 1);
  const int m1 = (int)(t % (n1 + 1));
  const int m0 = (int)(t / (n1 + 1));
  const double x = m0 * h0, y = m1 * h1, z = m2 * h2;
  const double r = sqrt(x * x + y * y + z * z);
  K[i] = (i == 0) ? g0 : 1.0 / (4.0 * M_PI * r);
}

// Derivative of the Hockney-Eastwood kernel along `axis` on the octant:
// D[m] = -x_a / (4 pi |x|^3), x = m h, with 0 (an odd function's value) at m = 0.
__global__ __launch_bounds__(256) void k_he_grad_kernel(double* D, int n0, int n1, int n2, double h0, double h1,
                                                        double h2, int axis) {
  const long long total = (long long)(n0 + 1) * (n1 + 1) * (n2 + 1);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int m2 = (int)(i % (n2 + 1));
  const long long t = i / (n2 + 1);
  const int m1 = (int)(t % (n1 + 1));
  const int m0 = (int)(t / (n1 + 1));
  const double x = m0 * h0, y = m1 * h1, z = m2 * h2;
  const double r2 = x * x + y * y + z * z;
  const double xa = axis == 0 ? x : (axis == 1 ? y : z);
  D[i] = (i == 0) ? 0.0 : -xa / (4.0 * M_PI * r2 * sqrt(r2));
}

// Samples of eq. (3): 2 sin^2(L|k|/2) / |k|^2, with L^2/2 at k = 0.
// s_d samples per axis; index l maps to the integer frequency l (dense
// non-negative grid, signed == false) or to l - s_d for l >= s_d / 2 (FFT
// order on the 4n grid, signed == true).  k_d = f_d * frequency.
__global__ __launch_bounds__(256) void k_vico_spectrum(double* G, int s0, int s1, int s2, double f0,
                                                       double f1, double f2, double L, int fft_order) {
  const long long total = (long long)s0 * s1 * s2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int l2 = (int)(i % s2);
  const long long t = i / s2;
  int l1 = (int)(t % s1);
  int l0 = (int)(t / s1);
  if (fft_order) {
    if (l0 >= s0 / 2) l0 -= s0;
    if (l1 >= s1 / 2) l1 -= s1;
    if (l2 >= s2 / 2) l2 -= s2;
  }
  const double kx = l0 * f0, ky = l1 * f1, kz = l2 * f2;
  const double k = sqrt(kx * kx + ky * ky + kz * kz);
  double v;
  if (k > 0.0) {
    const double s = sin(0.5 * L * k) / k;
    v = 2.0 * s * s;
  } else {
    v = 0.5 * L * L;
  }
  G[i] = v;
}

// Store the octant G[k0][k1][k2] (float64, dense) scaled, in the blocked layout
// out[((k1 * tiles + k2 / tile) * (n0 + 1) + k0) * tile + k2 % tile]; slots of
// the last tile beyond k2 = n2 are zero.
template <typename T>
__global__ __launch_bounds__(256) void k_store_octant(const double* __restrict__ G, T* __restrict__ out, int n0,
                                                      int n1, int n2, int tile, double scale) {
  const int tiles = (n2 + 1 + tile - 1) / tile;
  const long long total = (long long)(n1 + 1) * tiles * (n0 + 1) * tile;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int c = (int)(i % tile);
  long long t = i / tile;
  const int k0 = (int)(t % (n0 + 1));
  t /= (n0 + 1);
  const int tl = (int)(t % tiles);
  const int k1 = (int)(t / tiles);
  const int k2 = tl * tile + c;
  out[i] = k2 <= n2 ? (T)(scale * G[((long long)k0 * (n1 + 1) + k1) * (n2 + 1) + k2]) : T(0);
}

// ------------------------------------------------------------------ host side
static unsigned grid1(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t greens_he_kernel(double* K, const int n[3], const double h[3], double g0, hipStream_t s) {
  const long long total = (long long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
  hipLaunchKernelGGL(k_he_kernel, dim3(grid1(total)), dim3(256), 0, s, K, n[0], n[1], n[2], h[0], h[1], h[2], g0);
  return hipGetLastError();
}

hipError_t greens_he_grad_kernel(double* D, const int n[3], const double h[3], int axis, hipStream_t s) {
  const long long total = (long long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
  hipLaunchKernelGGL(k_he_grad_kernel, dim3(grid1(total)), dim3(256), 0, s, D, n[0], n[1], n[2], h[0], h[1], h[2],
                     axis);
  return hipGetLastError();
}

hipError_t greens_vico_spectrum(double* G, const int samples[3], const double f[3], double L, bool fft_order,
                                hipStream_t s) {
  const long long total = (long long)samples[0] * samples[1] * samples[2];
  hipLaunchKernelGGL(k_vico_spectrum, dim3(grid1(total)), dim3(256), 0, s, G, samples[0], samples[1], samples[2],
                     f[0], f[1], f[2], L, fft_order ? 1 : 0);
  return hipGetLastError();
}

// rocBLAS handles of the calling host thread, one per device (created on first
// use, destroyed when the thread ends): a handle carries its stream, so
// threads that precompute at the same time each use their own.
struct BlasHandles {
  std::map<int, rocblas_handle> h;
  ~BlasHandles() {
    for (auto& kv : h) (void)rocblas_destroy_handle(kv.second);
  }
};

static rocblas_handle blas_handle(int dev) {
  static thread_local BlasHandles handles;
  auto it = handles.h.find(dev);
  if (it != handles.h.end()) return it->second;
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
  handles.h[dev] = h;
  return h;
}

// Contract axis `axis` of the row-major array X[d0][d1][d2] with the matrix
// C[nout][d_axis] (row-major): Y has the same axis order with d_axis -> nout.
// Each case is one float64 GEMM in column-major terms (rocBLAS):
//   axis 0: Y (d1 d2 x nout) = X (d1 d2 x d0) C^T-as-stored (d0 x nout)
//   axis 1: per i0, Y_i0 (d2 x nout) = X_i0 (d2 x d1) C (d1 x nout)  (strided batch over i0)
//   axis 2: Y (nout x d0 d1) = C^T (nout x d2) X (d2 x d0 d1)
hipError_t greens_contract_axis(const double* X, double* Y, const double* C, const long long dims[3], int axis,
                                int nout, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  rocblas_handle h = blas_handle(dev);
  if (!h || rocblas_set_stream(h, s) != rocblas_status_success) return hipErrorInvalidValue;
  const long long d0 = dims[0], d1 = dims[1], d2 = dims[2];
  if (d0 * d1 > 0x7fffffffLL || d1 * d2 > 0x7fffffffLL) return hipErrorInvalidValue;
  const double one = 1.0, zero = 0.0;
  rocblas_status st;
  const rocblas_operation N = rocblas_operation_none, T = rocblas_operation_transpose;
  if (axis == 0) {
    const rocblas_int m = (rocblas_int)(d1 * d2);
    st = rocblas_dgemm(h, N, N, m, nout, (rocblas_int)d0, &one, X, m, C, (rocblas_int)d0, &zero, Y, m);
  } else if (axis == 1) {
    st = rocblas_dgemm_strided_batched(h, N, N, (rocblas_int)d2, nout, (rocblas_int)d1, &one, X, (rocblas_int)d2,
                                       (rocblas_stride)(d1 * d2), C, (rocblas_int)d1, 0, &zero, Y, (rocblas_int)d2,
                                       (rocblas_stride)nout * d2, (rocblas_int)d0);
  } else {
    st = rocblas_dgemm(h, T, N, nout, (rocblas_int)(d0 * d1), (rocblas_int)d2, &one, C, (rocblas_int)d2, X,
                       (rocblas_int)d2, &zero, Y, nout);
  }
  return st == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

hipError_t greens_store_octant(const double* G, void* out, bool f64, const int n[3], int tile, double scale,
                               hipStream_t s) {
  const long long tiles = (n[2] + 1 + tile - 1) / tile;
  const long long total = (long long)(n[1] + 1) * tiles * (n[0] + 1) * tile;
  if (f64)
    hipLaunchKernelGGL(k_store_octant<double>, dim3(grid1(total)), dim3(256), 0, s, G, (double*)out, n[0], n[1],
                       n[2], tile, scale);
  else
    hipLaunchKernelGGL(k_store_octant<float>, dim3(grid1(total)), dim3(256), 0, s, G, (float*)out, n[0], n[1],
                       n[2], tile, scale);
  return hipGetLastError();
}

}  // namespace fsp
