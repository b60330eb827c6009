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
// in place: a float64 matrix product, run by k_contract on the matrix cores.
// A DCT-I pairs its inputs l and P - l (equal cosines up to (-1)^m), so it is
// run folded: even outputs from the sums, odd outputs from the differences,
// half the products of the plain contraction.
#include <hip/hip_runtime.h>

#include <vector>

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

// Periodic axes: Y[m] = X[f0(m0)][f1(m1)][f2(m2)] on the (n+1)^3 octant, with
// f_a(m) = min(m, n_a - m) on a periodic axis (bit a of `periodic`), m on an
// open one: the kernel at each offset's nearest image over the axis's period.
__global__ __launch_bounds__(256) void k_fold_periodic(const double* __restrict__ X, double* __restrict__ Y, int n0,
                                                       int n1, int n2, int periodic) {
  const long long total = (long long)(n0 + 1) * (n1 + 1) * (n2 + 1);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int m2 = (int)(i % (n2 + 1));
  const long long t = i / (n2 + 1);
  int m1 = (int)(t % (n1 + 1));
  int m0 = (int)(t / (n1 + 1));
  if (periodic & 1) m0 = m0 < n0 - m0 ? m0 : n0 - m0;
  if (periodic & 2) m1 = m1 < n1 - m1 ? m1 : n1 - m1;
  if (periodic & 4) m2 = m2 < n2 - m2 ? m2 : n2 - m2;
  Y[i] = X[((long long)m0 * (n1 + 1) + m1) * (n2 + 1) + m2];
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

hipError_t greens_fold_periodic(const double* X, double* Y, const int n[3], int periodic, hipStream_t s) {
  const long long total = (long long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1);
  hipLaunchKernelGGL(k_fold_periodic, dim3(grid1(total)), dim3(256), 0, s, X, Y, n[0], n[1], n[2], periodic);
  return hipGetLastError();
}

hipError_t greens_vico_spectrum(double* G, const int samples[3], const double f[3], double L, bool fft_order,
                                hipStream_t s) {
  const long long total = (long long)samples[0] * samples[1] * samples[2];
  hipLaunchKernelGGL(k_vico_spectrum, dim3(grid1(total)), dim3(256), 0, s, G, samples[0], samples[1], samples[2],
                     f[0], f[1], f[2], L, fft_order ? 1 : 0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ contractions
// One per-axis transform of a precompute is a dense float64 contraction
//     Y(m, j) = sum_k C(m, k) X(k, j)
// of a small matrix C (the transform's rows m, at most n + 1 of them) with the
// data array X along its contracted axis k, for every column j of the other
// axes.  It runs on the matrix cores (v_mfma_f64_16x16x4f64): a block owns 64
// columns j and ALL output rows m (FT blocks of 16 rows), so each element of X
// is read from HBM once per axis; its four waves own 16 columns each and hold
// FT 16 x 16 accumulators.  K slices of 16 of C and X are staged through LDS.
//   X(k, j) = x[b x_bs + k x_sk + j x_sj]   (XJ: j contiguous, else k contiguous)
//   Y(m, j) = y[b y_bs + m y_sm + j y_sj]
// Folded DCT-I (P = fold_p > 0): the inputs k and P - k of a DCT-I have
// cosines equal up to (-1)^m, so even rows m = 2 r take the sums
// X(k) + X(P - k) (X(P / 2) alone at k = P / 2) with matrix ce [re][P / 2 + 1]
// and odd rows m = 2 r + 1 the differences X(k) - X(P - k) with matrix
// co [ro][P / 2]: the whole sum with half the products.  Plain (fold_p == 0):
// ce is [re][K] over X(k), and there are no odd rows.
// MFMA 16x16x4 f64 operands: lane l holds A(l % 16, l / 16) and B(l / 16, l % 16)
// of its 16 x 4 and 4 x 16 blocks; D(i, j) of the 16 x 16 block is register
// i / 4 of lane j + 16 (i % 4) (the float64 layout, checked on the device).
typedef double v4d __attribute__((ext_vector_type(4)));

struct ContractArgs {
  const double* cp;  // the matrix rows packed per K slice: [slice][16-row block f][k 16][row 16]
  const double* x;
  double* y;
  long long x_sk, x_sj, x_bs;
  long long y_sm, y_sj, y_bs;
  int re, ro;        // even (or all) rows and odd rows
  int kmax;          // contracted length (P / 2 + 1 folded)
  int N;             // columns j
  int fold_p;        // P (> 0: folded DCT-I)
  int fe, ftot;      // 16-row blocks of the even part, of both parts
  int mblocks, jtiles;
};

constexpr int CT_K = 16;        // K slice staged in LDS
constexpr int CT_THREADS = 256;
constexpr int CT_BN = 64;       // columns per block (16 per wave)
constexpr int CT_FT = 17;       // 16-row blocks per block (272 rows: n + 1 rows up to n = 256, folded or not)

template <bool XJ>
__global__ __launch_bounds__(CT_THREADS) void k_contract(ContractArgs g) {
  constexpr int FT = CT_FT;
  __shared__ double As[FT][CT_K][16 + 2];
  __shared__ double Bs[2][CT_K][CT_BN + 2];   // sums (or plain values), differences
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool fold = g.fold_p > 0;
  const int P = g.fold_p;
  // the m blocks of one column tile are neighbours in the (per-XCD) block order
  const int nblk = g.mblocks * g.jtiles;
  const int bid = (int)blockIdx.x;
  int tile = bid;
  if (nblk % 8 == 0) tile = (bid % 8) * (nblk / 8) + bid / 8;  // a bijection for whole octets
  const int mb = tile % g.mblocks, jt = tile / g.mblocks;
  const int f0 = mb * FT, j0 = jt * CT_BN;
  const long long bb = blockIdx.y;
  const double* X = g.x + bb * g.x_bs;
  double* Y = g.y + bb * g.y_bs;
  const int kmax = g.kmax;

  // global -> register staging of one K slice
  double ra[FT];                 // the image: row block u, k t / 16, row t % 16
  constexpr int BV = CT_K * CT_BN / CT_THREADS;   // 4 data positions per thread
  double rs[BV], rd[BV];
  auto load_slice = [&](int k0) {
    {
      // one K slice of this block's row blocks is one contiguous run of the image
      const double* src = g.cp + ((long long)(k0 / CT_K) * g.ftot + f0) * 256 + t;
#pragma unroll
      for (int u = 0; u < FT; ++u) ra[u] = f0 + u < g.ftot ? src[u * 256] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      int k, j;
      if (XJ) {  // 64 consecutive columns per wave and k
        j = t % CT_BN;
        k = (t / CT_BN) * BV + u;
      } else {   // 4 consecutive k per thread
        j = t / (CT_K / BV);
        k = (t % (CT_K / BV)) * BV + u;
      }
      const int gk = k0 + k, gj = j0 + j;
      double sv = 0.0, dv = 0.0;
      if (gj < g.N && gk < kmax) {
        const double* col = X + (long long)gj * g.x_sj;
        const double a = col[(long long)gk * g.x_sk];
        if (!fold) {
          sv = a;
        } else if (2 * gk == P) {
          sv = a;
        } else {
          const double c = col[(long long)(P - gk) * g.x_sk];
          sv = a + c;
          dv = a - c;
        }
      }
      rs[u] = sv;
      rd[u] = dv;
    }
  };
  auto store_slice = [&]() {
#pragma unroll
    for (int u = 0; u < FT; ++u) As[u][t / 16][t % 16] = ra[u];
#pragma unroll
    for (int u = 0; u < BV; ++u) {
      int k, j;
      if (XJ) {
        j = t % CT_BN;
        k = (t / CT_BN) * BV + u;
      } else {
        j = t / (CT_K / BV);
        k = (t % (CT_K / BV)) * BV + u;
      }
      Bs[0][k][j] = rs[u];
      Bs[1][k][j] = rd[u];
    }
  };

  v4d acc[FT];
#pragma unroll
  for (int u = 0; u < FT; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};

  const int nk = (kmax + CT_K - 1) / CT_K;
  load_slice(0);
  for (int ks = 0; ks < nk; ++ks) {
    __syncthreads();
    store_slice();
    __syncthreads();
    if (ks + 1 < nk) load_slice((ks + 1) * CT_K);  // in flight during the products
#pragma unroll
    for (int kk = 0; kk < CT_K; kk += 4) {
      const int kr = kk + lane / 16, c = lane % 16;
      const double bsum = Bs[0][kr][wave * 16 + c];
      const double bdif = Bs[1][kr][wave * 16 + c];
#pragma unroll
      for (int u = 0; u < FT; ++u) {
        const int f = f0 + u;
        if (f < g.ftot) {  // uniform in the block
          const double a = As[u][kr][c];
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, f < g.fe ? bsum : bdif, acc[u], 0, 0, 0);
        }
      }
    }
  }
  const int j = j0 + wave * 16 + lane % 16;
  if (j >= g.N) return;
#pragma unroll
  for (int u = 0; u < FT; ++u) {
    const int f = f0 + u;
    if (f >= g.ftot) break;
    const bool even = f < g.fe;
    const int base = (even ? f : f - g.fe) * 16;
    const int rows = even ? g.re : g.ro;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pr = base + lane / 16 + 4 * r;   // row of this part
      if (pr < rows) {
        const int m = fold ? 2 * pr + (even ? 0 : 1) : pr;
        Y[(long long)m * g.y_sm + (long long)j * g.y_sj] = acc[u][r];
      }
    }
  }
}

// Contract axis `axis` of the row-major array X[d0][d1][d2] with a matrix of
// nout rows: Y has the same axis order with d_axis -> nout.  `packed` is the
// matrix image of greens_pack_contract (folded when period > 0: then
// d_axis = period + 1).
//   axis 0: one item, X viewed as [d0][d1 d2]         (columns contiguous)
//   axis 1: d0 items, X[i0] viewed as [d1][d2]        (columns contiguous)
//   axis 2: one item, X viewed as [d0 d1][d2]: column j = row of X (k contiguous)
hipError_t greens_contract_axis(const double* X, double* Y, const double* packed, int period,
                                const long long dims[3], int axis, int nout, hipStream_t s) {
  const long long d0 = dims[0], d1 = dims[1], d2 = dims[2];
  const long long dax = dims[axis];
  const bool fold = period > 0;
  if (fold && (period % 2 != 0 || dax != period + 1)) return hipErrorInvalidValue;
  if (d0 * d1 > 0x7fffffffLL || d1 * d2 > 0x7fffffffLL || nout <= 0) return hipErrorInvalidValue;
  ContractArgs g{};
  g.cp = packed;
  g.fold_p = fold ? period : 0;
  g.re = fold ? (nout + 1) / 2 : nout;
  g.ro = fold ? nout / 2 : 0;
  g.kmax = fold ? period / 2 + 1 : (int)dax;
  g.fe = (g.re + 15) / 16;
  g.ftot = g.fe + (g.ro + 15) / 16;
  g.mblocks = (g.ftot + CT_FT - 1) / CT_FT;
  int batch = 1;
  bool xj = true;
  if (axis == 0 || axis == 1) {
    const long long inner = axis == 0 ? d1 * d2 : d2;
    g.x = X;
    g.x_sk = inner;
    g.x_sj = 1;
    g.x_bs = axis == 0 ? 0 : d1 * d2;
    g.y = Y;
    g.y_sm = inner;
    g.y_sj = 1;
    g.y_bs = axis == 0 ? 0 : (long long)nout * d2;
    g.N = (int)inner;
    batch = axis == 0 ? 1 : (int)d0;
  } else {
    g.x = X;
    g.x_sk = 1;
    g.x_sj = d2;
    g.x_bs = 0;
    g.y = Y;
    g.y_sm = 1;
    g.y_sj = nout;
    g.y_bs = 0;
    g.N = (int)(d0 * d1);
    xj = false;
  }
  g.jtiles = (g.N + CT_BN - 1) / CT_BN;
  const long long nblk = (long long)g.mblocks * g.jtiles;
  if (nblk > 0x7fffffffLL || batch > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblk, (unsigned)batch);
  if (xj)
    hipLaunchKernelGGL(k_contract<true>, grid, dim3(CT_THREADS), 0, s, g);
  else
    hipLaunchKernelGGL(k_contract<false>, grid, dim3(CT_THREADS), 0, s, g);
  return hipGetLastError();
}

// Matrix image read by k_contract for a transform of nout rows over an axis of
// `kin` inputs: folded (period > 0; kin = period + 1) from the even rows ce
// [ceil(nout / 2)][period / 2 + 1] and the odd rows co [nout / 2][period / 2],
// else from c = ce [nout][kin].  Layout [slice][row block][k 16][row 16], zero
// beyond each part's rows and length.
void greens_pack_contract(std::vector<double>& out, const std::vector<double>& ce, const std::vector<double>* co,
                          int nout, int kin, int period) {
  const bool fold = period > 0;
  const int re = fold ? (nout + 1) / 2 : nout, ro = fold ? nout / 2 : 0;
  const int ke = fold ? period / 2 + 1 : kin, ko = fold ? period / 2 : 0;
  const int fe = (re + 15) / 16, ftot = fe + (ro + 15) / 16;
  const int nk = (ke + CT_K - 1) / CT_K;
  out.assign((size_t)nk * ftot * 256, 0.0);
  for (int ks = 0; ks < nk; ++ks)
    for (int f = 0; f < ftot; ++f)
      for (int kq = 0; kq < 16; ++kq)
        for (int rq = 0; rq < 16; ++rq) {
          const int k = ks * 16 + kq;
          const bool even = f < fe;
          const int row = (even ? f : f - fe) * 16 + rq;
          double v = 0.0;
          if (even && row < re && k < ke) v = ce[(size_t)row * ke + k];
          if (!even && row < ro && k < ko) v = (*co)[(size_t)row * ko + k];
          out[(((size_t)ks * ftot + f) * 16 + kq) * 16 + rq] = v;
        }
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
