// fft_core.hpp -- radix plans, twiddle-table layout and register/LDS Stockham
// stages shared by the solve kernels (gfx950, wave64).
//
// A pencil of length L is transformed by a sequence of radix-R stages
// (Stockham autosort, so the output is in natural order with no bit
// reversal).  Stage s with radix R and span NS = R_0 * ... * R_{s-1} takes,
// for each butterfly b in [0, L/R), the inputs at rows b + r L/R, multiplies
// input r by w^(r k) with k = b mod NS and w = exp(-2 pi i / (NS R)), applies
// a length-R DFT and writes output m to row (b / NS) NS R + k + m NS.
//
// Work split: a tile of TC pencils is handled by TC * NQ threads; thread
// (c, q) owns pencil c of the tile and butterflies b = q + NQ j.  The first
// stage reads its inputs straight from global memory and the last stage
// leaves its outputs in registers, at rows b + m L/R, in the same thread that
// will store them; only the stages in between exchange data through LDS.
//
// Forward transforms use the plan in order; inverse transforms use it reversed
// (the last radix of the forward plan becomes the first of the inverse), so
// in a forward -> multiply -> inverse sequence the multiply and the first
// inverse stage need no data exchange.  The first radix of every plan is even:
// when only the lower half of the rows is non-zero (zero padding) a forward
// first stage skips inputs r >= R/2, and when only the lower half of an
// inverse is kept its last stage skips outputs m >= R/2.
#pragma once

#include <hip/hip_runtime.h>

namespace fsp {

// ---------------------------------------------------------------- plans
struct RadixPlan {
  int n;
  int r[4];
};

// Radix sequences for each supported pencil length (2^a or 3 * 2^a, 8..1024).
// Plan 0 is the default; plan 1 is an alternative (fewer, larger stages or
// more, smaller ones) the autotuner may pick: at 96, 192 and 384 it is the
// two-stage plan ending in radix 12 or 24, one LDS exchange fewer than plan 0.
// The first radix is always even and divides 32.
constexpr int NUM_PLANS = 2;

__host__ __device__ constexpr RadixPlan radix_plan(int L, int pid = 0) {
  if (pid == 1) {
    switch (L) {
      case 8: return {1, {8, 0, 0, 0}};
      case 12: return {2, {4, 3, 0, 0}};
      case 16: return {2, {4, 4, 0, 0}};
      case 24: return {3, {2, 4, 3, 0}};
      case 32: return {2, {16, 2, 0, 0}};
      case 48: return {3, {4, 4, 3, 0}};
      case 64: return {2, {16, 4, 0, 0}};
      case 96: return {2, {8, 12, 0, 0}};
      case 128: return {2, {8, 16, 0, 0}};
      case 192: return {2, {8, 24, 0, 0}};
      case 256: return {3, {8, 4, 8, 0}};
      case 384: return {2, {16, 24, 0, 0}};
      case 512: return {3, {8, 8, 8, 0}};
      case 768: return {4, {16, 4, 4, 3}};
      case 1024: return {3, {16, 8, 8, 0}};
      default: return {0, {0, 0, 0, 0}};
    }
  }
  switch (L) {
    case 8: return {1, {8, 0, 0, 0}};
    case 12: return {2, {4, 3, 0, 0}};
    case 16: return {1, {16, 0, 0, 0}};
    case 24: return {2, {8, 3, 0, 0}};
    case 32: return {2, {8, 4, 0, 0}};
    case 48: return {2, {16, 3, 0, 0}};
    case 64: return {2, {8, 8, 0, 0}};
    case 96: return {3, {8, 4, 3, 0}};
    case 128: return {2, {16, 8, 0, 0}};
    case 192: return {3, {8, 8, 3, 0}};
    case 256: return {2, {16, 16, 0, 0}};
    case 384: return {3, {16, 8, 3, 0}};
    case 512: return {2, {16, 32, 0, 0}};
    case 768: return {3, {16, 16, 3, 0}};
    case 1024: return {2, {32, 32, 0, 0}};
    default: return {0, {0, 0, 0, 0}};
  }
}

__host__ __device__ constexpr int plan_len(int L, int pid = 0) { return radix_plan(L, pid).n; }

// A plan is well formed when its radices multiply to L, each has a butterfly
// (Dft below), and the first is even and divides 32 (pruned first and last
// stages, constant twiddles).
__host__ __device__ constexpr bool plan_ok(int L, int pid) {
  const RadixPlan p = radix_plan(L, pid);
  if (p.n < 1 || p.n > 4 || p.r[0] % 2 != 0 || 32 % p.r[0] != 0) return false;
  int prod = 1;
  for (int i = 0; i < p.n; ++i) {
    const int r = p.r[i];
    if (r != 2 && r != 3 && r != 4 && r != 8 && r != 12 && r != 16 && r != 24 && r != 32) return false;
    prod *= r;
  }
  return prod == L;
}
__host__ __device__ constexpr bool plans_ok() {
  constexpr int lengths[] = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  for (int L : lengths)
    for (int pid = 0; pid < NUM_PLANS; ++pid)
      if (!plan_ok(L, pid)) return false;
  return true;
}
static_assert(plans_ok(), "every radix plan multiplies to its length and starts with an even radix dividing 32");

// Radix of stage s; rev selects the reversed plan used by inverse transforms.
__host__ __device__ constexpr int plan_radix(int L, int pid, bool rev, int s) {
  return rev ? radix_plan(L, pid).r[radix_plan(L, pid).n - 1 - s] : radix_plan(L, pid).r[s];
}

__host__ __device__ constexpr int plan_ns(int L, int pid, bool rev, int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= plan_radix(L, pid, rev, i);
  return ns;
}

// Twiddle table of one plan order: stage s >= 1 holds, for each k in [0, NS),
// six complex values w^k, w^2k, w^4k, w^8k, w^16k, w^3k with
// w = exp(-2 pi i / (NS R)); every other power w^rk (r < 32) is a product of
// at most three of them.
constexpr int TW_PER_K = 6;
__host__ __device__ constexpr int tw_power(int e) { return e == 5 ? 3 : (1 << e); }

__host__ __device__ constexpr int tw_stage_off(int L, int pid, bool rev, int s) {
  int off = 0;
  for (int i = 1; i < s; ++i) off += plan_ns(L, pid, rev, i) * TW_PER_K;
  return off;
}

__host__ __device__ constexpr int tw_order_size(int L, int pid, bool rev) {
  return tw_stage_off(L, pid, rev, plan_len(L, pid));
}

// Table for one length and plan: forward order, then reversed order.
__host__ __device__ constexpr int tw_size(int L, int pid) {
  return tw_order_size(L, pid, false) + tw_order_size(L, pid, true);
}
__host__ __device__ constexpr int tw_base(int L, int pid, bool rev) {
  return rev ? tw_order_size(L, pid, false) : 0;
}

// Complete twiddle table of one plan, for kernels that keep it in LDS: stage
// s >= 1 of an order holds w^(r k) for k in [0, NS) and r in [1, R) at
// k (R - 1) + r - 1 (so butterflies read from different LDS banks); forward
// order, then reversed order.  It follows the six-power table.
__host__ __device__ constexpr int twf_stage_size(int L, int pid, bool rev, int s) {
  return plan_ns(L, pid, rev, s) * (plan_radix(L, pid, rev, s) - 1);
}
__host__ __device__ constexpr int twf_stage_off(int L, int pid, bool rev, int s) {
  int off = 0;
  if (rev)
    for (int i = 1; i < plan_len(L, pid); ++i) off += twf_stage_size(L, pid, false, i);
  for (int i = 1; i < s; ++i) off += twf_stage_size(L, pid, rev, i);
  return off;
}
__host__ __device__ constexpr int twf_size(int L, int pid) { return twf_stage_off(L, pid, true, plan_len(L, pid)); }

// ---------------------------------------------------------------- complex
template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.x, -a.y}; }

// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// multiply by the constant (c, s) for the forward transform, (c, -s) for the inverse
template <bool INV, typename T>
__device__ __forceinline__ cx<T> mul_const(cx<T> a, T c, T s) {
  const T si = INV ? -s : s;
  return {a.x * c - a.y * si, a.x * si + a.y * c};
}

// ---------------------------------------------------------------- butterflies
// v[m] <- sum_r v[r] exp(-+ 2 pi i r m / R)   (- forward, + inverse)
template <int R, bool INV, typename T>
struct Dft;

template <bool INV, typename T>
struct Dft<2, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV, typename T>
struct Dft<3, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
    const cx<T> s = cadd(v[1], v[2]);
    const cx<T> d = mul_mi<INV>(csub(v[1], v[2]));
    const cx<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    v[0] = cadd(v[0], s);
    v[1] = {m.x + h * d.x, m.y + h * d.y};
    v[2] = {m.x - h * d.x, m.y - h * d.y};
  }
};

template <bool INV, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  const cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const cx<T> t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <bool INV, typename T>
struct Dft<4, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }
};

template <bool INV, typename T>
__device__ __forceinline__ void dft8(cx<T>* v, int st) {
  // v[0], v[st], ..., v[7 st]
  cx<T> e0 = v[0], e1 = v[2 * st], e2 = v[4 * st], e3 = v[6 * st];
  cx<T> o0 = v[st], o1 = v[3 * st], o2 = v[5 * st], o3 = v[7 * st];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  const T r = T(0.70710678118654752440);  // sqrt(1/2)
  o1 = mul_const<INV>(o1, r, -r);
  o2 = mul_mi<INV>(o2);
  o3 = mul_const<INV>(o3, -r, -r);
  v[0] = cadd(e0, o0);
  v[4 * st] = csub(e0, o0);
  v[st] = cadd(e1, o1);
  v[5 * st] = csub(e1, o1);
  v[2 * st] = cadd(e2, o2);
  v[6 * st] = csub(e2, o2);
  v[3 * st] = cadd(e3, o3);
  v[7 * st] = csub(e3, o3);
}

template <bool INV, typename T>
struct Dft<8, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) { dft8<INV>(v, 1); }
};

template <bool INV, typename T>
struct Dft<16, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    // 16 = 2 x 8: length-8 DFTs of the even and odd samples, then one radix-2 layer.
    cx<T> e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft8<INV>(e, 1);
    dft8<INV>(o, 1);
    const T c1 = T(0.92387953251128675613);  // cos(pi/8)
    const T s1 = T(0.38268343236508977173);  // sin(pi/8)
    const T r = T(0.70710678118654752440);
    // o[k] *= exp(-+ 2 pi i k / 16)
    o[1] = mul_const<INV>(o[1], c1, -s1);
    o[2] = mul_const<INV>(o[2], r, -r);
    o[3] = mul_const<INV>(o[3], s1, -c1);
    o[4] = mul_mi<INV>(o[4]);
    o[5] = mul_const<INV>(o[5], -s1, -c1);
    o[6] = mul_const<INV>(o[6], -r, -r);
    o[7] = mul_const<INV>(o[7], -c1, -s1);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 8] = csub(e[k], o[k]);
    }
  }
};

template <bool INV, typename T>
struct Dft<32, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    // 32 = 2 x 16: length-16 DFTs of the even and odd samples, then one radix-2 layer.
    cx<T> e[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    Dft<16, INV, T>::run(e);
    Dft<16, INV, T>::run(o);
    const T c1 = T(0.98078528040323044913);  // cos(pi/16)
    const T s1 = T(0.19509032201612826785);  // sin(pi/16)
    const T c2 = T(0.92387953251128675613);  // cos(pi/8)
    const T s2 = T(0.38268343236508977173);  // sin(pi/8)
    const T c3 = T(0.83146961230254523708);  // cos(3pi/16)
    const T s3 = T(0.55557023301960222474);  // sin(3pi/16)
    const T r = T(0.70710678118654752440);
    // o[k] *= exp(-+ 2 pi i k / 32)
    o[1] = mul_const<INV>(o[1], c1, -s1);
    o[2] = mul_const<INV>(o[2], c2, -s2);
    o[3] = mul_const<INV>(o[3], c3, -s3);
    o[4] = mul_const<INV>(o[4], r, -r);
    o[5] = mul_const<INV>(o[5], s3, -c3);
    o[6] = mul_const<INV>(o[6], s2, -c2);
    o[7] = mul_const<INV>(o[7], s1, -c1);
    o[8] = mul_mi<INV>(o[8]);
    o[9] = mul_const<INV>(o[9], -s1, -c1);
    o[10] = mul_const<INV>(o[10], -s2, -c2);
    o[11] = mul_const<INV>(o[11], -s3, -c3);
    o[12] = mul_const<INV>(o[12], -r, -r);
    o[13] = mul_const<INV>(o[13], -c3, -s3);
    o[14] = mul_const<INV>(o[14], -c2, -s2);
    o[15] = mul_const<INV>(o[15], -c1, -s1);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 16] = csub(e[k], o[k]);
    }
  }
};

// Multiplicative inverse of a modulo m (a, m coprime; 1 when m == 1).
__host__ __device__ constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

// Length N1 N2 DFT for coprime N1, N2 by the prime-factor (Good-Thomas) index
// maps, which need no twiddles between the two layers: input n = (N2 n1 + N1 n2)
// mod N feeds length-N1 DFTs over n1, then length-N2 DFTs over n2 give output
// k = (N2 u k1 + N1 t k2) mod N, u = N2^-1 mod N1, t = N1^-1 mod N2.
template <int N1, int N2, bool INV, typename T>
__device__ __forceinline__ void dft_pfa(cx<T>* v) {
  constexpr int N = N1 * N2;
  constexpr int U = inv_mod(N2 % N1, N1), TT = inv_mod(N1 % N2, N2);
  cx<T> a[N2][N1];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) a[n2][n1] = v[(N2 * n1 + N1 * n2) % N];
    Dft<N1, INV, T>::run(a[n2]);
  }
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    cx<T> b[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) b[n2] = a[n2][k1];
    Dft<N2, INV, T>::run(b);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) v[(N2 * U * k1 + N1 * TT * k2) % N] = b[k2];
  }
}

// Radices 12 = 3 x 4 and 24 = 8 x 3 (the last stage of the two-stage plans of
// lengths 3 * 2^a).
template <bool INV, typename T>
struct Dft<12, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) { dft_pfa<3, 4, INV, T>(v); }
};
template <bool INV, typename T>
struct Dft<24, INV, T> {
  static __device__ __forceinline__ void run(cx<T>* v) { dft_pfa<8, 3, INV, T>(v); }
};

// ---------------------------------------------------------------- pruned butterflies
// exp(-2 pi i r / R) = (tw_c, tw_s) for r < R / 2, R <= 32 (forward sign; the
// inverse conjugates through mul_const<INV>).
__host__ __device__ constexpr double tw_cos(int r, int R) {
  // cos(2 pi r / R) for the 16 angles r / R in [0, 1/2) with R | 32
  constexpr double c32[16] = {1.0,
                              0.98078528040323044913,
                              0.92387953251128675613,
                              0.83146961230254523708,
                              0.70710678118654752440,
                              0.55557023301960222474,
                              0.38268343236508977173,
                              0.19509032201612826785,
                              0.0,
                              -0.19509032201612826785,
                              -0.38268343236508977173,
                              -0.55557023301960222474,
                              -0.70710678118654752440,
                              -0.83146961230254523708,
                              -0.92387953251128675613,
                              -0.98078528040323044913};
  return c32[r * (32 / R)];
}
__host__ __device__ constexpr double tw_sin(int r, int R) {
  // sin(2 pi r / R) = cos(2 pi (r / R - 1/4)); for r / R < 1/4 use the cosine of the complement
  return (4 * r * (32 / R) >= 32) ? tw_cos(r * (32 / R) - 8, 32) : tw_cos(8 - r * (32 / R), 32);
}

// v[r] *= exp(-+ 2 pi i r / R) for a compile-time r (exact for r = 0 and r = R / 4)
template <int R, int r, bool INV, typename T>
__device__ __forceinline__ cx<T> twiddle_const(cx<T> a) {
  static_assert(32 % R == 0, "constant twiddles of radices dividing 32");
  if constexpr (r == 0) {
    return a;
  } else if constexpr (4 * r == R) {
    return mul_mi<INV>(a);
  } else {
    constexpr T c = T(tw_cos(r, R)), sn = T(-tw_sin(r, R));
    return mul_const<INV>(a, c, sn);
  }
}

template <int R, bool INV, typename T, int r = 0>
__device__ __forceinline__ void twiddle_all(cx<T>* b) {
  if constexpr (r < R / 2) {
    b[r] = twiddle_const<R, r, INV>(b[r]);
    twiddle_all<R, INV, T, r + 1>(b);
  }
}

// Length-R DFT of inputs whose upper half is zero (v[r], r >= R / 2, unread):
// output 2 m takes DFT_{R/2}(v[r]), output 2 m + 1 takes DFT_{R/2}(v[r] w_R^r).
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_half_in(cx<T>* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    v[1] = v[0];
  } else {
    cx<T> a[R / 2], b[R / 2];
#pragma unroll
    for (int r = 0; r < R / 2; ++r) a[r] = b[r] = v[r];
    twiddle_all<R, INV>(b);
    Dft<R / 2, INV, T>::run(a);
    Dft<R / 2, INV, T>::run(b);
#pragma unroll
    for (int m = 0; m < R / 2; ++m) {
      v[2 * m] = a[m];
      v[2 * m + 1] = b[m];
    }
  }
}

// Outputs m < R / 2 of a length-R DFT (the others are not computed):
// s[r] = v[r] + v[r + R/2] gives the even outputs, d[r] = (v[r] - v[r + R/2]) w_R^r
// the odd ones, each the first half of a length-R/2 DFT.
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_half_out(cx<T>* v) {
  if constexpr (R == 2) {
    v[0] = cadd(v[0], v[1]);
  } else if constexpr (R == 3 || R == 1) {
    Dft<R, INV, T>::run(v);
  } else {
    cx<T> s[R / 2], d[R / 2];
#pragma unroll
    for (int r = 0; r < R / 2; ++r) {
      s[r] = cadd(v[r], v[r + R / 2]);
      d[r] = csub(v[r], v[r + R / 2]);
    }
    twiddle_all<R, INV>(d);
    dft_half_out<R / 2, INV, T>(s);
    dft_half_out<R / 2, INV, T>(d);
#pragma unroll
    for (int m = 0; m < R / 4; ++m) {
      v[2 * m] = s[m];
      v[2 * m + 1] = d[m];
    }
  }
}

// ---------------------------------------------------------------- barriers
// Workgroup barrier for LDS reuse only: waits for this wave's LDS traffic,
// then synchronises the waves.  Global loads and stores stay in flight (the
// kernels never exchange data through global memory inside a launch), so a
// prefetch issued before the barrier keeps overlapping with the work after it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Keeps the compiler from moving memory operations across this point, so
// loads issued before it complete (in order) before those issued after.
__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }

// ---------------------------------------------------------------- stages
// Two consecutive complex values of the twiddle table in one load where the type allows.
template <typename T>
__device__ __forceinline__ void load_pair(const cx<T>* p, cx<T>& a, cx<T>& b) {
  if constexpr (sizeof(T) == 4) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    a = {q.x, q.y};
    b = {q.z, q.w};
  } else {
    a = p[0];
    b = p[1];
  }
}

// The six-power table values of one butterfly (those a radix R needs).
template <typename T>
struct TwBase {
  cx<T> w1, w2, w3, w4, w8, w16;
};

template <typename T, int R>
__device__ __forceinline__ void load_twbase(TwBase<T>& t, const cx<T>* __restrict__ tw, int k) {
  const cx<T>* e = tw + k * TW_PER_K;
  load_pair(e, t.w1, t.w2);
  if constexpr (R >= 4) load_pair(e + 4, t.w16, t.w3);
  if constexpr (R >= 8) load_pair(e + 2, t.w4, t.w8);
}

// v[r] *= w^(r k) (forward) or its conjugate (inverse), r = 1 .. R-1, from the
// loaded table values of butterfly k.
template <typename T, int R, bool INV>
__device__ __forceinline__ void apply_twbase(cx<T>* v, const TwBase<T>& t) {
  cx<T> w[R];
  w[1] = t.w1;
  if constexpr (R >= 3) w[2] = t.w2;
  if constexpr (R >= 4) w[3] = t.w3;
  if constexpr (R >= 8) {
    w[4] = t.w4;
    w[5] = cmul(t.w4, t.w1);
    w[6] = cmul(t.w4, t.w2);
    w[7] = cmul(t.w4, t.w3);
  }
  if constexpr (R >= 12) {
    w[8] = t.w8;
#pragma unroll
    for (int r = 9; r < (R < 16 ? R : 16); ++r) w[r] = cmul(t.w8, w[r - 8]);
  }
  if constexpr (R >= 24) {
    w[16] = t.w16;
#pragma unroll
    for (int r = 17; r < R; ++r) w[r] = cmul(t.w16, w[r - 16]);
  }
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], w[r]) : cmul(v[r], w[r]);
}

// v[r] *= w^(r k) (forward) or its conjugate (inverse), r = 1 .. R-1.
template <typename T, int R, int NS, bool INV>
__device__ __forceinline__ void apply_twiddles(cx<T>* v, const cx<T>* __restrict__ tw, int k) {
  if constexpr (NS > 1) {
    TwBase<T> t;
    load_twbase<T, R>(t, tw, k);
    apply_twbase<T, R, INV>(v, t);
  }
}

// v[r] *= w^(r k) or its conjugate from the complete table of the stage.
template <typename T, int R, int NS, bool INV>
__device__ __forceinline__ void apply_twiddles_full(cx<T>* v, const cx<T>* tf, int k) {
  if constexpr (NS > 1) {
    const cx<T>* e = tf + k * (R - 1) - 1;
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], e[r]) : cmul(v[r], e[r]);
  }
}

// Twiddles of stage S: from the six-power table tw (FULL == false) or from the
// complete table at tw (FULL == true).
template <typename T, int L, int PID, bool REV, int S, bool INV, bool FULL>
__device__ __forceinline__ void stage_twiddles(cx<T>* v, const cx<T>* tw, int k) {
  constexpr int R = plan_radix(L, PID, REV, S);
  constexpr int NS = plan_ns(L, PID, REV, S);
  if constexpr (FULL)
    apply_twiddles_full<T, R, NS, INV>(v, tw + twf_stage_off(L, PID, REV, S), k);
  else
    apply_twiddles<T, R, NS, INV>(v, tw + tw_base(L, PID, REV) + tw_stage_off(L, PID, REV, S), k);
}

// One middle stage: inputs from LDS, outputs back to LDS (in place, two barriers).
// idx(row) maps a pencil row to this thread's LDS slot.
template <typename T, int L, int PID, bool REV, int S, int NQ, bool INV, bool FULL = false, class IDX>
__device__ __forceinline__ void lds_stage(cx<T>* lds, const cx<T>* __restrict__ tw, int q, IDX idx) {
  constexpr int R = plan_radix(L, PID, REV, S);
  constexpr int NS = plan_ns(L, PID, REV, S);
  constexpr int NB = L / R;
  constexpr int J = (NB + NQ - 1) / NQ;
  cx<T> v[J][R];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int b = q + NQ * j;
    if ((NB % NQ == 0) || b < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[j][r] = lds[idx(b + r * NB)];
    }
  }
  lds_barrier();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int b = q + NQ * j;
    if ((NB % NQ == 0) || b < NB) {
      stage_twiddles<T, L, PID, REV, S, INV, FULL>(v[j], tw, b % NS);
      Dft<R, INV, T>::run(v[j]);
      const int base = (b / NS) * NS * R + (b % NS);
#pragma unroll
      for (int m = 0; m < R; ++m) lds[idx(base + m * NS)] = v[j][m];
    }
  }
  lds_barrier();
}

template <typename T, int L, int PID, bool REV, int S, int SEND, int NQ, bool INV, bool FULL = false, class IDX>
__device__ __forceinline__ void lds_stages(cx<T>* lds, const cx<T>* __restrict__ tw, int q, IDX idx) {
  if constexpr (S < SEND) {
    lds_stage<T, L, PID, REV, S, NQ, INV, FULL>(lds, tw, q, idx);
    lds_stages<T, L, PID, REV, S + 1, SEND, NQ, INV, FULL>(lds, tw, q, idx);
  }
}

// Last stage: inputs from LDS, outputs left in registers v[j][m] = row b + m L/R.
// HALF: only the outputs m < R / 2 are computed (the rest are left undefined).
template <typename T, int L, int PID, bool REV, int NQ, bool INV, bool FULL = false, bool HALF = false, int J, int R,
          class IDX>
__device__ __forceinline__ void lds_last_stage(const cx<T>* lds, const cx<T>* __restrict__ tw, int q,
                                               IDX idx, cx<T> (&v)[J][R]) {
  constexpr int S = plan_len(L, PID) - 1;
  constexpr int NS = plan_ns(L, PID, REV, S);
  constexpr int NB = L / R;
  static_assert(R == plan_radix(L, PID, REV, S), "register array matches the last radix");
  static_assert(J == (NB + NQ - 1) / NQ, "register array matches the butterfly split");
  static_assert(NS == NB, "last stage spans the pencil");
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int b = q + NQ * j;
    if ((NB % NQ == 0) || b < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[j][r] = lds[idx(b + r * NB)];
      stage_twiddles<T, L, PID, REV, S, INV, FULL>(v[j], tw, b);
      if constexpr (HALF)
        dft_half_out<R, INV, T>(v[j]);
      else
        Dft<R, INV, T>::run(v[j]);
    }
  }
}

// Last stage with the butterflies' table values already loaded (tb[j] for
// butterfly q + NQ j, a stage that spans the pencil: NS == NB).
template <typename T, int L, int PID, bool REV, int NQ, bool INV, int J, int R, class IDX>
__device__ __forceinline__ void lds_last_stage_pre(const cx<T>* lds, const TwBase<T> (&tb)[J], int q, IDX idx,
                                                   cx<T> (&v)[J][R]) {
  constexpr int NB = L / R;
  static_assert(R == plan_radix(L, PID, REV, plan_len(L, PID) - 1), "register array matches the last radix");
  static_assert(J == (NB + NQ - 1) / NQ, "register array matches the butterfly split");
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int b = q + NQ * j;
    if ((NB % NQ == 0) || b < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[j][r] = lds[idx(b + r * NB)];
      apply_twbase<T, R, INV>(v[j], tb[j]);
      Dft<R, INV, T>::run(v[j]);
    }
  }
}

// Table values of the last stage's butterflies q + NQ j.
template <typename T, int L, int PID, bool REV, int NQ, int J>
__device__ __forceinline__ void load_last_twbase(TwBase<T> (&tb)[J], const cx<T>* __restrict__ tw, int q) {
  constexpr int S = plan_len(L, PID) - 1;
  constexpr int R = plan_radix(L, PID, REV, S);
  constexpr int NB = L / R;
  const cx<T>* tws = tw + tw_base(L, PID, REV) + tw_stage_off(L, PID, REV, S);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int b = q + NQ * j;
    load_twbase<T, R>(tb[j], tws, (NB % NQ == 0) || b < NB ? b : 0);
  }
}

// Write first-stage outputs (span 1) to LDS: output m of butterfly b is row b R + m.
template <typename T, int R, int J, int NB, int NQ, class IDX>
__device__ __forceinline__ void write_first_outputs(cx<T>* lds, const cx<T> (&v)[J][R], int q, IDX idx) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int b = q + NQ * j;
    if ((NB % NQ == 0) || b < NB) {
#pragma unroll
      for (int m = 0; m < R; ++m) lds[idx(b * R + m)] = v[j][m];
    }
  }
}

// Exchange between the first stage (outputs of butterfly b at rows b R + m)
// and the last stage of a two-stage plan (inputs of butterfly b2 at rows
// b2 + r NB2) through an LDS array of real values: the real parts, then the
// imaginary parts, so the array is half the size of a complex one.  The
// caller has synchronised the array's previous use; three barriers inside.
template <typename T, int R, int J, int NB, int NQ, int R2, int J2, int NB2, class IDX>
__device__ __forceinline__ void exchange_split(T* lds, const cx<T> (&v)[J][R], cx<T> (&w)[J2][R2], int q,
                                               IDX idx) {
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if (part == 1) lds_barrier();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int b = q + NQ * j;
      if ((NB % NQ == 0) || b < NB) {
#pragma unroll
        for (int m = 0; m < R; ++m) lds[idx(b * R + m)] = part == 0 ? v[j][m].x : v[j][m].y;
      }
    }
    lds_barrier();
#pragma unroll
    for (int j = 0; j < J2; ++j) {
      const int b = q + NQ * j;
      if ((NB2 % NQ == 0) || b < NB2) {
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          if (part == 0)
            w[j][r].x = lds[idx(b + r * NB2)];
          else
            w[j][r].y = lds[idx(b + r * NB2)];
        }
      }
    }
  }
}

// The last stage on inputs already in registers (after exchange_split);
// FULL: tw is the complete table (as in lds_last_stage).
template <typename T, int L, int PID, bool REV, int NQ, bool INV, bool HALF, bool FULL = false, int J, int R>
__device__ __forceinline__ void last_stage_regs(cx<T> (&v)[J][R], const cx<T>* __restrict__ tw, int q) {
  constexpr int S = plan_len(L, PID) - 1;
  constexpr int NB = L / R;
  static_assert(R == plan_radix(L, PID, REV, S), "register array matches the last radix");
  static_assert(plan_ns(L, PID, REV, S) == NB, "last stage spans the pencil");
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int b = q + NQ * j;
    if ((NB % NQ == 0) || b < NB) {
      stage_twiddles<T, L, PID, REV, S, INV, FULL>(v[j], tw, b);
      if constexpr (HALF)
        dft_half_out<R, INV, T>(v[j]);
      else
        Dft<R, INV, T>::run(v[j]);
    }
  }
}

// Shape helpers for register arrays of the first / last stage.
template <int L, int PID, bool REV, int NQ>
struct FirstStage {
  static constexpr int R = plan_radix(L, PID, REV, 0);
  static constexpr int NB = L / R;
  static constexpr int J = (NB + NQ - 1) / NQ;
};
template <int L, int PID, bool REV, int NQ>
struct LastStage {
  static constexpr int R = plan_radix(L, PID, REV, plan_len(L, PID) - 1);
  static constexpr int NB = L / R;
  static constexpr int J = (NB + NQ - 1) / NQ;
};

}  // namespace fsp
