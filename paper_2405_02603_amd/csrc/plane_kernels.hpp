// plane_kernels.hpp -- axis-2 and axis-1 passes fused per i0-plane (small cubic-ish grids).
//
// For grids whose i0-plane of the axis-2 spectrum, X[i1][k] for i1 < n1 and
// k <= n2, fits in LDS, P1 and P2 run as one kernel and P4 and P5 as another:
// one block per plane (and item) keeps the plane in LDS between the axis-2
// and the axis-1 transforms, so the spectrum S is written once by the forward
// kernel and read once by the inverse kernel, and the axis-2 spectrum never
// goes to HBM.  The arithmetic is that of the separate passes with the same
// radix plans (same butterflies, same order): only where intermediate values
// live differs.                                     [Section 2.2, steps 1, 2, 4, 5]
//
//   k_plane_fwd  rows of rho (i0, i1): real transform of length 2 n2 of the
//                zero-padded row, as in P1, into the plane; then the columns
//                k of the plane: forward transform of length 2 n1 whose upper
//                half of inputs is the padding, as in P2; all 2 n1 rows to S.
//   k_plane_inv  columns k of S plane i0: inverse transform of length 2 n1,
//                rows < n1 kept, as in P4, into the plane; then the rows:
//                inverse real transform of length 2 n2, first n2 samples kept,
//                as in P5, to phi.
//
// The plane's rows use the row passes' padded pitch (row_slot).  Row phase:
// NQR threads per row, NT / NQR rows at a time.  Column phase: TC adjacent
// columns (consecutive lanes, contiguous in S) with NQC threads per pencil,
// column tiles in turn; the column stages exchange through a scratch array of
// L1 * TC complex values.
#pragma once

#include "solve_kernels.hpp"

namespace fsp {

struct PlaneArgs {
  const ItemPtrs* items;   // table of this launch's items, or NULL (then in / out)
  const void* in[MAX_ITEMS];   // forward: rho; inverse: S (or a gradient output's spectrum)
  void* out[MAX_ITEMS];        // forward: S; inverse: phi (or a gradient component)
  const void* twr;   // row twiddles (length n2, row plan) then exp(-i pi k / n2), k in [0, n2]
  const void* twc;   // column twiddles (length 2 n1, column plan)
  long long plane;   // complex elements between S planes i0 (2 n1 P)
  int pitch;         // P
};

// Shape of the plane kernels for n1 == n2 == N: row plan and threads per row,
// column plan, column tile and threads per pencil (TC * NQC threads a block,
// NT / NQR rows per row group).  tc == 0: not built for N.
struct PlaneCfg {
  int pidr, nqr, pidc, tc, nqc;
};

template <typename T>
__host__ __device__ constexpr PlaneCfg plane_cfg(int N) {
  if constexpr (sizeof(T) == 4) {
    switch (N) {
      case 32: return {0, 4, 0, 16, 8};
      case 48: return {0, 4, 0, 16, 12};
      case 64: return {0, 4, 0, 32, 8};
      case 96: return {0, 4, 0, 16, 24};
      case 128: return {0, 4, 1, 8, 32};
      default: return {0, 0, 0, 0, 0};
    }
  } else {
    switch (N) {
      case 32: return {0, 4, 0, 8, 8};
      case 48: return {0, 4, 0, 16, 12};
      case 64: return {0, 4, 0, 16, 8};
      default: return {0, 0, 0, 0, 0};
    }
  }
}

template <typename T>
__host__ __device__ constexpr int plane_lds_bytes(int N) {
  const PlaneCfg c = plane_cfg<T>(N);
  return (N * row_pitch(N) + 2 * N * c.tc) * 2 * (int)sizeof(T);
}

template <typename T, int N, int PIDR, int NQR, int PIDC, int TC, int NQC>
__global__ __launch_bounds__(TC* NQC) void k_plane_fwd(PlaneArgs a) {
  constexpr int LC = N, L1 = 2 * N, NT = TC * NQC, TRR = NT / NQR, G = N / TRR;
  static_assert(NT % NQR == 0 && N % TRR == 0, "row groups tile the plane");
  constexpr int PP = row_pitch(LC);
  constexpr int KR = plan_len(LC, PIDR), KC = plan_len(L1, PIDC);
  __shared__ cx<T> pl[N * PP];
  __shared__ cx<T> cs[KC > 1 ? L1 * TC : 1];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x;
  const cx<T>* rho = reinterpret_cast<const cx<T>*>(a.items ? a.items[blockIdx.y].rho : a.in[blockIdx.y]);
  cx<T>* S = reinterpret_cast<cx<T>*>(a.items ? a.items[blockIdx.y].work : a.out[blockIdx.y]);
  const cx<T>* twr = reinterpret_cast<const cx<T>*>(a.twr);
  const cx<T>* twc = reinterpret_cast<const cx<T>*>(a.twc);

  // ---- rows: every row group's input is requested before the first transform
  const int qr = tid % NQR, cr = tid / NQR;
  using F = FirstStage<LC, PIDR, false, NQR>;
  static_assert(F::R % 2 == 0, "forward plans start with an even radix");
  cx<T> raw[G][F::J][F::R / 2];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int i1 = g * TRR + cr;
    const cx<T>* in = rho + ((long long)i0 * N + i1) * (LC / 2);
    issue_fence();
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
      const int b = qr + NQR * j;
      const bool ok = (F::NB % NQR == 0) || b < F::NB;
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) raw[g][j][r] = ok ? ld_once(&in[b + r * F::NB]) : czero<T>();
    }
  }
  issue_fence();
  const cx<T>* pp = twr + tw_size(LC, PIDR);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int i1 = g * TRR + cr;
    auto idx = [i1](int e) { return i1 * PP + row_slot(e); };
    cx<T> v[F::J][F::R];
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) v[j][r] = raw[g][j][r];
      dft_half_in<F::R, false, T>(v[j]);  // the upper half of z is the zero padding
    }
    write_first_outputs<T, F::R, F::J, F::NB, NQR>(pl, v, qr, idx);
    lds_barrier();
    if constexpr (KR > 1) {
      lds_stages<T, LC, PIDR, false, 1, KR - 1, NQR, false>(pl, twr, qr, idx);
      using Ls = LastStage<LC, PIDR, false, NQR>;
      cx<T> w[Ls::J][Ls::R];
      lds_last_stage<T, LC, PIDR, false, NQR, false>(pl, twr, qr, idx, w);
      lds_barrier();
#pragma unroll
      for (int j = 0; j < Ls::J; ++j) {
        const int b = qr + NQR * j;
        if ((Ls::NB % NQR == 0) || b < Ls::NB) {
#pragma unroll
          for (int m = 0; m < Ls::R; ++m) pl[idx(b + m * Ls::NB)] = w[j][m];
        }
      }
      lds_barrier();
    }
    // split: the n2 + 1 non-negative frequencies of the real row, in place.  A
    // thread takes k and n2 - k together (k <= n2 / 2): it alone reads and
    // writes those two slots (k == 0 pairs with the slot n2, from z_0 alone).
    constexpr int JS = (LC / 2 + 1 + NQR - 1) / NQR;
#pragma unroll
    for (int j = 0; j < JS; ++j) {
      const int k = qr + NQR * j;
      if (k <= LC / 2) {
        const cx<T> Za = pl[idx(k)];
        const cx<T> Zb = pl[idx(k == 0 ? 0 : LC - k)];
        auto split = [](cx<T> A, cx<T> Bc, cx<T> w) {
          const cx<T> B = conjg(Bc);
          const cx<T> E = {T(0.5) * (A.x + B.x), T(0.5) * (A.y + B.y)};
          const cx<T> D = {T(0.5) * (A.x - B.x), T(0.5) * (A.y - B.y)};
          const cx<T> U = cmul(w, D);
          return cx<T>{E.x + U.y, E.y - U.x};
        };
        const cx<T> Xa = split(Za, Zb, pp[k]);         // X[k]
        const cx<T> Xb = split(Zb, Za, pp[LC - k]);    // X[n2 - k]
        pl[idx(k)] = Xa;
        if (k != LC / 2) pl[idx(LC - k)] = Xb;
      }
    }
  }
  lds_barrier();

  // ---- columns k <= n2 of the plane: axis-1 forward transforms, all 2 n1 rows to S
  const int c = tid % TC, q = tid / TC;
  using FC = FirstStage<L1, PIDC, false, NQC>;
  static_assert(FC::R % 2 == 0, "forward plans start with an even radix");
  constexpr int NTILE = (N + 1 + TC - 1) / TC;
  cx<T>* const Sb = S + (long long)i0 * a.plane;
  const unsigned P = (unsigned)a.pitch;
  auto cidx = [c](int row) { return row * TC + c; };
#pragma unroll 1
  for (int t = 0; t < NTILE; ++t) {
    const int k = t * TC + c;
    const bool kok = k <= N;
    const int ks = row_slot(kok ? k : N);
    cx<T> v[FC::J][FC::R];
#pragma unroll
    for (int j = 0; j < FC::J; ++j) {
      const int b = q + NQC * j;
      const bool ok = (FC::NB % NQC == 0) || b < FC::NB;
#pragma unroll
      for (int r = 0; r < FC::R; ++r)  // rows >= n1 are the zero padding
        v[j][r] = (ok && r < FC::R / 2) ? pl[(b + r * FC::NB) * PP + ks] : czero<T>();
      dft_half_in<FC::R, false, T>(v[j]);
    }
    if constexpr (KC == 1) {
#pragma unroll
      for (int j = 0; j < FC::J; ++j) {
        const int b = q + NQC * j;
        if (kok && ((FC::NB % NQC == 0) || b < FC::NB)) {
#pragma unroll
          for (int m = 0; m < FC::R; ++m) put<T, PASS_COL_FWD>(&Sb[(b + m * FC::NB) * P + k], v[j][m]);
        }
      }
    } else {
      if (t > 0) lds_barrier();  // the previous tile's last stage has read the scratch
      write_first_outputs<T, FC::R, FC::J, FC::NB, NQC>(cs, v, q, cidx);
      lds_barrier();
      lds_stages<T, L1, PIDC, false, 1, KC - 1, NQC, false>(cs, twc, q, cidx);
      using Lc = LastStage<L1, PIDC, false, NQC>;
      cx<T> w[Lc::J][Lc::R];
      lds_last_stage<T, L1, PIDC, false, NQC, false>(cs, twc, q, cidx, w);
#pragma unroll
      for (int j = 0; j < Lc::J; ++j) {
        const int b = q + NQC * j;
        if (kok && ((Lc::NB % NQC == 0) || b < Lc::NB)) {
#pragma unroll
          for (int m = 0; m < Lc::R; ++m) put<T, PASS_COL_FWD>(&Sb[(b + m * Lc::NB) * P + k], w[j][m]);
        }
      }
    }
  }
}

template <typename T, int N, int PIDR, int NQR, int PIDC, int TC, int NQC>
__global__ __launch_bounds__(TC* NQC) void k_plane_inv(PlaneArgs a) {
  constexpr int LC = N, L1 = 2 * N, NT = TC * NQC, TRR = NT / NQR, G = N / TRR;
  static_assert(NT % NQR == 0 && N % TRR == 0, "row groups tile the plane");
  constexpr int PP = row_pitch(LC);
  constexpr int KR = plan_len(LC, PIDR), KC = plan_len(L1, PIDC);
  __shared__ cx<T> pl[N * PP];
  __shared__ cx<T> cs[KC > 1 ? L1 * TC : 1];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x;
  const cx<T>* S = reinterpret_cast<const cx<T>*>(a.items ? a.items[blockIdx.y].work : a.in[blockIdx.y]);
  cx<T>* phi = reinterpret_cast<cx<T>*>(a.items ? a.items[blockIdx.y].phi : a.out[blockIdx.y]);
  const cx<T>* twr = reinterpret_cast<const cx<T>*>(a.twr);
  const cx<T>* twc = reinterpret_cast<const cx<T>*>(a.twc);

  // ---- columns k <= n2 of S plane i0: axis-1 inverse transforms, rows < n1 into the plane
  const int c = tid % TC, q = tid / TC;
  using FC = FirstStage<L1, PIDC, true, NQC>;
  constexpr int NTILE = (N + 1 + TC - 1) / TC;
  const cx<T>* const Sb = S + (long long)i0 * a.plane;
  const unsigned P = (unsigned)a.pitch;
  auto cidx = [c](int row) { return row * TC + c; };
  // the next tile's pencils are requested before the current tile is transformed
  auto load_tile = [&](int t, cx<T> (&raw)[FC::J][FC::R]) {
    const int k = t * TC + c;
    const bool kok = t < NTILE && k <= N;
#pragma unroll
    for (int j = 0; j < FC::J; ++j) {
      const int b = q + NQC * j;
      const bool ok = kok && ((FC::NB % NQC == 0) || b < FC::NB);
#pragma unroll
      for (int r = 0; r < FC::R; ++r) raw[j][r] = ok ? Sb[(b + r * FC::NB) * P + k] : czero<T>();
    }
  };
  cx<T> nxt[FC::J][FC::R];
  issue_fence();
  load_tile(0, nxt);
  issue_fence();
#pragma unroll 1
  for (int t = 0; t < NTILE; ++t) {
    const int k = t * TC + c;
    const bool kok = k <= N;
    const int ks = row_slot(kok ? k : N);
    cx<T> v[FC::J][FC::R];
#pragma unroll
    for (int j = 0; j < FC::J; ++j)
#pragma unroll
      for (int r = 0; r < FC::R; ++r) v[j][r] = nxt[j][r];
    issue_fence();
    load_tile(t + 1, nxt);
    issue_fence();
    if constexpr (KC == 1) {
#pragma unroll
      for (int j = 0; j < FC::J; ++j) {
        const int b = q + NQC * j;
        dft_half_out<FC::R, true, T>(v[j]);  // only rows < n1 are kept
        if (kok && ((FC::NB % NQC == 0) || b < FC::NB)) {
#pragma unroll
          for (int m = 0; m < FC::R / 2; ++m) pl[(b + m * FC::NB) * PP + ks] = v[j][m];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < FC::J; ++j) Dft<FC::R, true, T>::run(v[j]);
      if (t > 0) lds_barrier();  // the previous tile's last stage has read the scratch
      write_first_outputs<T, FC::R, FC::J, FC::NB, NQC>(cs, v, q, cidx);
      lds_barrier();
      lds_stages<T, L1, PIDC, true, 1, KC - 1, NQC, true>(cs, twc, q, cidx);
      using Lc = LastStage<L1, PIDC, true, NQC>;
      static_assert(Lc::R % 2 == 0, "inverse plans end with an even radix");
      cx<T> u[Lc::J][Lc::R];
      lds_last_stage<T, L1, PIDC, true, NQC, true, false, true>(cs, twc, q, cidx, u);
#pragma unroll
      for (int j = 0; j < Lc::J; ++j) {
        const int b = q + NQC * j;
        if (kok && ((Lc::NB % NQC == 0) || b < Lc::NB)) {
#pragma unroll
          for (int m = 0; m < Lc::R / 2; ++m) pl[(b + m * Lc::NB) * PP + ks] = u[j][m];
        }
      }
    }
  }
  lds_barrier();

  // ---- rows of the plane: inverse real transforms of length 2 n2, first n2 samples to phi
  const int qr = tid % NQR, cr = tid / NQR;
  const cx<T>* pp = twr + tw_size(LC, PIDR);
  using F = FirstStage<LC, PIDR, true, NQR>;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int i1 = g * TRR + cr;
    auto idx = [i1](int e) { return i1 * PP + row_slot(e); };
    cx<T> v[F::J][F::R];
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
      const int b = qr + NQR * j;
      if ((F::NB % NQR == 0) || b < F::NB) {
#pragma unroll
        for (int r = 0; r < F::R; ++r) {
          const int n = b + r * F::NB;
          const cx<T> X1 = pl[idx(n)];
          const cx<T> X2 = conjg(pl[idx(LC - n)]);
          const cx<T> A = cadd(X1, X2);
          const cx<T> B = cmulc(csub(X1, X2), pp[n]);
          v[j][r] = {A.x - B.y, A.y + B.x};
        }
        if constexpr (KR == 1)
          dft_half_out<F::R, true, T>(v[j]);  // only the first half of z is kept
        else
          Dft<F::R, true, T>::run(v[j]);
      }
    }
    cx<T>* out = phi + ((long long)i0 * N + i1) * (LC / 2);
    if constexpr (KR == 1) {
      static_assert(F::R % 2 == 0, "inverse plans end with an even radix");
#pragma unroll
      for (int j = 0; j < F::J; ++j) {
        const int b = qr + NQR * j;
        if ((F::NB % NQR == 0) || b < F::NB) {
#pragma unroll
          for (int m = 0; m < F::R / 2; ++m) put<T, PASS_ROW_INV>(&out[b + m * F::NB], v[j][m]);
        }
      }
    } else {
      lds_barrier();  // every thread of the row has read its pre-split inputs
      write_first_outputs<T, F::R, F::J, F::NB, NQR>(pl, v, qr, idx);
      lds_barrier();
      lds_stages<T, LC, PIDR, true, 1, KR - 1, NQR, true>(pl, twr, qr, idx);
      using Li = LastStage<LC, PIDR, true, NQR>;
      static_assert(Li::R % 2 == 0, "inverse plans end with an even radix");
      cx<T> u[Li::J][Li::R];
      lds_last_stage<T, LC, PIDR, true, NQR, true, false, true>(pl, twr, qr, idx, u);
#pragma unroll
      for (int j = 0; j < Li::J; ++j) {
        const int b = qr + NQR * j;
        if ((Li::NB % NQR == 0) || b < Li::NB) {
#pragma unroll
          for (int m = 0; m < Li::R / 2; ++m) put<T, PASS_ROW_INV>(&out[b + m * Li::NB], u[j][m]);
        }
      }
    }
  }
}

#define FSP_PLANE_SIZES(X) X(32) X(48) X(64) X(96) X(128)

// inv == false: passes 1-2 (rho -> S); inv == true: passes 4-5 (S -> phi), for
// n1 == n2 == N.  One block per plane i0 and item: grid (n0, items).
template <typename T>
hipError_t launch_plane(int N, int n0, bool inv, const PlaneArgs& a, int items, hipStream_t s) {
  bool found = false;
#define FSP_CASE(NV)                                                                                \
  if (N == NV) {                                                                                    \
    constexpr PlaneCfg c = plane_cfg<T>(NV);                                                        \
    if constexpr (c.tc > 0) {                                                                       \
      static_assert(plane_lds_bytes<T>(NV) <= 163840, "the plane and the column scratch fit in LDS"); \
      if (inv)                                                                                      \
        hipLaunchKernelGGL((k_plane_inv<T, NV, c.pidr, c.nqr, c.pidc, c.tc, c.nqc>), dim3(n0, items), \
                           dim3(c.tc * c.nqc), 0, s, a);                                            \
      else                                                                                          \
        hipLaunchKernelGGL((k_plane_fwd<T, NV, c.pidr, c.nqr, c.pidc, c.tc, c.nqc>), dim3(n0, items), \
                           dim3(c.tc * c.nqc), 0, s, a);                                            \
      found = true;                                                                                 \
    }                                                                                               \
  }
  FSP_PLANE_SIZES(FSP_CASE)
#undef FSP_CASE
  if (!found) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fsp
