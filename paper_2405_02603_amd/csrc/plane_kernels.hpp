// plane_kernels.hpp -- axis-2 and axis-1 passes fused per i0-plane (grids with n1 == n2).
//
// For grids whose i0-plane of the axis-2 spectrum, X[i1][k] for i1 < n1 and
// k <= n2, fits in LDS, P1 and P2 run as one kernel and P4 and P5 as another:
// one block per plane (and item) keeps the plane in LDS between the axis-2
// and the axis-1 transforms, so S is written once by the forward kernel and
// read once by the inverse kernel, and the axis-2 spectrum never goes to
// device memory.                                   [Section 2.2, steps 1, 2, 4, 5]
//
//   k_plane_fwd  rows of rho (i0, i1): real transform of length 2 n2 of the
//                zero-padded row, as in P1, into the plane; then each column k
//                of the plane: the axis-1 transform of length 2 n1 whose upper
//                half of inputs is the padding, as two transforms of length n1
//                in place in the column: its even outputs 2 m are DFT_n1(x)[m],
//                its odd outputs 2 m + 1 are DFT_n1(x_i w^i)[m] with
//                w = exp(-i pi / n1); all 2 n1 rows to S.
//   k_plane_inv  each column k of S plane i0: the inverse transform of length
//                2 n1, rows i < n1 kept, as two inverse transforms of length
//                n1 in place in the plane column, y_i = IDFT(X_even)_i +
//                conj(w^i) IDFT(X_odd)_i; then the rows: inverse real
//                transform of length 2 n2, first n2 samples kept, as in P5, to
//                phi.
//
// The block's LDS is the plane alone (rows at the row passes' padded pitch),
// so more blocks share a compute unit.  Rows and columns are transformed with
// the same length-n plan and twiddle table (n1 == n2), whose split table
// exp(-i pi k / n2) also gives the w^i above.  Row phase: NQR threads per row,
// NT / NQR rows at a time.  Column phase: TC adjacent columns (consecutive
// lanes, contiguous in S) with NQC threads per pencil, n2 / TC full column
// tiles and one tile for the column k = n2 alone; that tile's other lanes
// transform a column that holds no live data at that point (one already
// stored by the forward kernel, one yet to be filled by the inverse kernel)
// and store nothing.
#pragma once

#include "solve_kernels.hpp"

namespace fsp {

struct PlaneArgs {
  const ItemPtrs* items;   // table of this launch's items, or NULL (then in / out)
  const void* in[MAX_ITEMS];   // forward: rho; inverse: S (or a gradient output's spectrum)
  void* out[MAX_ITEMS];        // forward: S; inverse: phi (or a gradient component)
  const void* twr;   // twiddles of length n2 (plan PlaneCfg::pid) then exp(-i pi k / n2), k in [0, n2]
  long long plane;   // complex elements between S planes i0 (2 n1 P)
  int pitch;         // P
};

// Shape of the plane kernels for n1 == n2 == N: radix plan of length N (rows
// and columns), threads per row, column tile and threads per column pencil
// (TC * NQC threads a block, NT / NQR rows per row group), and the waves per
// SIMD the kernels are built for (the resident blocks' waves: registers are
// held to that).  tc == 0: not built.  Blocks with 64 KB or more of LDS use
// 4 or 8 waves: two such blocks of 6 waves did not share a compute unit on
// MI355X, two of 8 did.
struct PlaneCfg {
  int pid, nqr, tc, nqc, wpe;
};

template <typename T>
__host__ __device__ constexpr PlaneCfg plane_cfg(int N) {
  if constexpr (sizeof(T) == 4) {
    switch (N) {
      case 32: return {0, 4, 32, 4, 2};
      case 48: return {1, 4, 16, 12, 4};
      case 64: return {0, 4, 32, 8, 4};
      case 96: return {0, 16, 32, 16, 4};
      case 128: return {1, 4, 32, 16, 2};
      default: return {0, 0, 0, 0, 0};
    }
  } else {
    switch (N) {
      case 32: return {0, 4, 32, 4, 2};
      case 48: return {1, 4, 16, 12, 2};
      case 64: return {0, 4, 16, 8, 1};
      default: return {0, 0, 0, 0, 0};
    }
  }
}

template <typename T>
__host__ __device__ constexpr int plane_lds_bytes(int N) {
  return N * row_pitch(N) * 2 * (int)sizeof(T);
}

// One length-N transform of the pencils of a column tile, in place in the
// plane: first-stage outputs v (held by the caller) go to the column, the
// middle stages run there, the last stage's outputs are returned in w.  Four
// barriers at least; the caller has synchronised the column's previous use.
template <typename T, int N, int PID, bool INV, int NQC, class IDX, int J, int R, int JL, int RL>
__device__ __forceinline__ void plane_column_fft(cx<T>* pl, const cx<T>* tw, int q, IDX idx, const cx<T> (&v)[J][R],
                                                 cx<T> (&w)[JL][RL]) {
  constexpr int K = plan_len(N, PID);
  using Fs = FirstStage<N, PID, INV, NQC>;
  write_first_outputs<T, Fs::R, Fs::J, Fs::NB, NQC>(pl, v, q, idx);
  lds_barrier();
  lds_stages<T, N, PID, INV, 1, K - 1, NQC, INV>(pl, tw, q, idx);
  lds_last_stage<T, N, PID, INV, NQC, INV>(pl, tw, q, idx, w);
}

template <typename T, int N, int PID, int NQR, int TC, int NQC, int WPE>
__global__ __launch_bounds__(TC* NQC, WPE) void k_plane_fwd(PlaneArgs a) {
  constexpr int LC = N, NT = TC * NQC, TRR = NT / NQR, G = N / TRR;
  static_assert(NT % NQR == 0 && N % TRR == 0 && N % TC == 0, "row groups and column tiles tile the plane");
  constexpr int PP = row_pitch(LC);
  constexpr int K = plan_len(LC, PID);
  static_assert(K > 1, "the column transforms exchange through the plane");
  __shared__ cx<T> pl[N * PP];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x;
  const cx<T>* rho = reinterpret_cast<const cx<T>*>(a.items ? a.items[blockIdx.y].rho : a.in[blockIdx.y]);
  cx<T>* S = reinterpret_cast<cx<T>*>(a.items ? a.items[blockIdx.y].work : a.out[blockIdx.y]);
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.twr);
  const cx<T>* pp = tw + tw_size(LC, PID);  // exp(-i pi k / n2)

  // ---- rows: every row group's input is requested before the first transform
  const int qr = tid % NQR, cr = tid / NQR;
  using F = FirstStage<LC, PID, false, NQR>;
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
    lds_stages<T, LC, PID, false, 1, K - 1, NQR, false>(pl, tw, qr, idx);
    using Ls = LastStage<LC, PID, false, NQR>;
    cx<T> w[Ls::J][Ls::R];
    lds_last_stage<T, LC, PID, false, NQR, false>(pl, tw, qr, idx, w);
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
        auto split = [](cx<T> A, cx<T> Bc, cx<T> t) {
          const cx<T> B = conjg(Bc);
          const cx<T> E = {T(0.5) * (A.x + B.x), T(0.5) * (A.y + B.y)};
          const cx<T> D = {T(0.5) * (A.x - B.x), T(0.5) * (A.y - B.y)};
          const cx<T> U = cmul(t, D);
          return cx<T>{E.x + U.y, E.y - U.x};
        };
        const cx<T> Xa = split(Za, Zb, pp[k]);       // X[k]
        const cx<T> Xb = split(Zb, Za, pp[LC - k]);  // X[n2 - k]
        pl[idx(k)] = Xa;
        if (k != LC / 2) pl[idx(LC - k)] = Xb;
      }
    }
  }
  lds_barrier();

  // ---- columns k <= n2: even and odd outputs of the axis-1 forward transform
  const int c = tid % TC, q = tid / TC;
  using FC = FirstStage<N, PID, false, NQC>;
  using LC_ = LastStage<N, PID, false, NQC>;
  constexpr int NTILE = N / TC + 1;  // the last tile holds the column n2 alone
  cx<T>* const Sb = S + (long long)i0 * a.plane;
  const unsigned P = (unsigned)a.pitch;
#pragma unroll 1
  for (int t = 0; t < NTILE; ++t) {
    const int k = t * TC + c;
    const bool kok = k <= N;
    const int ks = row_slot(kok ? k : c);  // past n2: a column of the first tile, already stored
    auto cidx = [ks](int row) { return row * PP + ks; };
    cx<T> ve[FC::J][FC::R], vo[FC::J][FC::R];
#pragma unroll
    for (int j = 0; j < FC::J; ++j) {
      const int b = q + NQC * j;
      if ((FC::NB % NQC == 0) || b < FC::NB) {
#pragma unroll
        for (int r = 0; r < FC::R; ++r) {
          const int i1 = b + r * FC::NB;
          ve[j][r] = pl[cidx(i1)];
          vo[j][r] = cmul(ve[j][r], pp[i1]);
        }
        Dft<FC::R, false, T>::run(ve[j]);
        Dft<FC::R, false, T>::run(vo[j]);
      }
    }
    lds_barrier();  // the column's inputs are in registers before the transforms overwrite it
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half == 1) lds_barrier();  // the even transform's last stage has read the column
      cx<T> w[LC_::J][LC_::R];
      plane_column_fft<T, N, PID, false, NQC>(pl, tw, q, cidx, half == 0 ? ve : vo, w);
#pragma unroll
      for (int j = 0; j < LC_::J; ++j) {
        const int b = q + NQC * j;
        if (kok && ((LC_::NB % NQC == 0) || b < LC_::NB)) {
#pragma unroll
          for (int m = 0; m < LC_::R; ++m)
            put<T, PASS_COL_FWD>(&Sb[(2 * (b + m * LC_::NB) + half) * P + k], w[j][m]);
        }
      }
    }
    lds_barrier();  // the next tile's lanes past n2 reuse columns of the first tile
  }
}

template <typename T, int N, int PID, int NQR, int TC, int NQC, int WPE>
__global__ __launch_bounds__(TC* NQC, WPE) void k_plane_inv(PlaneArgs a) {
  constexpr int LC = N, NT = TC * NQC, TRR = NT / NQR, G = N / TRR;
  static_assert(NT % NQR == 0 && N % TRR == 0 && N % TC == 0, "row groups and column tiles tile the plane");
  constexpr int PP = row_pitch(LC);
  constexpr int K = plan_len(LC, PID);
  static_assert(K > 1, "the column transforms exchange through the plane");
  __shared__ cx<T> pl[N * PP];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x;
  const cx<T>* S = reinterpret_cast<const cx<T>*>(a.items ? a.items[blockIdx.y].work : a.in[blockIdx.y]);
  cx<T>* phi = reinterpret_cast<cx<T>*>(a.items ? a.items[blockIdx.y].phi : a.out[blockIdx.y]);
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.twr);
  const cx<T>* pp = tw + tw_size(LC, PID);  // exp(-i pi k / n2)

  // ---- columns k <= n2 of S plane i0: rows i < n1 of the axis-1 inverse transform
  const int c = tid % TC, q = tid / TC;
  using FC = FirstStage<N, PID, true, NQC>;
  using LC_ = LastStage<N, PID, true, NQC>;
  constexpr int NTILE = N / TC + 1;  // the column n2 alone comes first
  const cx<T>* const Sb = S + (long long)i0 * a.plane;
  const unsigned P = (unsigned)a.pitch;
  // tile t: the column n2 for t == 0, else columns (t - 1) TC + c
  auto col_of = [c](int t) { return t == 0 ? N + c : (t - 1) * TC + c; };
  // even rows 2 m and odd rows 2 m + 1 of the next tile are requested before
  // the current tile is transformed
  auto load_tile = [&](int t, cx<T> (&e)[FC::J][FC::R], cx<T> (&o)[FC::J][FC::R]) {
    const int k = col_of(t);
    const bool kok = t < NTILE && k <= N;
#pragma unroll
    for (int j = 0; j < FC::J; ++j) {
      const int b = q + NQC * j;
      const bool ok = kok && ((FC::NB % NQC == 0) || b < FC::NB);
#pragma unroll
      for (int r = 0; r < FC::R; ++r) {
        const unsigned row = 2 * (b + r * FC::NB);
        e[j][r] = ok ? Sb[row * P + k] : czero<T>();
        o[j][r] = ok ? Sb[(row + 1) * P + k] : czero<T>();
      }
    }
  };
  cx<T> ne[FC::J][FC::R], no[FC::J][FC::R];
  issue_fence();
  load_tile(0, ne, no);
  issue_fence();
#pragma unroll 1
  for (int t = 0; t < NTILE; ++t) {
    const int k = col_of(t);
    // past n2 (tile 0 only): a column of the first full tile, filled later
    const int ks = row_slot(k <= N ? k : c);
    auto cidx = [ks](int row) { return row * PP + ks; };
    cx<T> ve[FC::J][FC::R], vo[FC::J][FC::R];
#pragma unroll
    for (int j = 0; j < FC::J; ++j)
#pragma unroll
      for (int r = 0; r < FC::R; ++r) ve[j][r] = ne[j][r], vo[j][r] = no[j][r];
    issue_fence();
    load_tile(t + 1, ne, no);
    issue_fence();
#pragma unroll
    for (int j = 0; j < FC::J; ++j) {
      Dft<FC::R, true, T>::run(ve[j]);
      Dft<FC::R, true, T>::run(vo[j]);
    }
    cx<T> ye[LC_::J][LC_::R], yo[LC_::J][LC_::R];
    plane_column_fft<T, N, PID, true, NQC>(pl, tw, q, cidx, ve, ye);
    lds_barrier();  // the even transform's last stage has read the column
    plane_column_fft<T, N, PID, true, NQC>(pl, tw, q, cidx, vo, yo);
    lds_barrier();  // the odd transform's last stage has read the column
#pragma unroll
    for (int j = 0; j < LC_::J; ++j) {
      const int b = q + NQC * j;
      if ((LC_::NB % NQC == 0) || b < LC_::NB) {
#pragma unroll
        for (int m = 0; m < LC_::R; ++m) {
          const int i = b + m * LC_::NB;
          pl[cidx(i)] = cadd(ye[j][m], cmulc(yo[j][m], pp[i]));
        }
      }
    }
    lds_barrier();  // after tile 0, the next tile's columns may hold that tile's stray results
  }

  // ---- rows of the plane: inverse real transforms of length 2 n2, first n2 samples to phi
  const int qr = tid % NQR, cr = tid / NQR;
  using F = FirstStage<LC, PID, true, NQR>;
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
        Dft<F::R, true, T>::run(v[j]);
      }
    }
    cx<T>* out = phi + ((long long)i0 * N + i1) * (LC / 2);
    lds_barrier();  // every thread of the row has read its pre-split inputs
    write_first_outputs<T, F::R, F::J, F::NB, NQR>(pl, v, qr, idx);
    lds_barrier();
    lds_stages<T, LC, PID, true, 1, K - 1, NQR, true>(pl, tw, qr, idx);
    using Li = LastStage<LC, PID, true, NQR>;
    static_assert(Li::R % 2 == 0, "inverse plans end with an even radix");
    cx<T> u[Li::J][Li::R];
    lds_last_stage<T, LC, PID, true, NQR, true, false, true>(pl, tw, qr, idx, u);
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
      static_assert(plane_lds_bytes<T>(NV) <= 163840, "the plane fits in LDS"); \
      if (inv)                                                                                      \
        hipLaunchKernelGGL((k_plane_inv<T, NV, c.pid, c.nqr, c.tc, c.nqc, c.wpe>), dim3(n0, items),         \
                           dim3(c.tc * c.nqc), 0, s, a);                                            \
      else                                                                                          \
        hipLaunchKernelGGL((k_plane_fwd<T, NV, c.pid, c.nqr, c.tc, c.nqc, c.wpe>), dim3(n0, items),         \
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
