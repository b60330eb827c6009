// solve_launch.hpp -- tile shapes per pencil length and the host-side launchers
// of the five solve passes.  Included by one translation unit per precision.
#pragma once

#include "solve_kernels.hpp"

namespace fsp {

struct TileCfg {
  int tiles;  // TC (column passes: columns per block) or TR (row passes: rows per block)
  int nq;     // threads per pencil
};

// Column passes (pencil length L = 2 n, strided rows).  LDS = L * TC * sizeof(cx<T>).
template <typename T>
__host__ __device__ constexpr TileCfg col_cfg(int L) {
  constexpr bool d = sizeof(T) == 8;
  switch (L) {
    case 16: return {d ? 32 : 64, 1};
    case 24: return {d ? 32 : 64, 1};
    case 32: return {32, 4};
    case 48: return {d ? 32 : 64, 1};
    case 64: return {d ? 16 : 32, 8};
    case 96: return {d ? 16 : 32, 4};
    case 128: return {d ? 16 : 32, 8};
    case 192: return {d ? 8 : 16, 8};
    case 256: return {d ? 8 : 16, 16};
    case 384: return {d ? 8 : 16, 8};
    case 512: return {d ? 8 : 16, 16};
    case 768: return {d ? 4 : 8, 16};
    case 1024: return {d ? 4 : 8, 32};
    default: return {0, 0};
  }
}

// Row passes (pencil length LC = n2 complex, contiguous rows).  LDS = TR row_pitch(LC) sizeof(cx<T>).
template <typename T>
__host__ __device__ constexpr TileCfg row_cfg(int LC) {
  constexpr bool d = sizeof(T) == 8;
  switch (LC) {
    case 8: return {64, 1};
    case 12: return {64, 1};
    case 16: return {64, 1};
    case 24: return {64, 1};
    case 32: return {32, 4};
    case 48: return {d ? 32 : 64, 1};
    case 64: return {32, 8};
    case 96: return {32, 4};
    case 128: return {d ? 8 : 16, 8};
    case 192: return {d ? 8 : 16, 8};
    case 256: return {d ? 8 : 16, 16};
    case 384: return {d ? 4 : 8, 8};
    case 512: return {d ? 4 : 8, 16};
    default: return {0, 0};
  }
}

#define FSP_ROW_LENGTHS(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#define FSP_COL_LENGTHS(X) \
  X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

template <typename T>
hipError_t launch_p1(int LC, const RowArgs& a, int items, hipStream_t s) {
  switch (LC) {
#define FSP_CASE(LV)                                                                        \
  case LV: {                                                                                \
    constexpr TileCfg c = row_cfg<T>(LV);                                                   \
    const int blocks = (a.nrows + c.tiles - 1) / c.tiles;                                   \
    hipLaunchKernelGGL((k_row_r2c<T, LV, c.tiles, c.nq>), dim3(blocks, items), dim3(c.tiles * c.nq), 0, s, a); \
    break;                                                                                  \
  }
    FSP_ROW_LENGTHS(FSP_CASE)
#undef FSP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_p5(int LC, const RowArgs& a, int items, hipStream_t s) {
  switch (LC) {
#define FSP_CASE(LV)                                                                        \
  case LV: {                                                                                \
    constexpr TileCfg c = row_cfg<T>(LV);                                                   \
    const int blocks = (a.nrows + c.tiles - 1) / c.tiles;                                   \
    hipLaunchKernelGGL((k_row_c2r<T, LV, c.tiles, c.nq>), dim3(blocks, items), dim3(c.tiles * c.nq), 0, s, a); \
    break;                                                                                  \
  }
    FSP_ROW_LENGTHS(FSP_CASE)
#undef FSP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
int col_tiles(int L) {
  switch (L) {
#define FSP_CASE(LV) \
  case LV: return col_cfg<T>(LV).tiles;
    FSP_COL_LENGTHS(FSP_CASE)
#undef FSP_CASE
    default: return 0;
  }
}

// nouter: outer pencils groups (P2/P4: n0; P3: n1 + 1 pairs)
template <typename T>
hipError_t launch_col(int L, bool inverse, bool conv, const ColArgs& a, int items, hipStream_t s) {
  switch (L) {
#define FSP_CASE(LV)                                                                              \
  case LV: {                                                                                      \
    constexpr TileCfg c = col_cfg<T>(LV);                                                         \
    const dim3 grid((unsigned)(a.nouter * a.ntiles), (unsigned)items);                            \
    const dim3 block(c.tiles * c.nq);                                                             \
    if (conv)                                                                                     \
      hipLaunchKernelGGL((k_col_conv<T, LV, c.tiles, c.nq>), grid, block, 0, s, a);               \
    else if (inverse)                                                                             \
      hipLaunchKernelGGL((k_col_fft<T, LV, c.tiles, c.nq, true>), grid, block, 0, s, a);          \
    else                                                                                          \
      hipLaunchKernelGGL((k_col_fft<T, LV, c.tiles, c.nq, false>), grid, block, 0, s, a);         \
    break;                                                                                        \
  }
    FSP_COL_LENGTHS(FSP_CASE)
#undef FSP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Geometry of up to MAX_ITEMS solves of one shape, filled by the plans.
struct SolveGeom {
  int items;                 // solves in this group (1 .. MAX_ITEMS)
  int n0, n1, n2;
  int pitch;                 // P
  long long plane;           // complex elements between S planes i0 (>= 2 n1 P)
  int chunks;                // column chunks for passes 1-3 (1: whole passes)
  const void* tw_row;        // twiddles, length n2 (+ split table)
  const void* tw_c1;         // twiddles, length 2 n1
  const void* tw_c0;         // twiddles, length 2 n0
  const void* ghat[MAX_ITEMS];  // octant of each item, blocked [n1+1][tiles][n0+1][TC of P3]
  void* work[MAX_ITEMS];        // S of each item
  const void* rho[MAX_ITEMS];
  void* phi[MAX_ITEMS];
};

// Passes first..last of one solve (0 = P1 ... 4 = P5).
template <typename T>
hipError_t launch_solve(const SolveGeom& g, int first, int last, hipStream_t s) {
  const long long P = g.pitch;
  const long long plane = g.plane;  // complex elements per S plane i0
  RowArgs ra{};
  ra.nrows = g.n0 * g.n1;
  ra.n1 = g.n1;
  ra.pitch = g.pitch;
  ra.s_i0_stride = plane;
  ra.tw = g.tw_row;
  // P2 / P4: pencils along axis 1; outer = i0
  ColArgs ca{};
  for (int i = 0; i < g.items; ++i) ca.data[i] = g.work[i];
  ca.ncols = g.n2 + 1;
  ca.row_stride = P;
  ca.outer_stride = plane;
  ca.nouter = g.n0;
  ca.tw = g.tw_c1;
  // P3: pencils along axis 0; outer = k1 pairs
  ColArgs cc{};
  for (int i = 0; i < g.items; ++i) {
    cc.data[i] = g.work[i];
    cc.ghat[i] = g.ghat[i];
  }
  cc.ncols = g.n2 + 1;
  cc.row_stride = plane;
  cc.outer_stride = P;
  cc.nouter = g.n1 + 1;
  cc.tw = g.tw_c0;
  cc.n1 = g.n1;
  {
    const long long t0 = col_tiles<T>(2 * g.n0);
    cc.g_k1_stride = (g.n2 + 1 + t0 - 1) / t0 * (g.n0 + 1) * t0;
  }
  const int tc1 = col_tiles<T>(2 * g.n1), tc0 = col_tiles<T>(2 * g.n0);
  const int ncols = g.n2 + 1;
  auto set_cols = [&](ColArgs& c, int tcw, int c0, int c1) {
    c.col0 = c0;
    c.ncols = c1;
    c.ntiles = (c1 - c0 + tcw - 1) / tcw;
  };
  auto run = [&](int pass, int c0, int c1) -> hipError_t {
    switch (pass) {
      case 0:
        for (int i = 0; i < g.items; ++i) {
          ra.in[i] = g.rho[i];
          ra.out[i] = g.work[i];
        }
        return launch_p1<T>(g.n2, ra, g.items, s);
      case 1: set_cols(ca, tc1, c0, c1); return launch_col<T>(2 * g.n1, false, false, ca, g.items, s);
      case 2: set_cols(cc, tc0, c0, c1); return launch_col<T>(2 * g.n0, false, true, cc, g.items, s);
      case 3: set_cols(ca, tc1, c0, c1); return launch_col<T>(2 * g.n1, true, false, ca, g.items, s);
      case 4:
        for (int i = 0; i < g.items; ++i) {
          ra.in[i] = g.work[i];
          ra.out[i] = g.phi[i];
        }
        return launch_p5<T>(g.n2, ra, g.items, s);
      default: return hipErrorInvalidValue;
    }
  };
  hipError_t e = hipSuccess;
  if (g.chunks > 1 && first <= 1 && last >= 3) {
    // passes 1-3 column chunk by column chunk: a chunk's spectrum stays in the
    // memory-side cache between the three passes
    if (first == 0) e = run(0, 0, ncols);
    const int step = tc1 > tc0 ? tc1 : tc0;
    const int width = ((ncols + g.chunks - 1) / g.chunks + step - 1) / step * step;
    for (int c0 = 0; c0 < ncols && e == hipSuccess; c0 += width) {
      const int c1 = c0 + width < ncols ? c0 + width : ncols;
      for (int pass = 1; pass <= 3 && e == hipSuccess; ++pass) e = run(pass, c0, c1);
    }
    if (e == hipSuccess && last == 4) e = run(4, 0, ncols);
    return e;
  }
  for (int pass = first; pass <= last && e == hipSuccess; ++pass) e = run(pass, 0, ncols);
  return e;
}

}  // namespace fsp
