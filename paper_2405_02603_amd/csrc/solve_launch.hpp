// solve_launch.hpp -- tile shapes per pencil length and the host-side launchers
// of the five solve passes.  Included by one translation unit per precision.
#pragma once

#include "solve_kernels.hpp"
#include "plane_kernels.hpp"

namespace fsp {

struct TileCfg {
  int pid;    // radix plan (fft_core.hpp)
  int tiles;  // TC (column passes: columns per block) or TR (row passes: rows per block)
  int nq;     // threads per pencil
  int groups = 1;  // row passes: groups of `tiles` rows per block, transformed in turn
};

// Schedule variants per pencil length; variant 0 is the default and the
// autotuner may pick another.  Column passes of one length share TC (the
// Green's octant is stored in tiles of the axis-0 pass's TC).
constexpr int NUM_VARIANTS = 3;

template <typename T>
__host__ __device__ constexpr int col_tc(int L) {
  constexpr bool d = sizeof(T) == 8;
  switch (L) {
    case 16: case 24: case 48: return d ? 32 : 64;
    case 32: return 32;
    case 64: case 96: case 128: return d ? 16 : 32;
    case 192: case 256: case 384: case 512: return d ? 8 : 16;
    case 768: case 1024: return d ? 8 : 16;  // 128-byte row segments, as for 192-512
    default: return 0;
  }
}

// Column passes (pencil length L = 2 n, strided rows).  LDS = L * TC * sizeof(cx<T>).
template <typename T>
__host__ __device__ constexpr TileCfg col_cfg(int L, int v) {
  const int tc = col_tc<T>(L);
  // wider tiles (longer row segments, more LDS) for variant 2 of lengths 256-512;
  // the axis-0 pass never uses this shape (its variant 2 is the LDS-table or
  // the pipelined kernel)
  const int tw = 2 * tc;
  switch (L) {
    case 16: return v == 0 ? TileCfg{0, tc, 1} : v == 1 ? TileCfg{1, tc, 4} : TileCfg{1, tc, 2};
    case 24: return v == 0 ? TileCfg{0, tc, 1} : v == 1 ? TileCfg{1, tc, 2} : TileCfg{0, tc, 3};
    case 32: return v == 0 ? TileCfg{0, tc, 4} : v == 1 ? TileCfg{1, tc, 2} : TileCfg{0, tc, 8};
    case 48: return v == 0 ? TileCfg{0, tc, 1} : v == 1 ? TileCfg{1, tc, 4} : TileCfg{0, tc, 3};
    case 64: return v == 0 ? TileCfg{0, tc, 8} : v == 1 ? TileCfg{1, tc, 4} : TileCfg{0, tc, 4};
    case 96: return v == 0 ? TileCfg{0, tc, 4} : v == 1 ? TileCfg{1, tc, 4} : TileCfg{0, tc, 8};
    case 128: return v == 0 ? TileCfg{0, tc, 8} : v == 1 ? TileCfg{1, tc, 8} : TileCfg{0, tc, 16};
    case 192: return v == 0 ? TileCfg{0, tc, 8} : v == 1 ? TileCfg{1, tc, 8} : TileCfg{0, tc, 16};
    case 256: return v == 0 ? TileCfg{0, tc, 16} : v == 1 ? TileCfg{1, tc, 32} : TileCfg{0, tw, 16};
    case 384: return v == 0 ? TileCfg{0, tc, 8} : v == 1 ? TileCfg{1, tc, 16} : TileCfg{0, tw, 8};
    case 512: return v == 0 ? TileCfg{0, tc, 16} : v == 1 ? TileCfg{1, tc, 32} : TileCfg{0, tw, 16};
    // one block per compute unit at these lengths (L * TC complex of LDS): variant 2
    // adds threads per pencil instead of columns
    case 768: return v == 0 ? TileCfg{0, tc, 16} : v == 1 ? TileCfg{1, tc, 16} : TileCfg{0, tc, 32};
    case 1024: return v == 0 ? TileCfg{0, tc, 32} : v == 1 ? TileCfg{1, tc, 32} : TileCfg{1, tc, 64};
    default: return {0, 0, 0};
  }
}

// Row passes (pencil length LC = n2 complex, contiguous rows).  LDS = TR row_pitch(LC) sizeof(cx<T>).
template <typename T>
__host__ __device__ constexpr TileCfg row_cfg(int LC, int v) {
  constexpr bool d = sizeof(T) == 8;
  switch (LC) {
    case 8: return v == 0 ? TileCfg{0, 64, 1} : v == 1 ? TileCfg{0, 32, 1} : TileCfg{0, 16, 1};
    case 12: return v == 0 ? TileCfg{0, 64, 1} : v == 1 ? TileCfg{0, 32, 1} : TileCfg{0, 64, 3};
    case 16: return v == 0 ? TileCfg{0, 64, 1} : v == 1 ? TileCfg{1, 32, 4} : TileCfg{1, 64, 2};
    case 24: return v == 0 ? TileCfg{0, 64, 1} : v == 1 ? TileCfg{1, 32, 2} : TileCfg{0, 32, 3};
    case 32: return v == 0 ? TileCfg{0, 32, 4} : v == 1 ? TileCfg{1, 32, 2} : TileCfg{0, 16, 8};
    case 48: return v == 0 ? TileCfg{0, d ? 32 : 64, 1} : v == 1 ? TileCfg{1, 32, 4} : TileCfg{0, 32, 3};
    case 64: return v == 0 ? TileCfg{0, 32, 8} : v == 1 ? TileCfg{1, 32, 4} : TileCfg{0, 16, 8};
    // 96 and 128: a variant with 16 threads a row, 128-byte row segments per wave
    case 96: return v == 0 ? TileCfg{0, 32, 4} : v == 1 ? TileCfg{0, 8, 16} : TileCfg{0, 16, 8};
    case 128: return v == 0 ? TileCfg{0, d ? 8 : 16, 8} : v == 1 ? TileCfg{1, 16, 8} : TileCfg{1, 8, 16};
    case 192: return v == 0 ? TileCfg{0, d ? 8 : 16, 8} : v == 1 ? TileCfg{1, 16, 8} : TileCfg{0, 8, 16};
    // 256 in float32: small blocks of 4 rows, 2-4 groups each (more bytes in flight a thread)
    case 256:
      return d ? (v == 0 ? TileCfg{0, 8, 16} : v == 1 ? TileCfg{1, 8, 32} : TileCfg{1, 4, 32, 2})
               : (v == 0 ? TileCfg{0, 4, 16, 4} : v == 1 ? TileCfg{1, 4, 32, 2} : TileCfg{0, 4, 16, 2});
    case 384: return v == 0 ? TileCfg{0, d ? 4 : 8, 8} : v == 1 ? TileCfg{1, 8, 8} : TileCfg{0, 4, 16};
    // 512: the three-stage plan; 64 threads per row over 4 rows keeps 8 waves per SIMD
    case 512: return v == 0 ? TileCfg{1, 4, 64} : v == 1 ? TileCfg{1, 8, 32} : TileCfg{1, 16, 32};
    default: return {0, 0, 0};
  }
}

// Axis-0 pass variants: variant 0 as col_cfg, variant 1 as col_cfg or the
// split-exchange form (conv_split_wpe, below); variant 2 keeps the
// complete twiddle table in LDS, with the shape of variant 0 (else 1) when the
// table costs no resident block (conv_twf_fits) or saves registers
// (conv_twf_wide), and with the split exchanges too where variant 1 has them;
// else it is the pipelined persistent kernel (grid of at most
// CONV_PIPE_BLOCKS blocks) with the shape of variant 1.
constexpr int CONV_PIPE_BLOCKS = 1024;
constexpr int CONV_GATHER_MIN_BLOCKS = 2048;
constexpr int CONV_LDS_PER_CU = 163840;

// The table may not cost a resident block: as many blocks of the variant fit
// in a compute unit's LDS with it as without it.
template <typename T>
__host__ __device__ constexpr bool conv_twf_fits(int L, int v) {
  const TileCfg c = col_cfg<T>(L, v);
  const int base = L * c.tiles * 2 * (int)sizeof(T);
  const int with = base + twf_size(L, c.pid) * 2 * (int)sizeof(T);
  return plan_len(L, c.pid) > 1 && with <= CONV_LDS_PER_CU && CONV_LDS_PER_CU / with == CONV_LDS_PER_CU / base;
}

// 256-point pencils take the table although it costs a resident block by LDS
// (5 -> 4 blocks): in float32 the kernel then needs 111 VGPRs instead of 140,
// so 4 waves per SIMD reside instead of 3; in float64 registers hold 2 waves
// per SIMD either way, and the table's fewer instructions pay.
template <typename T>
__host__ __device__ constexpr bool conv_twf_wide(int L) {
  return L == 256;
}

template <typename T>
__host__ __device__ constexpr bool conv_twf(int L, int v) {
  return v == 2 && (conv_twf_fits<T>(L, 0) || conv_twf_fits<T>(L, 1) || conv_twf_wide<T>(L));
}

template <typename T>
__host__ __device__ constexpr bool conv_pipelined(int L, int v) {
  return v == 2 && !conv_twf<T>(L, v) && L >= 128 && plan_len(L, col_cfg<T>(L, 1).pid) > 1;
}

// Axis-0 pass variant 1 where conv_split_wpe(L) > 0: the shape of variant 0
// (a two-stage plan) with the exchange between its stages made through a real
// LDS array in two rounds, real parts then imaginary parts (half the LDS of a
// block), and the kernel built for that many waves per SIMD, so that more
// blocks share a compute unit.  Elsewhere variant 1 is col_cfg's.
template <typename T>
__host__ __device__ constexpr int conv_split_wpe(int L) {
  return sizeof(T) == 4 && L == 512 ? 3 : 0;
}

template <typename T>
__host__ __device__ constexpr TileCfg conv_cfg(int L, int v) {
  return conv_twf<T>(L, v) ? col_cfg<T>(L, conv_twf_fits<T>(L, 0) || conv_twf_wide<T>(L) ? 0 : 1)
         : conv_pipelined<T>(L, v)                ? col_cfg<T>(L, 1)
         : v == 1 && conv_split_wpe<T>(L) > 0     ? col_cfg<T>(L, 0)
                                                  : col_cfg<T>(L, v);
}

#define FSP_ROW_LENGTHS(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#define FSP_COL_LENGTHS(X) \
  X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define FSP_VARIANTS(X, LV) X(LV, 0) X(LV, 1) X(LV, 2)

template <typename T>
hipError_t launch_p1(int LC, int v, const RowArgs& a, int items, hipStream_t s) {
  bool found = false;
#define FSP_CASE_V(LV, VV)                                                                          \
  if (LC == LV && v == VV) {                                                                        \
    constexpr TileCfg c = row_cfg<T>(LV, VV);                                                       \
    const int blocks = (a.nrows + c.tiles * c.groups - 1) / (c.tiles * c.groups);                   \
    hipLaunchKernelGGL((k_row_r2c<T, LV, c.pid, c.tiles, c.nq, c.groups>), dim3(blocks, items),      \
                       dim3(c.tiles * c.nq), 0, s, a);                                              \
    found = true;                                                                                   \
  }
#define FSP_CASE(LV) FSP_VARIANTS(FSP_CASE_V, LV)
  FSP_ROW_LENGTHS(FSP_CASE)
#undef FSP_CASE
#undef FSP_CASE_V
  if (!found) return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_p5(int LC, int v, const RowArgs& a, int items, hipStream_t s) {
  bool found = false;
#define FSP_CASE_V(LV, VV)                                                                          \
  if (LC == LV && v == VV) {                                                                        \
    constexpr TileCfg c = row_cfg<T>(LV, VV);                                                       \
    const int blocks = (a.nrows + c.tiles * c.groups - 1) / (c.tiles * c.groups);                   \
    hipLaunchKernelGGL((k_row_c2r<T, LV, c.pid, c.tiles, c.nq, c.groups>), dim3(blocks, items),      \
                       dim3(c.tiles * c.nq), 0, s, a);                                              \
    found = true;                                                                                   \
  }
#define FSP_CASE(LV) FSP_VARIANTS(FSP_CASE_V, LV)
  FSP_ROW_LENGTHS(FSP_CASE)
#undef FSP_CASE
#undef FSP_CASE_V
  if (!found) return hipErrorInvalidValue;
  return hipGetLastError();
}

// Axis-0 pass of the gradient solve.  Variants 0 and 1: one launch writes
// every output from one forward transform, the spectrum held in registers
// through the outputs; for pencils of 256 and more variant 0 spreads a pencil
// over more threads, with plan 1: up to 1024 threads a block through 512
// (radix-8 stages), 512 threads beyond (a 1024-thread block is held to 128
// registers a thread); variant 1 is the column pass's variant 1.  Variant 2:
// one launch per output in the column pass's variant-0 shape (each reads the
// spectrum again, with fewer registers).  The tile stays col_tc (the layout
// of the tables).
template <typename T>
__host__ __device__ constexpr TileCfg grad_cfg(int L, int v) {
  const int tc = col_tc<T>(L);
  // (384: plan 0, whose first stages have 24 and 48 butterflies; plan 1's
  // radix-24 stage has only 16)
  if (v == 0 && L >= 256 && L <= 512) return {L == 384 ? 0 : 1, tc, 1024 / tc < L / 8 ? 1024 / tc : L / 8};
  if (v == 0 && L > 512) return {1, tc, 512 / tc};
  return col_cfg<T>(L, v == 2 ? 0 : v);
}

template <typename T>
int col_tiles(int L) {
  return col_tc<T>(L);
}

// Axis-0 launch geometry: when the last column is alone in its tile it is
// gathered over TC pairs k1 per block (ntail leading blocks) instead of
// filling one mostly empty tile per pair.  The gathered blocks read scattered
// rows and run longer than the others, so this pays only on grids of at least
// a.gather_min full-tile blocks.
inline ColArgs conv_gather(const ColArgs& a, int tc) {
  ColArgs b = a;
  const int span = a.ncols - a.col0;
  if (tc > 1 && span % tc == 1 && (long long)a.nouter * (span / tc) >= a.gather_min) {
    b.ntiles = span / tc;
    b.ntail = (a.nouter + tc - 1) / tc;
  } else {
    b.ntiles = (span + tc - 1) / tc;
    b.ntail = 0;
  }
  return b;
}

// kind: 0 forward (P2), 1 inverse (P4), 2 forward-multiply-inverse (P3)
template <typename T>
hipError_t launch_col(int L, int v, int kind, const ColArgs& a, int items, hipStream_t s) {
  bool found = false;
#define FSP_CASE_V(LV, VV)                                                                          \
  if (L == LV && v == VV) {                                                                         \
    constexpr TileCfg c = col_cfg<T>(LV, VV);                                                       \
    constexpr TileCfg cc = conv_cfg<T>(LV, VV);                                                     \
    static_assert(cc.tiles == col_tc<T>(LV), "the Green octant is blocked by col_tc columns");     \
    const dim3 grid((unsigned)(a.nouter * a.ntiles), (unsigned)items);                              \
    const dim3 block(c.tiles * c.nq);                                                               \
    if (kind == 2) {                                                                                \
      if (a.nout > 0) {                                                                             \
        /* the gradient solve: variants 0 and 1 all outputs, variant 2 exactly one */              \
        constexpr TileCfg gc = grad_cfg<T>(LV, VV);                                                 \
        if (items != 1 || a.nout > MAX_OUT || (VV == 2 && a.nout != 1)) return hipErrorInvalidValue; \
        const ColArgs b = conv_gather(a, gc.tiles);                                                 \
        const dim3 gridg((unsigned)(b.nouter * b.ntiles + b.ntail), 1u);                            \
        if constexpr (VV < 2)                                                                       \
          hipLaunchKernelGGL((k_col_conv<T, LV, gc.pid, gc.tiles, gc.nq, false, MAX_OUT>), gridg,   \
                             dim3(gc.tiles * gc.nq), 0, s, b);                                      \
        else                                                                                        \
          hipLaunchKernelGGL((k_col_conv<T, LV, gc.pid, gc.tiles, gc.nq, false, 1>), gridg,         \
                             dim3(gc.tiles * gc.nq), 0, s, b);                                      \
      } else if constexpr (conv_pipelined<T>(LV, VV)) {                                             \
        ColArgs b = a;                                                                              \
        b.ntail = 0;                                                                                \
        const int nb = b.nouter * b.ntiles < CONV_PIPE_BLOCKS ? b.nouter * b.ntiles : CONV_PIPE_BLOCKS; \
        hipLaunchKernelGGL((k_col_conv_pipe<T, LV, cc.pid, cc.tiles, cc.nq>), dim3(nb, items),      \
                           dim3(cc.tiles * cc.nq), 0, s, b);                                        \
      } else {                                                                                      \
        const ColArgs b = conv_gather(a, cc.tiles);                                                 \
        const dim3 gridc((unsigned)(b.nouter * b.ntiles + b.ntail), (unsigned)items);               \
        if constexpr (conv_twf<T>(LV, VV) && conv_split_wpe<T>(LV) > 0)                            \
          hipLaunchKernelGGL((k_col_conv<T, LV, cc.pid, cc.tiles, cc.nq, true, 0, true,             \
                                         conv_split_wpe<T>(LV)>),                                   \
                             gridc, dim3(cc.tiles * cc.nq), 0, s, b);                               \
        else if constexpr (conv_twf<T>(LV, VV))                                                     \
          hipLaunchKernelGGL((k_col_conv<T, LV, cc.pid, cc.tiles, cc.nq, true>), gridc,             \
                             dim3(cc.tiles * cc.nq), 0, s, b);                                      \
        else if constexpr (VV == 1 && conv_split_wpe<T>(LV) > 0)                                    \
          hipLaunchKernelGGL((k_col_conv<T, LV, cc.pid, cc.tiles, cc.nq, false, 0, true,            \
                                         conv_split_wpe<T>(LV)>),                                   \
                             gridc, dim3(cc.tiles * cc.nq), 0, s, b);                               \
        else                                                                                        \
          hipLaunchKernelGGL((k_col_conv<T, LV, cc.pid, cc.tiles, cc.nq>), gridc,                   \
                             dim3(cc.tiles * cc.nq), 0, s, b);                                      \
      }                                                                                             \
    } else if (kind == 1)                                                                           \
      hipLaunchKernelGGL((k_col_fft<T, LV, c.pid, c.tiles, c.nq, true>), grid, block, 0, s, a);     \
    else                                                                                            \
      hipLaunchKernelGGL((k_col_fft<T, LV, c.pid, c.tiles, c.nq, false>), grid, block, 0, s, a);    \
    found = true;                                                                                   \
  }
#define FSP_CASE(LV) FSP_VARIANTS(FSP_CASE_V, LV)
  FSP_COL_LENGTHS(FSP_CASE)
#undef FSP_CASE
#undef FSP_CASE_V
  if (!found) return hipErrorInvalidValue;
  return hipGetLastError();
}

// Fused axis-1 / axis-0 / axis-1 schedule for small cubic grids (n0 == n1):
// one block per TC columns holds the (i0, k1) slab in LDS.  tiles == 0 means
// unsupported.  LDS = (n N TC + groups TC 2n) sizeof(cx<T>) <= 160 KB.
constexpr int FUSED = 3;  // schedule value of passes 1..3 selecting the fused kernel
// Schedule value of passes 0 and 1 (both) or 3 and 4 (both) selecting the
// plane kernels (plane_kernels.hpp) for that pair.
constexpr int PLANE = 4;

template <typename T>
__host__ __device__ constexpr TileCfg slab_cfg(int L) {
  constexpr bool d = sizeof(T) == 8;
  switch (L) {
    case 16: return {0, d ? 16 : 32, 512};
    case 24: return {0, d ? 8 : 16, 512};
    case 32: return {0, d ? 8 : 16, 512};
    case 48: return {0, d ? 4 : 8, 512};
    case 64: return {0, d ? 2 : 4, 512};
    case 96: return {0, d ? 1 : 2, 512};
    case 128: return d ? TileCfg{0, 0, 0} : TileCfg{0, 2, 256};
    default: return {0, 0, 0};
  }
}

#define FSP_SLAB_LENGTHS(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

template <typename T>
hipError_t launch_slab(int L, const SlabArgs& a, int items, hipStream_t s) {
  bool found = false;
#define FSP_CASE(LV)                                                                                \
  if (L == LV) {                                                                                    \
    constexpr TileCfg c = slab_cfg<T>(LV);                                                          \
    if constexpr (c.tiles > 0) {                                                                    \
      hipLaunchKernelGGL((k_slab_conv<T, LV, 0, LV, 0, c.tiles, c.nq>), dim3(a.ntiles, items),      \
                         dim3(c.nq), 0, s, a);                                                      \
      found = true;                                                                                 \
    }                                                                                               \
  }
  FSP_SLAB_LENGTHS(FSP_CASE)
#undef FSP_CASE
  if (!found) return hipErrorInvalidValue;
  return hipGetLastError();
}

#ifdef FSP_SPLIT_LAUNCHERS
// The launchers are instantiated in their own translation units (compiled in
// parallel); the solve driver only references them.
extern template hipError_t launch_p1<float>(int, int, const RowArgs&, int, hipStream_t);
extern template hipError_t launch_p5<float>(int, int, const RowArgs&, int, hipStream_t);
extern template hipError_t launch_col<float>(int, int, int, const ColArgs&, int, hipStream_t);
extern template hipError_t launch_p1<double>(int, int, const RowArgs&, int, hipStream_t);
extern template hipError_t launch_p5<double>(int, int, const RowArgs&, int, hipStream_t);
extern template hipError_t launch_col<double>(int, int, int, const ColArgs&, int, hipStream_t);
extern template hipError_t launch_slab<float>(int, const SlabArgs&, int, hipStream_t);
extern template hipError_t launch_slab<double>(int, const SlabArgs&, int, hipStream_t);
extern template hipError_t launch_plane<float>(int, int, bool, const PlaneArgs&, int, hipStream_t);
extern template hipError_t launch_plane<double>(int, int, bool, const PlaneArgs&, int, hipStream_t);
#endif

// Geometry of up to MAX_ITEMS solves of one shape, filled by the plans.
struct SolveGeom {
  int items;                 // solves in this group (1 .. MAX_ITEMS; up to 65535 with items_dev)
  const ItemPtrs* items_dev; // device table of the group's buffers (then ghat/work/rho/phi are unused), or NULL
  int n0, n1, n2;
  int pitch;                 // P
  long long plane;           // complex elements between S planes i0 (>= 2 n1 P)
  int chunks;                // column chunks for passes 1-3 (1: whole passes)
  int gather_min;            // axis-0 blocks from which the lone last column is gathered
  int var[5];                // schedule variant of each pass
  const void* tw_row[5];     // twiddles of length n2 (+ split table) for the plan of P1 / P5
  const void* tw_c1[5];      // twiddles of length 2 n1 for the plan of P2 / P4
  const void* tw_c0;         // twiddles of length 2 n0 for the plan of P3
  const void* ghat[MAX_ITEMS];  // octant of each item, blocked [n1+1][tiles][n0+1][TC of P3]
  void* work[MAX_ITEMS];        // S of each item
  const void* rho[MAX_ITEMS];
  void* phi[MAX_ITEMS];
  // Gradient solve (one item; nout == 0 otherwise): the axis-0 pass reads S of
  // item 0 (once, or once per output with variant 2) and writes nout spectra,
  // which passes 4 and 5 take as items.  An output in place in S comes last.
  int nout;
  int ocomp[MAX_OUT];           // 0 potential, 1 + a derivative along axis a
  const void* oghat[MAX_OUT];   // table of each output
  void* owork[MAX_OUT];         // spectrum of each output (S itself for at most one)
  void* ophi[MAX_OUT];          // result of each output
};

// Passes first..last of one solve (0 = P1 ... 4 = P5).
template <typename T>
hipError_t launch_solve(const SolveGeom& g, int first, int last, hipStream_t s) {
  const long long P = g.pitch;
  const long long plane = g.plane;  // complex elements per S plane i0
  // items from the device table, or up to MAX_ITEMS in the kernel arguments
  const bool tab = g.items_dev != nullptr;
  if (!tab && (g.items < 1 || g.items > MAX_ITEMS)) return hipErrorInvalidValue;
  if (tab && (g.items < 1 || g.items > 65535 || g.nout)) return hipErrorInvalidValue;
  const int nfill = tab ? 0 : g.items;
  RowArgs ra{};
  ra.items = g.items_dev;
  ra.nrows = g.n0 * g.n1;
  ra.n1 = g.n1;
  ra.pitch = g.pitch;
  ra.s_i0_stride = plane;

  // P2 / P4: pencils along axis 1; outer = i0
  ColArgs ca{};
  ca.items = g.items_dev;
  for (int i = 0; i < nfill; ++i) ca.data[i] = g.work[i];
  ca.ncols = g.n2 + 1;
  ca.row_stride = P;
  ca.outer_stride = plane;
  ca.nouter = g.n0;

  // P3: pencils along axis 0; outer = k1 pairs
  ColArgs cc{};
  cc.items = g.items_dev;
  for (int i = 0; i < nfill; ++i) {
    cc.data[i] = g.work[i];
    cc.ghat[i] = g.ghat[i];
  }
  cc.nout = g.nout;
  for (int o = 0; o < g.nout; ++o) {
    cc.ocomp[o] = g.ocomp[o];
    cc.oghat[o] = g.oghat[o];
    cc.oout[o] = g.owork[o];
  }
  // P4 and P5 work on the P3 results
  void* const* after = g.nout ? g.owork : g.work;
  void* const* result = g.nout ? g.ophi : g.phi;
  const int npost = g.nout ? g.nout : g.items;
  cc.ncols = g.n2 + 1;
  cc.row_stride = plane;
  cc.outer_stride = P;
  cc.nouter = g.n1 + 1;
  cc.tw = g.tw_c0;
  cc.n1 = g.n1;
  cc.gather_min = g.gather_min;
  {
    const long long t0 = col_tiles<T>(2 * g.n0);
    cc.g_k1_stride = (g.n2 + 1 + t0 - 1) / t0 * (g.n0 + 1) * t0;
  }
  const int tc2 = col_cfg<T>(2 * g.n1, g.var[1]).tiles, tc4 = col_cfg<T>(2 * g.n1, g.var[3]).tiles;
  const int tc0 = col_tiles<T>(2 * g.n0);
  const int ncols = g.n2 + 1;
  auto set_cols = [&](ColArgs& c, int tcw, int c0, int c1) {
    c.col0 = c0;
    c.ncols = c1;
    c.ntiles = (c1 - c0 + tcw - 1) / tcw;
  };
  // passes 0-1 / 3-4 as the plane kernels: the pair runs at its first pass
  const bool plane_fwd = g.var[0] == PLANE, plane_inv = g.var[3] == PLANE;
  PlaneArgs pa{};
  pa.items = g.items_dev;
  pa.plane = plane;
  pa.pitch = g.pitch;
  auto run = [&](int pass, int c0, int c1) -> hipError_t {
    if ((pass == 1 && plane_fwd) || (pass == 4 && plane_inv)) return hipSuccess;
    if (pass == 0 && plane_fwd) {
      for (int i = 0; i < nfill; ++i) {
        pa.in[i] = g.rho[i];
        pa.out[i] = g.work[i];
      }
      pa.twr = g.tw_row[0];
      return launch_plane<T>(g.n2, g.n0, false, pa, g.items, s);
    }
    if (pass == 3 && plane_inv) {
      for (int i = 0; i < (tab ? 0 : npost); ++i) {
        pa.in[i] = after[i];
        pa.out[i] = result[i];
      }
      pa.twr = g.tw_row[4];
      return launch_plane<T>(g.n2, g.n0, true, pa, npost, s);
    }
    switch (pass) {
      case 0:
        for (int i = 0; i < nfill; ++i) {
          ra.in[i] = g.rho[i];
          ra.out[i] = g.work[i];
        }
        ra.tw = g.tw_row[0];
        return launch_p1<T>(g.n2, g.var[0], ra, g.items, s);
      case 1:
        set_cols(ca, tc2, c0, c1);
        ca.tw = g.tw_c1[1];
        return launch_col<T>(2 * g.n1, g.var[1], 0, ca, g.items, s);
      case 2:
        set_cols(cc, tc0, c0, c1);
        if (g.nout && g.var[2] == 2) {  // one launch per output, in order (an in-place one is last)
          hipError_t r = hipSuccess;
          for (int o = 0; o < g.nout && r == hipSuccess; ++o) {
            ColArgs c3 = cc;
            c3.nout = 1;
            c3.ocomp[0] = g.ocomp[o];
            c3.oghat[0] = g.oghat[o];
            c3.oout[0] = g.owork[o];
            r = launch_col<T>(2 * g.n0, 2, 2, c3, 1, s);
          }
          return r;
        }
        return launch_col<T>(2 * g.n0, g.var[2], 2, cc, g.items, s);
      case 3: {
        ColArgs c4 = ca;
        for (int i = 0; i < (tab ? 0 : npost); ++i) c4.data[i] = after[i];
        set_cols(c4, tc4, c0, c1);
        c4.tw = g.tw_c1[3];
        return launch_col<T>(2 * g.n1, g.var[3], 1, c4, npost, s);
      }
      case 4:
        for (int i = 0; i < (tab ? 0 : npost); ++i) {
          ra.in[i] = after[i];
          ra.out[i] = result[i];
        }
        ra.tw = g.tw_row[4];
        return launch_p5<T>(g.n2, g.var[4], ra, npost, s);
      default: return hipErrorInvalidValue;
    }
  };
  hipError_t e = hipSuccess;
  if (g.nout < 0 || g.nout > MAX_OUT || (g.nout && (g.items != 1 || g.var[1] == FUSED)))
    return hipErrorInvalidValue;  // one item, separate passes: the caller picks them
  // a plane pair is one kernel: a range holds both of its passes or neither
  if ((plane_fwd && (g.var[1] != PLANE || (first == 1 && last >= 1) || (first == 0 && last == 0))) ||
      (plane_inv && (g.var[4] != PLANE || (first <= 3 && last == 3) || (first == 4))) ||
      ((plane_fwd || plane_inv) && (g.n1 != g.n2 || g.chunks > 1 || g.var[1] == FUSED)))
    return hipErrorInvalidValue;
  if (g.var[1] == FUSED) {
    // passes 1-3 as one fused kernel over column tiles: a range holds all of
    // them or none (pass 0 or pass 4 alone)
    const bool mid = first <= 3 && last >= 1;
    if (mid && (first > 1 || last < 3)) return hipErrorInvalidValue;
    if (first == 0) e = run(0, 0, ncols);
    if (e != hipSuccess || !mid) return e == hipSuccess && last == 4 ? run(4, 0, ncols) : e;
    SlabArgs sa{};
    sa.items = g.items_dev;
    for (int i = 0; i < nfill; ++i) {
      sa.data[i] = g.work[i];
      sa.ghat[i] = g.ghat[i];
    }
    sa.tw1 = g.tw_c1[1];
    sa.tw0 = g.tw_c0;
    sa.plane = g.plane;
    sa.pitch = g.pitch;
    sa.ncols = ncols;
    const int tcs = slab_cfg<T>(2 * g.n1).tiles;
    sa.ntiles = (ncols + tcs - 1) / tcs;
    sa.gt = tc0;
    sa.g_k1_stride = cc.g_k1_stride;
    e = launch_slab<T>(2 * g.n1, sa, g.items, s);
    if (e == hipSuccess && last == 4) e = run(4, 0, ncols);
    return e;
  }
  if (g.chunks > 1 && first <= 1 && last >= 3) {
    // passes 1-3 column chunk by column chunk: a chunk's spectrum stays in the
    // memory-side cache between the three passes
    if (first == 0) e = run(0, 0, ncols);
    const int step = tc2 > tc0 ? (tc2 > tc4 ? tc2 : tc4) : (tc0 > tc4 ? tc0 : tc4);
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
