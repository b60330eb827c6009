// solve_kernels.hpp -- the five passes of one free-space solve (gfx950).
//
// Data layout.  rho and phi are [n0][n1][n2] real arrays.  The spectrum lives
// in one complex workspace S laid out [n0][2 n1][P] with P >= n2 + 1 a
// padded row pitch (rows start on 128-byte boundaries):
//
//   P1  rows of rho along axis 2: real transform of length 2 n2 of the
//       zero-padded row (computed as a complex transform of length n2 plus a
//       split step); writes the n2 + 1 non-negative frequencies to S rows
//       (i0, i1 < n1).                                   [Section 2.2, steps 1-2, 4]
//   P2  columns of S along axis 1: forward transform of length 2 n1 whose
//       upper half of inputs is the zero padding; writes all 2 n1 rows.
//   P3  columns of S along axis 0: forward transform of length 2 n0 (upper
//       half zero), multiply by the real, even transform of the mirror-
//       extended Green's function, inverse transform, keep rows < n0.
//                                                          [steps 3-5]
//   P4  columns of S along axis 1: inverse transform of length 2 n1, keep
//       rows < n1.
//   P5  rows of S along axis 2: inverse real transform of length 2 n2 from the
//       n2 + 1 stored frequencies, keep the first n2 samples -> phi. [step 5]
//
// Every pass reads and writes HBM once; the zero padding of rho2 and the
// unused half of phi2 are never stored.  The transforms are unnormalised: the
// stored Green's octant carries V / (8 n0 n1 n2).
//
// Column passes tile TC adjacent columns (contiguous in memory, so every row
// of a tile is one contiguous segment); row passes put consecutive lanes on
// consecutive elements of a row.
#pragma once

#include "fft_core.hpp"

namespace fsp {

// Up to MAX_ITEMS independent solves of one shape share a launch; blockIdx.y
// selects the item, whose buffers are passed by value in the kernel arguments.
constexpr int MAX_ITEMS = 16;
constexpr int MAX_OUT = 4;  // outputs of the gradient solve's axis-0 pass: three components and phi

// Buffers of one solve in a device-resident table.  A launch with a table
// (ColArgs/RowArgs/SlabArgs::items != NULL) reads item blockIdx.y's pointers
// from it when it runs, not from its arguments: a captured graph of such
// launches takes new rho / phi from an updated table without being captured
// again, and a launch may hold any number of items.
struct ItemPtrs {
  const void* rho;
  void* phi;
  void* work;        // S
  const void* ghat;  // the Green's octant, blocked as ColArgs::ghat
};

struct ColArgs {
  const ItemPtrs* items;      // table of this launch's items, or NULL (then data / ghat)
  void* data[MAX_ITEMS];      // S of each item
  const void* ghat[MAX_ITEMS];  // P3: Green's octant of each item, blocked [n1+1][tiles][n0+1][TC]
  const void* tw;             // twiddle table of this pencil length
  long long row_stride;       // complex elements between consecutive pencil rows
  long long outer_stride;     // complex elements between consecutive outer indices
  int col0;                   // first column handled by this launch
  int ncols;                  // end of the valid columns (n2 + 1 or a chunk end)
  int ntiles;                 // column tiles per outer index
  int nouter;                 // outer indices (P2/P4: n0; P3: n1 + 1 pairs)
  int n1;                     // P3: n1 (pairs k1 and 2 n1 - k1 share a Green's row)
  long long g_k1_stride;      // P3: reals between Green's blocks k1 (tiles (n0+1) TC)
  int ntail;                  // P3: leading blocks that gather column ncols - 1 over TC k1 pairs
  int gather_min;             // P3 (host side): grid size from which the launcher gathers
  // P3 with several outputs from one item (the gradient solve; nout == 0 otherwise)
  int nout;                   // outputs (1 .. MAX_OUT)
  int ocomp[MAX_OUT];         // multiply of output o: 0 potential (real); 1 + a derivative along axis a
  const void* oghat[MAX_OUT];   // table of output o, blocked as ghat
  void* oout[MAX_OUT];          // result spectrum of output o (may be data[0]: in place)
};

struct RowArgs {
  const ItemPtrs* items;      // table of this launch's items, or NULL (then in / out)
  const void* in[MAX_ITEMS];
  void* out[MAX_ITEMS];
  const void* tw;             // twiddles of length n2, then exp(-i pi k / n2), k in [0, n2]
  int nrows;                  // n0 * n1
  int n1;
  int pitch;                  // P
  long long s_i0_stride;      // complex elements between S planes (2 n1 P)
};

template <typename T>
__device__ __forceinline__ cx<T> czero() { return {T(0), T(0)}; }

// The buffers of this block's item (blockIdx.y): from the launch's table, else its arguments.
template <class A>
__device__ __forceinline__ void* item_work(const A& a) { return a.items ? a.items[blockIdx.y].work : a.data[blockIdx.y]; }
template <class A>
__device__ __forceinline__ const void* item_ghat(const A& a) {
  return a.items ? a.items[blockIdx.y].ghat : a.ghat[blockIdx.y];
}

// Load of a value that this launch reads exactly once (streamed, non-temporal).
template <typename T>
__device__ __forceinline__ cx<T> ld_once(const cx<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 w = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return {w.x, w.y};
}

// Store of a pass result.  Results that the next pass does not re-read soon
// are streamed past the caches (non-temporal); in float32 the axis-2 forward
// pass and the axis-1 passes keep normal stores, because their output is
// re-read by the next pass while part of it is still in the memory-side cache
// (measured: streaming those is slower, streaming the others is faster).
enum PassKind { PASS_ROW_FWD, PASS_COL_FWD, PASS_CONV, PASS_COL_INV, PASS_ROW_INV };

template <typename T, int KIND>
__device__ __forceinline__ void put(cx<T>* p, cx<T> v) {
  constexpr bool streamed = sizeof(T) == 8 || KIND == PASS_CONV || KIND == PASS_ROW_INV;
  if constexpr (streamed) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
  } else {
    *p = v;
  }
}

// LDS slot of element e of a row in the row passes: one pad slot after every
// 16 elements, so Stockham writes at strides of 16 or 32 elements fall on
// distinct banks.
__host__ __device__ constexpr int row_slot(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int row_pitch(int LC) { return row_slot(LC) + 1; }

// Pencil of thread column c: block b covers TC adjacent columns of outer index b / ntiles.
template <int TC>
__device__ __forceinline__ void place_column(const ColArgs& a, int c, int& col, int& outer, bool& ok) {
  const int tile = blockIdx.x % a.ntiles;
  outer = blockIdx.x / a.ntiles;
  col = a.col0 + tile * TC + c;
  ok = col < a.ncols;
}

// ----------------------------------------------------------------- P2 / P4
template <typename T, int L, int PID, int TC, int NQ, bool INV>
__global__ __launch_bounds__(TC* NQ) void k_col_fft(ColArgs a) {
  constexpr int K = plan_len(L, PID);
  __shared__ cx<T> lds[K > 1 ? L * TC : 1];
  const int tid = threadIdx.x;
  const int c = tid % TC, q = tid / TC;
  int col, outer;
  bool cok;
  place_column<TC>(a, c, col, outer, cok);
  cx<T>* base = reinterpret_cast<cx<T>*>(item_work(a)) + (long long)outer * a.outer_stride + col;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  const unsigned rs = (unsigned)a.row_stride;  // row offsets of one pencil fit in 32 bits (unsigned: no sign extension)
  auto idx = [c](int row) { return row * TC + c; };
  constexpr bool REV = INV;
  using F = FirstStage<L, PID, REV, NQ>;
  static_assert(INV || F::R % 2 == 0, "forward plans start with an even radix");

  cx<T> v[F::J][F::R];
#pragma unroll
  for (int j = 0; j < F::J; ++j) {
    const int b = q + NQ * j;
    const bool ok = cok && ((F::NB % NQ == 0) || b < F::NB);
#pragma unroll
    for (int r = 0; r < F::R; ++r) {
      // forward: rows >= L/2 are the zero padding and are never read
      const bool pad = !INV && r >= F::R / 2;
      v[j][r] = (ok && !pad) ? base[(b + r * F::NB) * rs] : czero<T>();
    }
    // forward: upper half of the inputs is zero; inverse with one stage: only
    // the lower half of the outputs is kept
    if constexpr (INV && K == 1)
      dft_half_out<F::R, true, T>(v[j]);
    else if constexpr (INV)
      Dft<F::R, true, T>::run(v[j]);
    else
      dft_half_in<F::R, false, T>(v[j]);
  }
  if constexpr (K == 1) {
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
      const int b = q + NQ * j;
      if (cok && ((F::NB % NQ == 0) || b < F::NB)) {
#pragma unroll
        for (int m = 0; m < F::R; ++m)
          if (!INV || m < F::R / 2) put<T, INV ? PASS_COL_INV : PASS_COL_FWD>(&base[(b + m * F::NB) * rs], v[j][m]);
      }
    }
  } else {
    write_first_outputs<T, F::R, F::J, F::NB, NQ>(lds, v, q, idx);
    lds_barrier();
    lds_stages<T, L, PID, REV, 1, K - 1, NQ, INV>(lds, tw, q, idx);
    using Ls = LastStage<L, PID, REV, NQ>;
    static_assert(!INV || Ls::R % 2 == 0, "inverse plans end with an even radix");
    cx<T> w[Ls::J][Ls::R];
    lds_last_stage<T, L, PID, REV, NQ, INV, false, INV>(lds, tw, q, idx, w);
#pragma unroll
    for (int j = 0; j < Ls::J; ++j) {
      const int b = q + NQ * j;
      if (cok && ((Ls::NB % NQ == 0) || b < Ls::NB)) {
#pragma unroll
        for (int m = 0; m < Ls::R; ++m)
          if (!INV || m < Ls::R / 2) put<T, INV ? PASS_COL_INV : PASS_COL_FWD>(&base[(b + m * Ls::NB) * rs], w[j][m]);
      }
    }
  }
}

// ----------------------------------------------------------------- P3
// Loads are issued in the order they are consumed (twiddles, Green's rows,
// the first pencil set, the second), so the first transform waits only for
// its own data while the second set is still arriving.  Two-stage plans load
// the table values of their forward butterflies once, for both sets.
// TWF: the plan's complete twiddle table is read into LDS once per block, so
// the butterflies load every power instead of multiplying it out of six.
// NOUT > 0 (the gradient solve): one forward transform per pencil set, then
// a.nout outputs (NOUT == 1: exactly one): output o multiplies by table
// a.oghat[o] (a.ocomp[o]: 0 the potential's, 1 + a the derivative along axis
// a) and goes to a.oout[o] (which may be S itself: a block reads each pencil
// set before it writes that set's outputs, and its two sets are different
// rows k1 and 2 n1 - k1).  One item per launch; separate instantiations, so
// the potential's kernel carries none of it.  With NOUT == 1 the spectrum is
// not held through a loop (fewer registers).
// SPLIT (two-stage plans): the exchanges go through a real-valued LDS array in
// two rounds (real parts, then imaginary parts) with a padded row pitch, half
// the LDS of a complex array, and the kernel is built for WPE waves per SIMD.
template <typename T, int L, int PID, int TC, int NQ, bool TWF = false, int NOUT = 0, bool SPLIT = false, int WPE = 1>
__global__ __launch_bounds__(TC* NQ, WPE) void k_col_conv(ColArgs a) {
  constexpr bool GRAD = NOUT > 0;
  constexpr int K = plan_len(L, PID);
  static_assert(!TWF || K > 1, "single-stage plans have no twiddles");
  static_assert(!SPLIT || K == 2, "split exchanges are built for two-stage plans");
  // the others keep their registers for occupancy (at 1024 points the preloaded values spill)
  constexpr bool PRE = K == 2 && !TWF && !GRAD && !SPLIT && sizeof(T) == 4 && L <= 512;
  constexpr int NT = TC * NQ;
  constexpr int TWN = TWF ? (twf_size(L, PID) + NT - 1) / NT : 1;  // table entries per thread
  constexpr int SP = TC + 1;  // split row pitch: rows R apart fall in other banks
  __shared__ cx<T> lds[K > 1 && !SPLIT ? L * TC : 1];
  __shared__ T ldss[SPLIT ? L * SP : 1];
  __shared__ cx<T> twl[TWF ? twf_size(L, PID) : 1];
  const int tid = threadIdx.x;
  const int c = tid % TC, q = tid / TC;
  int col, p;  // p: k1 in [0, n1]; the thread also handles 2 n1 - p
  bool cok;
  // The first ntail blocks take the last column (when it is the only column
  // of its tile) for TC pairs k1 each, so no block transforms a tile that is
  // mostly empty; their lanes differ in k1, the other blocks' lanes in column.
  const bool gathered = (int)blockIdx.x < a.ntail;
  if (gathered) {
    p = (int)blockIdx.x * TC + c;
    col = a.ncols - 1;
    cok = p <= a.n1;
    if (!cok) p = 0;  // addresses stay in range; nothing is loaded or stored
  } else {
    const int bid = (int)blockIdx.x - a.ntail;
    const int tile = bid % a.ntiles;
    p = bid / a.ntiles;
    col = a.col0 + tile * TC + c;
    cok = col < a.ncols;
  }
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  const unsigned rs = (unsigned)a.row_stride;  // row offsets of one pencil fit in 32 bits (unsigned: no sign extension)
  auto idx = [c](int row) { return row * TC + c; };
  auto idxs = [c](int row) { return row * SP + c; };
  using F = FirstStage<L, PID, false, NQ>;   // forward, first stage
  using Lf = LastStage<L, PID, false, NQ>;   // forward, last stage == inverse, first stage
  using Li = LastStage<L, PID, true, NQ>;    // inverse, last stage
  static_assert(F::R % 2 == 0, "forward plans start with an even radix");
  static_assert(Li::R % 2 == 0, "inverse plans end with an even radix");

  cx<T> twr[TWN];
  if constexpr (TWF) {
    const cx<T>* src = tw + tw_size(L, PID);
#pragma unroll
    for (int i = 0; i < TWN; ++i) {
      const int e = tid + NT * i;
      twr[i] = e < twf_size(L, PID) ? src[e] : czero<T>();
    }
  }
  TwBase<T> tbf[PRE ? Lf::J : 1];
  if constexpr (PRE) load_last_twbase<T, L, PID, false, NQ>(tbf, tw, q);

  // Green's values for the rows this thread holds after the forward transform;
  // the octant is stored in column tiles of TC, so a tile's rows are contiguous.
  // GRAD: the table of output o is a.oghat[o], in the same layout.
  const long long goff = (long long)p * a.g_k1_stride + (long long)(col / TC) * (L / 2 + 1) * TC + (col % TC);
  // Every lane's address lies inside the table (a lane past the last column
  // reads the zero-filled slots of the last column tile, and a gathered lane
  // past n1 reads row 0), so the loads need no predicate; those lanes' results
  // are never stored.
  auto load_g = [&](const void* table, T (&gv)[Lf::J][Lf::R]) {
    const T* g = reinterpret_cast<const T*>(table) + goff;
#pragma unroll
    for (int j = 0; j < Lf::J; ++j) {
      const int b = q + NQ * j;
      const bool ok = (Lf::NB % NQ == 0) || b < Lf::NB;
#pragma unroll
      for (int m = 0; m < Lf::R; ++m) {
        const int k0 = b + m * Lf::NB;
        const int kf = k0 <= L / 2 ? k0 : L - k0;
        gv[j][m] = ok ? g[kf * TC] : T(0);
      }
    }
  };
  T gv[Lf::J][Lf::R];
  load_g(GRAD ? a.oghat[0] : item_ghat(a), gv);
  // GRAD with registers to spare: the next output's table values are loaded
  // while the current output is transformed
  constexpr bool GPRE = NOUT > 1 && sizeof(T) * L / NQ <= 64;
  T gn[GPRE ? Lf::J : 1][GPRE ? Lf::R : 1];

  // k1 = p and its partner 2 n1 - p share the Green's rows; p = 0 and p = n1
  // have no partner.  `second` (a second pencil set follows, with barriers) is
  // block-uniform: gathered blocks always run it, and in the others p is the
  // block's own; `two` is the per-lane load/store mask of that set.
  const bool paired = !(p == 0 || p == a.n1);
  const bool second = gathered || paired;
  const bool two = cok && paired;
  const long long off_a = (long long)p * a.outer_stride + col;
  const long long off_b = (long long)(2 * a.n1 - p) * a.outer_stride + col;
  cx<T>* const data = reinterpret_cast<cx<T>*>(item_work(a));
  // The derivative tables are odd along their axis: their transform is -i T with
  // the real octant T read at the folded frequency and negated on the upper half
  // of that axis (k0 > n0; for axis 1 the partner 2 n1 - p; axis 2 holds k2 <= n2).
  auto multiply = [&](cx<T>& w, T g, int comp, int k0, bool upper_k1) {
    if (!GRAD || comp == 0) {
      w = cscale(w, g);
    } else {
      const bool neg = comp == 1 ? (k0 > L / 2) : (comp == 2 && upper_k1);
      const T t = neg ? -g : g;
      w = cx<T>{t * w.y, -t * w.x};  // w * (-i t)
    }
  };
  auto load_set = [&](const cx<T>* base, bool on, cx<T> (&raw)[F::J][F::R / 2]) {
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
      const int b = q + NQ * j;
      const bool ok = on && cok && ((F::NB % NQ == 0) || b < F::NB);
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) raw[j][r] = czero<T>();
      if (ok) {  // one branch around the butterfly's loads
#pragma unroll
        for (int r = 0; r < F::R / 2; ++r) raw[j][r] = ld_once(&base[(b + r * F::NB) * rs]);
      }
    }
  };
  const cx<T>* tws = TWF ? static_cast<const cx<T>*>(twl) : tw;
  // The spectrum of one pencil set (in the layout of the last forward stage)
  // times one table, back to space, the first half stored at base.
  auto finish = [&](const cx<T> (&w)[Lf::J][Lf::R], const T (&gt)[Lf::J][Lf::R], int comp, bool upper_k1,
                    cx<T>* base, bool st) {
    cx<T> x[Lf::J][Lf::R];
#pragma unroll
    for (int j = 0; j < Lf::J; ++j) {
      const int b = q + NQ * j;
#pragma unroll
      for (int m = 0; m < Lf::R; ++m) {
        x[j][m] = w[j][m];
        multiply(x[j][m], gt[j][m], comp, b + m * Lf::NB, upper_k1);
      }
      // K == 1: the whole inverse, of which only the lower half is kept; else its first stage (span 1)
      if constexpr (K == 1)
        dft_half_out<Lf::R, true, T>(x[j]);
      else
        Dft<Lf::R, true, T>::run(x[j]);
    }
    if constexpr (K == 1) {
#pragma unroll
      for (int j = 0; j < Lf::J; ++j) {
        const int b = q + NQ * j;
        if (st && ((Lf::NB % NQ == 0) || b < Lf::NB)) {
#pragma unroll
          for (int m = 0; m < Lf::R / 2; ++m) put<T, PASS_CONV>(&base[(b + m * Lf::NB) * rs], x[j][m]);
        }
      }
    } else {
      cx<T> u[Li::J][Li::R];
      lds_barrier();
      if constexpr (SPLIT) {
        exchange_split<T, Lf::R, Lf::J, Lf::NB, NQ, Li::R, Li::J, Li::NB>(ldss, x, u, q, idxs);
        last_stage_regs<T, L, PID, true, NQ, true, true, TWF>(u, tws, q);
      } else {
        write_first_outputs<T, Lf::R, Lf::J, Lf::NB, NQ>(lds, x, q, idx);
        lds_barrier();
        lds_stages<T, L, PID, true, 1, K - 1, NQ, true, TWF>(lds, tws, q, idx);
        lds_last_stage<T, L, PID, true, NQ, true, TWF, true>(lds, tws, q, idx, u);
      }
#pragma unroll
      for (int j = 0; j < Li::J; ++j) {
        const int b = q + NQ * j;
        if (st && ((Li::NB % NQ == 0) || b < Li::NB)) {
#pragma unroll
          for (int m = 0; m < Li::R / 2; ++m) put<T, PASS_CONV>(&base[(b + m * Li::NB) * rs], u[j][m]);
        }
      }
    }
  };
  // set: 0 for k1 = p, 1 for its partner (whose outputs come last in the block)
  auto run_set = [&](int set, const cx<T> (&raw)[F::J][F::R / 2], bool st) {
    const bool upper_k1 = set == 1;
    const long long off = set == 0 ? off_a : off_b;
    cx<T> v[F::J][F::R];
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) v[j][r] = raw[j][r];
      dft_half_in<F::R, false, T>(v[j]);  // the upper half is the zero padding
    }
    cx<T> w[Lf::J][Lf::R];
    if constexpr (K == 1) {
      static_assert(K > 1 || (F::J == Lf::J && F::R == Lf::R), "a one-stage plan is its own last stage");
#pragma unroll
      for (int j = 0; j < Lf::J; ++j)
#pragma unroll
        for (int m = 0; m < Lf::R; ++m) w[j][m] = v[j][m];
    } else if constexpr (SPLIT) {
      exchange_split<T, F::R, F::J, F::NB, NQ, Lf::R, Lf::J, Lf::NB>(ldss, v, w, q, idxs);
      last_stage_regs<T, L, PID, false, NQ, false, false, TWF>(w, tws, q);
    } else {
      write_first_outputs<T, F::R, F::J, F::NB, NQ>(lds, v, q, idx);
      lds_barrier();
      lds_stages<T, L, PID, false, 1, K - 1, NQ, false, TWF>(lds, tws, q, idx);
      if constexpr (PRE)
        lds_last_stage_pre<T, L, PID, false, NQ, false>(lds, tbf, q, idx, w);
      else
        lds_last_stage<T, L, PID, false, NQ, false, TWF>(lds, tws, q, idx, w);
    }
    if constexpr (!GRAD) {
      finish(w, gv, 0, upper_k1, data + off, st);
    } else {
      // every output from the one forward transform; the table values of
      // output 0 are in gv on entry (loaded at the start, or prefetched by the
      // other set's last output)
      // (one output: gv serves both sets)
      const int nout = NOUT == 1 ? 1 : a.nout;
#pragma unroll 1
      for (int o = 0; o < nout; ++o) {
        const bool last = set == 1 || !second;  // no set follows this one
        if constexpr (GPRE) {
          if (o + 1 < nout) load_g(a.oghat[o + 1], gn);
          else if (!last && nout > 1) load_g(a.oghat[0], gn);
        } else if ((o > 0 || set == 1) && nout > 1) {
          load_g(a.oghat[o], gv);
        }
        finish(w, gv, a.ocomp[o], upper_k1, reinterpret_cast<cx<T>*>(a.oout[o]) + off, st);
        if constexpr (GPRE) {
          if (nout > 1) {
#pragma unroll
            for (int j = 0; j < Lf::J; ++j)
#pragma unroll
              for (int m = 0; m < Lf::R; ++m) gv[j][m] = gn[j][m];
          }
        }
      }
    }
  };
  // GRAD where registers are short (long pencils per thread): the second set
  // is read after the first set's outputs, not held through them
  constexpr bool LATE_B = (NOUT > 1 && sizeof(T) * L / NQ >= 128) || (SPLIT && WPE >= 3);
  cx<T> raw_a[F::J][F::R / 2], raw_b[F::J][F::R / 2];
  issue_fence();
  load_set(data + off_a, true, raw_a);
  issue_fence();
  if constexpr (!LATE_B) load_set(data + off_b, two, raw_b);
  issue_fence();
  if constexpr (TWF) {  // the table arrived before the pencils; visible after the first barrier
#pragma unroll
    for (int i = 0; i < TWN; ++i) {
      const int e = tid + NT * i;
      if (e < twf_size(L, PID)) twl[e] = twr[i];
    }
  }
  run_set(0, raw_a, cok);
  if (second) {  // block-uniform: barriers inside
    if constexpr (LATE_B) load_set(data + off_b, two, raw_b);
    lds_barrier();
    run_set(1, raw_b, two);
  }
}

// ----------------------------------------------------------------- P3, pipelined
// Same computation as k_col_conv, but each block walks a sequence of pencil
// sets (items blockIdx.x, blockIdx.x + gridDim.x, ...; each item is the k1
// pair p, 2 n1 - p of one column tile) and loads the next set while it
// transforms the current one, so memory traffic and arithmetic overlap inside
// one block.  The Green's rows of a set are loaded at the start of its
// transform (the second set of a pair finds them in cache).
template <typename T, int L, int PID, int TC, int NQ>
__global__ __launch_bounds__(TC* NQ) void k_col_conv_pipe(ColArgs a) {
  constexpr int K = plan_len(L, PID);
  static_assert(K > 1, "pipelined pass needs an LDS exchange");
  __shared__ cx<T> lds[L * TC];
  const int tid = threadIdx.x;
  const int c = tid % TC, q = tid / TC;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  const unsigned rs = (unsigned)a.row_stride;  // row offsets of one pencil fit in 32 bits (unsigned: no sign extension)
  auto idx = [c](int row) { return row * TC + c; };
  using F = FirstStage<L, PID, false, NQ>;
  using Lf = LastStage<L, PID, false, NQ>;
  using Li = LastStage<L, PID, true, NQ>;
  static_assert(F::R % 2 == 0 && Li::R % 2 == 0, "plans start with an even radix");
  const int nitems = a.nouter * a.ntiles;
  cx<T>* data = reinterpret_cast<cx<T>*>(item_work(a));
  const T* ghat = reinterpret_cast<const T*>(item_ghat(a));

  // pencil set (item w, which) of this thread: its column base and Green's rows
  auto set_base = [&](int w, int which) -> cx<T>* {
    const int tile = w % a.ntiles, p = w / a.ntiles;
    const int k1 = which == 0 ? p : 2 * a.n1 - p;
    return data + (long long)k1 * a.outer_stride + (a.col0 + tile * TC + c);
  };
  auto set_green = [&](int w) -> const T* {
    const int tile = w % a.ntiles, p = w / a.ntiles;
    const int col = a.col0 + tile * TC + c;
    return ghat + (long long)p * a.g_k1_stride + (long long)(col / TC) * (L / 2 + 1) * TC + (col % TC);
  };
  auto set_ok = [&](int w) { return a.col0 + (w % a.ntiles) * TC + c < a.ncols; };
  auto paired = [&](int w) {
    const int p = w / a.ntiles;
    return p != 0 && p != a.n1;
  };
  auto load_set = [&](const cx<T>* base, bool on, cx<T> (&raw)[F::J][F::R / 2]) {
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
      const int b = q + NQ * j;
      const bool ok = on && ((F::NB % NQ == 0) || b < F::NB);
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) raw[j][r] = ok ? ld_once(&base[(b + r * F::NB) * rs]) : czero<T>();
    }
  };
  auto run_set = [&](cx<T>* base, const T* g, bool on, const cx<T> (&raw)[F::J][F::R / 2]) {
    cx<T> v[F::J][F::R];
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) v[j][r] = raw[j][r];
      dft_half_in<F::R, false, T>(v[j]);  // the upper half is the zero padding
    }
    write_first_outputs<T, F::R, F::J, F::NB, NQ>(lds, v, q, idx);
    lds_barrier();
    lds_stages<T, L, PID, false, 1, K - 1, NQ, false>(lds, tw, q, idx);
    cx<T> w[Lf::J][Lf::R];
    lds_last_stage<T, L, PID, false, NQ, false>(lds, tw, q, idx, w);
#pragma unroll
    for (int j = 0; j < Lf::J; ++j) {
      const int b = q + NQ * j;
      const bool ok = on && ((Lf::NB % NQ == 0) || b < Lf::NB);
#pragma unroll
      for (int m = 0; m < Lf::R; ++m) {
        const int k0 = b + m * Lf::NB;
        const int kf = k0 <= L / 2 ? k0 : L - k0;
        w[j][m] = cscale(w[j][m], ok ? g[kf * TC] : T(0));
      }
      Dft<Lf::R, true, T>::run(w[j]);
    }
    lds_barrier();
    write_first_outputs<T, Lf::R, Lf::J, Lf::NB, NQ>(lds, w, q, idx);
    lds_barrier();
    lds_stages<T, L, PID, true, 1, K - 1, NQ, true>(lds, tw, q, idx);
    cx<T> u[Li::J][Li::R];
    lds_last_stage<T, L, PID, true, NQ, true, false, true>(lds, tw, q, idx, u);
#pragma unroll
    for (int j = 0; j < Li::J; ++j) {
      const int b = q + NQ * j;
      if (on && ((Li::NB % NQ == 0) || b < Li::NB)) {
#pragma unroll
        for (int m = 0; m < Li::R / 2; ++m) put<T, PASS_CONV>(&base[(b + m * Li::NB) * rs], u[j][m]);
      }
    }
  };

  int w = blockIdx.x, which = 0;
  if (w >= nitems) return;  // uniform per block
  cx<T> raw[F::J][F::R / 2];
  load_set(set_base(w, which), set_ok(w), raw);
  while (true) {
    int w2 = w, which2 = which + 1;
    if (which2 == 2 || !paired(w)) {
      w2 = w + gridDim.x;
      which2 = 0;
    }
    const bool more = w2 < nitems;  // uniform per block
    cx<T> raw2[F::J][F::R / 2];
    if (more) load_set(set_base(w2, which2), set_ok(w2), raw2);
    run_set(set_base(w, which), set_green(w), set_ok(w), raw);
    if (!more) break;
    lds_barrier();
    w = w2;
    which = which2;
#pragma unroll
    for (int j = 0; j < F::J; ++j)
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) raw[j][r] = raw2[j][r];
  }
}

// ----------------------------------------------------------------- P2+P3+P4 fused (small grids)
// One block holds the whole (i0, k1) slab of TC adjacent columns in LDS,
// laid out [i0][k1][c] (c fastest), and performs the axis-1 forward transform,
// the axis-0 forward transform, Green's multiply and inverse, and the axis-1
// inverse transform there: S is read once and written once.  Every stage works
// on all pencils of the slab at once: a thread takes the butterflies
// u = tid + NT j (c fastest, then butterfly, then pencil), reads their inputs,
// waits at a barrier, then writes their outputs in place.
template <typename T, int L, int PID, bool REV, int S, int NP, int TC, int NT, bool INV, bool PAD, class PIDX>
__device__ __forceinline__ void slab_stage(cx<T>* lds, const cx<T>* __restrict__ tw, int tid, PIDX pidx) {
  constexpr int R = plan_radix(L, PID, REV, S);
  constexpr int NS = plan_ns(L, PID, REV, S);
  constexpr int NB = L / R;
  constexpr int UNITS = NP * TC * NB;
  constexpr int J = (UNITS + NT - 1) / NT;
  const cx<T>* tws = tw + tw_base(L, PID, REV) + tw_stage_off(L, PID, REV, S);
  cx<T> v[J][R];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int u = tid + NT * j;
    if (UNITS % NT == 0 || u < UNITS) {
      const int c = u % TC, b = (u / TC) % NB, pp = u / (TC * NB);
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[j][r] = (PAD && r >= R / 2) ? czero<T>() : lds[pidx(pp, b + r * NB, c)];
    }
  }
  lds_barrier();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int u = tid + NT * j;
    if (UNITS % NT == 0 || u < UNITS) {
      const int c = u % TC, b = (u / TC) % NB, pp = u / (TC * NB);
      apply_twiddles<T, R, NS, INV>(v[j], tws, b % NS);
      Dft<R, INV, T>::run(v[j]);
      const int base = (b / NS) * NS * R + (b % NS);
#pragma unroll
      for (int m = 0; m < R; ++m) lds[pidx(pp, base + m * NS, c)] = v[j][m];
    }
  }
  lds_barrier();
}

// All stages of one transform of every pencil of the slab, in LDS.
template <typename T, int L, int PID, bool REV, int S, int NP, int TC, int NT, bool INV, bool PAD, class PIDX>
__device__ __forceinline__ void slab_fft(cx<T>* lds, const cx<T>* __restrict__ tw, int tid, PIDX pidx) {
  if constexpr (S < plan_len(L, PID)) {
    slab_stage<T, L, PID, REV, S, NP, TC, NT, INV, PAD && S == 0>(lds, tw, tid, pidx);
    slab_fft<T, L, PID, REV, S + 1, NP, TC, NT, INV, PAD>(lds, tw, tid, pidx);
  }
}

// N0 = L0 / 2, N1 = L1 / 2.  tw1: twiddles of length L1 (plan PID1), tw0: of
// length L0 (plan PID0); ghat blocked in column tiles of GT.
struct SlabArgs {
  const ItemPtrs* items;      // table of this launch's items, or NULL (then data / ghat)
  void* data[MAX_ITEMS];
  const void* ghat[MAX_ITEMS];
  const void* tw1;
  const void* tw0;
  long long plane;   // complex elements between S planes i0
  int pitch;         // P
  int ncols;         // n2 + 1
  int ntiles;        // column tiles of TC
  int gt;            // column tile of the Green's octant
  long long g_k1_stride;
};

template <typename T, int L1, int PID1, int L0, int PID0, int TC, int NT>
__global__ __launch_bounds__(NT) void k_slab_conv(SlabArgs a) {
  constexpr int N0 = L0 / 2, N1 = L1 / 2;
  __shared__ cx<T> lds[N0 * L1 * TC];
  const int tid = threadIdx.x;
  const int col0 = blockIdx.x * TC;
  cx<T>* S = reinterpret_cast<cx<T>*>(item_work(a));
  const T* ghat = reinterpret_cast<const T*>(item_ghat(a));
  const cx<T>* tw1 = reinterpret_cast<const cx<T>*>(a.tw1);
  const cx<T>* tw0 = reinterpret_cast<const cx<T>*>(a.tw0);
  // load rows (i0, i1 < N1) of the tile
  for (int e = tid; e < N0 * N1 * TC; e += NT) {
    const int c = e % TC, i1 = (e / TC) % N1, i0 = e / (TC * N1);
    const int col = col0 + c;
    lds[(i0 * L1 + i1) * TC + c] = col < a.ncols ? S[i0 * a.plane + (long long)i1 * a.pitch + col] : czero<T>();
  }
  lds_barrier();
  // axis-1 forward: pencils (i0, c) along k1; upper half of the inputs is padding
  auto along1 = [](int i0, int k1, int c) { return (i0 * L1 + k1) * TC + c; };
  slab_fft<T, L1, PID1, false, 0, N0, TC, NT, false, true>(lds, tw1, tid, along1);
  // axis 0: pencils (k1, c) along i0 (length L0, rows >= N0 live only in registers)
  {
    using F = FirstStage<L0, PID0, false, 1>;
    constexpr int K = plan_len(L0, PID0);
    static_assert(K >= 1, "plan");
    // The axis-0 pencils are longer than the slab holds (rows N0..L0-1 are the
    // zero padding and the discarded half), so each is transformed in registers
    // by one thread group: NQ0 threads per pencil, pencils in turn.
    constexpr int NQ0 = (L0 / F::R) < (NT / TC) ? (L0 / F::R) : (NT / TC);
    // pencils of one column handled together, limited so that slab + scratch fit in LDS
    constexpr int SLAB_BYTES = N0 * L1 * TC * (int)sizeof(cx<T>);
    constexpr int PEN_ONE = TC * L0 * (int)sizeof(cx<T>);
    constexpr int G_THREADS = NT / (NQ0 * TC);
    constexpr int G_LDS = (163840 - 1024 - SLAB_BYTES) / PEN_ONE - 1;
    constexpr int GROUPS = G_THREADS < G_LDS ? G_THREADS : (G_LDS > 0 ? G_LDS : 1);
    // one extra group of scratch: threads beyond GROUPS groups run the same
    // stage code (every thread takes the barriers) on that dummy region
    __shared__ cx<T> pen[K > 1 ? (GROUPS + 1) * TC * L0 : 1];
    const int c = tid % TC, q = (tid / TC) % NQ0, gsel = tid / (TC * NQ0);
    const int gpen = gsel < GROUPS ? gsel : GROUPS;
    auto pidx = [&](int row) { return (gpen * L0 + row) * TC + c; };
    for (int k1b = 0; k1b < L1; k1b += GROUPS) {
      const int k1 = k1b + gsel;
      const bool act = gsel < GROUPS && k1 < L1 && tid < GROUPS * TC * NQ0;
      const int col = col0 + c;
      // forward first stage from the slab
      cx<T> v[F::J][F::R];
#pragma unroll
      for (int j = 0; j < F::J; ++j) {
        const int b = q + NQ0 * j;
        const bool ok = act && ((F::NB % NQ0 == 0) || b < F::NB);
#pragma unroll
        for (int r = 0; r < F::R; ++r)
          v[j][r] = (ok && r < F::R / 2) ? lds[(b + r * F::NB) * L1 * TC + k1 * TC + c] : czero<T>();
        dft_half_in<F::R, false, T>(v[j]);
      }
      if constexpr (K == 1) {
        const int k1f = k1 <= N1 ? k1 : L1 - k1;
        const T* g = ghat + (long long)k1f * a.g_k1_stride + (long long)(col / a.gt) * (N0 + 1) * a.gt + (col % a.gt);
#pragma unroll
        for (int j = 0; j < F::J; ++j) {
          const int b = q + NQ0 * j;
          const bool ok = act && col < a.ncols && ((F::NB % NQ0 == 0) || b < F::NB);
#pragma unroll
          for (int m = 0; m < F::R; ++m) {
            const int k0 = b + m * F::NB;
            const int kf = k0 <= N0 ? k0 : L0 - k0;
            v[j][m] = cscale(v[j][m], ok ? g[kf * a.gt] : T(0));
          }
          dft_half_out<F::R, true, T>(v[j]);  // rows >= N0 are dropped
        }
        lds_barrier();
#pragma unroll
        for (int j = 0; j < F::J; ++j) {
          const int b = q + NQ0 * j;
          if (act && ((F::NB % NQ0 == 0) || b < F::NB)) {
#pragma unroll
            for (int m = 0; m < F::R / 2; ++m) lds[(b + m * F::NB) * L1 * TC + k1 * TC + c] = v[j][m];
          }
        }
        lds_barrier();
      } else {
        using Lf = LastStage<L0, PID0, false, NQ0>;
        using Li = LastStage<L0, PID0, true, NQ0>;
        using F2 = FirstStage<L0, PID0, false, NQ0>;
        cx<T> v2[F2::J][F2::R];
#pragma unroll
        for (int j = 0; j < F2::J; ++j) {
          const int b = q + NQ0 * j;
          const bool ok = act && ((F2::NB % NQ0 == 0) || b < F2::NB);
#pragma unroll
          for (int r = 0; r < F2::R; ++r)
            v2[j][r] = (ok && r < F2::R / 2) ? lds[(b + r * F2::NB) * L1 * TC + k1 * TC + c] : czero<T>();
          dft_half_in<F2::R, false, T>(v2[j]);
        }
        write_first_outputs<T, F2::R, F2::J, F2::NB, NQ0>(pen, v2, q, pidx);
        lds_barrier();
        lds_stages<T, L0, PID0, false, 1, K - 1, NQ0, false>(pen, tw0, q, pidx);
        cx<T> w[Lf::J][Lf::R];
        lds_last_stage<T, L0, PID0, false, NQ0, false>(pen, tw0, q, pidx, w);
        const int k1f = k1 <= N1 ? k1 : L1 - k1;
        const T* g = ghat + (long long)k1f * a.g_k1_stride + (long long)(col / a.gt) * (N0 + 1) * a.gt + (col % a.gt);
#pragma unroll
        for (int j = 0; j < Lf::J; ++j) {
          const int b = q + NQ0 * j;
          const bool ok = act && col < a.ncols && ((Lf::NB % NQ0 == 0) || b < Lf::NB);
#pragma unroll
          for (int m = 0; m < Lf::R; ++m) {
            const int k0 = b + m * Lf::NB;
            const int kf = k0 <= N0 ? k0 : L0 - k0;
            w[j][m] = cscale(w[j][m], ok ? g[kf * a.gt] : T(0));
          }
          Dft<Lf::R, true, T>::run(w[j]);
        }
        lds_barrier();
        write_first_outputs<T, Lf::R, Lf::J, Lf::NB, NQ0>(pen, w, q, pidx);
        lds_barrier();
        lds_stages<T, L0, PID0, true, 1, K - 1, NQ0, true>(pen, tw0, q, pidx);
        cx<T> u[Li::J][Li::R];
        lds_last_stage<T, L0, PID0, true, NQ0, true, false, true>(pen, tw0, q, pidx, u);
        // back into the slab, rows < N0 (all of this group's reads of the slab are done)
#pragma unroll
        for (int j = 0; j < Li::J; ++j) {
          const int b = q + NQ0 * j;
          if (act && ((Li::NB % NQ0 == 0) || b < Li::NB)) {
#pragma unroll
            for (int m = 0; m < Li::R / 2; ++m) lds[(b + m * Li::NB) * L1 * TC + k1 * TC + c] = u[j][m];
          }
        }
        lds_barrier();
      }
    }
  }
  // axis-1 inverse: pencils (i0, c) along k1, in LDS
  slab_fft<T, L1, PID1, true, 0, N0, TC, NT, true, false>(lds, tw1, tid, along1);
  // store rows (i0, i1 < N1)
  for (int e = tid; e < N0 * N1 * TC; e += NT) {
    const int c = e % TC, i1 = (e / TC) % N1, i0 = e / (TC * N1);
    const int col = col0 + c;
    if (col < a.ncols) put<T, PASS_COL_INV>(&S[i0 * a.plane + (long long)i1 * a.pitch + col], lds[(i0 * L1 + i1) * TC + c]);
  }
}

// ----------------------------------------------------------------- P1
// Row of n2 = LC reals x (zero-padded to 2 LC): z[n] = x[2n] + i x[2n+1]
// (n < LC/2, zero above), Z = DFT_LC(z), then for k in [0, LC]
//   X[k] = (Z[k] + conj Z[LC-k]) / 2 - i e^{-i pi k / LC} (Z[k] - conj Z[LC-k]) / 2.
// A block transforms G groups of TR rows, one after the other, and requests
// every group's input first: a thread keeps G times the bytes in flight.
template <typename T, int LC, int PID, int TR, int NQ, int G = 1>
__global__ __launch_bounds__(TR* NQ) void k_row_r2c(RowArgs a) {
  constexpr int K = plan_len(LC, PID);
  constexpr int LP = row_pitch(LC);
  __shared__ cx<T> lds[TR * LP];
  const int tid = threadIdx.x;
  const int q = tid % NQ, c = tid / NQ;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  auto idx = [c](int e) { return c * LP + row_slot(e); };
  using F = FirstStage<LC, PID, false, NQ>;
  static_assert(F::R % 2 == 0, "forward plans start with an even radix");
  // every group's input is requested before the first group is transformed
  cx<T> raw[G][F::J][F::R / 2];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = ((int)blockIdx.x * G + g) * TR + c;
    const bool rok = row < a.nrows;
    const void* src = a.items ? a.items[blockIdx.y].rho : a.in[blockIdx.y];
    const cx<T>* in = reinterpret_cast<const cx<T>*>(src) + (long long)row * (LC / 2);
    issue_fence();
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
      const int b = q + NQ * j;
      const bool ok = rok && ((F::NB % NQ == 0) || b < F::NB);
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) raw[g][j][r] = ok ? ld_once(&in[b + r * F::NB]) : czero<T>();
    }
  }
  issue_fence();
  const cx<T>* pp = tw + tw_size(LC, PID);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = ((int)blockIdx.x * G + g) * TR + c;
    const bool rok = row < a.nrows;
    if (g > 0) lds_barrier();
    cx<T> v[F::J][F::R];
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
#pragma unroll
      for (int r = 0; r < F::R / 2; ++r) v[j][r] = raw[g][j][r];
      dft_half_in<F::R, false, T>(v[j]);  // the upper half of z is the zero padding
    }
    if constexpr (K == 1) {
      write_first_outputs<T, F::R, F::J, F::NB, NQ>(lds, v, q, idx);
    } else {
      write_first_outputs<T, F::R, F::J, F::NB, NQ>(lds, v, q, idx);
      lds_barrier();
      lds_stages<T, LC, PID, false, 1, K - 1, NQ, false>(lds, tw, q, idx);
      using Ls = LastStage<LC, PID, false, NQ>;
      cx<T> w[Ls::J][Ls::R];
      lds_last_stage<T, LC, PID, false, NQ, false>(lds, tw, q, idx, w);
      lds_barrier();
#pragma unroll
      for (int j = 0; j < Ls::J; ++j) {
        const int b = q + NQ * j;
        if ((Ls::NB % NQ == 0) || b < Ls::NB) {
#pragma unroll
          for (int m = 0; m < Ls::R; ++m) lds[idx(b + m * Ls::NB)] = w[j][m];
        }
      }
    }
    lds_barrier();
    if (rok) {
      const int i0 = row / a.n1, i1 = row - i0 * a.n1;
      void* dst = a.items ? a.items[blockIdx.y].work : a.out[blockIdx.y];
      cx<T>* out = reinterpret_cast<cx<T>*>(dst) + (long long)i0 * a.s_i0_stride + (long long)i1 * a.pitch;
      constexpr int JO = (LC + 1 + NQ - 1) / NQ;
#pragma unroll
      for (int j = 0; j < JO; ++j) {
        const int k = q + NQ * j;
        if (k <= LC) {
          const cx<T> A = lds[idx(k == LC ? 0 : k)];
          const cx<T> B = conjg(lds[idx(k == 0 ? 0 : LC - k)]);
          const cx<T> E = {T(0.5) * (A.x + B.x), T(0.5) * (A.y + B.y)};
          const cx<T> D = {T(0.5) * (A.x - B.x), T(0.5) * (A.y - B.y)};
          const cx<T> U = cmul(pp[k], D);
          put<T, PASS_ROW_FWD>(&out[k], cx<T>{E.x + U.y, E.y - U.x});
        }
      }
    }
  }
}

// ----------------------------------------------------------------- P5
// From X[k], k in [0, LC] (half spectrum of a real row of length 2 LC):
//   Y[n] = (X[n] + conj X[LC-n]) + i e^{+i pi n / LC} (X[n] - conj X[LC-n]),
//   z = inverse DFT_LC(Y), x[2n] = Re z[n], x[2n+1] = Im z[n]; keep n < LC/2.
// G groups of TR rows per block, every group's input requested first, as in P1.
template <typename T, int LC, int PID, int TR, int NQ, int G = 1>
__global__ __launch_bounds__(TR* NQ) void k_row_c2r(RowArgs a) {
  constexpr int K = plan_len(LC, PID);
  constexpr int LP = row_pitch(LC);
  __shared__ cx<T> lds[TR * LP];
  const int tid = threadIdx.x;
  const int q = tid % NQ, c = tid / NQ;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  auto idx = [c](int e) { return c * LP + row_slot(e); };
  constexpr int JI = (LC + 1 + NQ - 1) / NQ;
  cx<T> raw[G][JI];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = ((int)blockIdx.x * G + g) * TR + c;
    const bool rok = row < a.nrows;
    const int i0 = row / a.n1, i1 = row - i0 * a.n1;
    const void* src = a.items ? a.items[blockIdx.y].work : a.in[blockIdx.y];
    const cx<T>* in = reinterpret_cast<const cx<T>*>(src) + (long long)i0 * a.s_i0_stride + (long long)i1 * a.pitch;
    issue_fence();
#pragma unroll
    for (int j = 0; j < JI; ++j) {
      const int k = q + NQ * j;
      raw[g][j] = (rok && k <= LC) ? ld_once(&in[k]) : czero<T>();
    }
  }
  issue_fence();
  const cx<T>* pp = tw + tw_size(LC, PID);
  using F = FirstStage<LC, PID, true, NQ>;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = ((int)blockIdx.x * G + g) * TR + c;
    const bool rok = row < a.nrows;
    if (g > 0) lds_barrier();
#pragma unroll
    for (int j = 0; j < JI; ++j) {
      const int k = q + NQ * j;
      if (k <= LC) lds[idx(k)] = raw[g][j];
    }
    lds_barrier();
    cx<T> v[F::J][F::R];
#pragma unroll
    for (int j = 0; j < F::J; ++j) {
      const int b = q + NQ * j;
      if ((F::NB % NQ == 0) || b < F::NB) {
#pragma unroll
        for (int r = 0; r < F::R; ++r) {
          const int n = b + r * F::NB;
          const cx<T> X1 = lds[idx(n)];
          const cx<T> X2 = conjg(lds[idx(LC - n)]);
          const cx<T> A = cadd(X1, X2);
          const cx<T> B = cmulc(csub(X1, X2), pp[n]);
          v[j][r] = {A.x - B.y, A.y + B.x};
        }
        if constexpr (K == 1)
          dft_half_out<F::R, true, T>(v[j]);  // only the first half of z is kept
        else
          Dft<F::R, true, T>::run(v[j]);
      }
    }
    void* dst = a.items ? a.items[blockIdx.y].phi : a.out[blockIdx.y];
    cx<T>* out = reinterpret_cast<cx<T>*>(dst) + (long long)row * (LC / 2);
    if constexpr (K == 1) {
      static_assert(F::R % 2 == 0, "inverse plans end with an even radix");
      if (rok) {
#pragma unroll
        for (int j = 0; j < F::J; ++j) {
          const int b = q + NQ * j;
          if ((F::NB % NQ == 0) || b < F::NB) {
#pragma unroll
            for (int m = 0; m < F::R / 2; ++m) put<T, PASS_ROW_INV>(&out[b + m * F::NB], v[j][m]);
          }
        }
      }
    } else {
      lds_barrier();
      write_first_outputs<T, F::R, F::J, F::NB, NQ>(lds, v, q, idx);
      lds_barrier();
      lds_stages<T, LC, PID, true, 1, K - 1, NQ, true>(lds, tw, q, idx);
      using Li = LastStage<LC, PID, true, NQ>;
      static_assert(Li::R % 2 == 0, "inverse plans end with an even radix");
      cx<T> u[Li::J][Li::R];
      lds_last_stage<T, LC, PID, true, NQ, true, false, true>(lds, tw, q, idx, u);
      if (rok) {
#pragma unroll
        for (int j = 0; j < Li::J; ++j) {
          const int b = q + NQ * j;
          if ((Li::NB % NQ == 0) || b < Li::NB) {
#pragma unroll
            for (int m = 0; m < Li::R / 2; ++m) put<T, PASS_ROW_INV>(&out[b + m * Li::NB], u[j][m]);
          }
        }
      }
    }
  }
}

}  // namespace fsp
