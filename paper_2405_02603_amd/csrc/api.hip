// api.hip -- plans, buffers, precompute driver and the C ABI declared in fsp.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "fft_core.hpp"
#include "fsp.h"
#include "internal.hpp"
#include "solve_launch.hpp"

namespace fsp {
hipError_t solve_f32(const SolveGeom& g, int first, int last, hipStream_t s);
hipError_t solve_f64(const SolveGeom& g, int first, int last, hipStream_t s);
hipError_t greens_he_kernel(double* K, const int n[3], const double h[3], double g0, hipStream_t s);
hipError_t greens_he_grad_kernel(double* D, const int n[3], const double h[3], int axis, hipStream_t s);
hipError_t greens_vico_spectrum(double* G, const int samples[3], const double f[3], double L, bool fft_order,
                                hipStream_t s);
hipError_t greens_contract_axis(const double* X, double* Y, const double* packed, int period,
                                const long long dims[3], int axis, int nout, hipStream_t s);
void greens_pack_contract(std::vector<double>& out, const std::vector<double>& ce, const std::vector<double>* co,
                          int nout, int kin, int period);
hipError_t greens_fold_periodic(const double* X, double* Y, const int n[3], int periodic, hipStream_t s);
hipError_t greens_store_octant(const double* G, void* out, bool f64, const int n[3], int tile, double scale,
                               hipStream_t s);
int conv_tile_f32(int L);
int conv_tile_f64(int L);
}  // namespace fsp

namespace {

thread_local std::string g_err;

fsp_status fail(fsp_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

fsp_status fail_hip(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return FSP_ERR_DEVICE;
}

bool supported_edge(int n) {
  switch (n) {
    case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
    case 128: case 192: case 256: case 384: case 512:
      return true;
    default:
      return false;
  }
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// exp(-2 pi i t / d) in long double, rounded once
void cis_neg(long long t, long long d, long double* c, long double* s) {
  const long double pi = 3.141592653589793238462643383279502884L;
  t %= d;
  const long double a = 2.0L * pi * (long double)t / (long double)d;
  *c = cosl(a);
  *s = -sinl(a);
}

template <typename T>
void push_c(std::vector<char>& buf, long double re, long double im) {
  T v[2] = {(T)re, (T)im};
  const char* p = reinterpret_cast<const char*>(v);
  buf.insert(buf.end(), p, p + sizeof(v));
}

// Twiddles of one pencil length: forward order then reversed order (fft_core.hpp layout):
// per stage s >= 1 and k in [0, NS): w^(p k) for p = 1, 2, 4, 8, 16, 3, w = exp(-2 pi i / (NS R)).
template <typename T>
void append_twiddles(std::vector<char>& buf, int L, int pid) {
  for (int rev = 0; rev < 2; ++rev) {
    const int K = fsp::plan_len(L, pid);
    for (int s = 1; s < K; ++s) {
      const int R = fsp::plan_radix(L, pid, rev != 0, s);
      const int NS = fsp::plan_ns(L, pid, rev != 0, s);
      for (int k = 0; k < NS; ++k)
        for (int e = 0; e < fsp::TW_PER_K; ++e) {
          long double c, sn;
          cis_neg((long long)k * fsp::tw_power(e), (long long)NS * R, &c, &sn);
          push_c<T>(buf, c, sn);
        }
    }
  }
}

// Complete table of one plan (fsp::twf_stage_off order): w^(r k) for each stage.
template <typename T>
void append_full_twiddles(std::vector<char>& buf, int L, int pid) {
  for (int rev = 0; rev < 2; ++rev) {
    for (int s = 1; s < fsp::plan_len(L, pid); ++s) {
      const int R = fsp::plan_radix(L, pid, rev != 0, s);
      const int NS = fsp::plan_ns(L, pid, rev != 0, s);
      for (int k = 0; k < NS; ++k)
        for (int r = 1; r < R; ++r) {
          long double c, sn;
          cis_neg((long long)k * r, (long long)NS * R, &c, &sn);
          push_c<T>(buf, c, sn);
        }
    }
  }
}

// cos and sin of pi j / half for j in [0, 2 half): every matrix entry below
// has an angle pi t / half with t an exact integer reduced mod 2 half, so one
// long-double table per matrix replaces a trigonometric call per entry.
struct TrigTable {
  std::vector<long double> c, s;
  explicit TrigTable(int half) : c(2 * (size_t)half), s(2 * (size_t)half) {
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < 2 * half; ++j) {
      c[j] = cosl(pi * (long double)j / (long double)half);
      s[j] = sinl(pi * (long double)j / (long double)half);
    }
  }
};

// DCT-I rows m < nout of a length period + 1 transform, C[m][l] = w_l cos(pi l m / period)
// (w = 1 at l = 0 and l = period, else 2), folded for the contraction kernel,
// which pairs inputs l and period - l: Ce[r][l] = w_l cos(pi l (2r) / period), l in [0, period / 2], acts
// on the sums X[l] + X[period - l] (X[period / 2] alone at l = period / 2), and
// Co[r][l] = w_l cos(pi l (2r + 1) / period), l in [0, period / 2), on the
// differences X[l] - X[period - l]; the cosines of l and period - l agree up to
// (-1)^m, so this is the whole sum with half the products.
void dct1_fold_matrices(std::vector<double>& Ce, std::vector<double>& Co, int nout, int period) {
  const int half = period / 2;
  const TrigTable tt(period);
  const int re = (nout + 1) / 2, ro = nout / 2;
  Ce.assign((size_t)re * (half + 1), 0.0);
  Co.assign((size_t)ro * half, 0.0);
  for (int m = 0; m < nout; ++m) {
    const bool even = m % 2 == 0;
    const int k = even ? half + 1 : half;
    double* row = even ? &Ce[(size_t)(m / 2) * k] : &Co[(size_t)(m / 2) * k];
    // angle index l m mod 2 period, stepped; w c is exact in double for w = 1, 2
    long long t = 0;
    for (int l = 0; l < k; ++l) {
      row[l] = (l == 0 ? 1.0 : 2.0) * (double)tt.c[t];
      t += m;
      if (t >= 2LL * period) t %= 2LL * period;
    }
  }
}

// Octant rows of the inverse DFT of real, even data on a grid of s = 4n points:
// C[m][l] = cos(2 pi l m / s), m <= n.
void dft_cos_matrix(std::vector<double>& C, int nout, int s) {
  const TrigTable tt(s / 2);  // 2 pi t / s = pi t / (s / 2), s even
  C.resize((size_t)nout * s);
  for (int m = 0; m < nout; ++m)
    for (int l = 0; l < s; ++l) {
      const long long t = ((long long)l * m) % s;
      C[(size_t)m * s + l] = (double)tt.c[t];
    }
}

// Rows m < nout of the sine sum that turns the (period+1) non-negative
// frequency samples l of an even spectrum into the derivative of its inverse
// transform along that axis: C[m][l] = 2 (-kfac l) sin(pi l m / period)
// (the end samples carry sin = 0).
void sine_k_matrix(std::vector<double>& C, int nout, int period, double kfac) {
  const int nin = period + 1;
  const TrigTable tt(period);
  C.assign((size_t)nout * nin, 0.0);
  for (int m = 0; m < nout; ++m)
    for (int l = 1; l < period; ++l) {
      const long long t = ((long long)l * m) % (2LL * period);
      C[(size_t)m * nin + l] = (double)(-2.0L * kfac * l * tt.s[t]);
    }
}

// The same on the full grid of s samples in FFT order (signed frequency
// l' = l or l - s): C[m][l] = -(kfac l') sin(2 pi l m / s).
void dft_sin_k_matrix(std::vector<double>& C, int nout, int s, double kfac) {
  const TrigTable tt(s / 2);
  C.resize((size_t)nout * s);
  for (int m = 0; m < nout; ++m)
    for (int l = 0; l < s; ++l) {
      const long long t = ((long long)l * m) % s;
      const long long ls = l < s / 2 ? l : l - s;
      C[(size_t)m * s + l] = (double)(-(long double)kfac * ls * tt.s[t]);
    }
}

// Sine transform of an odd table on [0, n] (0 at both ends), the transform of
// its odd extension to 2n points up to a factor -i: C[k][m] = 2 sin(pi k m / n).
void dst1_matrix(std::vector<double>& C, int n) {
  const TrigTable tt(n);
  C.assign((size_t)(n + 1) * (n + 1), 0.0);
  for (int k = 0; k <= n; ++k)
    for (int m = 1; m < n; ++m) {
      const long long t = ((long long)k * m) % (2LL * n);
      C[(size_t)k * (n + 1) + m] = (double)(2.0L * tt.s[t]);
    }
}

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  hipError_t enter(int dev) {
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != dev) {
      e = hipSetDevice(dev);
      if (e != hipSuccess) return e;
      changed = true;
    }
    return hipSuccess;
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

// Workspace of fsp_solve_static: one array per GPU (every device that loads
// this code object holds its own copy until the process ends).  In host code
// the name stands for no device address: the address of a device's copy comes
// from hipGetSymbolAddress with that device current (scratch_address).
static __device__ __align__(256) unsigned char scratch[FSP_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of its copy of scratch

// The device address of `scratch` on device dev, which must be current.
// Looked up once per device and kept.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return hipSuccess;
}

}  // namespace

struct fsp_plan_s {
  fsp_plan_desc d{};
  int n[3]{};
  double h[3]{};
  double V = 0, L = 0, alpha = 1.1, g0 = 0;
  int rb = 4;     // bytes per real
  int pitch = 0;  // complex elements per S row
  int gtile = 0;  // column tile of the blocked Green's octant
  long long plane = 0;  // complex elements between S planes i0
  int chunks = 1;       // column chunks for passes 1-3
  int gather_min = fsp::CONV_GATHER_MIN_BLOCKS;  // axis-0 grid size from which the lone column is gathered
  size_t tw_row_off[fsp::NUM_PLANS]{}, tw_c1_off[fsp::NUM_PLANS]{}, tw_c0_off[fsp::NUM_PLANS]{}, oct_off = 0;
  bool grad = false;        // FSP_WANT_GRAD: derivative octants and three more spectra
  int periodic = 0;         // bit a: axis a periodic (its kernel table folded to the nearest image)
  size_t grad_off[3]{};     // offsets of the derivative octants in the Green's buffer
  int grad_p3 = -1;         // axis-0 variant of the gradient solve (-1: from the schedule)
  size_t work1_bytes = 0;   // one workspace S (the gradient's other spectra follow it)
  int var[5]{};  // schedule variant of each pass
  int sep[5]{};  // the fastest separate-pass variants found by fsp_autotune (whatever schedule it kept)
  size_t ghat_bytes = 0, work_bytes = 0, pre_bytes = 0;
  std::vector<char> tw_host;      // image of [0, oct_off) of the Green's buffer
  std::vector<double> cmat_host;  // cosine matrices used by the precompute
  void* ghat = nullptr;
  void* work = nullptr;
  bool own_ghat = false, own_work = false;
  const void* ghat_read = nullptr;  // buffer the solves read (own or shared)
  bool bound = false, ready = false;
  int device = -1;
};

namespace {

template <typename T>
void build_twiddles(fsp_plan_s* p) {
  std::vector<char>& b = p->tw_host;
  b.clear();
  for (int pid = 0; pid < fsp::NUM_PLANS; ++pid) {
    p->tw_row_off[pid] = b.size();
    append_twiddles<T>(b, p->n[2], pid);
    for (int k = 0; k <= p->n[2]; ++k) {  // split table exp(-i pi k / n2)
      long double c, s;
      cis_neg(k, 2LL * p->n[2], &c, &s);
      push_c<T>(b, c, s);
    }
    b.resize(align_up(b.size(), 256), 0);
  }
  for (int pid = 0; pid < fsp::NUM_PLANS; ++pid) {
    p->tw_c1_off[pid] = b.size();
    append_twiddles<T>(b, 2 * p->n[1], pid);
    b.resize(align_up(b.size(), 256), 0);
  }
  for (int pid = 0; pid < fsp::NUM_PLANS; ++pid) {
    p->tw_c0_off[pid] = b.size();
    append_twiddles<T>(b, 2 * p->n[0], pid);
    append_full_twiddles<T>(b, 2 * p->n[0], pid);  // read by the axis-0 kernel's LDS-table variant
    b.resize(align_up(b.size(), 256), 0);
  }
  p->oct_off = b.size();
}

// Schedules found by the autotuner, per (n0, n1, n2, precision); new plans of a
// tuned shape start with the tuned schedule.
struct TuneKey {
  int n0, n1, n2, prec;
  bool operator<(const TuneKey& o) const {
    return std::tie(n0, n1, n2, prec) < std::tie(o.n0, o.n1, o.n2, o.prec);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::array<int, 11>> g_tuned;  // schedule, the gradient's axis-0 variant, separate variants

double model_bytes(const fsp_plan_s* p) {
  // P1 reads rho, writes (n2+1) n1 n0 complex; P2 reads that, writes 2 n1 (n2+1) n0;
  // P3 reads/writes 2 n1 (n2+1) n0 and reads the octant; P4 mirrors P2, P5 mirrors P1.
  // The fused slab (passes 1-3) reads and writes the (n2+1) n1 n0 rows once; a
  // plane pair reads rho and writes S (0-1), or reads S and writes phi (3-4).
  const double n0 = p->n[0], n1 = p->n[1], n2 = p->n[2], s = p->rb;
  const double real_grid = n0 * n1 * n2;
  const double half1 = n0 * n1 * (n2 + 1) * 2;      // reals in (n2+1) n1 n0 complex
  const double half2 = n0 * 2 * n1 * (n2 + 1) * 2;  // reals in 2 n1 (n2+1) n0 complex
  const double octant = (n0 + 1) * (n1 + 1) * (n2 + 1);
  if (p->var[1] == fsp::FUSED) return (2 * real_grid + 4 * half1 + octant) * s;
  const double fwd = p->var[0] == fsp::PLANE ? real_grid + half2 : real_grid + 2 * half1 + half2;
  const double inv = p->var[3] == fsp::PLANE ? real_grid + half2 : real_grid + 2 * half1 + half2;
  return (fwd + 2 * half2 + octant + inv) * s;
}

}  // namespace

extern "C" {

const char* fsp_status_str(fsp_status s) {
  switch (s) {
    case FSP_OK: return "FSP_OK";
    case FSP_ERR_INVALID_ARG: return "FSP_ERR_INVALID_ARG";
    case FSP_ERR_UNSUPPORTED_SIZE: return "FSP_ERR_UNSUPPORTED_SIZE";
    case FSP_ERR_BOX_ASPECT: return "FSP_ERR_BOX_ASPECT";
    case FSP_ERR_OUT_OF_MEMORY: return "FSP_ERR_OUT_OF_MEMORY";
    case FSP_ERR_NOT_READY: return "FSP_ERR_NOT_READY";
    case FSP_ERR_DEVICE: return "FSP_ERR_DEVICE";
  }
  return "FSP_ERR_UNKNOWN";
}

const char* fsp_last_error(void) { return g_err.c_str(); }

const char* fsp_version(void) { return "fsp 0.1.0 gfx950"; }

// Doubles in the matrix image of one axis contraction (fsp::greens_pack_contract):
// nout rows over kin inputs, folded when period > 0.
static size_t image_elems(int nout, int kin, int period) {
  const bool fold = period > 0;
  const size_t re = fold ? (nout + 1) / 2 : nout, ro = fold ? nout / 2 : 0;
  const size_t ke = fold ? period / 2 + 1 : kin;
  return (ke + 15) / 16 * ((re + 15) / 16 + (ro + 15) / 16) * 256;
}

fsp_status fsp_plan_create(const fsp_plan_desc* desc, fsp_plan* out) {
  if (!desc || !out) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_create: NULL argument");
  *out = nullptr;
  const fsp_plan_desc& d = *desc;
  if (d.greens < FSP_HOCKNEY || d.greens > FSP_VICO_DCT)
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_create: unknown greens value");
  if (d.prec != FSP_F32 && d.prec != FSP_F64) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_create: unknown prec value");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(d.lo[a]) || !std::isfinite(d.hi[a]) || !(d.hi[a] > d.lo[a]))
      return fail(FSP_ERR_INVALID_ARG, "fsp_plan_create: box needs finite lo < hi on every axis");
    if (!supported_edge(d.n[a]))
      return fail(FSP_ERR_UNSUPPORTED_SIZE,
                  "fsp_plan_create: n[" + std::to_string(a) + "] = " + std::to_string(d.n[a]) +
                      " is not 2^a or 3*2^a in [8, 512]");
    if (d.greens == FSP_VICO && d.n[a] > 256)
      return fail(FSP_ERR_UNSUPPORTED_SIZE, "fsp_plan_create: the (4N)^3 Vico-Greengard route is limited to n <= 256");
  }
  const unsigned periodic_bits = FSP_PERIODIC_0 | FSP_PERIODIC_1 | FSP_PERIODIC_2;
  if (d.flags & ~((unsigned)FSP_WANT_GRAD | periodic_bits))
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_create: unknown flags");
  if ((d.flags & FSP_WANT_GRAD) && (d.flags & periodic_bits))
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_create: periodic axes are not supported with FSP_WANT_GRAD");
  const double alpha = d.alpha == 0.0 ? 1.1 : d.alpha;
  if (!std::isfinite(alpha) || !(alpha > 1.0))
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_create: alpha must exceed 1 (0 selects 1.1)");
  fsp_plan_s* p = new (std::nothrow) fsp_plan_s();
  if (!p) return fail(FSP_ERR_OUT_OF_MEMORY, "fsp_plan_create: host allocation failed");
  p->d = d;
  p->alpha = alpha;
  p->periodic = ((d.flags & FSP_PERIODIC_0) ? 1 : 0) | ((d.flags & FSP_PERIODIC_1) ? 2 : 0) |
                ((d.flags & FSP_PERIODIC_2) ? 4 : 0);
  p->g0 = std::isnan(d.g0) ? 1.0 / (4.0 * M_PI) : d.g0;
  double diag2 = 0, minlen = 1e300;
  for (int a = 0; a < 3; ++a) {
    p->n[a] = d.n[a];
    const double len = d.hi[a] - d.lo[a];
    p->h[a] = len / d.n[a];
    diag2 += len * len;
    minlen = std::min(minlen, len);
  }
  p->V = p->h[0] * p->h[1] * p->h[2];
  p->L = alpha * std::sqrt(diag2);
  if (d.greens != FSP_HOCKNEY && p->L > 3.0 * minlen) {
    delete p;
    return fail(FSP_ERR_BOX_ASPECT,
                "fsp_plan_create: Vico-Greengard window alpha*|diag| exceeds 3 x the shortest box edge");
  }
  p->rb = d.prec == FSP_F64 ? 8 : 4;
  const int cb = 2 * p->rb;
  p->pitch = (int)align_up((size_t)p->n[2] + 1, 128 / cb);
  if (d.prec == FSP_F64)
    build_twiddles<double>(p);
  else
    build_twiddles<float>(p);
  p->gtile = d.prec == FSP_F64 ? fsp::conv_tile_f64(2 * p->n[0]) : fsp::conv_tile_f32(2 * p->n[0]);
  {
    const size_t tiles = (p->n[2] + 1 + p->gtile - 1) / p->gtile;
    const size_t oct = align_up((size_t)(p->n[1] + 1) * tiles * (p->n[0] + 1) * p->gtile * p->rb, 256);
    p->grad = (d.flags & FSP_WANT_GRAD) != 0;
    for (int a = 0; a < 3; ++a) p->grad_off[a] = p->grad ? p->oct_off + (a + 1) * oct : 0;
    p->ghat_bytes = p->oct_off + (p->grad ? 4 : 1) * oct;
  }
  {
    long long pad = 0;
    if (const char* e = std::getenv("FSP_PLANE_PAD")) pad = std::atoll(e);
    p->plane = 2LL * p->n[1] * p->pitch + pad;
    if (const char* e = std::getenv("FSP_CHUNKS")) p->chunks = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("FSP_CONV_GATHER_MIN")) p->gather_min = std::max(0, std::atoi(e));
  }
  p->work1_bytes = align_up((size_t)p->n[0] * p->plane * cb, 256);
  p->work_bytes = (p->grad ? 4 : 1) * p->work1_bytes;  // the gradient: S and three more spectra
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(TuneKey{p->n[0], p->n[1], p->n[2], d.prec});
    if (it != g_tuned.end()) {
      for (int i = 0; i < 5; ++i) p->var[i] = it->second[i];
      p->grad_p3 = it->second[5];
      for (int i = 0; i < 5; ++i) p->sep[i] = it->second[6 + i];
    }
  }
  // the column kernels address a pencil's rows with 32-bit element offsets
  if ((long long)(2 * p->n[0]) * p->plane >= (1LL << 31)) {
    delete p;
    return fail(FSP_ERR_UNSUPPORTED_SIZE, "fsp_plan_create: workspace plane offsets exceed 32 bits");
  }
  // transient float64 precompute buffers (two ping-pong arrays) + cosine matrices
  const size_t n0 = p->n[0], n1 = p->n[1], n2 = p->n[2];
  size_t a = 0, b = 0;
  if (d.greens == FSP_HOCKNEY) {
    a = b = (n0 + 1) * (n1 + 1) * (n2 + 1);
  } else if (d.greens == FSP_VICO_DCT) {
    a = (2 * n0 + 1) * (2 * n1 + 1) * (2 * n2 + 1);
    b = (2 * n1 + 1) * (2 * n2 + 1) * (n0 + 1);
  } else {
    a = 64 * n0 * n1 * n2;
    b = 16 * n1 * n2 * (n0 + 1);
  }
  size_t cm = 0;  // matrix images of every component (the same sizes component_matrices builds)
  for (int comp = 0; comp < (p->grad ? 4 : 1); ++comp)
    for (int ax = 0; ax < 3; ++ax) {
      const int m = p->n[ax];
      const bool deriv = comp == ax + 1;
      if (d.greens == FSP_VICO_DCT)
        cm += deriv ? image_elems(m + 1, 2 * m + 1, 0) : image_elems(m + 1, 2 * m + 1, 2 * m);
      else if (d.greens == FSP_VICO)
        cm += image_elems(m + 1, 4 * m, 0);
      cm += deriv ? image_elems(m + 1, m + 1, 0) : image_elems(m + 1, m + 1, m);
    }
  p->pre_bytes = align_up(a * 8, 256) + align_up(b * 8, 256) + align_up(cm * 8, 256);
  *out = p;
  g_err.clear();
  return FSP_OK;
}

fsp_status fsp_plan_bytes(fsp_plan p, size_t* ghat_bytes, size_t* work_bytes) {
  if (!p) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_bytes: NULL plan");
  if (ghat_bytes) *ghat_bytes = p->ghat_bytes;
  if (work_bytes) *work_bytes = p->work_bytes;
  return FSP_OK;
}

fsp_status fsp_plan_precompute_bytes(fsp_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_precompute_bytes: NULL argument");
  *bytes = p->pre_bytes;
  return FSP_OK;
}

fsp_status fsp_plan_model_bytes(fsp_plan p, double* bytes) {
  if (!p || !bytes) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_model_bytes: NULL argument");
  *bytes = model_bytes(p);
  return FSP_OK;
}

fsp_status fsp_plan_ghat_layout(fsp_plan p, size_t* octant_offset, int* tile) {
  if (!p) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_ghat_layout: NULL plan");
  if (octant_offset) *octant_offset = p->oct_off;
  if (tile) *tile = p->gtile;
  return FSP_OK;
}

fsp_status fsp_plan_octant_offset(fsp_plan p, int component, size_t* offset) {
  if (!p || !offset) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_octant_offset: NULL argument");
  if (component < 0 || component > 3 || (component > 0 && !p->grad))
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_octant_offset: component must be 0, or 1-3 on a plan with FSP_WANT_GRAD");
  *offset = component == 0 ? p->oct_off : p->grad_off[component - 1];
  return FSP_OK;
}

static void release_buffers(fsp_plan_s* p) {
  if (p->own_ghat && p->ghat) (void)hipFree(p->ghat);
  if (p->own_work && p->work) (void)hipFree(p->work);
  p->ghat = p->work = nullptr;
  p->own_ghat = p->own_work = false;
  p->ghat_read = nullptr;
  p->bound = p->ready = false;
}

fsp_status fsp_plan_bind(fsp_plan p, void* ghat_dev, void* work_dev) {
  if (!p) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_bind: NULL plan");
  if ((reinterpret_cast<uintptr_t>(ghat_dev) | reinterpret_cast<uintptr_t>(work_dev)) & 255u)
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_bind: buffers must be 256-byte aligned");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "fsp_plan_bind: hipGetDevice");
  release_buffers(p);
  p->device = dev;
  if (p->work1_bytes <= FSP_STATIC_SCRATCH_BYTES) {
    // set-up time: find this device's fsp_solve_static workspace now, so that
    // call does no lookup later (a failure here is retried, and reported, there)
    void* ws = nullptr;
    if (scratch_address(dev, &ws) != hipSuccess) (void)hipGetLastError();
  }
  if (ghat_dev) {
    p->ghat = ghat_dev;
  } else {
    e = hipMalloc(&p->ghat, p->ghat_bytes);
    if (e != hipSuccess) {
      p->ghat = nullptr;
      (void)hipGetLastError();
      return fail(FSP_ERR_OUT_OF_MEMORY, "fsp_plan_bind: hipMalloc of the Green's buffer failed");
    }
    p->own_ghat = true;
  }
  if (work_dev) {
    p->work = work_dev;
  } else {
    e = hipMalloc(&p->work, p->work_bytes);
    if (e != hipSuccess) {
      p->work = nullptr;
      (void)hipGetLastError();
      release_buffers(p);
      return fail(FSP_ERR_OUT_OF_MEMORY, "fsp_plan_bind: hipMalloc of the workspace failed");
    }
    p->own_work = true;
  }
  p->ghat_read = p->ghat;
  p->bound = true;
  return FSP_OK;
}

fsp_status fsp_plan_share_ghat(fsp_plan dst, fsp_plan src) {
  if (!dst || !src) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_share_ghat: NULL plan");
  const fsp_plan_desc &a = dst->d, &b = src->d;
  bool same = a.greens == b.greens && a.prec == b.prec && dst->alpha == src->alpha && dst->g0 == src->g0 &&
              dst->periodic == src->periodic;
  for (int i = 0; i < 3; ++i) same = same && a.n[i] == b.n[i] && a.lo[i] == b.lo[i] && a.hi[i] == b.hi[i];
  if (!same) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_share_ghat: plans differ in kernel, grid, box or precision");
  if (dst->grad && !src->grad)
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_share_ghat: the destination needs derivative tables the source lacks");
  if (!src->ready) return fail(FSP_ERR_NOT_READY, "fsp_plan_share_ghat: source plan has no precomputed transform");
  if (!dst->bound) return fail(FSP_ERR_NOT_READY, "fsp_plan_share_ghat: bind the destination plan first");
  if (src->device != dst->device) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_share_ghat: plans on different devices");
  dst->ghat_read = src->ghat_read;
  dst->ready = true;
  return FSP_OK;
}

// Matrix images depend only on the transform's sizes (and, for the derivative
// forms, on the frequency step kfac), not on the plan: each is built once per
// process and shared.  The cache is cleared when it holds many images (plans
// with FSP_WANT_GRAD on ever-changing boxes); images in use stay alive.
extern "C++" {
using ImagePtr = std::shared_ptr<const std::vector<double>>;
std::mutex g_image_mu;
std::map<std::tuple<int, int, int, int, uint64_t>, ImagePtr> g_images;

template <class Build>
ImagePtr cached_image(int kind, int nout, int kin, int period, double kfac, Build build) {
  uint64_t bits = 0;
  std::memcpy(&bits, &kfac, sizeof bits);
  const auto key = std::make_tuple(kind, nout, kin, period, bits);
  {
    std::lock_guard<std::mutex> lk(g_image_mu);
    auto it = g_images.find(key);
    if (it != g_images.end()) return it->second;
  }
  auto img = std::make_shared<std::vector<double>>();
  build(*img);
  std::lock_guard<std::mutex> lk(g_image_mu);
  if (g_images.size() >= 256) g_images.clear();
  g_images[key] = img;
  return img;
}
}  // extern "C++"

// One axis contraction of a precompute: the offset of its matrix image
// (fsp::greens_pack_contract) and, for a DCT-I run folded, its period.
struct AxisOp {
  size_t off = 0;
  int period = 0;  // > 0: folded DCT-I of this period
};

// Matrices of one component's precompute, in the order they are used: for
// Vico-Greengard the three spectrum -> kernel contractions, then the three
// kernel -> transform contractions.  Component 0 is the potential; component
// 1 + a the derivative along axis a, whose axis-a matrices are the sine forms.
static void component_matrices(const fsp_plan_s* p, int comp, std::vector<double>& cm, std::vector<AxisOp>& ops) {
  const int* n = p->n;
  const int gk = p->d.greens;
  const int ax = comp - 1;
  enum { IMG_DCT1, IMG_SINE_K, IMG_DFT_COS, IMG_DFT_SIN_K, IMG_DST1 };
  auto push = [&](const ImagePtr& img, int period) {
    AxisOp op;
    op.period = period;
    op.off = cm.size();
    cm.insert(cm.end(), img->begin(), img->end());
    ops.push_back(op);
  };
  // a plain matrix of nout rows over kin inputs, or a DCT-I run folded
  auto add = [&](int kind, int nout, int kin, double kfac, void (*fill)(std::vector<double>&, int, int, double)) {
    push(cached_image(kind, nout, kin, 0, kfac,
                      [&](std::vector<double>& img) {
                        std::vector<double> c;
                        fill(c, nout, kin, kfac);
                        fsp::greens_pack_contract(img, c, nullptr, nout, kin, 0);
                      }),
         0);
  };
  auto add_dct1 = [&](int nout, int period) {
    push(cached_image(IMG_DCT1, nout, period + 1, period, 0.0,
                      [&](std::vector<double>& img) {
                        std::vector<double> ce, co;
                        dct1_fold_matrices(ce, co, nout, period);
                        fsp::greens_pack_contract(img, ce, &co, nout, period + 1, period);
                      }),
         period);
  };
  if (gk == FSP_VICO_DCT) {
    for (int a = 0; a < 3; ++a) {
      if (a == ax)
        add(IMG_SINE_K, n[a] + 1, 2 * n[a] + 1, M_PI / (2.0 * n[a] * p->h[a]),
            [](std::vector<double>& c, int nout, int kin, double kf) { sine_k_matrix(c, nout, kin - 1, kf); });
      else
        add_dct1(n[a] + 1, 2 * n[a]);
    }
  } else if (gk == FSP_VICO) {
    for (int a = 0; a < 3; ++a) {
      if (a == ax)
        add(IMG_DFT_SIN_K, n[a] + 1, 4 * n[a], 2.0 * M_PI / (4.0 * n[a] * p->h[a]),
            [](std::vector<double>& c, int nout, int kin, double kf) { dft_sin_k_matrix(c, nout, kin, kf); });
      else
        add(IMG_DFT_COS, n[a] + 1, 4 * n[a], 0.0,
            [](std::vector<double>& c, int nout, int kin, double) { dft_cos_matrix(c, nout, kin); });
    }
  }
  for (int a = 0; a < 3; ++a) {
    if (a == ax)
      add(IMG_DST1, n[a] + 1, n[a] + 1, 0.0, [](std::vector<double>& c, int, int kin, double) { dst1_matrix(c, kin - 1); });
    else
      add_dct1(n[a] + 1, n[a]);
  }
}

fsp_status fsp_precompute(fsp_plan p, void* stream) {
  if (!p) return fail(FSP_ERR_INVALID_ARG, "fsp_precompute: NULL plan");
  if (!p->bound) return fail(FSP_ERR_NOT_READY, "fsp_precompute: bind buffers first");
  DeviceGuard guard;
  hipError_t e = guard.enter(p->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_precompute: hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int* n = p->n;
  const int gk = p->d.greens;
  const int ncomp = p->grad ? 4 : 1;
  // all components' matrices, uploaded once (the host image outlives the copy)
  std::vector<double>& cm = p->cmat_host;
  cm.clear();
  std::vector<AxisOp> ops;
  for (int c = 0; c < ncomp; ++c) component_matrices(p, c, cm, ops);
  const size_t per_comp = ops.size() / ncomp;
  const size_t n0 = n[0], n1 = n[1], n2 = n[2];
  size_t a_elems, b_elems;
  if (gk == FSP_HOCKNEY) {
    a_elems = b_elems = (n0 + 1) * (n1 + 1) * (n2 + 1);
  } else if (gk == FSP_VICO_DCT) {
    a_elems = (2 * n0 + 1) * (2 * n1 + 1) * (2 * n2 + 1);
    b_elems = (2 * n1 + 1) * (2 * n2 + 1) * (n0 + 1);
  } else {
    a_elems = 64 * n0 * n1 * n2;
    b_elems = 16 * n1 * n2 * (n0 + 1);
  }
  double *A = nullptr, *B = nullptr, *C = nullptr;
  e = hipMallocAsync((void**)&A, a_elems * 8, s);
  if (e == hipSuccess) e = hipMallocAsync((void**)&B, b_elems * 8, s);
  if (e == hipSuccess) e = hipMallocAsync((void**)&C, cm.size() * 8, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (A) (void)hipFreeAsync(A, s);
    if (B) (void)hipFreeAsync(B, s);
    return fail(FSP_ERR_OUT_OF_MEMORY, "fsp_precompute: transient float64 buffers could not be allocated");
  }
  p->ready = false;
  e = hipMemcpyAsync(C, cm.data(), cm.size() * 8, hipMemcpyHostToDevice, s);
  for (int comp = 0; comp < ncomp && e == hipSuccess; ++comp) {
    size_t mi = comp * per_comp;
    long long dims[3];  // current layout dims, leading axis first
    double scale = p->V / (8.0 * n0 * n1 * n2);  // folds V and the 1/M^3 of the inverse transform
    double* X = A;
    double* Y = B;
    int axis = 0;
    auto contract = [&](int nout) {
      // axes in order 0, 1, 2: dims[axis] -> nout, layout order unchanged
      const AxisOp& op = ops[mi];
      if (e == hipSuccess)
        e = fsp::greens_contract_axis(X, Y, C + op.off, op.period, dims, axis, nout, s);
      ++mi;
      dims[axis] = nout;
      axis = (axis + 1) % 3;
      std::swap(X, Y);
    };
    if (gk == FSP_HOCKNEY) {
      if (comp == 0)
        e = fsp::greens_he_kernel(X, n, p->h, p->g0, s);
      else
        e = fsp::greens_he_grad_kernel(X, n, p->h, comp - 1, s);
      dims[0] = n0 + 1;
      dims[1] = n1 + 1;
      dims[2] = n2 + 1;
    } else {
      const bool full = gk == FSP_VICO;
      int samples[3];
      double f[3];
      for (int a = 0; a < 3; ++a) {
        samples[a] = full ? 4 * n[a] : 2 * n[a] + 1;
        f[a] = M_PI / (2.0 * n[a] * p->h[a]);  // k = 2 pi l / (4 n h)
      }
      e = fsp::greens_vico_spectrum(X, samples, f, p->L, full, s);
      dims[0] = samples[0];
      dims[1] = samples[1];
      dims[2] = samples[2];
      for (int a = 0; a < 3; ++a) contract(n[a] + 1);
      // inverse transform on the 4n grid: 1 / prod(4 n_d h_d) = 1 / (64 n0 n1 n2 V)
      scale /= 64.0 * n0 * n1 * n2 * p->V;
    }
    if (p->periodic && e == hipSuccess) {  // the kernel octant (in X) folded to the nearest image
      e = fsp::greens_fold_periodic(X, Y, n, p->periodic, s);
      std::swap(X, Y);
    }
    for (int a = 0; a < 3; ++a) contract(n[a] + 1);
    const size_t off = comp == 0 ? p->oct_off : p->grad_off[comp - 1];
    if (e == hipSuccess)
      e = fsp::greens_store_octant(X, static_cast<char*>(p->ghat) + off, p->d.prec == FSP_F64, n, p->gtile, scale, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(p->ghat, p->tw_host.data(), p->tw_host.size(), hipMemcpyHostToDevice, s);
  (void)hipFreeAsync(A, s);
  (void)hipFreeAsync(B, s);
  (void)hipFreeAsync(C, s);
  if (e != hipSuccess) return fail_hip(e, "fsp_precompute");
  p->ghat_read = p->ghat;
  p->ready = true;
  return FSP_OK;
}

// Shape fields shared by every item of a launch group (items filled by the caller).
static fsp::SolveGeom group_geom(const fsp_plan_s* p, const int* var);
static fsp::SolveGeom group_geom(const fsp_plan_s* p) { return group_geom(p, p->var); }

// Shape fields with an explicit schedule.
static fsp::SolveGeom group_geom(const fsp_plan_s* p, const int* var) {
  fsp::SolveGeom g{};
  g.items = 0;
  g.n0 = p->n[0];
  g.n1 = p->n[1];
  g.n2 = p->n[2];
  g.pitch = p->pitch;
  g.plane = p->plane;
  g.chunks = p->chunks;
  g.gather_min = p->gather_min;
  const char* gb = static_cast<const char*>(p->ghat_read);
  for (int i = 0; i < 5; ++i) g.var[i] = var[i];
  // the radix plan of a variant may differ between the precisions
  const bool f64 = p->d.prec == FSP_F64;
  const fsp::PlaneCfg pcf = f64 ? fsp::plane_cfg<double>(p->n[2]) : fsp::plane_cfg<float>(p->n[2]);
  const bool plane_fwd = var[0] == fsp::PLANE, plane_inv = var[3] == fsp::PLANE;
  auto row_pid = [&](int v) { return f64 ? fsp::row_cfg<double>(p->n[2], v).pid : fsp::row_cfg<float>(p->n[2], v).pid; };
  const int pr1 = plane_fwd ? pcf.pid : row_pid(var[0]);
  const int pr5 = plane_inv ? pcf.pid : row_pid(var[4]);
  const bool fused = var[1] == fsp::FUSED;
  auto col_pid = [&](int L, int v) { return f64 ? fsp::col_cfg<double>(L, v).pid : fsp::col_cfg<float>(L, v).pid; };
  const int pc2 = fused || plane_fwd ? 0 : col_pid(2 * p->n[1], var[1]);
  const int pc4 = fused || plane_inv ? 0 : col_pid(2 * p->n[1], var[3]);
  const int pc3 = fused ? 0
                  : f64 ? fsp::conv_cfg<double>(2 * p->n[0], var[2]).pid
                        : fsp::conv_cfg<float>(2 * p->n[0], var[2]).pid;
  for (int i = 0; i < 5; ++i) g.tw_row[i] = g.tw_c1[i] = nullptr;
  g.tw_row[0] = gb + p->tw_row_off[pr1];
  g.tw_row[4] = gb + p->tw_row_off[pr5];
  g.tw_c1[1] = gb + p->tw_c1_off[pc2];
  g.tw_c1[3] = gb + p->tw_c1_off[pc4];
  g.tw_c0 = gb + p->tw_c0_off[pc3];
  return g;
}

static void add_item(fsp::SolveGeom& g, const fsp_plan_s* p, const void* rho, void* phi) {
  const int i = g.items++;
  g.ghat[i] = static_cast<const char*>(p->ghat_read) + p->oct_off;
  g.work[i] = p->work;
  g.rho[i] = rho;
  g.phi[i] = phi;
}

// Same grid, precision and layout (schedules may differ).
static bool same_geometry(const fsp_plan_s* a, const fsp_plan_s* b) {
  return a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2] && a->d.prec == b->d.prec &&
         a->pitch == b->pitch && a->plane == b->plane && a->chunks == b->chunks && a->gather_min == b->gather_min;
}

static bool same_shape(const fsp_plan_s* a, const fsp_plan_s* b) {
  bool same = a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2] && a->d.prec == b->d.prec &&
              a->pitch == b->pitch && a->plane == b->plane && a->chunks == b->chunks &&
              a->gather_min == b->gather_min;
  for (int i = 0; i < 5; ++i) same = same && a->var[i] == b->var[i];
  return same;
}

static hipError_t run_group(const fsp::SolveGeom& g, bool f64, int first, int last, hipStream_t s) {
  return f64 ? fsp::solve_f64(g, first, last, s) : fsp::solve_f32(g, first, last, s);
}

static fsp_status solve_one(fsp_plan p, const void* rho, void* phi, hipStream_t s, int first = 0, int last = 4) {
  fsp::SolveGeom g = group_geom(p);
  add_item(g, p, rho, phi);
  hipError_t e = run_group(g, p->d.prec == FSP_F64, first, last, s);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve");
  return FSP_OK;
}

// Items of equal shape share launches (up to MAX_ITEMS per launch); launch
// group k goes to streams[k % nstreams].
static fsp_status enqueue_batch(int count, const fsp_plan* plans, const void* const* rho, void* const* phi,
                                const hipStream_t* streams, int nstreams) {
  std::vector<char> done(count, 0);
  int group = 0;
  for (int i = 0; i < count; ++i) {
    if (done[i]) continue;
    fsp::SolveGeom g = group_geom(plans[i]);
    for (int j = i; j < count; ++j) {
      if (done[j] || !same_shape(plans[i], plans[j])) continue;
      add_item(g, plans[j], rho[j], phi[j]);
      done[j] = 1;
      if (g.items == fsp::MAX_ITEMS) {
        hipError_t e = run_group(g, plans[i]->d.prec == FSP_F64, 0, 4, streams[group++ % nstreams]);
        if (e != hipSuccess) return fail_hip(e, "fsp_solve_batched");
        g = group_geom(plans[i]);
      }
    }
    if (g.items) {
      hipError_t e = run_group(g, plans[i]->d.prec == FSP_F64, 0, 4, streams[group++ % nstreams]);
      if (e != hipSuccess) return fail_hip(e, "fsp_solve_batched");
    }
  }
  return FSP_OK;
}

static fsp_status check_batch(const char* who, int count, const fsp_plan* plans, const void* const* rho,
                              void* const* phi) {
  if (count < 0) return fail(FSP_ERR_INVALID_ARG, std::string(who) + ": negative count");
  if (count == 0) return FSP_OK;
  if (!plans || !rho || !phi) return fail(FSP_ERR_INVALID_ARG, std::string(who) + ": NULL argument");
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !rho[i] || !phi[i])
      return fail(FSP_ERR_INVALID_ARG, std::string(who) + ": NULL entry " + std::to_string(i));
    if (!plans[i]->ready)
      return fail(FSP_ERR_NOT_READY, std::string(who) + ": plan " + std::to_string(i) + " is not ready");
    if (plans[i]->device != plans[0]->device)
      return fail(FSP_ERR_INVALID_ARG, std::string(who) + ": plans on different devices");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i] || plans[j]->work == plans[i]->work)
        return fail(FSP_ERR_INVALID_ARG, std::string(who) + ": two entries share a workspace");
  }
  return FSP_OK;
}

}  // extern "C"

// Library-internal entry points of the serving engine (internal.hpp).
namespace fsp {
namespace internal {

hipError_t solve_items(fsp_plan geo, int count, const void* const* rho, void* const* phi, void* const* work,
                       const void* const* octant, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int i0 = 0; i0 < count && e == hipSuccess; i0 += fsp::MAX_ITEMS) {
    fsp::SolveGeom g = group_geom(geo);
    for (int i = i0; i < count && g.items < fsp::MAX_ITEMS; ++i) {
      const int k = g.items++;
      g.rho[k] = rho[i];
      g.phi[k] = phi[i];
      g.work[k] = work[i];
      g.ghat[k] = octant[i];
    }
    e = run_group(g, geo->d.prec == FSP_F64, 0, 4, s);
  }
  return e;
}

size_t work1_bytes(fsp_plan p) { return p->work1_bytes; }
size_t ghat_bytes(fsp_plan p) { return p->ghat_bytes; }
size_t precompute_bytes(fsp_plan p) { return p->pre_bytes; }
const void* octant(fsp_plan p) { return static_cast<const char*>(p->ghat_read) + p->oct_off; }

fsp_status bind_ghat(fsp_plan p, void* ghat_dev) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "bind_ghat: hipGetDevice");
  release_buffers(p);
  p->device = dev;
  p->ghat = ghat_dev;
  p->ghat_read = ghat_dev;
  p->bound = true;  // no workspace: the plan is only precomputed and read
  return FSP_OK;
}

const char* last_error() { return g_err.c_str(); }
void set_error(const std::string& msg) { g_err = msg; }

}  // namespace internal
}  // namespace fsp

extern "C" {

fsp_status fsp_solve(fsp_plan p, const void* rho, void* phi, void* stream) {
  if (!p || !rho || !phi) return fail(FSP_ERR_INVALID_ARG, "fsp_solve: NULL argument");
  if (!p->ready) return fail(FSP_ERR_NOT_READY, "fsp_solve: plan has no bound buffers or no precomputed transform");
  DeviceGuard guard;
  hipError_t e = guard.enter(p->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve: hipSetDevice");
  return solve_one(p, rho, phi, reinterpret_cast<hipStream_t>(stream));
}

fsp_status fsp_solve_static(fsp_plan p, const void* rho, void* phi, void* stream) {
  if (!p || !rho || !phi) return fail(FSP_ERR_INVALID_ARG, "fsp_solve_static: NULL argument");
  if (p->work1_bytes > FSP_STATIC_SCRATCH_BYTES)
    return fail(FSP_ERR_UNSUPPORTED_SIZE, "fsp_solve_static: the plan's workspace of " +
                                              std::to_string(p->work1_bytes) + " bytes exceeds the static " +
                                              std::to_string((size_t)FSP_STATIC_SCRATCH_BYTES) + "-byte scratch");
  if (!p->ready) return fail(FSP_ERR_NOT_READY, "fsp_solve_static: plan has no bound buffers or no precomputed transform");
  DeviceGuard guard;
  hipError_t e = guard.enter(p->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve_static: hipSetDevice");
  void* ws = nullptr;
  e = scratch_address(p->device, &ws);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve_static: hipGetSymbolAddress of the scratch array");
  fsp::SolveGeom g = group_geom(p);
  add_item(g, p, rho, phi);
  g.work[0] = ws;  // the plan's own workspace is not touched
  e = run_group(g, p->d.prec == FSP_F64, 0, 4, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail_hip(e, "fsp_solve_static");
  return FSP_OK;
}

fsp_status fsp_solve_passes(fsp_plan p, const void* rho, void* phi, int first, int last, void* stream) {
  if (!p) return fail(FSP_ERR_INVALID_ARG, "fsp_solve_passes: NULL plan");
  if (first < 0 || last > 4 || first > last) return fail(FSP_ERR_INVALID_ARG, "fsp_solve_passes: need 0 <= first <= last <= 4");
  if ((first == 0 && !rho) || (last == 4 && !phi)) return fail(FSP_ERR_INVALID_ARG, "fsp_solve_passes: NULL rho/phi for its pass");
  if (p->var[1] == fsp::FUSED && first <= 3 && last >= 1 && (first > 1 || last < 3))
    return fail(FSP_ERR_INVALID_ARG, "fsp_solve_passes: the fused schedule runs passes 1-3 together");
  if (p->var[0] == fsp::PLANE && (first == 1 || (first == 0 && last == 0)))
    return fail(FSP_ERR_INVALID_ARG, "fsp_solve_passes: the plane schedule runs passes 0-1 together");
  if (p->var[3] == fsp::PLANE && (first == 4 || (first <= 3 && last == 3)))
    return fail(FSP_ERR_INVALID_ARG, "fsp_solve_passes: the plane schedule runs passes 3-4 together");
  if (!p->ready) return fail(FSP_ERR_NOT_READY, "fsp_solve_passes: plan has no bound buffers or no precomputed transform");
  DeviceGuard guard;
  hipError_t e = guard.enter(p->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve_passes: hipSetDevice");
  return solve_one(p, rho, phi, reinterpret_cast<hipStream_t>(stream), first, last);
}

// The gradient solve of one item: separate passes 1-3, the axis-0 pass in the
// gradient's own variants (p3; -1 follows the schedule).  The three components
// go to the workspace's other spectra, phi (when not NULL) in place in S, last;
// passes 4 and 5 take the outputs as the items of one launch each.
static fsp::SolveGeom grad_geom(const fsp_plan_s* p, const void* rho, void* phi, void* grad, int p3) {
  int var[5];
  for (int i = 0; i < 5; ++i) var[i] = p->var[i];
  if (var[1] == fsp::FUSED) var[1] = var[2] = var[3] = 0;
  if (p3 >= 0) var[2] = p3;
  fsp::SolveGeom g = group_geom(p, var);
  const int gp = p->d.prec == FSP_F64 ? fsp::grad_cfg<double>(2 * p->n[0], var[2]).pid
                                      : fsp::grad_cfg<float>(2 * p->n[0], var[2]).pid;
  g.tw_c0 = static_cast<const char*>(p->ghat_read) + p->tw_c0_off[gp];
  add_item(g, p, rho, nullptr);
  const size_t field = (size_t)p->n[0] * p->n[1] * p->n[2] * p->rb;
  const char* gb = static_cast<const char*>(p->ghat_read);
  for (int a = 0; a < 3; ++a) {
    g.ocomp[a] = 1 + a;
    g.oghat[a] = gb + p->grad_off[a];
    g.owork[a] = static_cast<char*>(p->work) + (a + 1) * p->work1_bytes;
    g.ophi[a] = grad ? static_cast<char*>(grad) + a * field : nullptr;
  }
  g.nout = 3;
  if (phi) {
    g.ocomp[3] = 0;
    g.oghat[3] = gb + p->oct_off;
    g.owork[3] = p->work;
    g.ophi[3] = phi;
    g.nout = 4;
  }
  return g;
}

fsp_status fsp_solve_grad(fsp_plan p, const void* rho, void* phi, void* grad, void* stream) {
  if (!p || !rho || !grad) return fail(FSP_ERR_INVALID_ARG, "fsp_solve_grad: NULL argument");
  if (!p->grad) return fail(FSP_ERR_INVALID_ARG, "fsp_solve_grad: the plan was created without FSP_WANT_GRAD");
  if (!p->ready) return fail(FSP_ERR_NOT_READY, "fsp_solve_grad: plan has no bound buffers or no precomputed transform");
  const size_t field = (size_t)p->n[0] * p->n[1] * p->n[2] * p->rb;
  if (phi) {
    const char *g0 = static_cast<const char*>(grad), *f = static_cast<const char*>(phi);
    if (f < g0 + 3 * field && g0 < f + field)
      return fail(FSP_ERR_INVALID_ARG, "fsp_solve_grad: phi overlaps grad");
  }
  DeviceGuard guard;
  hipError_t e = guard.enter(p->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve_grad: hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool f64 = p->d.prec == FSP_F64;
  e = run_group(grad_geom(p, rho, phi, grad, p->grad_p3), f64, 0, 4, s);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve_grad");
  return FSP_OK;
}

fsp_status fsp_plan_get_schedule(fsp_plan p, int* variants) {
  if (!p || !variants) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_get_schedule: NULL argument");
  for (int i = 0; i < 5; ++i) variants[i] = p->var[i];
  return FSP_OK;
}

static bool fused_supported(const fsp_plan_s* p) {
  if (p->n[0] != p->n[1] || p->chunks != 1) return false;
  return p->d.prec == FSP_F64 ? fsp::slab_cfg<double>(2 * p->n[1]).tiles > 0
                              : fsp::slab_cfg<float>(2 * p->n[1]).tiles > 0;
}

static bool plane_supported(const fsp_plan_s* p) {
  if (p->n[1] != p->n[2] || p->chunks != 1) return false;
  return p->d.prec == FSP_F64 ? fsp::plane_cfg<double>(p->n[2]).tc > 0 : fsp::plane_cfg<float>(p->n[2]).tc > 0;
}

fsp_status fsp_plan_set_schedule(fsp_plan p, const int* variants) {
  if (!p || !variants) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_set_schedule: NULL argument");
  const bool fused = variants[1] == fsp::FUSED;
  if (fused && (variants[2] != fsp::FUSED || variants[3] != fsp::FUSED || !fused_supported(p)))
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_set_schedule: the fused schedule needs passes 1-3 all set to 3, "
                                     "n0 == n1 and a grid small enough for the slab to fit in LDS");
  const bool plane_fwd = variants[0] == fsp::PLANE || variants[1] == fsp::PLANE;
  const bool plane_inv = variants[3] == fsp::PLANE || variants[4] == fsp::PLANE;
  if ((plane_fwd && (variants[0] != fsp::PLANE || variants[1] != fsp::PLANE)) ||
      (plane_inv && (variants[3] != fsp::PLANE || variants[4] != fsp::PLANE)) ||
      ((plane_fwd || plane_inv) && !plane_supported(p)))
    return fail(FSP_ERR_INVALID_ARG, "fsp_plan_set_schedule: the plane schedule needs passes 0 and 1 (or 3 and 4) "
                                     "both set to 4, n1 == n2 and a plane that fits in LDS");
  for (int i = 0; i < 5; ++i) {
    const bool mid = i >= 1 && i <= 3;
    const bool in_plane = (i <= 1 && plane_fwd) || (i >= 3 && plane_inv);
    if (variants[i] < 0 || (variants[i] >= fsp::NUM_VARIANTS && !(mid && fused) && !in_plane))
      return fail(FSP_ERR_INVALID_ARG, "fsp_plan_set_schedule: variant out of range");
    if (mid && !fused && variants[i] == fsp::FUSED)
      return fail(FSP_ERR_INVALID_ARG, "fsp_plan_set_schedule: variant out of range");
  }
  for (int i = 0; i < 5; ++i) p->var[i] = variants[i];
  p->grad_p3 = -1;  // the gradient solve follows this schedule
  return FSP_OK;
}

// Median of n (<= 8) timings: robust against the odd slow repetition.
static float median_ms(float* v, int n) {
  std::sort(v, v + n);
  return n % 2 ? v[n / 2] : 0.5f * (v[n / 2 - 1] + v[n / 2]);
}

fsp_status fsp_autotune(fsp_plan p, const void* rho, void* phi, int reps, void* stream, float* times_ms) {
  if (!p || !rho || !phi) return fail(FSP_ERR_INVALID_ARG, "fsp_autotune: NULL argument");
  {
    // the timed solves write phi many times: an overlap would corrupt rho
    const size_t field = (size_t)p->n[0] * p->n[1] * p->n[2] * p->rb;
    const char *r = static_cast<const char*>(rho), *f = static_cast<const char*>(phi);
    if (r < f + field && f < r + field) return fail(FSP_ERR_INVALID_ARG, "fsp_autotune: phi overlaps rho");
  }
  if (!p->ready) return fail(FSP_ERR_NOT_READY, "fsp_autotune: plan has no bound buffers or no precomputed transform");
  if (reps < 1 || reps > 8) return fail(FSP_ERR_INVALID_ARG, "fsp_autotune: reps must be in [1, 8]");
  DeviceGuard guard;
  hipError_t e = guard.enter(p->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_autotune: hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int best[5];
  for (int i = 0; i < 5; ++i) best[i] = p->var[i];
  if (best[1] == fsp::FUSED) best[1] = best[2] = best[3] = 0;  // tune the separate passes first
  if (best[0] == fsp::PLANE) best[0] = best[1] = 0;
  if (best[3] == fsp::PLANE) best[3] = best[4] = 0;
  // Each variant is timed inside full solves (the pass reads what the pass
  // before it just wrote, as in a real solve): events around the pass only.
  for (int pass = 0; pass < 5 && e == hipSuccess; ++pass) {
    float best_ms = 1e30f;
    for (int v = 0; v < fsp::NUM_VARIANTS && e == hipSuccess; ++v) {
      for (int i = 0; i < 5; ++i) p->var[i] = best[i];
      p->var[pass] = v;
      float rep_ms[8] = {};
      for (int r = 0; r <= reps && e == hipSuccess; ++r) {  // r == 0 warms up
        fsp_status st = pass > 0 ? solve_one(p, rho, phi, s, 0, pass - 1) : FSP_OK;
        if (st == FSP_OK) e = hipEventRecord(e0, s);
        if (st == FSP_OK && e == hipSuccess) st = solve_one(p, rho, phi, s, pass, pass);
        if (st == FSP_OK && e == hipSuccess) e = hipEventRecord(e1, s);
        if (st == FSP_OK && e == hipSuccess && pass < 4) st = solve_one(p, rho, phi, s, pass + 1, 4);
        if (st != FSP_OK) {  // the solve's own error is the one reported
          for (int i = 0; i < 5; ++i) p->var[i] = best[i];
          if (e0) (void)hipEventDestroy(e0);
          if (e1) (void)hipEventDestroy(e1);
          return st;
        }
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (r > 0) rep_ms[r - 1] = ms;
      }
      const float ms = median_ms(rep_ms, reps);
      if (times_ms) times_ms[pass * fsp::NUM_VARIANTS + v] = ms;
      if (e == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best[pass] = v;
      }
    }
  }
  for (int i = 0; i < 5; ++i) p->sep[i] = best[i];
  // whole-solve schedules built from the best separate variants: the separate
  // passes, the fused slab (passes 1-3), the plane kernels for passes 0-1 and
  // 3-4 (both pairs, or either alone); each timed as a full solve, the fastest kept
  if (e == hipSuccess) {
    fsp_status st_sched = FSP_OK;
    auto time_solve = [&](const int* sched, float* out) -> hipError_t {
      for (int i = 0; i < 5; ++i) p->var[i] = sched[i];
      hipError_t r = hipSuccess;
      float rep_ms[8] = {};
      for (int k = 0; k <= reps && r == hipSuccess; ++k) {
        r = hipEventRecord(e0, s);
        if (r == hipSuccess && (st_sched = solve_one(p, rho, phi, s)) != FSP_OK) return hipErrorInvalidValue;
        if (r == hipSuccess) r = hipEventRecord(e1, s);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        if (k > 0) rep_ms[k - 1] = ms;
      }
      *out = median_ms(rep_ms, reps);
      return r;
    };
    const int P = fsp::PLANE, Fu = fsp::FUSED;
    const int cand[5][5] = {{best[0], best[1], best[2], best[3], best[4]},
                            {best[0], Fu, Fu, Fu, best[4]},
                            {P, P, best[2], P, P},
                            {P, P, best[2], best[3], best[4]},
                            {best[0], best[1], best[2], P, P}};
    const bool ok[5] = {true, fused_supported(p), plane_supported(p), plane_supported(p), plane_supported(p)};
    float t[5] = {0, 0, 0, 0, 0};
    int pick = 0;
    for (int c = 0; c < 5 && e == hipSuccess; ++c) {
      if (!ok[c]) continue;
      e = time_solve(cand[c], &t[c]);
      if (st_sched != FSP_OK) {
        for (int i = 0; i < 5; ++i) p->var[i] = best[i];
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return st_sched;
      }
      if (e == hipSuccess && t[c] < t[pick]) pick = c;
    }
    if (times_ms) {
      times_ms[5 * fsp::NUM_VARIANTS] = t[1];
      times_ms[5 * fsp::NUM_VARIANTS + 1] = t[0];
      for (int c = 2; c < 5; ++c) times_ms[5 * fsp::NUM_VARIANTS + c] = t[c];
    }
    if (e == hipSuccess)
      for (int i = 0; i < 5; ++i) best[i] = cand[pick][i];
  }
  for (int i = 0; i < 5; ++i) p->var[i] = best[i];
  // the gradient solve's axis-0 pass (four outputs), each of its variants
  if (e == hipSuccess && p->grad) {
    const bool f64 = p->d.prec == FSP_F64;
    float best_ms = 1e30f;
    int best_v = 0;
    for (int v = 0; v < fsp::NUM_VARIANTS && e == hipSuccess; ++v) {
      const fsp::SolveGeom g = grad_geom(p, rho, phi, nullptr, v);
      float rep_ms[8] = {};
      for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        e = run_group(g, f64, 0, 1, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = run_group(g, f64, 2, 2, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (r > 0) rep_ms[r - 1] = ms;
      }
      const float ms = median_ms(rep_ms, reps);
      if (e == hipSuccess && ms < best_ms) best_ms = ms, best_v = v;
    }
    if (e == hipSuccess) p->grad_p3 = best_v;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail_hip(e, "fsp_autotune");
  // leave a correct result in phi with the tuned schedule
  fsp_status st = solve_one(p, rho, phi, s);
  if (st != FSP_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::array<int, 11> a;
    for (int i = 0; i < 5; ++i) a[i] = best[i];
    auto it = g_tuned.find(TuneKey{p->n[0], p->n[1], p->n[2], p->d.prec});
    a[5] = p->grad ? p->grad_p3 : it != g_tuned.end() ? it->second[5] : -1;
    for (int i = 0; i < 5; ++i) a[6 + i] = p->sep[i];
    g_tuned[TuneKey{p->n[0], p->n[1], p->n[2], p->d.prec}] = a;
  }
  return FSP_OK;
}

fsp_status fsp_solve_batched(int count, const fsp_plan* plans, const void* const* rho, void* const* phi,
                             void* stream) {
  fsp_status st = check_batch("fsp_solve_batched", count, plans, rho, phi);
  if (st != FSP_OK || count == 0) return st;
  DeviceGuard guard;
  hipError_t e = guard.enter(plans[0]->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_solve_batched: hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return enqueue_batch(count, plans, rho, phi, &s, 1);
}

fsp_status fsp_autotune_batch(int count, const fsp_plan* plans, const void* const* rho, void* const* phi, int reps,
                              void* stream) {
  fsp_status st = check_batch("fsp_autotune_batch", count, plans, rho, phi);
  if (st != FSP_OK || count == 0) return st;
  if (reps < 1 || reps > 8) return fail(FSP_ERR_INVALID_ARG, "fsp_autotune_batch: reps must be in [1, 8]");
  for (int i = 0; i < count; ++i) {
    const size_t field = (size_t)plans[i]->n[0] * plans[i]->n[1] * plans[i]->n[2] * plans[i]->rb;
    const char *r = static_cast<const char*>(rho[i]), *f = static_cast<const char*>(phi[i]);
    if (r < f + field && f < r + field) return fail(FSP_ERR_INVALID_ARG, "fsp_autotune_batch: a phi overlaps its rho");
  }
  DeviceGuard guard;
  hipError_t e = guard.enter(plans[0]->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_autotune_batch: hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::vector<char> done(count, 0);
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    if (done[i]) continue;
    std::vector<fsp_plan> gp;
    std::vector<const void*> gr;
    std::vector<void*> gf;
    for (int j = i; j < count; ++j) {
      if (done[j] || !same_geometry(plans[i], plans[j])) continue;
      done[j] = 1;
      gp.push_back(plans[j]);
      gr.push_back(rho[j]);
      gf.push_back(phi[j]);
    }
    const fsp_plan p0 = gp[0];
    // the schedule and separate variants last tuned for this shape, else the first plan's
    int base[5], sp[5];
    for (int k = 0; k < 5; ++k) base[k] = p0->var[k], sp[k] = p0->sep[k];
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tuned.find(TuneKey{p0->n[0], p0->n[1], p0->n[2], p0->d.prec});
      if (it != g_tuned.end())
        for (int k = 0; k < 5; ++k) base[k] = it->second[k], sp[k] = it->second[6 + k];
    }
    if (base[1] == fsp::FUSED) continue;  // the fused slab: nothing to choose between
    std::vector<std::array<int, 5>> orig;
    for (fsp_plan q : gp) orig.push_back({q->var[0], q->var[1], q->var[2], q->var[3], q->var[4]});
    // median time of the group's solves enqueued together with schedule c
    auto time_group = [&](const int* c, float* out) {
      for (fsp_plan q : gp)
        for (int k = 0; k < 5; ++k) q->var[k] = c[k];
      float rep_ms[8] = {};
      for (int r = 0; r <= reps && e == hipSuccess; ++r) {  // r == 0 warms up
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
          st = enqueue_batch((int)gp.size(), gp.data(), gr.data(), gf.data(), &s, 1);
          if (st != FSP_OK) return;
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (r > 0) rep_ms[r - 1] = ms;
      }
      *out = median_ms(rep_ms, reps);
    };
    const int P = fsp::PLANE;
    const int cand[4][5] = {{sp[0], sp[1], base[2], sp[3], sp[4]},
                            {P, P, base[2], sp[3], sp[4]},
                            {sp[0], sp[1], base[2], P, P},
                            {P, P, base[2], P, P}};
    const int ncand = plane_supported(p0) ? 4 : 1;
    float best_ms = 1e30f;
    int cur[5] = {cand[0][0], cand[0][1], cand[0][2], cand[0][3], cand[0][4]};
    bool timed = false;
    for (int c = 0; c < ncand && e == hipSuccess && st == FSP_OK; ++c) {
      float ms = 0;
      time_group(cand[c], &ms);
      if (e == hipSuccess && st == FSP_OK && ms < best_ms) {
        best_ms = ms, timed = true;
        for (int k = 0; k < 5; ++k) cur[k] = cand[c][k];
      }
    }
    // then each separate pass in turn: its other variants, timed with the group
    // (a variant that wins alone need not win when the group's launches are
    // wider, e.g. where occupancy decides)
    for (int q = 0; q < 5 && timed && e == hipSuccess && st == FSP_OK; ++q) {
      if (cur[q] == P) continue;
      for (int v = 0; v < fsp::NUM_VARIANTS && e == hipSuccess && st == FSP_OK; ++v) {
        if (v == cur[q]) continue;
        int trial[5] = {cur[0], cur[1], cur[2], cur[3], cur[4]};
        trial[q] = v;
        float ms = 0;
        time_group(trial, &ms);
        if (e == hipSuccess && st == FSP_OK && ms < best_ms) {
          best_ms = ms;
          cur[q] = v;
        }
      }
    }
    for (size_t m = 0; m < gp.size(); ++m)
      for (int k = 0; k < 5; ++k) gp[m]->var[k] = timed ? cur[k] : orig[m][k];
    if (st != FSP_OK) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != FSP_OK) return st;
  if (e != hipSuccess) return fail_hip(e, "fsp_autotune_batch");
  return FSP_OK;
}

fsp_status fsp_plan_destroy(fsp_plan p) {
  if (!p) return fail(FSP_ERR_INVALID_ARG, "fsp_plan_destroy: NULL plan");
  if (p->own_ghat || p->own_work) {
    DeviceGuard guard;
    (void)guard.enter(p->device);
    release_buffers(p);
  }
  delete p;
  return FSP_OK;
}

}  // extern "C"

struct fsp_batch_s {
  std::vector<fsp_plan> plans;
  std::vector<int> slot;            // table slot of solve i
  // launch groups: equal shapes, contiguous table slots [first, first + count)
  struct Group {
    int first, count;
    fsp_plan plan;                  // a member (the group's shape and schedule)
  };
  std::vector<Group> groups;
  std::vector<fsp::ItemPtrs> host;  // the table as last written (slot order)
  fsp::ItemPtrs* table = nullptr;   // the device table the captured kernels read
  int device = 0;
  // Graph layout.  The leading groups (largest first) run in turn on
  // `branches` branches; the last `tail` groups (the smallest) then run
  // together on `tail_branches` branches, each group (largest first) put on
  // the branch with the fewest model bytes so far, once the leading ones are
  // done.  Measured on the 64-solve mix: the largest group alone first, then
  // the other four on three branches (0.792 ms; 0.798 on four, 0.802 on two,
  // 0.827 all in turn, 0.851 all five side by side).  Groups that overlap
  // the largest slow its kernels more than they fill idle compute units.
  int branches = 1;
  int tail = 8;
  int tail_branches = 3;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// New inputs and outputs of up to SET_ITEMS table slots, written by one launch
// (the values travel in the kernel arguments, so the update is ordered on the
// caller's stream like any kernel and needs no host staging buffer).
constexpr int SET_ITEMS = 64;
struct SetItemsArgs {
  fsp::ItemPtrs* table;
  int count;
  int slot[SET_ITEMS];
  const void* rho[SET_ITEMS];
  void* phi[SET_ITEMS];
};

__global__ __launch_bounds__(SET_ITEMS) void k_set_items(SetItemsArgs a) {
  const int i = threadIdx.x;
  if (i < a.count) {
    a.table[a.slot[i]].rho = a.rho[i];
    a.table[a.slot[i]].phi = a.phi[i];
  }
}

// Capture the group launches of a batch as one graph whose launch groups run
// on parallel branches; every launch reads its items' buffers from the table.
hipError_t capture_batch(fsp_batch_s* b) {
  const int nb = b->branches;
  const int ng = (int)b->groups.size();
  const int nt = std::max(0, std::min(b->tail, ng - 1));  // trailing groups
  const int ntb = std::max(0, std::min(nt, b->tail_branches));  // their branches
  const int ns = nb + ntb;
  hipStream_t cs = nullptr;
  std::vector<hipStream_t> side(ns, nullptr);
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join(ns, nullptr), mid(nb, nullptr);
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  for (int i = 0; i < ns && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&side[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (int i = 0; i < ns && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
  for (int i = 0; i < nb && nt > 0 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&mid[i], hipEventDisableTiming);
  bool capturing = false;
  if (e == hipSuccess) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    capturing = e == hipSuccess;
  }
  if (e == hipSuccess) e = hipEventRecord(fork, cs);
  for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipStreamWaitEvent(side[i], fork, 0);
  auto launch_group = [&](int k, hipStream_t st) {
    const fsp_batch_s::Group& gr = b->groups[k];
    fsp::SolveGeom g = group_geom(gr.plan);
    g.items = gr.count;
    g.items_dev = b->table + gr.first;
    e = run_group(g, gr.plan->d.prec == FSP_F64, 0, 4, st);
  };
  for (int k = 0; k < ng - nt && e == hipSuccess; ++k) launch_group(k, side[k % nb]);
  if (nt > 0) {  // the trailing groups start together once every leading group is done
    for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipEventRecord(mid[i], side[i]);
    for (int t = 0; t < ntb && e == hipSuccess; ++t)
      for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipStreamWaitEvent(side[nb + t], mid[i], 0);
    // each (largest first) to the branch with the fewest model bytes so far
    std::vector<double> load(ntb, 0.0);
    for (int k = ng - nt; k < ng && e == hipSuccess; ++k) {
      const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[t] += model_bytes(b->groups[k].plan) * b->groups[k].count;
      launch_group(k, side[nb + t]);
    }
  }
  for (int i = 0; i < ns && e == hipSuccess; ++i) e = hipEventRecord(join[i], side[i]);
  for (int i = 0; i < ns && e == hipSuccess; ++i) e = hipStreamWaitEvent(cs, join[i], 0);
  if (capturing) {
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) {
      b->graph = g;
      e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  for (auto ev : join)
    if (ev) (void)hipEventDestroy(ev);
  for (auto ev : mid)
    if (ev) (void)hipEventDestroy(ev);
  if (fork) (void)hipEventDestroy(fork);
  for (auto st : side)
    if (st) (void)hipStreamDestroy(st);
  if (cs) (void)hipStreamDestroy(cs);
  return e;
}

void free_batch(fsp_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->table) (void)hipFree(b->table);
  delete b;
}

}  // namespace

extern "C" {

fsp_status fsp_batch_create(int count, const fsp_plan* plans, const void* const* rho, void* const* phi,
                            fsp_batch* out) {
  if (!out) return fail(FSP_ERR_INVALID_ARG, "fsp_batch_create: NULL out");
  *out = nullptr;
  if (count <= 0) return fail(FSP_ERR_INVALID_ARG, "fsp_batch_create: count must be positive");
  fsp_status st = check_batch("fsp_batch_create", count, plans, rho, phi);
  if (st != FSP_OK) return st;
  fsp_batch_s* b = new (std::nothrow) fsp_batch_s();
  if (!b) return fail(FSP_ERR_OUT_OF_MEMORY, "fsp_batch_create: host allocation failed");
  b->plans.assign(plans, plans + count);
  b->device = plans[0]->device;
  b->slot.assign(count, -1);
  // one launch group per shape, its items in consecutive table slots
  for (int i = 0; i < count; ++i) {
    if (b->slot[i] >= 0) continue;
    fsp_batch_s::Group gr{(int)b->host.size(), 0, plans[i]};
    for (int j = i; j < count; ++j) {
      if (b->slot[j] >= 0 || !same_shape(plans[i], plans[j])) continue;
      if (gr.count == 65535) break;  // the launch grid's item axis
      b->slot[j] = (int)b->host.size();
      fsp::ItemPtrs it;
      it.rho = rho[j];
      it.phi = phi[j];
      it.work = plans[j]->work;
      it.ghat = static_cast<const char*>(plans[j]->ghat_read) + plans[j]->oct_off;
      b->host.push_back(it);
      ++gr.count;
    }
    b->groups.push_back(gr);
  }
  for (int i = 0; i < count; ++i)
    if (b->slot[i] < 0) {  // a shape with more than 65535 solves: its own groups
      fsp_batch_s::Group gr{(int)b->host.size(), 0, plans[i]};
      for (int j = i; j < count && gr.count < 65535; ++j) {
        if (b->slot[j] >= 0 || !same_shape(plans[i], plans[j])) continue;
        b->slot[j] = (int)b->host.size();
        b->host.push_back(fsp::ItemPtrs{rho[j], phi[j], plans[j]->work,
                                        static_cast<const char*>(plans[j]->ghat_read) + plans[j]->oct_off});
        ++gr.count;
      }
      b->groups.push_back(gr);
    }
  // the group that moves the most bytes starts first, on the first branch
  std::stable_sort(b->groups.begin(), b->groups.end(), [](const fsp_batch_s::Group& x, const fsp_batch_s::Group& y) {
    return model_bytes(x.plan) * x.count > model_bytes(y.plan) * y.count;
  });
  if (const char* env = std::getenv("FSP_BATCH_BRANCHES")) b->branches = std::max(1, std::min(16, std::atoi(env)));
  if (const char* env = std::getenv("FSP_BATCH_TAIL")) b->tail = std::max(0, std::min(8, std::atoi(env)));
  if (const char* env = std::getenv("FSP_BATCH_TAIL_BRANCHES")) b->tail_branches = std::max(1, std::min(8, std::atoi(env)));
  DeviceGuard guard;
  hipError_t e = guard.enter(b->device);
  if (e == hipSuccess) e = hipMalloc(&b->table, b->host.size() * sizeof(fsp::ItemPtrs));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b->table = nullptr;
    free_batch(b);
    return fail(FSP_ERR_OUT_OF_MEMORY, "fsp_batch_create: device table allocation failed");
  }
  e = hipMemcpy(b->table, b->host.data(), b->host.size() * sizeof(fsp::ItemPtrs), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_batch(b);
    return fail_hip(e, "fsp_batch_create: table upload");
  }
  *out = b;
  return FSP_OK;
}

fsp_status fsp_batch_set_io(fsp_batch b, const void* const* rho, void* const* phi, void* stream) {
  if (!b || !rho || !phi) return fail(FSP_ERR_INVALID_ARG, "fsp_batch_set_io: NULL argument");
  const int count = (int)b->plans.size();
  for (int i = 0; i < count; ++i)
    if (!rho[i] || !phi[i]) return fail(FSP_ERR_INVALID_ARG, "fsp_batch_set_io: NULL entry " + std::to_string(i));
  DeviceGuard guard;
  hipError_t e = guard.enter(b->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_batch_set_io: hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int i0 = 0; i0 < count && e == hipSuccess; i0 += SET_ITEMS) {
    SetItemsArgs a{};
    a.table = b->table;
    a.count = std::min(SET_ITEMS, count - i0);
    for (int k = 0; k < a.count; ++k) {
      const int i = i0 + k;
      a.slot[k] = b->slot[i];
      a.rho[k] = rho[i];
      a.phi[k] = phi[i];
      b->host[b->slot[i]].rho = rho[i];
      b->host[b->slot[i]].phi = phi[i];
    }
    hipLaunchKernelGGL(k_set_items, dim3(1), dim3(SET_ITEMS), 0, s, a);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail_hip(e, "fsp_batch_set_io");
  return FSP_OK;
}

fsp_status fsp_batch_launch(fsp_batch b, void* stream) {
  if (!b) return fail(FSP_ERR_INVALID_ARG, "fsp_batch_launch: NULL batch");
  DeviceGuard guard;
  hipError_t e = guard.enter(b->device);
  if (e != hipSuccess) return fail_hip(e, "fsp_batch_launch: hipSetDevice");
  if (!b->exec) {
    e = capture_batch(b);
    if (e != hipSuccess) return fail_hip(e, "fsp_batch_launch: graph capture");
  }
  e = hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail_hip(e, "fsp_batch_launch: hipGraphLaunch");
  return FSP_OK;
}

fsp_status fsp_batch_destroy(fsp_batch b) {
  if (!b) return fail(FSP_ERR_INVALID_ARG, "fsp_batch_destroy: NULL batch");
  DeviceGuard guard;
  (void)guard.enter(b->device);
  free_batch(b);
  return FSP_OK;
}

}  // extern "C"
