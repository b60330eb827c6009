// Scenarios for the CPU build of the serving engine (see mock_device.cpp).
// Prints "name key value" lines; exits non-zero when an invariant fails:
//   no device fault (every pointer a solve or precompute uses is live),
//   the bytes held never exceed the budget, every request ends done or
//   rejected, and a request is rejected only when it alone exceeds the budget.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <random>
#include <vector>

#include "fsp.h"
#include "fsp_serve.h"
#include "internal.hpp"

namespace mock {
extern long long faults, solves, precomputes;
}

static size_t need_of(const fsp_request& r) {
  fsp_plan_desc d{};
  for (int a = 0; a < 3; ++a) {
    d.n[a] = r.n[a];
    d.lo[a] = r.lo[a];
    d.hi[a] = r.hi[a];
  }
  d.greens = r.greens;
  d.prec = r.prec;
  fsp_plan p = nullptr;
  fsp_plan_create(&d, &p);
  const size_t n = fsp::internal::ghat_bytes(p) + fsp::internal::precompute_bytes(p) + fsp::internal::work1_bytes(p);
  fsp_plan_destroy(p);
  return n;
}

static int run(const char* name, std::vector<fsp_request>& reqs, size_t budget, int slots, int fold) {
  fsp_server s = nullptr;
  if (fsp_server_create(budget, slots, fold, &s) != FSP_OK) {
    std::printf("%s create_failed 1\n", name);
    return 1;
  }
  const long long f0 = mock::faults;
  std::vector<fsp_request_result> res(reqs.size());
  const fsp_status st = fsp_server_run(s, (int)reqs.size(), reqs.data(), res.data(), 0.0, 60.0);
  fsp_server_stats stats{};
  fsp_server_get_stats(s, &stats);
  int bad = st != FSP_OK;
  int done = 0, rejected = 0;
  for (size_t i = 0; i < reqs.size(); ++i) {
    if (res[i].status == FSP_OK) {
      ++done;
    } else if (res[i].status == FSP_ERR_OUT_OF_MEMORY) {
      ++rejected;
      if (need_of(reqs[i]) <= budget) bad = 1;  // rejected though it fits an empty engine
    } else {
      bad = 1;
    }
  }
  const long long faults = mock::faults - f0;
  if (faults || stats.peak_held_bytes > budget) bad = 1;
  std::printf("%s requests %zu\n%s done %d\n%s rejected %d\n%s faults %lld\n%s peak_held %zu\n%s budget %zu\n"
              "%s evictions %lld\n%s launches %lld\n%s ok %d\n",
              name, reqs.size(), name, done, name, rejected, name, faults, name, (size_t)stats.peak_held_bytes, name,
              budget, name, stats.evictions, name, stats.launches, name, !bad);
  fsp_server_destroy(s);
  return bad;
}

static fsp_request make(int n, int greens, int prec, double a, double t, void* buf) {
  fsp_request r{};
  r.t_arrival = t;
  r.n[0] = r.n[1] = r.n[2] = n;
  r.greens = greens;
  r.prec = prec;
  for (int k = 0; k < 3; ++k) {
    r.lo[k] = -a;
    r.hi[k] = a * (k == 2 ? 1.5 : 1.0);
  }
  r.rho = buf;
  r.phi = buf;
  return r;
}

int main() {
  void* buf = nullptr;
  hipMalloc(&buf, 1 << 20);
  int bad = 0;
  {
    // the tight-budget case: one 96^3 admission with a refresh fits, the cache of
    // every box and size does not
    std::vector<fsp_request> reqs;
    for (int i = 0; i < 12; ++i) reqs.push_back(make(i % 2 == 0 ? 96 : 48, FSP_VICO_DCT, FSP_F32, 1.0 - 0.1 * (i % 3),
                                                     0.0, buf));
    const size_t budget = (size_t)(need_of(reqs[0]) * 1.05);
    bad |= run("tight", reqs, budget, 1, 2);
  }
  std::mt19937 rng(12345);
  const int sizes[] = {8, 16, 24, 32, 48, 64, 96};
  for (int trial = 0; trial < 60; ++trial) {
    std::vector<fsp_request> reqs;
    const int count = 10 + (int)(rng() % 120);
    size_t total = 0, biggest = 0;
    for (int i = 0; i < count; ++i) {
      const int n = sizes[rng() % 7];
      reqs.push_back(make(n, (int)(rng() % 3), (int)(rng() % 2), 0.5 + 0.1 * (rng() % 4), 0.0, buf));
      total += need_of(reqs.back());
      biggest = std::max(biggest, need_of(reqs.back()));
    }
    // budgets from below the biggest request (some rejections) to above everything
    const double f = 0.5 + 0.25 * (rng() % 12);
    const size_t budget = std::max<size_t>(1, (size_t)(biggest * f + (rng() % 3 == 0 ? total : 0)));
    char name[32];
    std::snprintf(name, sizeof name, "random%d", trial);
    bad |= run(name, reqs, budget, 1 + (int)(rng() % 6), 1 + (int)(rng() % 12));
  }
  hipFree(buf);
  std::printf("all ok %d\n", !bad);
  return bad;
}
