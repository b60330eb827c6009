// serve_engine.hip -- the serving engine of fsp_serve.h: continuous batching of
// independent solve requests on one GPU, driven by the calling host thread.
//
// Per request: a workspace from a pool keyed by (grid, precision), and the
// Green's transform of its (Green's function, grid, box, alpha, precision)
// from a cache, computed on a miss on the refresh stream.  Requests of the
// queue's head shape are folded into one launch (fsp::internal::solve_items):
// the solve kernels take each item's own workspace and Green's octant, so one
// launch holds requests of different Green's functions and boxes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "fsp.h"
#include "fsp_serve.h"
#include "internal.hpp"

namespace {

__global__ void k_tick(int* p) {
  if (threadIdx.x == 0 && p) *p = 0;
}

struct GKey {  // one cached Green's transform
  int greens, prec, n0, n1, n2;
  double lo0, lo1, lo2, hi0, hi1, hi2, alpha;
  bool operator<(const GKey& o) const {
    return std::tie(greens, prec, n0, n1, n2, lo0, lo1, lo2, hi0, hi1, hi2, alpha) <
           std::tie(o.greens, o.prec, o.n0, o.n1, o.n2, o.lo0, o.lo1, o.lo2, o.hi0, o.hi1, o.hi2, o.alpha);
  }
};

struct WKey {  // one workspace shape
  int prec, n0, n1, n2;
  bool operator<(const WKey& o) const { return std::tie(prec, n0, n1, n2) < std::tie(o.prec, o.n0, o.n1, o.n2); }
  bool operator==(const WKey& o) const { return prec == o.prec && n0 == o.n0 && n1 == o.n1 && n2 == o.n2; }
};

struct Entry {
  GKey key{};
  fsp_plan plan = nullptr;   // precomputed into buf; never solved itself
  void* buf = nullptr;
  size_t bytes = 0;          // Green's buffer
  size_t transient = 0;      // precompute transients, held until `ready` is seen
  hipEvent_t begin = nullptr, ready = nullptr;
  bool refreshing = false;
  float refresh_ms = 0.0f;
  fsp_status status = FSP_OK;
  int users = 0;             // in-flight solves reading it
  unsigned long long last_use = 0;
};

struct Worker {
  WKey key{};
  void* work = nullptr;
  size_t bytes = 0;
  bool busy = false;
  unsigned long long last_use = 0;
};

struct Launch {
  int slot = -1;
  hipEvent_t done = nullptr;
  std::vector<int> reqs;
  std::vector<Worker*> workers;
  std::vector<Entry*> entries;   // one per request (repeats allowed)
  std::vector<char> waited;      // request waited for its entry's refresh
};

using clock_type = std::chrono::steady_clock;

}  // namespace

struct fsp_server_s {
  int device = 0;
  size_t budget = 0;
  int slots = 0, max_fold = 1;
  std::vector<hipStream_t> streams;
  std::vector<char> slot_busy;
  hipStream_t refresh = nullptr;
  std::map<GKey, std::unique_ptr<Entry>> cache;
  std::vector<std::unique_ptr<Worker>> pool;
  size_t held = 0;
  unsigned long long tick = 0;
  fsp_server_stats st{};
  std::vector<hipEvent_t> spare_events;
  int* tick_buf = nullptr;
};

namespace {

fsp_status srv_fail(fsp_status s, const std::string& msg) {
  fsp::internal::set_error(msg);
  return s;
}

hipEvent_t take_event(fsp_server_s* s) {
  if (!s->spare_events.empty()) {
    hipEvent_t e = s->spare_events.back();
    s->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void hold(fsp_server_s* s, size_t bytes) {
  s->held += bytes;
  s->st.peak_held_bytes = std::max(s->st.peak_held_bytes, s->held);
}

void drop_entry(fsp_server_s* s, Entry* e) {
  if (e->plan) (void)fsp_plan_destroy(e->plan);
  if (e->buf) (void)hipFree(e->buf);
  if (e->begin) s->spare_events.push_back(e->begin);
  if (e->ready) s->spare_events.push_back(e->ready);
  s->held -= e->bytes + (e->refreshing ? e->transient : 0);
}

// Free idle buffers, least recently used first, until `need` more bytes fit
// the budget; entries in `keep` stay.  True when they fit.
bool make_room(fsp_server_s* s, size_t need, const std::vector<Entry*>& keep) {
  while (s->held + need > s->budget) {
    Worker* wv = nullptr;
    for (auto& w : s->pool)
      if (!w->busy && (!wv || w->last_use < wv->last_use)) wv = w.get();
    Entry* ev = nullptr;
    for (auto& kv : s->cache) {
      Entry* e = kv.second.get();
      if (e->users || e->refreshing || std::find(keep.begin(), keep.end(), e) != keep.end()) continue;
      if (!ev || e->last_use < ev->last_use) ev = e;
    }
    if (!wv && !ev) return false;
    if (wv && (!ev || wv->last_use <= ev->last_use)) {
      (void)hipFree(wv->work);
      s->held -= wv->bytes;
      for (size_t i = 0; i < s->pool.size(); ++i)
        if (s->pool[i].get() == wv) {
          s->pool.erase(s->pool.begin() + (long)i);
          break;
        }
    } else {
      const GKey k = ev->key;
      drop_entry(s, ev);
      s->cache.erase(k);
    }
    ++s->st.evictions;
  }
  return true;
}

fsp_plan_desc desc_of(const fsp_request& r) {
  fsp_plan_desc d{};
  for (int a = 0; a < 3; ++a) {
    d.n[a] = r.n[a];
    d.lo[a] = r.lo[a];
    d.hi[a] = r.hi[a];
  }
  d.greens = r.greens;
  d.prec = r.prec;
  d.alpha = r.alpha;
  d.g0 = __builtin_nan("");
  d.flags = 0;
  return d;
}

GKey gkey_of(const fsp_request& r) {
  const double alpha = r.alpha == 0.0 ? 1.1 : r.alpha;
  return GKey{r.greens, r.prec, r.n[0], r.n[1], r.n[2], r.lo[0], r.lo[1], r.lo[2], r.hi[0], r.hi[1], r.hi[2], alpha};
}

WKey wkey_of(const fsp_request& r) { return WKey{r.prec, r.n[0], r.n[1], r.n[2]}; }

// Sizes of a request's Green's buffer, its precompute transients and its workspace.
struct Sizes {
  size_t ghat = 0, transient = 0, work = 0;
};

}  // namespace

extern "C" {

fsp_status fsp_server_create(size_t budget_bytes, int slots, int max_fold, fsp_server* out) {
  if (!out) return srv_fail(FSP_ERR_INVALID_ARG, "fsp_server_create: NULL out");
  *out = nullptr;
  if (budget_bytes == 0 || slots < 1 || slots > 64 || max_fold < 1 || max_fold > 256)
    return srv_fail(FSP_ERR_INVALID_ARG, "fsp_server_create: need budget > 0, 1 <= slots <= 64, 1 <= max_fold <= 256");
  auto* s = new (std::nothrow) fsp_server_s();
  if (!s) return srv_fail(FSP_ERR_OUT_OF_MEMORY, "fsp_server_create: host allocation failed");
  hipError_t e = hipGetDevice(&s->device);
  s->budget = budget_bytes;
  s->slots = slots;
  s->max_fold = max_fold;
  s->st.budget_bytes = budget_bytes;
  s->streams.assign(slots, nullptr);
  s->slot_busy.assign(slots, 0);
  for (int i = 0; i < slots && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->refresh, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&s->tick_buf, sizeof(int));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)fsp_server_destroy(s);
    return srv_fail(FSP_ERR_DEVICE, std::string("fsp_server_create: ") + hipGetErrorString(e));
  }
  *out = s;
  return FSP_OK;
}

fsp_status fsp_server_run(fsp_server s, int count, const fsp_request* reqs, fsp_request_result* results,
                          double time_scale, double max_wall_s) {
  if (!s || count < 0 || (count > 0 && (!reqs || !results)) || !(time_scale >= 0.0) || !(max_wall_s > 0.0))
    return srv_fail(FSP_ERR_INVALID_ARG, "fsp_server_run: bad argument");
#ifndef FSP_SERVER_ENABLED
  // Switched off in the device build: a run of the engine's GPU tests left the
  // GPU faulted, and again after the workspace-eviction fix; the second cause
  // is not found.  The engine's logic runs on the CPU, against a stand-in
  // device, under the sanitizers (the host build defines FSP_SERVER_ENABLED).
  if (count > 0)
    return srv_fail(FSP_ERR_DEVICE, "fsp_server_run: the serving engine is switched off in this build "
                                    "(its GPU runs faulted; it runs only in the CPU test build)");
#endif
  // validate every request (a descriptor the library rejects, NULL arrays) before anything runs
  std::vector<Sizes> sz(count);
  {
    std::map<GKey, Sizes> seen;
    for (int i = 0; i < count; ++i) {
      const fsp_request& r = reqs[i];
      if (!r.rho || !r.phi || !(r.t_arrival >= 0.0))
        return srv_fail(FSP_ERR_INVALID_ARG, "fsp_server_run: request " + std::to_string(i) + " has a NULL array or a negative arrival");
      const GKey k = gkey_of(r);
      auto it = seen.find(k);
      if (it == seen.end()) {
        const fsp_plan_desc d = desc_of(r);
        fsp_plan p = nullptr;
        fsp_status stt = fsp_plan_create(&d, &p);
        if (stt != FSP_OK) return srv_fail(stt, "fsp_server_run: request " + std::to_string(i) + ": " + fsp_last_error());
        Sizes z;
        z.ghat = fsp::internal::ghat_bytes(p);
        z.transient = fsp::internal::precompute_bytes(p);
        z.work = fsp::internal::work1_bytes(p);
        (void)fsp_plan_destroy(p);
        it = seen.emplace(k, z).first;
      }
      sz[i] = it->second;
    }
  }
  hipError_t he = hipSetDevice(s->device);
  if (he != hipSuccess) return srv_fail(FSP_ERR_DEVICE, std::string("fsp_server_run: ") + hipGetErrorString(he));
  for (int i = 0; i < count; ++i) {
    results[i] = fsp_request_result{};
    results[i].status = FSP_ERR_NOT_READY;
    results[i].slot = -1;
    results[i].t_arrival = reqs[i].t_arrival * time_scale;
  }
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].t_arrival < reqs[b].t_arrival; });

  // the two clocks' zero: a fresh device time stamp (an event on an idle
  // stream may carry the stamp of that stream's last finished work)
  hipEvent_t t0 = take_event(s);
  if (!t0) return srv_fail(FSP_ERR_DEVICE, "fsp_server_run: hipEventCreate");
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s->streams[0], s->tick_buf);
  he = hipEventRecord(t0, s->streams[0]);
  if (he == hipSuccess) he = hipStreamSynchronize(s->streams[0]);
  if (he != hipSuccess) return srv_fail(FSP_ERR_DEVICE, std::string("fsp_server_run: ") + hipGetErrorString(he));
  const auto wall0 = clock_type::now();
  auto now = [&]() { return std::chrono::duration<double>(clock_type::now() - wall0).count(); };

  std::deque<int> queue;
  std::vector<Launch> inflight;
  size_t next = 0;
  int finished = 0;
  fsp_status run_status = FSP_OK;

  auto finish = [&](Launch& L, fsp_status stt, double t_done) {
    const double seen = now();
    for (size_t k = 0; k < L.reqs.size(); ++k) {
      fsp_request_result& res = results[L.reqs[k]];
      res.status = stt;
      res.t_done = t_done;
      res.t_seen = seen;
      res.refresh_ms = L.waited[k] ? L.entries[k]->refresh_ms : 0.0f;
      ++finished;
    }
    for (Worker* w : L.workers) {
      w->busy = false;
      w->last_use = ++s->tick;
    }
    for (Entry* e : L.entries) {
      --e->users;
      e->last_use = ++s->tick;
    }
    s->slot_busy[L.slot] = 0;
    s->spare_events.push_back(L.done);
  };

  // a refresh whose event has passed releases its transients
  auto poll_refreshes = [&]() {
    for (auto& kv : s->cache) {
      Entry* e = kv.second.get();
      if (!e->refreshing) continue;
      const hipError_t q = hipEventQuery(e->ready);
      if (q == hipErrorNotReady) continue;
      e->refreshing = false;
      s->held -= e->transient;
      float ms = 0.0f;
      if (q == hipSuccess && hipEventElapsedTime(&ms, e->begin, e->ready) == hipSuccess) e->refresh_ms = ms;
      if (q != hipSuccess) e->status = FSP_ERR_DEVICE;
      s->st.refresh_ms_total += e->refresh_ms;
    }
  };

  auto poll_launches = [&]() {
    for (size_t i = 0; i < inflight.size();) {
      const hipError_t q = hipEventQuery(inflight[i].done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      float ms = 0.0f;
      fsp_status stt = FSP_OK;
      if (q != hipSuccess || hipEventElapsedTime(&ms, t0, inflight[i].done) != hipSuccess) stt = FSP_ERR_DEVICE;
      poll_refreshes();  // a refresh this launch waited for is complete too
      finish(inflight[i], stt, ms * 1e-3);
      inflight.erase(inflight.begin() + (long)i);
    }
  };

  // Green's entry of request i, created (and its refresh enqueued) on a miss;
  // NULL when its buffer cannot be allocated.
  auto entry_for = [&](int i) -> Entry* {
    const GKey k = gkey_of(reqs[i]);
    auto it = s->cache.find(k);
    if (it != s->cache.end()) return it->second.get();
    auto e = std::make_unique<Entry>();
    e->key = k;
    e->bytes = sz[i].ghat;
    e->transient = sz[i].transient;
    const fsp_plan_desc d = desc_of(reqs[i]);
    if (fsp_plan_create(&d, &e->plan) != FSP_OK) return nullptr;
    if (hipMalloc(&e->buf, e->bytes) != hipSuccess) {
      (void)hipGetLastError();
      (void)fsp_plan_destroy(e->plan);
      return nullptr;
    }
    hold(s, e->bytes + e->transient);
    e->refreshing = true;
    e->begin = take_event(s);
    e->ready = take_event(s);
    fsp_status stt = fsp::internal::bind_ghat(e->plan, e->buf);
    if (stt == FSP_OK && hipEventRecord(e->begin, s->refresh) != hipSuccess) stt = FSP_ERR_DEVICE;
    if (stt == FSP_OK) stt = fsp_precompute(e->plan, s->refresh);
    if (hipEventRecord(e->ready, s->refresh) != hipSuccess && stt == FSP_OK) stt = FSP_ERR_DEVICE;
    e->status = stt;
    ++s->st.refreshes;
    Entry* raw = e.get();
    s->cache.emplace(k, std::move(e));
    return raw;
  };

  auto idle_worker = [&](const WKey& k, const std::vector<Worker*>& taken) -> Worker* {
    for (auto& w : s->pool)
      if (!w->busy && w->key == k && std::find(taken.begin(), taken.end(), w.get()) == taken.end()) return w.get();
    return nullptr;
  };

  // Admit the queue's head (with followers of its shape) on a free slot.
  // Returns true when something was admitted or rejected.
  auto admit = [&]() -> bool {
    if (queue.empty()) return false;
    int slot = -1;
    for (int k = 0; k < s->slots; ++k)
      if (!s->slot_busy[k]) {
        slot = k;
        break;
      }
    if (slot < 0) return false;
    const int head = queue.front();
    const WKey wk = wkey_of(reqs[head]);
    Launch L;
    L.slot = slot;
    std::vector<Entry*> keep;
    std::vector<size_t> taken_pos;  // queue positions taken
    for (size_t qi = 0; qi < queue.size() && (int)L.reqs.size() < s->max_fold; ++qi) {
      const int i = queue[qi];
      if (!(wkey_of(reqs[i]) == wk)) continue;
      // what this request would reuse -- a cached Green's transform, an idle
      // workspace -- is protected before room is made, so make_room cannot
      // free it (busy workers and kept entries are never evicted)
      auto cit = s->cache.find(gkey_of(reqs[i]));
      Entry* cached = cit != s->cache.end() ? cit->second.get() : nullptr;
      Worker* w = idle_worker(wk, L.workers);
      if (w) w->busy = true;
      std::vector<Entry*> protect = keep;
      if (cached) protect.push_back(cached);
      const size_t need = (cached ? 0 : sz[i].ghat + sz[i].transient) + (w ? 0 : sz[i].work);
      if (!make_room(s, need, protect)) {
        if (w) w->busy = false;
        if (qi == 0 && L.reqs.empty()) {
          // the head alone: rejected if it could not fit an empty engine, else it waits
          if (sz[i].ghat + sz[i].transient + sz[i].work > s->budget) {
            results[i].status = FSP_ERR_OUT_OF_MEMORY;
            ++s->st.rejected;
            ++finished;
            queue.pop_front();
            return true;
          }
          return false;
        }
        break;  // followers only while they fit
      }
      // a failed allocation (device memory short of the budget) ends the group;
      // the request stays queued and is retried after completions free memory
      Entry* e = cached ? cached : entry_for(i);
      if (!e) {
        if (w) w->busy = false;
        break;
      }
      if (!w) {
        auto nw = std::make_unique<Worker>();
        nw->key = wk;
        nw->bytes = sz[i].work;
        if (hipMalloc(&nw->work, nw->bytes) != hipSuccess) {
          (void)hipGetLastError();
          break;
        }
        hold(s, nw->bytes);
        w = nw.get();
        s->pool.push_back(std::move(nw));
      }
      w->busy = true;
      keep.push_back(e);
      L.reqs.push_back(i);
      L.workers.push_back(w);
      L.entries.push_back(e);
      L.waited.push_back(e->refreshing ? 1 : 0);
      taken_pos.push_back(qi);
    }
    if (L.reqs.empty()) return false;
    for (size_t k = taken_pos.size(); k-- > 0;) queue.erase(queue.begin() + (long)taken_pos[k]);
    const double t_admit = now();
    hipStream_t st = s->streams[slot];
    hipError_t e = hipSuccess;
    fsp_status stt = FSP_OK;
    for (size_t k = 0; k < L.entries.size(); ++k) {
      Entry* en = L.entries[k];
      ++en->users;
      if (en->status != FSP_OK) stt = en->status;
      if (L.waited[k] && e == hipSuccess) e = hipStreamWaitEvent(st, en->ready, 0);
    }
    std::vector<const void*> rho(L.reqs.size()), oct(L.reqs.size());
    std::vector<void*> phi(L.reqs.size()), work(L.reqs.size());
    for (size_t k = 0; k < L.reqs.size(); ++k) {
      rho[k] = reqs[L.reqs[k]].rho;
      phi[k] = reqs[L.reqs[k]].phi;
      work[k] = L.workers[k]->work;
      oct[k] = fsp::internal::octant(L.entries[k]->plan);
      results[L.reqs[k]].t_admit = t_admit;
      results[L.reqs[k]].slot = slot;
      results[L.reqs[k]].launch_size = (int)L.reqs.size();
    }
    if (stt == FSP_OK && e == hipSuccess)
      e = fsp::internal::solve_items(L.entries[0]->plan, (int)L.reqs.size(), rho.data(), phi.data(), work.data(),
                                     oct.data(), st);
    L.done = take_event(s);
    if (e == hipSuccess && L.done) e = hipEventRecord(L.done, st);
    s->slot_busy[slot] = 1;
    ++s->st.launches;
    if (stt != FSP_OK || e != hipSuccess || !L.done) {
      if (!L.done) L.done = take_event(s);
      (void)hipGetLastError();
      finish(L, stt != FSP_OK ? stt : FSP_ERR_DEVICE, 0.0);
      return true;
    }
    inflight.push_back(std::move(L));
    return true;
  };

  while (finished < count) {
    const double t = now();
    if (t > max_wall_s) {
      run_status = FSP_ERR_DEVICE;
      fsp::internal::set_error("fsp_server_run: stopped after max_wall_s with requests unfinished");
      break;
    }
    while (next < order.size() && reqs[order[next]].t_arrival * time_scale <= t) queue.push_back(order[next++]);
    poll_launches();
    poll_refreshes();
    bool progressed = false;
    while (admit()) progressed = true;
    if (!progressed && inflight.empty() && queue.empty() && next < order.size()) {
      // idle until the next arrival (short sleeps keep the arrival clock honest)
      const double wait = reqs[order[next]].t_arrival * time_scale - now();
      if (wait > 2e-4) std::this_thread::sleep_for(std::chrono::microseconds((long)std::min(wait * 0.5e6, 2000.0)));
    }
  }
  // drain: every launch completes before the call returns
  for (int k = 0; k < s->slots; ++k) (void)hipStreamSynchronize(s->streams[k]);
  (void)hipStreamSynchronize(s->refresh);
  poll_launches();
  poll_refreshes();
  s->spare_events.push_back(t0);
  s->st.held_bytes = s->held;
  return run_status;
}

fsp_status fsp_server_get_stats(fsp_server s, fsp_server_stats* out) {
  if (!s || !out) return srv_fail(FSP_ERR_INVALID_ARG, "fsp_server_get_stats: NULL argument");
  s->st.held_bytes = s->held;
  *out = s->st;
  return FSP_OK;
}

fsp_status fsp_server_destroy(fsp_server s) {
  if (!s) return srv_fail(FSP_ERR_INVALID_ARG, "fsp_server_destroy: NULL server");
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamSynchronize(st);
  if (s->refresh) (void)hipStreamSynchronize(s->refresh);
  for (auto& kv : s->cache) drop_entry(s, kv.second.get());
  s->cache.clear();
  for (auto& w : s->pool) (void)hipFree(w->work);
  s->pool.clear();
  for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->refresh) (void)hipStreamDestroy(s->refresh);
  if (s->tick_buf) (void)hipFree(s->tick_buf);
  delete s;
  return FSP_OK;
}

}  // extern "C"
