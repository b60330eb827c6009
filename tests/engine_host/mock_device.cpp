// The stand-in device of tests/engine_host/hip/hip_runtime.h and the library
// calls the serving engine makes (plans, precompute, the solve launch), for a
// CPU build of serve_engine.hip.  Every device pointer a solve or a precompute
// receives is checked against the live allocations: a use of freed (or never
// allocated) device memory is counted as a device fault.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "fsp.h"
#include "internal.hpp"

MockIdx threadIdx, blockIdx;

// Streams hold queues of operations that run later, in stream order: a
// kernel (with the device ranges it touches), an event record, a wait for
// another stream's event.  Work advances when the engine queries an event or
// synchronizes, and also a little at random on every query (the device runs
// on its own), so an operation may run long after it was enqueued.  A device
// range is checked when its operation RUNS: memory freed after enqueue and
// before that is a fault.  hipFree does not wait for queued work (the stricter
// of the two behaviours a runtime may have).
struct MockEvent;
struct Op {
  int kind;                      // 0 kernel, 1 record, 2 wait
  std::vector<std::pair<const char*, size_t>> ranges;
  std::string what;
  MockEvent* ev = nullptr;       // record: the event
  MockStream* wait_stream = nullptr;  // wait: stream and index of the awaited record,
  long long wait_pos = -1;            // as they were when the wait was enqueued
};
struct MockStream {
  int id;
  std::deque<Op> ops;
  long long done_ops = 0;        // operations run so far
};
struct MockEvent {
  MockStream* stream = nullptr;  // stream of the last record
  long long pos = -1;            // its index on that stream (-1: never recorded)
  long long epoch = 0;           // records so far
  double t = 0;
};

namespace mock {
std::map<const char*, size_t> live;   // device allocations: base -> bytes
long long faults = 0, mallocs = 0, frees = 0, solves = 0, precomputes = 0;
double clock_ms = 0;
std::vector<MockStream*> streams;
unsigned rng_state = 7;
unsigned rnd() {
  rng_state = rng_state * 1103515245u + 12345u;
  return rng_state >> 16;
}

bool inside(const void* p, size_t bytes) {
  const char* c = static_cast<const char*>(p);
  auto it = live.upper_bound(c);
  if (it == live.begin()) return false;
  --it;
  return c >= it->first && c + bytes <= it->first + it->second;
}

void fault(const std::string& what) {
  ++faults;
  std::fprintf(stderr, "mock device fault: %s\n", what.c_str());
}


// Run the next operation of s if it can run; true when it ran.
bool step(MockStream* s) {
  if (s->ops.empty()) return false;
  Op& op = s->ops.front();
  if (op.kind == 2 && op.wait_stream && op.wait_stream->done_ops <= op.wait_pos) return false;
  if (op.kind == 0)
    for (auto& r : op.ranges)
      if (!inside(r.first, r.second)) fault(op.what + " touches memory that is no longer allocated");
  if (op.kind == 1) {
    clock_ms += 0.01;
    op.ev->t = clock_ms;
  }
  s->ops.pop_front();
  ++s->done_ops;
  return true;
}

// Advance stream s until event e's record has run (running other streams as needed).
void run_until(MockEvent* e) {
  for (int guard = 0; guard < 1000000 && e->stream && e->stream->done_ops <= e->pos; ++guard) {
    if (!step(e->stream))
      for (MockStream* o : streams) step(o);   // s waits on another stream
  }
}

void drift() {  // the device makes some progress on its own
  for (MockStream* o : streams)
    for (unsigned k = rnd() % 3; k > 0; --k) step(o);
}

void enqueue(MockStream* s, Op op) {
  if (!s) s = streams.empty() ? nullptr : streams[0];
  if (!s) return;
  s->ops.push_back(std::move(op));
}
}  // namespace mock

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipMalloc(void** p, size_t bytes) {
  char* b = static_cast<char*>(std::malloc(bytes ? bytes : 1));
  if (!b) return hipErrorOutOfMemory;
  mock::live[b] = bytes;
  ++mock::mallocs;
  *p = b;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  auto it = mock::live.find(static_cast<const char*>(p));
  if (it == mock::live.end()) {
    mock::fault("hipFree of memory that is not a live allocation");
    return hipErrorInvalidValue;
  }
  mock::live.erase(it);
  ++mock::frees;
  std::free(p);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  static int next = 0;
  *s = new MockStream{next++, {}, 0};
  mock::streams.push_back(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  while (!s->ops.empty())
    if (!mock::step(s))
      for (MockStream* o : mock::streams) mock::step(o);
  mock::streams.erase(std::find(mock::streams.begin(), mock::streams.end(), s));
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  for (int guard = 0; guard < 1000000 && !s->ops.empty(); ++guard)
    if (!mock::step(s))
      for (MockStream* o : mock::streams) mock::step(o);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  Op op;
  op.kind = 2;
  op.wait_stream = e->stream;
  op.wait_pos = e->pos;
  mock::enqueue(s, std::move(op));
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new MockEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (!s) s = mock::streams.empty() ? nullptr : mock::streams[0];
  e->stream = s;
  e->pos = s->done_ops + (long long)s->ops.size();
  ++e->epoch;
  Op op;
  op.kind = 1;
  op.ev = e;
  mock::enqueue(s, std::move(op));
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  mock::drift();
  if (!e->stream || e->stream->done_ops > e->pos) return hipSuccess;
  return hipErrorNotReady;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)(b->t - a->t);
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock error"; }

// ------------------------------------------------------------------ library calls
struct fsp_plan_s {
  fsp_plan_desc d;
  size_t ghat = 0, work = 0, pre = 0;
  void* buf = nullptr;
};

namespace {
thread_local std::string g_err;
bool supported(int n) {
  switch (n) {
    case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 192: case 256:
    case 384: case 512: return true;
    default: return false;
  }
}
}  // namespace

extern "C" {
fsp_status fsp_plan_create(const fsp_plan_desc* d, fsp_plan* out) {
  if (!d || !out) return FSP_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    if (!supported(d->n[a])) {
      g_err = "unsupported size";
      return FSP_ERR_UNSUPPORTED_SIZE;
    }
  auto* p = new fsp_plan_s();
  p->d = *d;
  const size_t s = d->prec == FSP_F64 ? 8 : 4;
  const size_t n0 = d->n[0], n1 = d->n[1], n2 = d->n[2];
  p->ghat = 4096 + (n0 + 1) * (n1 + 1) * (n2 + 16) * s;
  p->work = n0 * 2 * n1 * (n2 + 16) * 2 * s;
  p->pre = d->greens == FSP_HOCKNEY ? 16 * (n0 + 1) * (n1 + 1) * (n2 + 1)
                                    : 12 * (2 * n0 + 1) * (2 * n1 + 1) * (2 * n2 + 1);
  *out = p;
  return FSP_OK;
}
fsp_status fsp_plan_destroy(fsp_plan p) {
  if (!p) return FSP_ERR_INVALID_ARG;
  delete p;
  return FSP_OK;
}
fsp_status fsp_precompute(fsp_plan p, void* stream) {
  if (!p || !p->buf) return FSP_ERR_NOT_READY;
  if (!mock::inside(p->buf, p->ghat)) mock::fault("precompute into memory that is not live (at enqueue)");
  Op op;
  op.kind = 0;
  op.what = "precompute";
  op.ranges.push_back({static_cast<const char*>(p->buf), p->ghat});
  mock::enqueue(static_cast<hipStream_t>(stream), std::move(op));
  ++mock::precomputes;
  return FSP_OK;
}
const char* fsp_last_error(void) { return g_err.c_str(); }
}

namespace fsp {
namespace internal {
hipError_t solve_items(fsp_plan geo, int count, const void* const* rho, void* const* phi, void* const* work,
                       const void* const* octant, hipStream_t s) {
  Op op;
  op.kind = 0;
  op.what = "solve";
  if (!mock::inside(geo->buf, geo->ghat)) mock::fault("solve enqueued with the twiddles of a freed Green's buffer");
  op.ranges.push_back({static_cast<const char*>(geo->buf), geo->ghat});
  for (int i = 0; i < count; ++i) {
    if (!work[i] || !mock::inside(work[i], geo->work)) mock::fault("solve enqueued with a workspace that is not live");
    if (!octant[i] || !mock::inside(octant[i], 1)) mock::fault("solve enqueued with an octant that is not live");
    if (!rho[i] || !phi[i]) mock::fault("solve with a NULL array");
    op.ranges.push_back({static_cast<const char*>(work[i]), geo->work});
    op.ranges.push_back({static_cast<const char*>(octant[i]), 1});
  }
  mock::enqueue(s, std::move(op));
  ++mock::solves;
  return hipSuccess;
}
size_t work1_bytes(fsp_plan p) { return p->work; }
size_t ghat_bytes(fsp_plan p) { return p->ghat; }
size_t precompute_bytes(fsp_plan p) { return p->pre; }
const void* octant(fsp_plan p) { return static_cast<const char*>(p->buf) + 64; }
fsp_status bind_ghat(fsp_plan p, void* buf) {
  p->buf = buf;
  return FSP_OK;
}
const char* last_error() { return g_err.c_str(); }
void set_error(const std::string& m) { g_err = m; }
}  // namespace internal
}  // namespace fsp
