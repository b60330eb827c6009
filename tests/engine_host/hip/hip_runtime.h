// Host-only stand-in for the HIP runtime, used to compile the serving engine
// (serve_engine.hip) as plain C++ on the CPU under AddressSanitizer: device
// memory is host memory whose live blocks are tracked, streams are inert,
// events complete after a few queries, kernels run on the host.
#pragma once

#include <cstddef>

typedef int hipError_t;
enum : int { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNotReady = 600 };
typedef struct MockStream* hipStream_t;
typedef struct MockEvent* hipEvent_t;
constexpr unsigned hipStreamNonBlocking = 1u;

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct MockIdx {
  unsigned x = 0, y = 0, z = 0;
};
extern MockIdx threadIdx, blockIdx;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) kernel(__VA_ARGS__)

hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipMalloc(void** p, size_t bytes);
template <class T>
hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
hipError_t hipFree(void* p);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
