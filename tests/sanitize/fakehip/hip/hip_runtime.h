// Host-only stand-in for the HIP runtime, for building the library's host
// code (table construction, the C ABI's argument handling, the request
// dispatcher's threads and queues) under ASan / UBSan / TSan on a machine
// without a GPU.  "Device" memory is host memory, streams run nothing
// asynchronously: a kernel launch executes the kernel serially on the
// calling thread (only element-wise kernels are meant to run this way),
// events are complete as soon as they are recorded.  Test infrastructure
// only; never part of the library build.
#pragma once
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <atomic>

#define __host__
#define __device__
#define __forceinline__ inline
#define __global__
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__

typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidSymbol = 13,
  hipErrorNotReady = 600,
};
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 16 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };

struct uint2 { unsigned int x, y; };
struct uint4 { unsigned int x, y, z, w; };
inline uint2 make_uint2(unsigned int x, unsigned int y) { return uint2{x, y}; }
inline uint4 make_uint4(unsigned int x, unsigned int y, unsigned int z, unsigned int w) { return uint4{x, y, z, w}; }
struct dim3 {
  unsigned int x = 1, y = 1, z = 1;
  dim3() = default;
  dim3(unsigned int a, unsigned int b = 1, unsigned int c = 1) : x(a), y(b), z(c) {}
};
inline thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;

struct fakehip_stream { int dummy; };
struct fakehip_event { std::atomic<int> recorded{0}; };
typedef fakehip_stream* hipStream_t;
typedef fakehip_event* hipEvent_t;

inline hipError_t hipMalloc(void** p, size_t n) {
  *p = std::aligned_alloc(256, (n + 255) / 256 * 256 + 256);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDeviceCount(int* c) { *c = 1; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "fake HIP error"; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new fakehip_stream{0}; return hipSuccess; }
inline hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new fakehip_event(); return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->recorded.store(1); return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
template <typename K>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, size_t) { *n = 1; return hipSuccess; }
#define HIP_SYMBOL(x) ((const void*)&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }

// A launch runs every thread of every block in turn on the calling thread.
template <typename K, typename... A>
void fakehip_launch(K kernel, dim3 grid, dim3 block, A... args) {
  gridDim = grid;
  blockDim = block;
  for (unsigned bx = 0; bx < grid.x; ++bx)
    for (unsigned tx = 0; tx < block.x; ++tx) {
      blockIdx = dim3(bx);
      threadIdx = dim3(tx);
      kernel(args...);
    }
}
#define hipLaunchKernelGGL(kernel, grid, block, shm, stream, ...) fakehip_launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)
