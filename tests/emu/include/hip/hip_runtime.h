// Host emulation of the HIP language and runtime subset that libsgspm uses.
//
// Test infrastructure only: the kernel sources compile with g++ against this
// header, every launch runs its workgroups on the CPU (one fiber per work-item,
// __syncthreads and wave shuffles as scheduling points), device allocations are
// host allocations of the exact size, and LDS is one host array whose bytes
// past the launch's dynamic size are poisoned for AddressSanitizer.  Built with
// -fsanitize=address, every global and LDS access of a kernel is checked
// against its allocation.  Nothing here is part of the library.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#define __global__
#define __device__
#define __host__
#define __shared__
#define __constant__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))

using std::isfinite;
using std::isinf;
using std::isnan;
using std::signbit;

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern dim3 threadIdx, blockIdx, blockDim, gridDim;

// min and max of the device library (by value, in the common type)
template <typename A, typename B> inline typename std::common_type<A, B>::type min(A a, B b) { return a < b ? a : b; }
template <typename A, typename B> inline typename std::common_type<A, B>::type max(A a, B b) { return a < b ? b : a; }

void __syncthreads();
float __shfl_down(float v, unsigned d, int width = 64);
double __shfl_down(double v, unsigned d, int width = 64);
int __shfl_down(int v, unsigned d, int width = 64);

// ---- runtime
typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotSupported = 801,
  hipErrorLaunchFailure = 719,
} hipError_t;
typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;
typedef enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed } hipStreamCaptureMode;
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph* hipGraph_t;
typedef struct hipGraphExec* hipGraphExec_t;
typedef struct hipGraphNode* hipGraphNode_t;
#define hipStreamNonBlocking 0x1
#define hipEventDisableSystemFence 0x20000000
#define HIP_SYMBOL(x) ((const void*)&(x))

hipError_t hipMalloc(void** p, size_t n);
template <typename T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st = nullptr);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st = nullptr);
hipError_t hipMemset(void* d, int v, size_t n);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int* d);
hipError_t hipSetDevice(int d);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* n, char* log, size_t sz);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGetSymbolAddress(void** p, const void* sym);

// ---- launches
namespace emu {
struct Launch {
  void (*body)(void*);
  void* ctx;
};
// Runs the workgroups of a launch (all, or a spread subset when the emulator is
// told to sample) with `lds` bytes of dynamic LDS; records an error for an
// invalid geometry instead of running.
void run_launch(const char* name, dim3 grid, dim3 block, size_t lds, const Launch& l);
template <typename F> void body_thunk(void* p) { (*static_cast<F*>(p))(); }
template <typename... KA, typename... A>
void launch(const char* name, void (*k)(KA...), dim3 grid, dim3 block, size_t lds, hipStream_t, A&&... args) {
  auto f = [&]() { k(args...); };
  run_launch(name, grid, block, lds, Launch{&body_thunk<decltype(f)>, &f});
}
}  // namespace emu
#define hipLaunchKernelGGL(K, G, B, L, S, ...) ::emu::launch(#K, K, G, B, L, S, __VA_ARGS__)
