// Host emulation of the parts of the HIP runtime and device language that
// the library's sources use, for the CPU test that runs the real kernel
// sources on the host under AddressSanitizer.  A workgroup's threads are
// cooperative fibers; barriers, wave-wide exchanges (shuffles, DPP moves,
// permlane swaps) and readfirstlane synchronise the fibers they involve, and
// a barrier that some participants can never reach is reported.  Device
// memory is host memory.
#pragma once
#include <math.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct alignas(16) float4 {
  float x, y, z, w;
};
struct alignas(16) double2 {
  double x, y;
};
struct alignas(8) float2 {
  float x, y;
};

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx {
  unsigned x, y, z;
};
extern EmuIdx threadIdx, blockIdx, blockDim, gridDim;

typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotSupported = 801
};
enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
};
typedef struct EmuStream* hipStream_t;
typedef struct EmuEvent* hipEvent_t;
typedef struct EmuGraph* hipGraph_t;
typedef struct EmuGraphExec* hipGraphExec_t;
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1
};

hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t s);
hipError_t hipMemcpy(void* d, const void* s, size_t bytes, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t bytes,
                          hipMemcpyKind k, hipStream_t st);
hipError_t hipMemcpy2D(void* d, size_t dp, const void* s, size_t sp,
                       size_t w, size_t h, hipMemcpyKind k);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetDevice(int* d);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, char*,
                               size_t);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
#define HIP_SYMBOL(x) (&(x))
template <typename S>
hipError_t hipGetSymbolAddress(void** p, S* sym) {
  *p = (void*)sym;
  return hipSuccess;
}

// device-side builtins
void __syncthreads();
double __shfl_xor(double v, int mask, int width = 64);
float __shfl_xor(float v, int mask, int width = 64);
int __shfl_xor(int v, int mask, int width = 64);
inline unsigned __umulhi(unsigned a, unsigned b) {
  return (unsigned)(((uint64_t)a * (uint64_t)b) >> 32);
}
int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                   bool bound_ctrl);
struct EmuPair {
  unsigned v[2];
  unsigned operator[](int i) const { return v[i]; }
};
EmuPair emu_permlane32_swap(unsigned a, unsigned b, bool fi, bool bc);
EmuPair emu_permlane16_swap(unsigned a, unsigned b, bool fi, bool bc);
int emu_readfirstlane(int v);
#define __builtin_amdgcn_update_dpp emu_update_dpp
#define __builtin_amdgcn_permlane32_swap emu_permlane32_swap
#define __builtin_amdgcn_permlane16_swap emu_permlane16_swap
#define __builtin_amdgcn_readfirstlane emu_readfirstlane

// fibers of a workgroup never interleave inside one call: plain updates
inline int atomicOr(int* p, int v) {
  const int o = *p;
  *p = o | v;
  return o;
}

using std::isfinite;
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }

// kernel launches run every workgroup to completion before returning
void emu_launch(dim3 grid, dim3 block, const std::function<void()>& body);
#define HIP_KERNEL_NAME(...) __VA_ARGS__
template <typename... KArgs, typename... Args>
void hipLaunchKernelGGL(void (*k)(KArgs...), dim3 grid, dim3 block,
                        size_t shmem, hipStream_t s, Args... args) {
  (void)shmem;
  (void)s;
  emu_launch(grid, block, [&]() { k(args...); });
}
