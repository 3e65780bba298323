// Host build of the library's HIP sources, for checking them on the CPU (test
// infrastructure: the package never loads what is built from this header).
//
// The kernels compile as ordinary C++ (clang, x86-64).  Each lane of a
// workgroup is a fiber (emu_runtime.cpp); workgroups of a launch run one after
// another; the wave-level operations the kernels use (FP64 MFMA 16x16x4, DPP
// row permutations, readlane, shuffles) take the values of all live lanes of
// the wave at once, as the hardware does.  Shared memory is a static object per
// kernel, device memory is host memory, and the runtime calls the host code
// makes are served by plain host functions.
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...)
#define __constant__ static
#define __align__(n) __attribute__((aligned(n)))
#ifdef EMU_LDS_SECTION
// every shared-memory object in one linker section, so that the runtime can
// find (and fill, and shadow) all of it
#define __shared__ static __attribute__((section("emu_lds")))
#else
#define __shared__ static
#endif

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotSupported = 801 };
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef int hipStreamCaptureStatus;
enum { hipStreamCaptureStatusNone = 0 };
enum hipMemcpyKind {
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
};
enum hipDeviceAttribute_t {
  hipDeviceAttributeMultiprocessorCount = 1,
  hipDeviceAttributeWallClockRate = 2
};
#define HIP_MEMORY_SCOPE_AGENT 2
#define __HIP_MEMORY_SCOPE_AGENT 2
#define HIP_SYMBOL(X) ((const void*)&(X))

namespace emu {
struct Lane {
  dim3 tid;
};
extern Lane* g_cur;
extern dim3 g_block, g_bdim, g_gdim;
void launch(dim3 grid, dim3 block, const std::function<void()>& body);
void syncthreads(const char* file, int line);
double shfl(double v, int src, const char* file, int line);
double shfl_xor(double v, int mask, const char* file, int line);
int readlane(int v, int lane, const char* file, int line);
int mov_dpp(int v, int ctrl, const char* file, int line);
typedef double v4 __attribute__((ext_vector_type(4)));
v4 mfma_f64(double a, double b, v4 c, const char* file, int line);
uint64_t clock64();
void sleep_yield();
}  // namespace emu

#define threadIdx (emu::g_cur->tid)
#define blockIdx (emu::g_block)
#define blockDim (emu::g_bdim)
#define gridDim (emu::g_gdim)

#define __syncthreads() emu::syncthreads(__FILE__, __LINE__)
#define __shfl(v, s, w) emu::shfl((v), (s), __FILE__, __LINE__)
#define __shfl_xor(v, m, w) emu::shfl_xor((v), (m), __FILE__, __LINE__)
#define __builtin_amdgcn_readlane(v, l) emu::readlane((v), (l), __FILE__, __LINE__)
#define __builtin_amdgcn_mov_dpp(v, c, rm, bm, bc) emu::mov_dpp((v), (c), __FILE__, __LINE__)
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) \
  emu::mfma_f64((a), (b), (c), __FILE__, __LINE__)
// the kernels refine these estimates by Newton steps; exact values here
#define __builtin_amdgcn_rsq(x) (1.0 / sqrt((double)(x)))
#define __builtin_amdgcn_rcp(x) (1.0 / (double)(x))
#define __builtin_amdgcn_s_sleep(n) emu::sleep_yield()
#define __builtin_amdgcn_fence(order, scope) __atomic_thread_fence(order)
#define wall_clock64() emu::clock64()
#define __threadfence() __atomic_thread_fence(__ATOMIC_SEQ_CST)

static inline long long __double_as_longlong(double x) {
  long long r;
  memcpy(&r, &x, 8);
  return r;
}
static inline double __longlong_as_double(long long x) {
  double r;
  memcpy(&r, &x, 8);
  return r;
}

static inline int atomicCAS(int* p, int cmp, int val) {
  __atomic_compare_exchange_n(p, &cmp, val, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
static inline unsigned atomicCAS(unsigned* p, unsigned cmp, unsigned val) {
  __atomic_compare_exchange_n(p, &cmp, val, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
static inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }

template <class T>
static inline T min(T a, T b) { return b < a ? b : a; }
template <class T>
static inline T max(T a, T b) { return a < b ? b : a; }

#define hipLaunchKernelGGL(K, G, B, SHM, ST, ...) \
  emu::launch(dim3(G), dim3(B), [=]() { K(__VA_ARGS__); })

extern "C" {
hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st);
hipError_t hipStreamSynchronize(hipStream_t st);
hipError_t hipStreamIsCapturing(hipStream_t st, hipStreamCaptureStatus* s);
hipError_t hipGetDevice(int* d);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t st);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetLastError(void);
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetSymbolAddress(void** p, const void* sym);
}
template <class F>
static inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F, int, size_t) {
  *n = 1;
  return hipSuccess;
}
