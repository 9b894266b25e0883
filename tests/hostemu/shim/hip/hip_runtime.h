// Test-only host stand-in for <hip/hip_runtime.h>: it lets the library's
// kernel sources compile as ordinary host C++ (kernels become functions, a
// wave has one lane, device memory is host memory, launches compile to
// nothing), so that tests/test_host_emulation.py can run the per-ray code of
// the kernels under the host's AddressSanitizer, UndefinedBehaviorSanitizer
// and MemorySanitizer.  The library itself is never built against it.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline __attribute__((always_inline))
#define __shared__ static
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
struct emu_dim3 { unsigned x = 0, y = 0, z = 0; };
inline thread_local emu_dim3 threadIdx, blockIdx, blockDim{64, 1, 1}, gridDim{1, 1, 1};
struct dim3 { unsigned x, y, z; dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
// one lane per wave: a ballot is the lane's own predicate
inline unsigned long long __ballot(int p) { return p ? 1ull : 0ull; }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
template <typename T> inline T __shfl(T v, int, int = 64) { return v; }
template <typename T> inline T __shfl_xor(T v, int, int = 64) { return v; }
inline void __syncthreads() {}
template <typename T> inline T atomicAdd(T *p, T v) { T o = *p; *p = o + v; return o; }
inline float __expf(float x) { return expf(x); }
inline float __logf(float x) { return logf(x); }
inline float __sinf(float x) { return sinf(x); }
inline float __cosf(float x) { return cosf(x); }
inline float rsqrtf(float x) { return 1.0f / sqrtf(x); }
#define __builtin_amdgcn_rcpf(x) (1.0f / (float)(x))
#define __builtin_amdgcn_rcp(x) (1.0 / (double)(x))
#define __builtin_amdgcn_rsq(x) (1.0 / sqrt((double)(x)))
#define __builtin_amdgcn_sqrt(x) sqrt((double)(x))
inline int emu_frexp_exp(double x) { int e; frexp(x, &e); return e; }
inline double emu_frexp_mant(double x) { int e; return frexp(x, &e); }
#define __builtin_amdgcn_frexp_exp(x) emu_frexp_exp(x)
#define __builtin_amdgcn_frexp_mant(x) emu_frexp_mant(x)
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, ...) (c)
#define __builtin_amdgcn_fence(...) ((void)0)
#define __builtin_amdgcn_wave_barrier() ((void)0)
// runtime API: host memory, no launches; hardware estimates replaced by
// their exact definitions
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum { hipDeviceAttributeMultiprocessorCount = 0 };
#define hipEventDisableTiming 0
inline hipError_t hipMalloc(void **p, size_t n) { *p = malloc(n ? n : 1); return *p ? 0 : 2; }
template <typename T> inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc((void **)p, n); }
inline hipError_t hipFree(void *p) { free(p); return 0; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return 0; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t = 0) { memcpy(d, s, n); return 0; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
inline hipError_t hipSetDevice(int) { return 0; }
inline hipError_t hipGetLastError() { return 0; }
inline const char *hipGetErrorString(hipError_t) { return "emu"; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = nullptr; return 0; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = nullptr; return 0; }
inline hipError_t hipEventDestroy(hipEvent_t) { return 0; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = 0) { return 0; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return 0; }
inline hipError_t hipEventElapsedTime(float *m, hipEvent_t, hipEvent_t) { *m = 0; return 0; }
inline hipError_t hipMemGetInfo(size_t *f, size_t *t) { *f = *t = (size_t)1 << 36; return 0; }
inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return 0; }
inline hipError_t hipDeviceGetAttribute(int *v, int, int) { *v = 256; return 0; }
template <typename K> inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, K, int, size_t) { *n = 1; return 0; }
#define hipGetSymbolAddress(p, s) (*(p) = (void *)&(s), 0)
#define HIP_SYMBOL(s) s
#define hipLaunchKernelGGL(...) ((void)0)
using std::sqrt; using std::fabs; using std::floor; using std::fmin; using std::fmax; using std::exp;
using std::log; using std::sin; using std::cos; using std::fma; using std::rint; using std::ldexp;
using std::isnan; using std::isfinite; using std::log1p; using std::expm1; using std::pow; using std::ceil;
inline float __fdividef(float a, float b) { return a / b; }
template <typename T> inline T min(T a, T b) { return a < b ? a : b; }
template <typename T> inline T max(T a, T b) { return a > b ? a : b; }
