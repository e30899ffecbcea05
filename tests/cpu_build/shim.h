// One-lane stand-ins for the HIP device built-ins used by gt_device.h, so
// the tracker's per-lane logic can be compiled for and run on a CPU (test
// infrastructure; the library itself is never built this way).  A wave has
// one lane and a workgroup one wave: ballots return that lane's bit, ranks
// are 0, shuffles and read-first-lane are the identity, barriers are empty.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#undef __device__
#undef __host__
#undef __global__
#undef __forceinline__
#undef __shared__
#undef __launch_bounds__
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __shared__ static
#define __launch_bounds__(x)
#undef threadIdx
#undef blockIdx
#undef blockDim
#undef gridDim
struct CpuDim3 {
    unsigned x = 0, y = 0, z = 0;
};
static thread_local CpuDim3 threadIdx, blockIdx, blockDim{1, 1, 1}, gridDim{1, 1, 1};

static inline uint64_t __ballot(int p) { return p ? 1ull : 0ull; }
static inline int __popcll(unsigned long long m) { return __builtin_popcountll(m); }
static inline int __ffsll(unsigned long long m) { return __builtin_ffsll((long long)m); }
static inline unsigned __lane_id() { return 0; }
template <typename T> static inline T __shfl(T v, int) { return v; }
template <typename T> static inline T __shfl_up(T v, unsigned) { return v; }   // no lane below lane 0
template <typename T> static inline T __shfl_xor(T v, int) { return v; }
static inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t, uint32_t c) { return c; }
static inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t, uint32_t c) { return c; }
template <typename T> static inline T __builtin_amdgcn_readfirstlane(T v) { return v; }
static inline void __builtin_amdgcn_s_sleep(int) {}
static inline uint32_t __builtin_amdgcn_s_getreg(int) { return 0; }
static inline void __syncthreads() {}
static inline long long __double_as_longlong(double d) { long long v; std::memcpy(&v, &d, 8); return v; }
static inline double __longlong_as_double(long long v) { double d; std::memcpy(&d, &v, 8); return d; }
static inline uint32_t __float_as_uint(float f) { uint32_t v; std::memcpy(&v, &f, 4); return v; }
static inline float __uint_as_float(uint32_t v) { float f; std::memcpy(&f, &v, 4); return f; }
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
template <typename T> static inline T atomicAdd(T *p, T v) { T o = *p; *p = o + v; return o; }
template <typename T, typename V> static inline T cpu_atomic_fetch_add(T *p, V v, int, int) {
    T o = *p;
    *p = o + (T)v;
    return o;
}
#define __hip_atomic_fetch_add cpu_atomic_fetch_add
template <typename T> static inline T cpu_atomic_load(T *p, int, int) { return *p; }
#define __hip_atomic_load cpu_atomic_load
#undef __HIP_MEMORY_SCOPE_WORKGROUP
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
#undef __HIP_MEMORY_SCOPE_AGENT
#define __HIP_MEMORY_SCOPE_AGENT 0
template <typename A, typename B> static inline A min(A a, B b) { return a < (A)b ? a : (A)b; }
template <typename A, typename B> static inline A max(A a, B b) { return a > (A)b ? a : (A)b; }
#define GT_AS(n)
