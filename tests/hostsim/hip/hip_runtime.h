// Host stand-in for the HIP runtime header, for the CPU build of the
// marching kernel in tests/hostsim (test infrastructure only).
//
// A block of the kernel runs as one OS thread per GPU thread.  Barriers
// and wave operations are real rendezvous between those threads (with a
// time limit that reports a thread that never arrives, e.g. a barrier or a
// shuffle inside divergent code).  __shared__ objects go into their own
// section, which the driver fills with 0xff bytes (NaN in FP32 and FP64,
// 255 as a solid flag) before every block, so a read of LDS that the block
// has not written shows up in the results.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static __attribute__((section("hostsim_lds")))

struct int2 {
  int x, y;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }
struct dim3 {
  unsigned x = 0, y = 0, z = 0;
};
typedef int hipError_t;
typedef struct hostsim_stream* hipStream_t;
typedef struct hostsim_event* hipEvent_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };

namespace hostsim {

extern thread_local dim3 thread_idx, block_idx;

// Rendezvous of every live thread of the block; aborts with `what` if the
// others do not arrive in time.
void block_barrier(const char* what);
// Rendezvous of the 64 lanes of the caller's wave: each lane publishes one
// 64-bit word and receives all 64.
void wave_gather(uint64_t mine, uint64_t all[64], const char* what);
[[noreturn]] void fail(const char* fmt, ...);

template <typename T>
T shfl(T v, int src, const char* what) {
  static_assert(sizeof(T) <= 8, "64-bit words at most");
  uint64_t w = 0;
  std::memcpy(&w, &v, sizeof(T));
  uint64_t all[64];
  wave_gather(w, all, what);
  const uint64_t r = all[src];
  T out;
  std::memcpy(&out, &r, sizeof(T));
  return out;
}

}  // namespace hostsim

#define threadIdx hostsim::thread_idx
#define blockIdx hostsim::block_idx

inline void __syncthreads() { hostsim::block_barrier("__syncthreads"); }

template <typename T>
T __shfl_xor(T v, int mask, int width = 64) {
  if (width != 64) hostsim::fail("__shfl_xor: width %d", width);
  return hostsim::shfl(v, (int)(threadIdx.x & 63) ^ mask, "__shfl_xor");
}
template <typename T>
T __shfl_down(T v, unsigned d, int width = 64) {
  if (width != 64) hostsim::fail("__shfl_down: width %d", width);
  const int src = (int)(threadIdx.x & 63) + (int)d;
  return hostsim::shfl(v, src < 64 ? src : (int)(threadIdx.x & 63), "__shfl_down");
}
inline int __any(int pred) {
  uint64_t all[64];
  hostsim::wave_gather((uint64_t)(pred != 0), all, "__any");
  int any = 0;
  for (int l = 0; l < 64; l++) any |= (int)all[l];
  return any;
}
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }
inline unsigned long long atomicAdd(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}

// Round-to-nearest FP64 operations (the build uses -ffp-contract=off).
inline double __dadd_rn(double a, double b) { return a + b; }
inline double __dsub_rn(double a, double b) { return a - b; }
inline double __dmul_rn(double a, double b) { return a * b; }
// The hardware reciprocal is within an ulp of 1/x; the kernel refines it
// with a Newton step.
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }
