// lc_reduce.hpp -- wave and block sums of the fused kernels, in a fixed
// order (so a colloid's force has the same bits on every run).
#pragma once

#include <hip/hip_runtime.h>

namespace lc {

template <typename R>
__device__ inline R wave_sum(R v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sums over the 64 lanes of a full wave of NV <= 16 doubles per lane, in a
// fixed order.  The values are padded to P = 2^LOG; at exchange s the lanes
// split on lane bit 5-s, each keeping one half of its values and adding the
// partner's copy of that half, so P-1 shuffles reduce all of them at once;
// the remaining lane bits are then summed.  Lane l returns the total of
// value (l >> (6 - LOG)), repeated in 64 >> LOG consecutive lanes.
template <int NV>
struct WaveSums {
  static constexpr int LOG = NV <= 1 ? 0 : NV <= 2 ? 1 : NV <= 4 ? 2 : NV <= 8 ? 3 : 4;
  static constexpr int P = 1 << LOG;
  static constexpr int REP = 64 >> LOG;   // lanes holding each total
  __device__ static double run(const double (&v)[NV]) {
    static_assert(NV <= 16, "at most 16 values");
    double w[P];
#pragma unroll
    for (int i = 0; i < P; i++) w[i] = i < NV ? v[i] : 0.0;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < LOG; s++) {
      const int half = P >> (s + 1);
      const bool hi = (lane >> (5 - s)) & 1;
#pragma unroll
      for (int j = 0; j < half; j++) {
        const double send = hi ? w[j] : w[j + half];
        const double keep = hi ? w[j + half] : w[j];
        w[j] = keep + __shfl_xor(send, 32 >> s, 64);
      }
    }
    double r = w[0];
#pragma unroll
    for (int o = REP >> 1; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
    return r;
  }
  __device__ static int index() { return (threadIdx.x & 63) >> (6 - LOG); }
  __device__ static bool writer() { return ((threadIdx.x & 63) & (REP - 1)) == 0 && index() < NV; }
};

// Reduce n doubles per thread over the block into out[k * stride],
// k = 0..n-1 (threads < n).
template <int NT, int NV>
__device__ inline void block_sum(double (&v)[NV], double* sred, double* out, long long stride = 1) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6;
  {
    const double s = WaveSums<NV>::run(v);
    if (WaveSums<NV>::writer()) sred[w * NV + WaveSums<NV>::index()] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int i = 0; i < NW; i++) s += sred[i * NV + threadIdx.x];
    out[threadIdx.x * stride] = s;
  }
}

}  // namespace lc
