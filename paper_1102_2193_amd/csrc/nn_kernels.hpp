// nn_kernels.hpp -- launch interface of the warm-start network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcnn {

struct Case {
  double pos[3];
  double a0;
  double pitch;
  int anchoring;
  int pad_;
  double q_amp;
  double q_eq;
};

hipError_t launch_features(int L, const Case& c, uint16_t* x0, float* f32, hipStream_t s);
// mode 0: bias + SiLU (z and bf16 activation); 1: bias, FP32 out; 2: times
// silu'(zprev), bf16 out; 3: FP32 out
hipError_t launch_conv(int cinp, int coutp, int mode, int L, const uint16_t* x, const uint16_t* w, const float* bias,
                       const float* zprev, float* zout, uint16_t* aout, hipStream_t s);
// The first layer (16 -> 32, mode 0 or 4) with its input features computed
// in the halo staging instead of read; xf (if not null) receives them
// (BF16 [V][16], as launch_features without f32 writes).
hipError_t launch_conv_feat(int mode, int L, const Case& c, const uint16_t* w, const float* bias, float* zout,
                            uint16_t* aout, uint16_t* xf, hipStream_t s);
// Weight and bias gradients of a layer: per-block partials (nblk blocks of
// tpb tiles; 27 coutp cinp + coutp floats each), then their fixed-order sum
// into dW [cout][cin][27] and db [cout].
hipError_t launch_wgrad(int cinp, int coutp, int L, int nblk, int tpb, const uint16_t* dz, const uint16_t* x,
                        float* part, hipStream_t s);
hipError_t launch_wgrad_reduce(int nblk, int coutp, int cinp, int cout, int cin, const float* part, float* dW,
                               float* db, hipStream_t s);
// The same sums, each followed by the layer's Adam step on that weight or
// bias (as launch_adam with update 1) instead of being stored.
hipError_t launch_wgrad_adam(int nblk, int coutp, int cinp, int cout, int cin, const float* part, float* W, float* b,
                             float* mW, float* vW, float* mb, float* vb, float lr, float c1, float c2, uint16_t* wf,
                             uint16_t* wb, hipStream_t s);
hipError_t launch_loss(int L, const Case& c, const float* out, const float* Qt, const uint8_t* fluid, double inv_nf,
                       uint16_t* dz, double* part, hipStream_t s);
template <typename R>
hipError_t launch_warm(int L, const Case& c, const float* out, R* Q, long long nsites, long long off, hipStream_t s);
hipError_t launch_adam(int cout, int cin, int coutp, int cinp, float* W, float* b, const float* dW, const float* db,
                       float* mW, float* vW, float* mb, float* vb, float lr, float c1, float c2, int update,
                       uint16_t* wf, uint16_t* wb, hipStream_t s);
hipError_t launch_pack(long long V, int C, int CP, const float* src, uint16_t* dst, hipStream_t s);
hipError_t launch_unpack(long long V, int C, int CP, const float* src, float* dst, hipStream_t s);

}  // namespace lcnn
