/*
 * lc_nn.h -- C ABI of the learned warm start: a small 3D convolutional
 * network that predicts the relaxed Q field around a colloid in a
 * cholesteric from the colloid's radius, the pitch and the anchoring, used
 * as the initial condition of the plain relaxation (the method of
 * Lintuvuori, Marenduzzo, Stratford and Cates, Soft Matter 2011, Sec. 2,
 * stays the judge of the result).  Not part of the paper.
 *
 * Network: 12 input channels -> conv 3x3x3 (12->32) SiLU -> (32->32) SiLU
 * -> (32->32) SiLU -> (32->5) linear = dQ, periodic padding.  Tap
 * t = (dz+1)*9 + (dy+1)*3 + (dx+1); y[o](p) = b[o] + sum_{c,t} W[o][c][t]
 * x[c](p + d_t).  Weights are FP32 masters with BF16 copies; every
 * convolution multiplies BF16 operands on the matrix cores with FP32
 * accumulation.  Q_warm = Q_helix + q_eq * dQ.
 * Input channels: clip((|x-R| - a)/8, -1, 2); unit vector from R (3);
 * helix Q / amplitude (5); a/16; 32/pitch; +1 homeotropic / -1 planar.
 * Loss: mean over fluid sites of |Q_warm - Q_target|_F^2; Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).
 *
 * Conventions as in lc.h: int status codes (LC_OK ...), FP64 or FP32 host
 * arrays in [component][z][y][x] order, work on the stream given at
 * creation, getters synchronise.  The grid is one cubic box of edge L, a
 * multiple of 8 from 8 to 1024.
 */
#ifndef LC_NN_H
#define LC_NN_H

#include "lc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lc_nn lc_nn;

/* One warm-start case: colloid centre and radius, cholesteric pitch (helix
 * n(z) = (cos 2 pi z/p, sin 2 pi z/p, 0)), anchoring (LC_ANCHOR_NORMAL or
 * LC_ANCHOR_PLANAR), helix amplitude of Q_helix and the bulk order q_eq. */
typedef struct lc_nn_case {
  double pos[3];
  double a0;
  double pitch;
  int anchoring;
  int pad_;
  double q_amp;
  double q_eq;
} lc_nn_case;

/* Create a network for an L^3 grid with weights from a seeded generator:
 * W ~ U(-s, s), s = sqrt(6 / (27 C_in)), b = 0 (splitmix64 stream of seed).
 * L must be a multiple of 8 in [8, 1024] (else LC_EINVAL). */
int lc_nn_create(int L, unsigned long long seed, void* hip_stream, lc_nn** out);
void lc_nn_destroy(lc_nn* nn);
const char* lc_nn_last_error(const lc_nn* nn);

/* Layer l (0..3) parameters, FP32: W [C_out][C_in][27], b [C_out]. Setting
 * them resets the optimiser state. */
int lc_nn_set_layer(lc_nn* nn, int layer, const float* W, const float* b);
int lc_nn_get_layer(lc_nn* nn, int layer, float* W, float* b);

/* Weights to and from a file (the optimiser state is not saved; loading
 * resets it, as lc_nn_set_layer does).  Format: magic "LCNNWTS1", int
 * version 1, int layer count 4, then per layer int C_out, C_in, 27, 0 and
 * the FP32 W [C_out][C_in][27] and b [C_out], native byte order.  The
 * weights do not depend on L.  LC_EINVAL if the file cannot be opened or
 * written, or is not a weight file of this network (the network is then
 * unchanged). */
int lc_nn_save(lc_nn* nn, const char* path);
int lc_nn_load(lc_nn* nn, const char* path);

/* Input features of a case: 12 x L^3 floats (may be NULL to only build
 * them on the device). */
int lc_nn_features(lc_nn* nn, const lc_nn_case* c, float* feat_out);

/* Inference pass: dQ (5 x L^3, FP64 host).  (lc_nn_train_step runs its own
 * forward pass, keeping the pre-activations for the backward pass.) */
int lc_nn_predict(lc_nn* nn, const lc_nn_case* c, double* dQ_out);

/* Write Q_helix + q_eq * dQ into box `box` of a context (whose box must be
 * L^3).  Runs the forward pass on the device; no host round trip. */
int lc_nn_warm_start(lc_nn* nn, const lc_nn_case* c, lc_ctx* ctx, int box);

/* One training step on one case: forward, loss against Q_target (5 x L^3
 * FP64) over the sites where fluid[s] != 0, backward, Adam with learning
 * rate lr.  loss_out (may be NULL) receives the loss before the update. */
int lc_nn_train_step(lc_nn* nn, const lc_nn_case* c, const double* Q_target, const unsigned char* fluid,
                     float lr, double* loss_out);

/* Layer-level entry points (for checking the kernels):
 * forward of layer l on a given input x (C_in x L^3, FP32 values that are
 * rounded to BF16 as the kernels do): z_out (C_out x L^3) before the
 * activation.  Backward of layer l given dz (C_out x L^3, rounded to BF16):
 * dW [C_out][C_in][27], db [C_out] and dx (C_in x L^3, before the
 * previous layer's activation derivative). */
int lc_nn_layer_forward(lc_nn* nn, int layer, const float* x, float* z_out);
int lc_nn_layer_backward(lc_nn* nn, int layer, const float* x, const float* dz, float* dW, float* db,
                         float* dx);

/* Mean duration (ms, HIP events on the network's stream) of one forward
 * pass and of one training step on case c over n repetitions:
 * out[0] forward, out[1] training step. */
int lc_nn_time(lc_nn* nn, const lc_nn_case* c, const double* Q_target, const unsigned char* fluid, int n,
               double out[2]);

#ifdef __cplusplus
}
#endif
#endif
