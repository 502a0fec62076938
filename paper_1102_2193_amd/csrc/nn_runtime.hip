// nn_runtime.hip -- host runtime of the warm-start network (include/lc_nn.h).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/lc_nn.h"
#include "lc_internal.hpp"
#include "nn_kernels.hpp"

namespace {

constexpr int NL = 4;
constexpr int CIN[NL] = {12, 32, 32, 32}, COUT[NL] = {32, 32, 32, 5};
constexpr int CINP[NL] = {16, 32, 32, 32}, COUTP[NL] = {32, 32, 32, 16};

std::string g_nn_error;

uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

struct lc_nn {
  int L = 0;
  long long V = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  float *W[NL] = {}, *b[NL] = {}, *mW[NL] = {}, *vW[NL] = {}, *mb[NL] = {}, *vb[NL] = {}, *dW[NL] = {}, *db[NL] = {};
  uint16_t *wf[NL] = {}, *wb[NL] = {};
  uint16_t* x0 = nullptr;              // features [V][16]
  float* z[3] = {};                    // pre-activations [V][32]
  uint16_t* a[3] = {};                 // activations [V][32]
  float* out = nullptr;                // dQ [V][16]
  uint16_t* g4 = nullptr;              // d loss / d out [V][16]
  uint16_t* g[3] = {};                 // d loss / d z_l [V][32]
  float* wpart = nullptr;               // weight- and bias-gradient block partials
  int wblk = 0, tpb = 0;
  double* lpart = nullptr;
  int lblk = 0;
  float* Qt = nullptr;
  uint8_t* fluid = nullptr;
  float* tmpf = nullptr;               // [V][32] scratch for the layer-level calls
  uint16_t *tmph = nullptr, *tmph2 = nullptr;
  int step = 0;
  std::string err;
};

namespace {

int nfail(lc_nn* n, int code, const std::string& m) {
  if (n) n->err = m;
  else g_nn_error = m;
  return code;
}

#define NNCHK(nn, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return nfail(nn, LC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

lcnn::Case to_case(const lc_nn_case* c) {
  lcnn::Case k;
  memset(&k, 0, sizeof(k));
  for (int a = 0; a < 3; a++) k.pos[a] = c->pos[a];
  k.a0 = c->a0;
  k.pitch = c->pitch;
  k.anchoring = c->anchoring;
  k.q_amp = c->q_amp;
  k.q_eq = c->q_eq;
  return k;
}

int check_case(lc_nn* n, const lc_nn_case* c) {
  if (!c) return nfail(n, LC_EINVAL, "case is NULL");
  if (!(c->pitch > 0) || !(c->a0 > 0) || !isfinite(c->q_amp) || !isfinite(c->q_eq))
    return nfail(n, LC_EINVAL, "bad case parameters");
  return LC_OK;
}

// refresh the BF16 copies of layer l (no update)
int refresh_bf16(lc_nn* n, int l) {
  NNCHK(n, lcnn::launch_adam(COUT[l], CIN[l], COUTP[l], CINP[l], n->W[l], n->b[l], nullptr, nullptr, nullptr, nullptr,
                             nullptr, nullptr, 0.f, 1.f, 1.f, 0, n->wf[l], n->wb[l], n->stream));
  return LC_OK;
}

// Forward pass; `keep` stores the pre-activations for a backward pass.
int forward(lc_nn* n, const lcnn::Case& k, bool keep) {
  // layer 0 computes its input features itself (kept in x0 for the weight
  // gradient when training)
  NNCHK(n, lcnn::launch_conv_feat(keep ? 0 : 4, n->L, k, n->wf[0], n->b[0], n->z[0], n->a[0], keep ? n->x0 : nullptr,
                                  n->stream));
  const uint16_t* in = n->a[0];
  for (int l = 1; l < NL - 1; l++) {
    NNCHK(n, lcnn::launch_conv(CINP[l], COUTP[l], keep ? 0 : 4, n->L, in, n->wf[l], n->b[l], nullptr, n->z[l],
                               n->a[l], n->stream));
    in = n->a[l];
  }
  NNCHK(n, lcnn::launch_conv(CINP[3], COUTP[3], 1, n->L, in, n->wf[3], n->b[3], nullptr, n->out, nullptr, n->stream));
  return LC_OK;
}

// gradients of layer l from dz (bf16 [V][COUTP]) and its input x
int layer_grads(lc_nn* n, int l, const uint16_t* dz, const uint16_t* x) {
  NNCHK(n, lcnn::launch_wgrad(CINP[l], COUTP[l], n->L, n->wblk, n->tpb, dz, x, n->wpart, n->stream));
  NNCHK(n, lcnn::launch_wgrad_reduce(n->wblk, COUTP[l], CINP[l], COUT[l], CIN[l], n->wpart, n->dW[l], n->db[l],
                                     n->stream));
  return LC_OK;
}

// Backward pass and Adam step.  Per layer, from the last: the data
// gradient for the layer below (with the layer's old BF16 weights), then the
// weight and bias gradients, summed and applied by one fused kernel.
int backward_and_update(lc_nn* n, float lr) {
  n->step++;
  const float c1 = 1.f - powf(0.9f, (float)n->step), c2 = 1.f - powf(0.999f, (float)n->step);
  const uint16_t* dz = n->g4;
  for (int l = NL - 1; l >= 0; l--) {
    const uint16_t* x = l == 0 ? n->x0 : n->a[l - 1];
    if (l > 0)
      // d loss / d z_{l-1} = (W^T * dz) times silu'(z_{l-1})
      NNCHK(n, lcnn::launch_conv(COUTP[l], CINP[l], 2, n->L, dz, n->wb[l], nullptr, n->z[l - 1], nullptr,
                                 n->g[l - 1], n->stream));
    NNCHK(n, lcnn::launch_wgrad(CINP[l], COUTP[l], n->L, n->wblk, n->tpb, dz, x, n->wpart, n->stream));
    NNCHK(n, lcnn::launch_wgrad_adam(n->wblk, COUTP[l], CINP[l], COUT[l], CIN[l], n->wpart, n->W[l], n->b[l],
                                     n->mW[l], n->vW[l], n->mb[l], n->vb[l], lr, c1, c2, n->wf[l], n->wb[l],
                                     n->stream));
    if (l > 0) dz = n->g[l - 1];
  }
  return LC_OK;
}

int upload_targets(lc_nn* n, const double* Qt, const unsigned char* fluid, double* inv_nf) {
  std::vector<float> q((size_t)5 * n->V);
  for (long long i = 0; i < 5 * n->V; i++) q[i] = (float)Qt[i];
  long long nf = 0;
  for (long long i = 0; i < n->V; i++) nf += fluid[i] != 0;
  if (nf == 0) return nfail(n, LC_EINVAL, "no fluid site");
  *inv_nf = 1.0 / (double)nf;
  NNCHK(n, hipMemcpyAsync(n->Qt, q.data(), sizeof(float) * q.size(), hipMemcpyHostToDevice, n->stream));
  NNCHK(n, hipMemcpyAsync(n->fluid, fluid, n->V, hipMemcpyHostToDevice, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

int loss(lc_nn* n, const lcnn::Case& k, double inv_nf, double* loss_out) {
  NNCHK(n, lcnn::launch_loss(n->L, k, n->out, n->Qt, n->fluid, inv_nf, n->g4, n->lpart, n->stream));
  if (loss_out) {
    std::vector<double> h(n->lblk);
    NNCHK(n, hipMemcpyAsync(h.data(), n->lpart, sizeof(double) * n->lblk, hipMemcpyDeviceToHost, n->stream));
    NNCHK(n, hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (double v : h) s += v;
    *loss_out = s * inv_nf;
  }
  return LC_OK;
}

}  // namespace

extern "C" {

int lc_nn_create(int L, unsigned long long seed, void* hip_stream, lc_nn** out) {
  if (!out) return nfail(nullptr, LC_EINVAL, "out is NULL");
  *out = nullptr;
  if (L < 8 || L % 8 || L > 1024) return nfail(nullptr, LC_EINVAL, "L must be a multiple of 8 in [8, 1024]");
  lc_nn* n = new lc_nn();
  n->L = L;
  n->V = (long long)L * L * L;
  auto bail = [&](int code, const std::string& m) {
    lc_nn_destroy(n);
    return nfail(nullptr, code, m);
  };
  if (hip_stream) n->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess) return bail(LC_EDEVICE, "stream");
    n->own_stream = true;
  }
  const long long V = n->V;
  const int ntile = (L / 8) * (L / 8) * (L / 4);
  n->tpb = (ntile + 255) / 256;
  n->wblk = (ntile + n->tpb - 1) / n->tpb;
  n->lblk = (int)((V + 255) / 256);
  bool ok = true;
  auto dmalloc = [&](void** p, size_t sz) {
    if (ok && hipMalloc(p, sz) != hipSuccess) ok = false;
    if (ok && hipMemsetAsync(*p, 0, sz, n->stream) != hipSuccess) ok = false;
  };
  for (int l = 0; l < NL; l++) {
    const size_t nw = (size_t)COUT[l] * CIN[l] * 27;
    dmalloc((void**)&n->W[l], nw * 4);
    dmalloc((void**)&n->mW[l], nw * 4);
    dmalloc((void**)&n->vW[l], nw * 4);
    dmalloc((void**)&n->dW[l], nw * 4);
    // the convolution epilogues read the bias at every padded channel (zero there)
    dmalloc((void**)&n->b[l], COUTP[l] * 4);
    dmalloc((void**)&n->mb[l], COUT[l] * 4);
    dmalloc((void**)&n->vb[l], COUT[l] * 4);
    dmalloc((void**)&n->db[l], COUT[l] * 4);
    dmalloc((void**)&n->wf[l], (size_t)27 * COUTP[l] * CINP[l] * 2);
    dmalloc((void**)&n->wb[l], (size_t)27 * COUTP[l] * CINP[l] * 2);
  }
  dmalloc((void**)&n->x0, V * 16 * 2);
  for (int l = 0; l < 3; l++) {
    dmalloc((void**)&n->z[l], V * 32 * 4);
    dmalloc((void**)&n->a[l], V * 32 * 2);
    dmalloc((void**)&n->g[l], V * 32 * 2);
  }
  dmalloc((void**)&n->out, V * 16 * 4);
  dmalloc((void**)&n->g4, V * 16 * 2);
  dmalloc((void**)&n->wpart, (size_t)n->wblk * (27 * 32 * 32 + 32) * 4);
  dmalloc((void**)&n->lpart, (size_t)n->lblk * 8);
  dmalloc((void**)&n->Qt, V * 5 * 4);
  dmalloc((void**)&n->fluid, V);
  dmalloc((void**)&n->tmpf, V * 32 * 4);
  dmalloc((void**)&n->tmph, V * 32 * 2);
  dmalloc((void**)&n->tmph2, V * 32 * 2);
  if (!ok) return bail(LC_ENOMEM, "device allocation failed");
  // seeded uniform init, W ~ U(-s, s), s = sqrt(6 / (27 C_in))
  for (int l = 0; l < NL; l++) {
    const size_t nw = (size_t)COUT[l] * CIN[l] * 27;
    std::vector<float> w(nw);
    const double s = sqrt(6.0 / (27.0 * CIN[l]));
    const uint64_t base = seed * 0xD1B54A32D192ED03ull + (uint64_t)(l + 1) * 0x9E3779B97F4A7C15ull;
    for (size_t i = 0; i < nw; i++) {
      const double u = (double)(splitmix64(base + i) >> 11) * (1.0 / 9007199254740992.0);
      w[i] = (float)(s * (2.0 * u - 1.0));
    }
    if (hipMemcpyAsync(n->W[l], w.data(), nw * 4, hipMemcpyHostToDevice, n->stream) != hipSuccess)
      return bail(LC_EDEVICE, "upload");
    if (refresh_bf16(n, l) != LC_OK) return bail(LC_EDEVICE, n->err);
  }
  if (hipStreamSynchronize(n->stream) != hipSuccess) return bail(LC_EDEVICE, "initialisation failed");
  *out = n;
  return LC_OK;
}

void lc_nn_destroy(lc_nn* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  for (int l = 0; l < NL; l++) {
    void* p[] = {n->W[l], n->b[l], n->mW[l], n->vW[l], n->mb[l], n->vb[l], n->dW[l], n->db[l], n->wf[l], n->wb[l]};
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
  void* q[] = {n->x0, n->z[0], n->z[1], n->z[2], n->a[0], n->a[1], n->a[2], n->g[0], n->g[1], n->g[2], n->out,
               n->g4, n->wpart, n->lpart, n->Qt, n->fluid, n->tmpf, n->tmph, n->tmph2};
  for (void* p : q)
    if (p) (void)hipFree(p);
  if (n->own_stream && n->stream) (void)hipStreamDestroy(n->stream);
  delete n;
}

const char* lc_nn_last_error(const lc_nn* n) { return n ? n->err.c_str() : g_nn_error.c_str(); }

int lc_nn_set_layer(lc_nn* n, int l, const float* W, const float* b) {
  if (!n) return LC_EINVAL;
  if (l < 0 || l >= NL || !W || !b) return nfail(n, LC_EINVAL, "bad layer or NULL array");
  const size_t nw = (size_t)COUT[l] * CIN[l] * 27;
  NNCHK(n, hipMemcpyAsync(n->W[l], W, nw * 4, hipMemcpyHostToDevice, n->stream));
  NNCHK(n, hipMemcpyAsync(n->b[l], b, COUT[l] * 4, hipMemcpyHostToDevice, n->stream));
  for (int k = 0; k < NL; k++) {
    NNCHK(n, hipMemsetAsync(n->mW[k], 0, (size_t)COUT[k] * CIN[k] * 27 * 4, n->stream));
    NNCHK(n, hipMemsetAsync(n->vW[k], 0, (size_t)COUT[k] * CIN[k] * 27 * 4, n->stream));
    NNCHK(n, hipMemsetAsync(n->mb[k], 0, COUT[k] * 4, n->stream));
    NNCHK(n, hipMemsetAsync(n->vb[k], 0, COUT[k] * 4, n->stream));
  }
  n->step = 0;
  int rc = refresh_bf16(n, l);
  if (rc) return rc;
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

int lc_nn_get_layer(lc_nn* n, int l, float* W, float* b) {
  if (!n) return LC_EINVAL;
  if (l < 0 || l >= NL || !W || !b) return nfail(n, LC_EINVAL, "bad layer or NULL array");
  NNCHK(n, hipMemcpyAsync(W, n->W[l], (size_t)COUT[l] * CIN[l] * 27 * 4, hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipMemcpyAsync(b, n->b[l], COUT[l] * 4, hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

// Weight file: magic, version, layer count, then per layer its shape
// (C_out, C_in, taps) and the FP32 W and b, native byte order.
const char kWeightMagic[8] = {'L', 'C', 'N', 'N', 'W', 'T', 'S', '1'};

int lc_nn_save(lc_nn* n, const char* path) {
  if (!n) return LC_EINVAL;
  if (!path) return nfail(n, LC_EINVAL, "path is NULL");
  std::vector<std::vector<float>> W(NL), b(NL);
  for (int l = 0; l < NL; l++) {
    W[l].resize((size_t)COUT[l] * CIN[l] * 27);
    b[l].resize(COUT[l]);
    int rc = lc_nn_get_layer(n, l, W[l].data(), b[l].data());
    if (rc) return rc;
  }
  FILE* fp = fopen(path, "wb");
  if (!fp) return nfail(n, LC_EINVAL, std::string("cannot open ") + path + " for writing");
  const int head[2] = {1, NL};
  bool ok = fwrite(kWeightMagic, 1, 8, fp) == 8 && fwrite(head, sizeof(int), 2, fp) == 2;
  for (int l = 0; l < NL && ok; l++) {
    const int shape[4] = {COUT[l], CIN[l], 27, 0};
    ok = fwrite(shape, sizeof(int), 4, fp) == 4 && fwrite(W[l].data(), 4, W[l].size(), fp) == W[l].size() &&
         fwrite(b[l].data(), 4, b[l].size(), fp) == b[l].size();
  }
  ok = (fclose(fp) == 0) && ok;
  if (!ok) return nfail(n, LC_EINVAL, std::string("writing ") + path + " failed");
  return LC_OK;
}

int lc_nn_load(lc_nn* n, const char* path) {
  if (!n) return LC_EINVAL;
  if (!path) return nfail(n, LC_EINVAL, "path is NULL");
  FILE* fp = fopen(path, "rb");
  if (!fp) return nfail(n, LC_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  int head[2];
  std::vector<std::vector<float>> W(NL), b(NL);
  bool ok = fread(magic, 1, 8, fp) == 8 && memcmp(magic, kWeightMagic, 8) == 0 &&
            fread(head, sizeof(int), 2, fp) == 2 && head[0] == 1 && head[1] == NL;
  for (int l = 0; l < NL && ok; l++) {
    int shape[4];
    ok = fread(shape, sizeof(int), 4, fp) == 4 && shape[0] == COUT[l] && shape[1] == CIN[l] && shape[2] == 27;
    if (!ok) break;
    W[l].resize((size_t)COUT[l] * CIN[l] * 27);
    b[l].resize(COUT[l]);
    ok = fread(W[l].data(), 4, W[l].size(), fp) == W[l].size() && fread(b[l].data(), 4, b[l].size(), fp) == b[l].size();
  }
  ok = ok && fgetc(fp) == EOF;
  fclose(fp);
  if (!ok) return nfail(n, LC_EINVAL, std::string(path) + " is not a weight file of this network");
  for (int l = 0; l < NL; l++) {
    int rc = lc_nn_set_layer(n, l, W[l].data(), b[l].data());
    if (rc) return rc;
  }
  return LC_OK;
}

int lc_nn_features(lc_nn* n, const lc_nn_case* c, float* feat_out) {
  if (!n) return LC_EINVAL;
  int rc = check_case(n, c);
  if (rc) return rc;
  const lcnn::Case k = to_case(c);
  NNCHK(n, lcnn::launch_features(n->L, k, n->x0, n->tmpf, n->stream));
  if (feat_out)
    NNCHK(n, hipMemcpyAsync(feat_out, n->tmpf, sizeof(float) * 12 * n->V, hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

int lc_nn_predict(lc_nn* n, const lc_nn_case* c, double* dQ_out) {
  if (!n) return LC_EINVAL;
  int rc = check_case(n, c);
  if (rc) return rc;
  if ((rc = forward(n, to_case(c), false)) != LC_OK) return rc;
  if (dQ_out) {
    std::vector<float> h((size_t)n->V * 16);
    NNCHK(n, hipMemcpyAsync(h.data(), n->out, sizeof(float) * h.size(), hipMemcpyDeviceToHost, n->stream));
    NNCHK(n, hipStreamSynchronize(n->stream));
    for (long long v = 0; v < n->V; v++)
      for (int k = 0; k < 5; k++) dQ_out[k * n->V + v] = h[v * 16 + k];
  }
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

int lc_nn_warm_start(lc_nn* n, const lc_nn_case* c, lc_ctx* ctx, int box) {
  if (!n) return LC_EINVAL;
  int rc = check_case(n, c);
  if (rc) return rc;
  LcQView q;
  if ((rc = lc_internal_q_view(ctx, box, &q)) != LC_OK) return nfail(n, rc, "bad context or box");
  if (q.nx != n->L || q.ny != n->L || q.nz != n->L) return nfail(n, LC_EINVAL, "box is not L^3");
  NNCHK(n, hipStreamSynchronize(q.stream));
  const lcnn::Case k = to_case(c);
  if ((rc = forward(n, k, false)) != LC_OK) return rc;
  NNCHK(n, q.prec == LC_FP32 ? lcnn::launch_warm<float>(n->L, k, n->out, (float*)q.Q, q.nsites, q.off, n->stream)
                             : lcnn::launch_warm<double>(n->L, k, n->out, (double*)q.Q, q.nsites, q.off, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

int lc_nn_train_step(lc_nn* n, const lc_nn_case* c, const double* Q_target, const unsigned char* fluid, float lr,
                     double* loss_out) {
  if (!n) return LC_EINVAL;
  int rc = check_case(n, c);
  if (rc) return rc;
  if (!Q_target || !fluid || !(lr >= 0.f)) return nfail(n, LC_EINVAL, "bad training arguments");
  double inv_nf;
  if ((rc = upload_targets(n, Q_target, fluid, &inv_nf)) != LC_OK) return rc;
  const lcnn::Case k = to_case(c);
  if ((rc = forward(n, k, true)) != LC_OK) return rc;
  if ((rc = loss(n, k, inv_nf, loss_out)) != LC_OK) return rc;
  if ((rc = backward_and_update(n, lr)) != LC_OK) return rc;
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

int lc_nn_layer_forward(lc_nn* n, int l, const float* x, float* z_out) {
  if (!n) return LC_EINVAL;
  if (l < 0 || l >= NL || !x || !z_out) return nfail(n, LC_EINVAL, "bad layer or NULL array");
  const long long V = n->V;
  NNCHK(n, hipMemcpyAsync(n->tmpf, x, sizeof(float) * CIN[l] * V, hipMemcpyHostToDevice, n->stream));
  NNCHK(n, lcnn::launch_pack(V, CIN[l], CINP[l], n->tmpf, n->tmph, n->stream));
  // z into the layer's own buffer (layers 0-2) or the output buffer (layer 3)
  float* zb = l < 3 ? n->z[l] : n->out;
  NNCHK(n, lcnn::launch_conv(CINP[l], COUTP[l], l < 3 ? 0 : 1, n->L, n->tmph, n->wf[l], n->b[l], nullptr, zb,
                             l < 3 ? n->a[l] : nullptr, n->stream));
  NNCHK(n, lcnn::launch_unpack(V, COUT[l], COUTP[l], zb, n->tmpf, n->stream));
  NNCHK(n, hipMemcpyAsync(z_out, n->tmpf, sizeof(float) * COUT[l] * V, hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  return LC_OK;
}

int lc_nn_layer_backward(lc_nn* n, int l, const float* x, const float* dz, float* dW, float* db, float* dx) {
  if (!n) return LC_EINVAL;
  if (l < 0 || l >= NL || !x || !dz || !dW || !db || !dx) return nfail(n, LC_EINVAL, "bad layer or NULL array");
  const long long V = n->V;
  NNCHK(n, hipMemcpyAsync(n->tmpf, x, sizeof(float) * CIN[l] * V, hipMemcpyHostToDevice, n->stream));
  NNCHK(n, lcnn::launch_pack(V, CIN[l], CINP[l], n->tmpf, n->tmph, n->stream));
  NNCHK(n, hipMemcpyAsync(n->tmpf, dz, sizeof(float) * COUT[l] * V, hipMemcpyHostToDevice, n->stream));
  NNCHK(n, lcnn::launch_pack(V, COUT[l], COUTP[l], n->tmpf, n->tmph2, n->stream));
  int rc = layer_grads(n, l, n->tmph2, n->tmph);
  if (rc) return rc;
  NNCHK(n, lcnn::launch_conv(COUTP[l], CINP[l], 3, n->L, n->tmph2, n->wb[l], nullptr, nullptr, n->tmpf, nullptr,
                             n->stream));
  std::vector<float> h((size_t)V * CINP[l]);
  NNCHK(n, hipMemcpyAsync(h.data(), n->tmpf, sizeof(float) * h.size(), hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipMemcpyAsync(dW, n->dW[l], sizeof(float) * COUT[l] * CIN[l] * 27, hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipMemcpyAsync(db, n->db[l], sizeof(float) * COUT[l], hipMemcpyDeviceToHost, n->stream));
  NNCHK(n, hipStreamSynchronize(n->stream));
  for (long long v = 0; v < V; v++)
    for (int k = 0; k < CIN[l]; k++) dx[k * V + v] = h[v * CINP[l] + k];
  return LC_OK;
}

int lc_nn_time(lc_nn* n, const lc_nn_case* c, const double* Q_target, const unsigned char* fluid, int reps,
               double out[2]) {
  if (!n || !out || reps < 1) return LC_EINVAL;
  int rc = check_case(n, c);
  if (rc) return rc;
  double inv_nf;
  if ((rc = upload_targets(n, Q_target, fluid, &inv_nf)) != LC_OK) return rc;
  const lcnn::Case k = to_case(c);
  hipEvent_t e0, e1, e2;
  NNCHK(n, hipEventCreate(&e0));
  NNCHK(n, hipEventCreate(&e1));
  NNCHK(n, hipEventCreate(&e2));
  NNCHK(n, hipEventRecord(e0, n->stream));
  for (int r = 0; r < reps; r++)
    if ((rc = forward(n, k, false)) != LC_OK) return rc;
  NNCHK(n, hipEventRecord(e1, n->stream));
  for (int r = 0; r < reps; r++) {
    if ((rc = forward(n, k, true)) != LC_OK) return rc;
    if ((rc = loss(n, k, inv_nf, nullptr)) != LC_OK) return rc;
    if ((rc = backward_and_update(n, 0.f)) != LC_OK) return rc;
  }
  NNCHK(n, hipEventRecord(e2, n->stream));
  NNCHK(n, hipEventSynchronize(e2));
  float t1 = 0.f, t2 = 0.f;
  NNCHK(n, hipEventElapsedTime(&t1, e0, e1));
  NNCHK(n, hipEventElapsedTime(&t2, e1, e2));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  out[0] = t1 / reps;
  out[1] = t2 / reps;
  return LC_OK;
}

}  // extern "C"
