// nn_kernels.hip -- gfx950 kernels of the warm-start network (include/lc_nn.h).
//
// Activations are BF16, channels-last [voxel][C] with C padded to 16 or 32.
// A 3x3x3 periodic convolution is an implicit GEMM over the voxels of an
// 8x8x4 tile, the output channels and K = 27 taps x input channels.  Each
// wave owns one z-layer of the tile (64 voxels = four blocks of 16) and
// multiplies BF16 fragments on the matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation; a 16-channel input takes two taps per instruction).
// Fragment layout for a wave of 64 lanes: A[i][k] -> lane i + 16*(k/KB),
// element k%KB; B[k][j] -> lane j + 16*(k/KB), element k%KB (KB = K/4
// consecutive k per lane); D[i][j] -> lane j + 16*(i/4), element i%4.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lc_arch.hpp"
#include "lc_reduce.hpp"
#include "nn_kernels.hpp"

namespace lcnn {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

__device__ inline uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// logistic function with the hardware reciprocal (within 1 ulp; the result
// is rounded to BF16 or enters a derivative factor)
__device__ inline float sigmoidf_(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

constexpr int TX = 8, TY = 8, TZ = 4, TV = TX * TY * TZ;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;

__device__ inline int wrap1(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// ---------------------------------------------------------------------
// input features
// ---------------------------------------------------------------------
// The 16 input channels of voxel (x, y, z) (Sec. 3 geometry of the case:
// clipped signed distance to the surface, outward normal, unit helix of
// the pitch, radius, pitch and anchoring sign, four zeros) in FP64 (the
// reference values, also written as FP32 when f32 is requested) or FP32,
// which the BF16 rounding cannot tell apart except at rounding ties.
template <typename R>
__device__ inline void features_at(int L, const Case& c, int x, int y, int z, R f[16]) {
  const R h = (R)0.5 * (R)L;
  R r[3] = {(R)x - (R)c.pos[0], (R)y - (R)c.pos[1], (R)z - (R)c.pos[2]};
  for (int k = 0; k < 3; k++) r[k] = r[k] > h ? r[k] - (R)L : (r[k] < -h ? r[k] + (R)L : r[k]);
  const R rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  const R sd = (rn - (R)c.a0) * (R)0.125;
  f[0] = sd < (R)-1 ? (R)-1 : (sd > (R)2 ? (R)2 : sd);
  const R irn = rn > (R)0 ? (R)1 / rn : (R)0;
  for (int k = 0; k < 3; k++) f[1 + k] = r[k] * irn;
  // helix phase 2 pi z / pitch, reduced exactly in units of pi
  R sz, cz;
  if constexpr (sizeof(R) == 8)
    sincospi(2.0 * z / c.pitch, &sz, &cz);
  else
    sincospif((float)(2 * z) / (float)c.pitch, &sz, &cz);
  const R third = (R)1 / (R)3;
  f[4] = cz * cz - third;
  f[5] = cz * sz;
  f[6] = 0;
  f[7] = sz * sz - third;
  f[8] = 0;
  f[9] = (R)c.a0 / (R)16;
  f[10] = (R)32 / (R)c.pitch;
  f[11] = c.anchoring == 2 ? (R)-1 : (R)1;
  for (int k = 12; k < 16; k++) f[k] = 0;
}
// the 16 channels as BF16 pairs
template <typename R>
__device__ inline void pack16(const R f[16], unsigned pk[8]) {
#pragma unroll
  for (int k = 0; k < 8; k++) pk[k] = (unsigned)f2bf((float)f[2 * k]) | ((unsigned)f2bf((float)f[2 * k + 1]) << 16);
}

template <bool F64>
__global__ void __launch_bounds__(256) k_features(int L, Case c, uint16_t* __restrict__ x0, float* __restrict__ f32) {
  using R = typename std::conditional<F64, double, float>::type;
  const long long V = (long long)L * L * L;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  // V < 2^31 (the grid is limited to L <= 1024)
  const unsigned u = (unsigned)v, LL = (unsigned)L * (unsigned)L;
  const int z = (int)(u / LL), y = (int)((u - (unsigned)z * LL) / (unsigned)L), x = (int)(u - (unsigned)z * LL - (unsigned)y * L);
  R f[16];
  features_at<R>(L, c, x, y, z, f);
  // the voxel's 16 BF16 channels as two 16-byte stores
  unsigned pk[8];
  pack16<R>(f, pk);
  *(u4*)(x0 + v * 16) = u4{pk[0], pk[1], pk[2], pk[3]};
  *(u4*)(x0 + v * 16 + 8) = u4{pk[4], pk[5], pk[6], pk[7]};
  if constexpr (F64)
    for (int k = 0; k < 12; k++) f32[k * V + v] = (float)f[k];
}

// ---------------------------------------------------------------------
// convolution as implicit GEMM on the matrix cores
// ---------------------------------------------------------------------
// x [V][CIN] bf16, w [27][COUT][CIN] bf16.  MODE 0: z = acc + b, store z
// (FP32) and bf16(silu(z)); MODE 1: z = acc + b (FP32); MODE 2: acc times
// silu'(zprev) stored as bf16 (data gradient through an activation);
// MODE 3: acc stored as FP32 (plain data gradient); MODE 4: as MODE 0
// without keeping z (inference).
// FEAT (first layer): the input is not read but computed, the 16 features
// of every halo voxel from the case cs (the FP32 values k_features<false>
// stores); xf, if not null, receives them for the tile's own voxels.
template <int CIN, int COUT, int MODE, bool FEAT = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    k_conv(int L, const uint16_t* __restrict__ x, const uint16_t* __restrict__ w, const float* __restrict__ bias,
           const float* __restrict__ zprev, float* __restrict__ zout, uint16_t* __restrict__ aout, Case cs,
           uint16_t* __restrict__ xf) {
  // Every K step is one v_mfma_f32_16x16x32_bf16: 32 input channels of one
  // tap, or (16-channel inputs) the 16 channels of two taps, lane groups
  // kq = 0, 1 taking tap 2s and kq = 2, 3 tap 2s + 1 (tap 27 of the last
  // pair has zero fragments).  Each lane's A and B fragments hold the same
  // eight consecutive (tap, channel) pairs, so the products pair up
  // whatever order the instruction assigns to them within a K block.
  static_assert(CIN == 16 || CIN == 32, "16 or 32 input channels");
  constexpr bool PAIR = CIN == 16;
  constexpr int NK = PAIR ? 14 : 27;
  // LDS layout of the halo: voxel (hx, hy, hz) at hx CIN + hy RS + hz PZ
  // elements, the voxels of an x-row packed.  A 16-byte LDS read serves 16
  // lanes per cycle, lane groups {0-3, 12-15, 20-23, 24-27}, {4-7, 8-11,
  // 16-19, 28-31} and the same in 32-63 (measured on gfx950 with the
  // bank-conflict counter); each group reads all 16 voxels of a fragment
  // (of one tap), half at the lane's first channel chunk and half at the
  // next, and with rows 10.5 voxels apart (32 channels) or 512 bytes apart
  // (16 channels) the 16 addresses fall in distinct banks.  The packed rows
  // keep four blocks' halos within one CU's LDS.
  constexpr int RS = PAIR ? 256 : HX * CIN + CIN / 2, PZ = HY * RS, SB = 8;
  using Chunk = u4;
  __shared__ __align__(16) uint16_t sx[HZ * PZ];
  const int tid = threadIdx.x;
  const int ntx = L / TX, nty = L / TY;
  const int b = blockIdx.x;
  const int x0 = (b % ntx) * TX, y0 = ((b / ntx) % nty) * TY, z0 = (b / (ntx * nty)) * TZ;
  const int wv = tid >> 6, lane = tid & 63;
  const int ri = lane & 15, kq = lane >> 4;
  // the lane's tap within a pair and first input channel
  const int hi = PAIR ? kq >> 1 : 0, ch = PAIR ? 8 * (kq & 1) : 8 * kq;
  // Operand roles: A = weights (M = output channels), B = activations
  // (N = voxels), so that a lane's accumulators are output channels of one
  // voxel: D[i][j] sits in lane j + 16 (i / 4), element i % 4.  Row i of M
  // block mb is output channel oc(mb, i).  With 32 outputs and only BF16
  // stored (inference) oc = 8 (i / 4) + 4 mb + i % 4, so lane (j, kq)
  // holds channels 8 kq .. 8 kq + 7 of voxel j (one 16-byte store); when
  // FP32 values are stored or read oc = 16 mb + i, so that the four lanes
  // of a voxel cover 16 consecutive channels (64 bytes) per M block.
  constexpr int NM = COUT / 16, PF = 4;
  constexpr bool OCT = COUT == 32 && MODE == 4;
  auto oc = [](int mb, int i) { return OCT ? 8 * (i >> 2) + 4 * mb + (i & 3) : 16 * mb + i; };
  f4 acc[NM][4];   // [M block][voxel block]
#pragma unroll
  for (int mb = 0; mb < NM; mb++)
#pragma unroll
    for (int nb = 0; nb < 4; nb++) acc[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
  // LDS offset of tap t from the centre voxel
  auto tap_off = [](int t) { return (t % 3 - 1) * CIN + ((t / 3) % 3 - 1) * RS + (t / 9 - 1) * PZ; };
  // weight fragments of steps k+1 .. k+PF-1 are in flight while step k runs
  // on the matrix cores; the first PF are loaded before the halo
  u4 wq[PF][NM];
  auto load_w = [&](int k, u4 (&wf)[NM]) {
    const bool pad = PAIR && k == NK - 1 && hi;   // tap 27: zero
    const int t = pad ? 26 : (PAIR ? 2 * k + hi : k);
#pragma unroll
    for (int mb = 0; mb < NM; mb++) {
      const u4 v = *(const u4*)(w + ((long long)(t * COUT + oc(mb, ri)) * CIN + ch));
      wf[mb] = pad ? u4{0u, 0u, 0u, 0u} : v;
    }
  };
#pragma unroll
  for (int k = 0; k < PF; k++) load_w(k, wq[k]);
  // halo staging: every load is issued before the first store to LDS, so
  // their latencies overlap
  constexpr int CH = CIN / SB, NIT = (HV * CH + 255) / 256;
  if constexpr (FEAT) {
    static_assert(CIN == 16, "16 feature channels");
#pragma unroll
    for (int it = 0; it < (HV + 255) / 256; it++) {
      const int v = tid + it * 256;
      if (v < HV) {
        const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
        const int gx = wrap1(x0 - 1 + hx, L), gy = wrap1(y0 - 1 + hy, L), gz = wrap1(z0 - 1 + hz, L);
        float f[16];
        unsigned pk[8];
        features_at<float>(L, cs, gx, gy, gz, f);
        pack16<float>(f, pk);
        uint16_t* d = sx + hx * CIN + hy * RS + hz * PZ;
        *(u4*)d = u4{pk[0], pk[1], pk[2], pk[3]};
        *(u4*)(d + 8) = u4{pk[4], pk[5], pk[6], pk[7]};
        if (xf && hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && hz >= 1 && hz <= TZ) {
          uint16_t* g = xf + (gx + (long long)L * (gy + (long long)L * gz)) * 16;
          *(u4*)g = u4{pk[0], pk[1], pk[2], pk[3]};
          *(u4*)(g + 8) = u4{pk[4], pk[5], pk[6], pk[7]};
        }
      }
    }
  } else {
    Chunk tmp[NIT];
    int soff[NIT];
#pragma unroll
    for (int it = 0; it < NIT; it++) {
      const int e = tid + it * 256;
      if (e < HV * CH) {
        const int v = e / CH, c = e - v * CH;
        const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
        const int gx = wrap1(x0 - 1 + hx, L), gy = wrap1(y0 - 1 + hy, L), gz = wrap1(z0 - 1 + hz, L);
        const long long gv = gx + (long long)L * (gy + (long long)L * gz);
        tmp[it] = *(const Chunk*)(x + gv * CIN + SB * c);
        soff[it] = hx * CIN + hy * RS + hz * PZ + SB * c;
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; it++) {
      const int e = tid + it * 256;
      if (e < HV * CH) *(Chunk*)(sx + soff[it]) = tmp[it];
    }
  }
  __syncthreads();
  // voxel block nb of the wave: x = ri & 7, y = 2 nb + (ri >> 3)
  const uint16_t* sa = sx + ((ri & 7) + 1) * CIN + ((ri >> 3) + 1) * RS + (wv + 1) * PZ + ch;
#pragma unroll
  for (int k = 0; k < NK; k++) {
    const int off = PAIR ? (hi ? tap_off(k == NK - 1 ? 26 : 2 * k + 1) : tap_off(2 * k)) : tap_off(k);
#pragma unroll
    for (int nb = 0; nb < 4; nb++) {
      const u4 xv = *(const u4*)(sa + off + 2 * nb * RS);
#pragma unroll
      for (int mb = 0; mb < NM; mb++)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, wq[k % PF][mb]),
                                                              __builtin_bit_cast(bf8, xv), acc[mb][nb], 0, 0, 0);
    }
    if (k + PF < NK) load_w(k + PF, wq[k % PF]);
  }
  // epilogue: lane (ri, kq) owns, for each M block mb, the four channels
  // oc(mb, 4 kq) .. + 3 of voxel (ri & 7, 2 nb + (ri >> 3)) of the wave's
  // layer.  Every value it reads (bias, z of the previous pass) is loaded
  // before its first store, so that no load waits behind the stores.
  const long long gv0 = (x0 + (ri & 7)) + (long long)L * ((y0 + (ri >> 3)) + (long long)L * (z0 + wv));
  // The inference forms (MODE 4, and MODE 1, the output layer) store with
  // the non-temporal hint: their results are read once, by the next layer
  // or by the loss, and the hint took 5-11% off these kernels; the training
  // forms keep ordinary stores, whose results the backward pass reads again
  // (the hint made them 7-23% slower).
  auto store = [](auto v, auto* p) {
    if constexpr (MODE == 4 || MODE == 1) __builtin_nontemporal_store(v, p);
    else *p = v;
  };
  f4 bj[NM], zq[MODE == 2 ? 4 : 1][NM];
#pragma unroll
  for (int mb = 0; mb < NM; mb++)
    bj[mb] = (MODE == 0 || MODE == 1 || MODE == 4) ? *(const f4*)(bias + oc(mb, 4 * kq)) : f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (MODE == 2) {
#pragma unroll
    for (int nb = 0; nb < 4; nb++)
#pragma unroll
      for (int mb = 0; mb < NM; mb++) zq[nb][mb] = *(const f4*)(zprev + (gv0 + 2LL * nb * L) * COUT + oc(mb, 4 * kq));
  }
#pragma unroll
  for (int nb = 0; nb < 4; nb++) {
    const long long base = (gv0 + 2LL * nb * L) * COUT;
    unsigned pk[NM][2];
#pragma unroll
    for (int mb = 0; mb < NM; mb++) {
      f4 v = acc[mb][nb];
      if constexpr (MODE == 0 || MODE == 1 || MODE == 4) v += bj[mb];
      if constexpr (MODE == 0 || MODE == 1 || MODE == 3) store(v, (f4*)(zout + base + oc(mb, 4 * kq)));
      if constexpr (MODE == 0 || MODE == 2 || MODE == 4) {
        float a[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          if constexpr (MODE == 2) {
            const float zp = zq[nb][mb][e], sg = sigmoidf_(zp);
            a[e] = v[e] * (sg * (1.0f + zp * (1.0f - sg)));
          } else {
            a[e] = v[e] * sigmoidf_(v[e]);
          }
        }
        pk[mb][0] = (unsigned)f2bf(a[0]) | ((unsigned)f2bf(a[1]) << 16);
        pk[mb][1] = (unsigned)f2bf(a[2]) | ((unsigned)f2bf(a[3]) << 16);
        if constexpr (!OCT) store(u2{pk[mb][0], pk[mb][1]}, (u2*)(aout + base + oc(mb, 4 * kq)));
      }
    }
    if constexpr (OCT) store(u4{pk[0][0], pk[0][1], pk[1][0], pk[1][1]}, (u4*)(aout + base + 8 * kq));
  }
}

// one Adam step of parameter w with gradient g (beta1 0.9, beta2 0.999,
// eps 1e-8; c1, c2 the bias corrections of the step)
__device__ inline float adam_step(float w, float g, float& m, float& v, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  m = b1 * m + (1.f - b1) * g;
  v = b2 * v + (1.f - b2) * g * g;
  return w - lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ---------------------------------------------------------------------
// weight gradient: dW[t][o][c] = sum_p dz[p][o] x[p + d_t][c]
// ---------------------------------------------------------------------
// An implicit GEMM with K = voxels, on v_mfma_f32_16x16x32_bf16: the 32
// voxels of one instruction are four x-rows of the 8x8x4 tile, lane group
// kq taking row 4 ks + kq (8 voxels per lane), so both operands of a lane
// are eight consecutive voxels of one channel.  dz is staged as rows
// sd[o][p]; the input halo is staged three times, shifted by dx = -1, 0, +1
// (sxs[dx+1][c][halo row][i] = x at halo x = i + 1 + dx), so that for every
// tap the eight voxels of a lane are one aligned 16-byte LDS read.  A
// 16-byte LDS read serves the lane groups {0-3, 12-15, 20-23, 24-27},
// {4-7, 8-11, 16-19, 28-31} (and the same in 32-63) one per cycle: with
// row strides of 34 and 62 16-byte chunks (2 mod 4) the eight lanes of
// each row half that a group holds fall in distinct banks.  The staging
// loads each input voxel once (a halo row's ten voxels per item) and
// writes 16-byte row segments.
// Block b accumulates over tiles [b*tpb, (b+1)*tpb) and writes its partial
// sums part[b][27][COUT][CIN] followed by the bias-gradient partials
// part[b][27 COUT CIN + o] = sum of dz[p][o] over its voxels (row sums of
// the staged dz, 16 threads per channel); wave w of the kWgThreads / 64
// owns taps w, w + 8, ... (at most four).
constexpr int kWgThreads = 512;
template <int CIN, int COUT>
__global__ void __launch_bounds__(kWgThreads)
    k_wgrad(int L, int tpb, const uint16_t* __restrict__ dz, const uint16_t* __restrict__ x, float* __restrict__ part) {
  constexpr int NROW = HY * HZ;           // halo x-rows of a tile
  constexpr int PS = TV + 16;             // sd row stride (elements)
  constexpr int CSTR = NROW * 8 + 16;     // sxs channel stride (elements)
  __shared__ __align__(16) uint16_t sd[COUT * PS];           // [o][p]
  __shared__ __align__(16) uint16_t sxs[3 * CIN * CSTR];    // [dx+1][c][halo row][i]
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int ri = lane & 15, kq = lane >> 4;
  const int ntx = L / TX, nty = L / TY, ntz = L / TZ, ntile = ntx * nty * ntz;
  constexpr int NW = kWgThreads / 64, NTAP = (27 + NW - 1) / NW;
  f4 acc[NTAP][COUT / 16][CIN / 16];
#pragma unroll
  for (int a = 0; a < NTAP; a++)
#pragma unroll
    for (int m = 0; m < COUT / 16; m++)
#pragma unroll
      for (int n = 0; n < CIN / 16; n++) acc[a][m][n] = f4{0.f, 0.f, 0.f, 0.f};
  static_assert(COUT * 16 <= kWgThreads && TV == 16 * 16, "16 threads of 16 voxels per dz row");
  float bacc = 0.f;   // bias gradient: this thread's 16 voxels of row tid / 16, over the tiles
  // staging items: (halo row, channel octet) of the input, whose ten voxels
  // are loaded once and written as the three shifted copies, on threads
  // [0, NXI); (tile x-row, channel octet) of dz on threads [NXI, NXI + NDI).
  // An item writes one 16-byte segment (eight voxels of one channel) per
  // channel and copy.
  constexpr int DO = COUT / 8, XO = CIN / 8;
  // Item numbering: 16 consecutive threads take 16 consecutive rows of one
  // octet, so that the 16 lanes of a 16-byte store write 16 consecutive
  // chunks of one channel row (the halo's 60 rows padded to 64 items).
  constexpr int NXI = 64 * XO, NDI = (TV / TX) * DO;
  static_assert(NXI + NDI <= kWgThreads && TX == 8 && NROW <= 64, "one staging item per thread, 8-voxel rows");
  auto xitem = [](int e, int& oc, int& row) { oc = (e / 16) % XO, row = e % 16 + 16 * (e / (16 * XO)); };
  auto ditem = [](int e, int& oc, int& p8) { oc = (e / 16) % DO, p8 = e % 16 + 16 * (e / (16 * DO)); };
  // element k (0..7) of the octets of voxels v[0..7] as one 16-byte segment
  auto seg8 = [](const u4* v, int k) {
    const int d = k >> 1, sh = 16 * (k & 1);
    unsigned o[4];
#pragma unroll
    for (int q = 0; q < 4; q++)
      o[q] = ((v[2 * q][d] >> sh) & 0xffffu) | (((v[2 * q + 1][d] >> sh) & 0xffffu) << 16);
    return u4{o[0], o[1], o[2], o[3]};
  };
  // the global loads of a tile's items: all issued before the first LDS
  // store; the next tile's are issued once this tile's are stored, so they
  // overlap this tile's matrix-core work
  u4 tv[HX];
  auto load_items = [&](int tile) {
    const int x0 = (tile % ntx) * TX, y0 = ((tile / ntx) % nty) * TY, z0 = (tile / (ntx * nty)) * TZ;
    int oc, row;
    xitem(tid, oc, row);
    if (tid < NXI && row < NROW) {
      const int hy = row % HY, hz = row / HY;
      const long long gyz = (long long)L * (wrap1(y0 - 1 + hy, L) + (long long)L * wrap1(z0 - 1 + hz, L));
#pragma unroll
      for (int i = 0; i < HX; i++) tv[i] = *(const u4*)(x + (wrap1(x0 - 1 + i, L) + gyz) * CIN + 8 * oc);
    } else if (tid >= NXI && tid < NXI + NDI) {
      int dc, p8;
      ditem(tid - NXI, dc, p8);
      const int ly = p8 % TY, lz = p8 / TY;
      const long long gv = x0 + (long long)L * ((y0 + ly) + (long long)L * (z0 + lz));
#pragma unroll
      for (int j = 0; j < TX; j++) tv[j] = *(const u4*)(dz + (gv + j) * COUT + 8 * dc);
    }
  };
  const int tile_beg = (int)blockIdx.x * tpb, tile_end = min(tile_beg + tpb, ntile);
  if (tile_beg < tile_end) load_items(tile_beg);
  // the barriers below order LDS accesses only (lc::lds_sync), so the next
  // tile's loads stay in flight across them
  for (int tile = tile_beg; tile < tile_end; tile++) {
    lc::lds_sync();   // the previous tile's LDS reads are done
    int oc, row;
    xitem(tid, oc, row);
    if (tid < NXI && row < NROW) {
#pragma unroll
      for (int cp = 0; cp < 3; cp++)
#pragma unroll
        for (int k = 0; k < 8; k++) *(u4*)(sxs + (cp * CIN + 8 * oc + k) * CSTR + row * 8) = seg8(tv + cp, k);
    } else if (tid >= NXI && tid < NXI + NDI) {
      int dc, p8;
      ditem(tid - NXI, dc, p8);
#pragma unroll
      for (int k = 0; k < 8; k++) *(u4*)(sd + (8 * dc + k) * PS + 8 * p8) = seg8(tv, k);
    }
    if (tile + 1 < tile_end) load_items(tile + 1);
    lc::lds_sync();
    if (tid < COUT * 16) {
      const u4* r = (const u4*)(sd + (tid >> 4) * PS + 16 * (tid & 15));
      float t = 0.f;
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const u4 v = r[h];
#pragma unroll
        for (int d = 0; d < 4; d++) t += bf2f((uint16_t)(v[d] & 0xffffu)) + bf2f((uint16_t)(v[d] >> 16));
      }
      bacc += t;
    }
#pragma unroll
    for (int a = 0; a < NTAP; a++) {
      const int t = wv + NW * a;
      if (t >= 27) break;
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dzz = t / 9 - 1;
#pragma unroll 2
      for (int ks = 0; ks < TV / 32; ks++) {
        const int r = 4 * ks + kq;   // x-row of the tile: voxels 8r .. 8r+7
        const int hrow = (r % TY + 1 + dy) + HY * (r / TY + 1 + dzz);
        u4 bq[CIN / 16];
#pragma unroll
        for (int n = 0; n < CIN / 16; n++)
          bq[n] = *(const u4*)(sxs + ((dx + 1) * CIN + n * 16 + ri) * CSTR + hrow * 8);
#pragma unroll
        for (int m = 0; m < COUT / 16; m++) {
          const u4 af = *(const u4*)(sd + (m * 16 + ri) * PS + 8 * r);
#pragma unroll
          for (int n = 0; n < CIN / 16; n++)
            acc[a][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, af),
                                                                __builtin_bit_cast(bf8, bq[n]), acc[a][m][n], 0, 0, 0);
        }
      }
    }
  }
  float* out = part + (long long)blockIdx.x * (27 * COUT * CIN + COUT);
  // bias: the 16 threads of a row are 16 consecutive lanes of one wave
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) bacc += __shfl_xor(bacc, o, 16);
  if (tid < COUT * 16 && (tid & 15) == 0) out[27 * COUT * CIN + (tid >> 4)] = bacc;
#pragma unroll
  for (int a = 0; a < NTAP; a++) {
    const int t = wv + NW * a;
    if (t >= 27) break;
#pragma unroll
    for (int m = 0; m < COUT / 16; m++)
#pragma unroll
      for (int n = 0; n < CIN / 16; n++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int o = m * 16 + 4 * kq + e, c = n * 16 + ri;
          out[(t * COUT + o) * CIN + c] = acc[a][m][n][e];
        }
  }
}

// Sum of the weight-gradient block partials part[k][t][o][c] (padded
// COUTP x CINP) into dW[o][c][t] for the real channel counts, and of the
// bias partials that follow them into db[o].  A workgroup
// takes 64 consecutive partial entries (coalesced rows); wave w sums blocks
// w, w+4, ... and the four wave sums are added in wave order, so the result
// does not depend on timing.  ADAM: instead of storing the gradient, the
// thread that summed it takes the layer's Adam step on that weight (W, its
// moments and both BF16 copies, as k_adam) or bias.
struct AdamArgs {
  float *W, *b, *mW, *vW, *mb, *vb;
  float lr, c1, c2;
  uint16_t *wf, *wb;
};
template <bool ADAM>
__global__ void __launch_bounds__(256)
    k_wgrad_reduce(int nblk, int COUTP, int CINP, int cout, int cin, const float* __restrict__ part,
                   float* __restrict__ dW, float* __restrict__ db, AdamArgs ad) {
  __shared__ float s[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = 27 * COUTP * CINP, np = nw + COUTP;   // weight entries, then the biases
  const int i = blockIdx.x * 64 + lane;
  float acc = 0.f;
  if (i < np)
    for (int k0 = w; k0 < nblk; k0 += 64) {
      // sixteen loads in flight, added in the order k = w, w + 4, ...
      float t[16];
#pragma unroll
      for (int j = 0; j < 16; j++) {
        const int k = k0 + 4 * j;
        t[j] = k < nblk ? part[(long long)k * np + i] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 16; j++) acc += t[j];
    }
  s[w][lane] = acc;
  __syncthreads();
  if (w == 0 && i < np) {
    const float t4 = ((s[0][lane] + s[1][lane]) + s[2][lane]) + s[3][lane];
    if (i < nw) {
      const int c = i % CINP, o = (i / CINP) % COUTP, t = i / (CINP * COUTP);
      if (o < cout && c < cin) {
        const int e = (o * cin + c) * 27 + t;
        if constexpr (ADAM) {
          const float wn = adam_step(ad.W[e], t4, ad.mW[e], ad.vW[e], ad.lr, ad.c1, ad.c2);
          ad.W[e] = wn;
          const uint16_t h = f2bf(wn);
          ad.wf[(t * COUTP + o) * CINP + c] = h;
          ad.wb[((26 - t) * CINP + c) * COUTP + o] = h;
        } else {
          dW[e] = t4;
        }
      }
    } else if (i - nw < cout) {
      const int o = i - nw;
      if constexpr (ADAM)
        ad.b[o] = adam_step(ad.b[o], t4, ad.mb[o], ad.vb[o], ad.lr, ad.c1, ad.c2);
      else
        db[o] = t4;
    }
  }
}

// ---------------------------------------------------------------------
// loss and its gradient; warm-start output
// ---------------------------------------------------------------------
// unit helix Q at layer z for the given pitch (phase 2 pi z / pitch,
// reduced exactly in units of pi)
__device__ inline void helix_unit(double pitch, int z, double h[5]) {
  double s, c;
  sincospi(2.0 * z / pitch, &s, &c);
  h[0] = c * c - 1.0 / 3.0; h[1] = c * s; h[2] = 0.0; h[3] = s * s - 1.0 / 3.0; h[4] = 0.0;
}

// out [V][16] (channels 0..4 = dQ); Qt [5][V]; grad dz [V][16] bf16;
// part[b] = block sum of |d|^2 over fluid voxels (FP64).
__global__ void __launch_bounds__(256)
    k_loss(int L, Case c, const float* __restrict__ out, const float* __restrict__ Qt, const uint8_t* __restrict__ fluid,
           double inv_nf, uint16_t* __restrict__ dz, double* __restrict__ part) {
  __shared__ double sred[4];
  const long long V = (long long)L * L * L;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double l2 = 0.0;
  if (v < V) {
    const int z = (int)((unsigned)v / ((unsigned)L * (unsigned)L));
    double h[5];
    helix_unit(c.pitch, z, h);
    const f4 o4 = *(const f4*)(out + v * 16);   // channels 0-3 in one load
    const float o[5] = {o4[0], o4[1], o4[2], o4[3], out[v * 16 + 4]};
    float d[5];
    for (int k = 0; k < 5; k++) d[k] = (float)(c.q_amp * h[k]) + (float)c.q_eq * o[k] - Qt[k * V + v];
    const bool f = fluid[v] != 0;
    if (f) {
      const double xx = d[0], xy = d[1], xz = d[2], yy = d[3], yz = d[4];
      l2 = 2.0 * (xx * xx + yy * yy + xx * yy + xy * xy + xz * xz + yz * yz);
    }
    const float sc = f ? (float)(c.q_eq * inv_nf) : 0.f;
    const float g[5] = {4.f * d[0] + 2.f * d[3], 4.f * d[1], 4.f * d[2], 4.f * d[3] + 2.f * d[0], 4.f * d[4]};
    // channels 0-4 of the voxel's 16 (the rest zero) as two 16-byte stores
    const unsigned p0 = (unsigned)f2bf(sc * g[0]) | ((unsigned)f2bf(sc * g[1]) << 16);
    const unsigned p1 = (unsigned)f2bf(sc * g[2]) | ((unsigned)f2bf(sc * g[3]) << 16);
    const unsigned p2 = (unsigned)f2bf(sc * g[4]);
    *(u4*)(dz + v * 16) = u4{p0, p1, p2, 0u};
    *(u4*)(dz + v * 16 + 8) = u4{0u, 0u, 0u, 0u};
  }
  double lv[1] = {l2};
  lc::block_sum<256, 1>(lv, sred, part + blockIdx.x);
}

// Q_warm = q_amp * helix + q_eq * dQ into a field [5][nsites] at offset off
template <typename R>
__global__ void __launch_bounds__(256)
    k_warm(int L, Case c, const float* __restrict__ out, R* __restrict__ Q, long long nsites, long long off) {
  const long long V = (long long)L * L * L;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  double h[5];
  helix_unit(c.pitch, (int)((unsigned)v / ((unsigned)L * (unsigned)L)), h);
  for (int k = 0; k < 5; k++) Q[k * nsites + off + v] = (R)(c.q_amp * h[k] + c.q_eq * (double)out[v * 16 + k]);
}

// ---------------------------------------------------------------------
// Adam on the FP32 masters and the BF16 copies
// ---------------------------------------------------------------------
// W [cout][cin][27] and b [cout]; wf [27][COUTP][CINP] (forward), wb
// [27][CINP][COUTP] with the mirrored tap (data gradient).
__global__ void __launch_bounds__(256)
    k_adam(int cout, int cin, int COUTP, int CINP, float* __restrict__ W, float* __restrict__ b, const float* __restrict__ dW,
           const float* __restrict__ db, float* __restrict__ mW, float* __restrict__ vW, float* __restrict__ mb,
           float* __restrict__ vb, float lr, float c1, float c2, int update, uint16_t* __restrict__ wf,
           uint16_t* __restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nW = cout * cin * 27;
  if (e < nW) {
    float w = W[e];
    if (update) {
      w = adam_step(w, dW[e], mW[e], vW[e], lr, c1, c2);
      W[e] = w;
    }
    const int t = e % 27, c = (e / 27) % cin, o = e / (27 * cin);
    const uint16_t h = f2bf(w);
    wf[(t * COUTP + o) * CINP + c] = h;
    wb[((26 - t) * CINP + c) * COUTP + o] = h;
  } else if (e < nW + cout && update) {
    const int o = e - nW;
    b[o] = adam_step(b[o], db[o], mb[o], vb[o], lr, c1, c2);
  }
}

// conversions for the layer-level entry points: FP32 [C][V] <-> padded
// BF16 / FP32 channels-last
__global__ void k_pack_bf16(long long V, int C, int CP, const float* __restrict__ src, uint16_t* __restrict__ dst) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  for (int k = 0; k < CP; k++) dst[v * CP + k] = k < C ? f2bf(src[k * V + v]) : (uint16_t)0;
}
__global__ void k_unpack_f32(long long V, int C, int CP, const float* __restrict__ src, float* __restrict__ dst) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  for (int k = 0; k < C; k++) dst[k * V + v] = src[v * CP + k];
}

// ---------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------
hipError_t launch_features(int L, const Case& c, uint16_t* x0, float* f32, hipStream_t s) {
  const long long V = (long long)L * L * L;
  if (f32)
    k_features<true><<<(unsigned)((V + 255) / 256), 256, 0, s>>>(L, c, x0, f32);
  else
    k_features<false><<<(unsigned)((V + 255) / 256), 256, 0, s>>>(L, c, x0, f32);
  return hipGetLastError();
}

hipError_t launch_conv(int cinp, int coutp, int mode, int L, const uint16_t* x, const uint16_t* w, const float* bias,
                       const float* zprev, float* zout, uint16_t* aout, hipStream_t s) {
  const int nblk = (L / TX) * (L / TY) * (L / TZ);
#define LCNN_CONV(CI, CO, M)                                                            \
  if (cinp == CI && coutp == CO && mode == M) {                                         \
    k_conv<CI, CO, M><<<nblk, 256, 0, s>>>(L, x, w, bias, zprev, zout, aout, Case{}, nullptr); \
    return hipGetLastError();                                                           \
  }
  LCNN_CONV(16, 32, 0)
  LCNN_CONV(32, 32, 0)
  LCNN_CONV(16, 32, 4)
  LCNN_CONV(32, 32, 4)
  LCNN_CONV(32, 16, 1)
  LCNN_CONV(32, 32, 2)
  LCNN_CONV(16, 32, 2)
  LCNN_CONV(32, 32, 3)
  LCNN_CONV(16, 32, 3)
  LCNN_CONV(32, 16, 3)
#undef LCNN_CONV
  return hipErrorInvalidValue;
}

hipError_t launch_conv_feat(int mode, int L, const Case& c, const uint16_t* w, const float* bias, float* zout,
                            uint16_t* aout, uint16_t* xf, hipStream_t s) {
  const int nblk = (L / TX) * (L / TY) * (L / TZ);
  if (mode == 0)
    k_conv<16, 32, 0, true><<<nblk, 256, 0, s>>>(L, nullptr, w, bias, nullptr, zout, aout, c, xf);
  else if (mode == 4)
    k_conv<16, 32, 4, true><<<nblk, 256, 0, s>>>(L, nullptr, w, bias, nullptr, zout, aout, c, xf);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_wgrad(int cinp, int coutp, int L, int nblk, int tpb, const uint16_t* dz, const uint16_t* x,
                        float* part, hipStream_t s) {
#define LCNN_WG(CI, CO)                                                  \
  if (cinp == CI && coutp == CO) {                                       \
    k_wgrad<CI, CO><<<nblk, kWgThreads, 0, s>>>(L, tpb, dz, x, part);    \
    return hipGetLastError();                                            \
  }
  LCNN_WG(16, 32)
  LCNN_WG(32, 32)
  LCNN_WG(32, 16)
#undef LCNN_WG
  return hipErrorInvalidValue;
}

hipError_t launch_wgrad_reduce(int nblk, int coutp, int cinp, int cout, int cin, const float* part, float* dW,
                               float* db, hipStream_t s) {
  const int np = 27 * coutp * cinp + coutp;
  k_wgrad_reduce<false><<<(np + 63) / 64, 256, 0, s>>>(nblk, coutp, cinp, cout, cin, part, dW, db, AdamArgs{});
  return hipGetLastError();
}

hipError_t launch_wgrad_adam(int nblk, int coutp, int cinp, int cout, int cin, const float* part, float* W, float* b,
                             float* mW, float* vW, float* mb, float* vb, float lr, float c1, float c2, uint16_t* wf,
                             uint16_t* wb, hipStream_t s) {
  const int np = 27 * coutp * cinp + coutp;
  const AdamArgs ad{W, b, mW, vW, mb, vb, lr, c1, c2, wf, wb};
  k_wgrad_reduce<true><<<(np + 63) / 64, 256, 0, s>>>(nblk, coutp, cinp, cout, cin, part, nullptr, nullptr, ad);
  return hipGetLastError();
}

hipError_t launch_loss(int L, const Case& c, const float* out, const float* Qt, const uint8_t* fluid, double inv_nf,
                       uint16_t* dz, double* part, hipStream_t s) {
  const long long V = (long long)L * L * L;
  k_loss<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(L, c, out, Qt, fluid, inv_nf, dz, part);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_warm(int L, const Case& c, const float* out, R* Q, long long nsites, long long off, hipStream_t s) {
  const long long V = (long long)L * L * L;
  k_warm<R><<<(unsigned)((V + 255) / 256), 256, 0, s>>>(L, c, out, Q, nsites, off);
  return hipGetLastError();
}
template hipError_t launch_warm<float>(int, const Case&, const float*, float*, long long, long long, hipStream_t);
template hipError_t launch_warm<double>(int, const Case&, const float*, double*, long long, long long, hipStream_t);

hipError_t launch_adam(int cout, int cin, int coutp, int cinp, float* W, float* b, const float* dW, const float* db,
                       float* mW, float* vW, float* mb, float* vb, float lr, float c1, float c2, int update,
                       uint16_t* wf, uint16_t* wb, hipStream_t s) {
  const int n = cout * cin * 27 + cout;
  k_adam<<<(n + 255) / 256, 256, 0, s>>>(cout, cin, coutp, cinp, W, b, dW, db, mW, vW, mb, vb, lr, c1, c2, update,
                                         wf, wb);
  return hipGetLastError();
}

hipError_t launch_pack(long long V, int C, int CP, const float* src, uint16_t* dst, hipStream_t s) {
  k_pack_bf16<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(V, C, CP, src, dst);
  return hipGetLastError();
}
hipError_t launch_unpack(long long V, int C, int CP, const float* src, float* dst, hipStream_t s) {
  k_unpack_f32<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(V, C, CP, src, dst);
  return hipGetLastError();
}

}  // namespace lcnn
