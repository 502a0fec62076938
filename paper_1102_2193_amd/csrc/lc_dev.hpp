// lc_dev.hpp -- device-side definitions of the hybrid LB/FD library for
// gfx950: box descriptor, D3Q19 lattice, colloid geometry, Q-tensor algebra.
//
// Physics follows Lintuvuori, Marenduzzo, Stratford, Cates, Soft Matter
// 2011: free energy Eq. (1), Beris-Edwards Eq. (2), stress Eq. (4),
// bounce-back on links and the hybrid boundary treatment of Sec. 2.2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lc {

// One box of the batch.  Host and device share this layout.
struct BoxDev {
  int nx, ny, nz, hydro;
  long long off;            // first site of the box in the concatenated arrays
  int tile_base, ntx, nty, ntz;          // fused-kernel tiles of this box
  int col0, ncol;                        // its colloids: entries col0 .. col0+ncol-1 of the table
  double tau, rho0, A0, gamma, K, q0, xi, Gamma;
  double itau, fsrc;                     // 1/tau and 1 - 1/(2 tau)
  double body[3];
  int adv, st27;                         // advection order (1..3); 27-point Q stencil
};

// Colloids of a box keep their surfaces at least this far apart (lattice
// units) at the start of every step: no fluid node then has links or faces
// to two colloids, so each link, face, ghost node and moving-boundary event
// belongs to one colloid.
constexpr double kColloidGap = 3.0;
constexpr int kMaxColloids = 16;   // per box

// One colloid (Sec. 2.2).  Host and device share this layout; the position
// (and a free colloid's velocities) advance on the device.
struct ColDev {
  int box, motion, anchoring, pad_;
  // centre at the start of a step, by the step's buffer parity: the
  // post-step kernel of a step writes the other slot
  double pos[2][3];
  double a0, vel[3], omega[3], S0, W;
  double fext[3], mass, inertia;          // free motion (motion == 2)
  int slot_base;                          // its fused-kernel slots: slot_base + tile (or column block + ncb * plane)
  int ghost_base, ghost_ext;              // ghost launch: thread range, candidate cube edge
  int event_ext;                          // candidate cube edge of the moving-boundary events
  int post_blk0, post_nblk;               // blocks of the post-step kernel for this colloid
};

// D3Q19: rest, 6 axis links, 12 diagonal links; opposite links adjacent.
__host__ __device__ constexpr int cx(int i) {
  return i == 1 || i == 7 || i == 9 || i == 11 || i == 13 ? 1
       : i == 2 || i == 8 || i == 10 || i == 12 || i == 14 ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i) {
  return i == 3 || i == 7 || i == 10 || i == 15 || i == 17 ? 1
       : i == 4 || i == 8 || i == 9 || i == 16 || i == 18 ? -1 : 0;
}
__host__ __device__ constexpr int cz(int i) {
  return i == 5 || i == 11 || i == 14 || i == 15 || i == 18 ? 1
       : i == 6 || i == 12 || i == 13 || i == 16 || i == 17 ? -1 : 0;
}
// c_i . v for direction i with the zero components left out: a product
// with a zero component is not folded away in IEEE arithmetic and would
// cost an instruction.  The nonzero terms are added in x, y, z order, as
// the full dot product adds them.
template <typename R>
__device__ __forceinline__ R cdot(int i, const R v[3]) {
  const int c[3] = {cx(i), cy(i), cz(i)};
  R s = (R)0;
  bool first = true;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    if (c[k] == 0) continue;
    const R t = c[k] > 0 ? v[k] : -v[k];
    s = first ? t : s + t;
    first = false;
  }
  return s;
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wgt(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

__device__ inline int wrapc(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Minimum-image displacement; kept free of fused multiply-adds so that the
// solid/fluid decision is taken exactly as an unfused FP64 evaluation.
__device__ inline double minimg(double d, int L) {
  if (d > 0.5 * L) d = __dsub_rn(d, (double)L);
  else if (d < -0.5 * L) d = __dadd_rn(d, (double)L);
  return d;
}

__device__ inline void rel_pos(const BoxDev& B, const double R[3], double px, double py,
                               double pz, double r[3]) {
  r[0] = minimg(__dsub_rn(px, R[0]), B.nx);
  r[1] = minimg(__dsub_rn(py, R[1]), B.ny);
  r[2] = minimg(__dsub_rn(pz, R[2]), B.nz);
}

// Solid iff |x - R|^2 < a0^2 with the nominal radius and position (Sec. 2.2).
__device__ inline bool inside(const BoxDev& B, const ColDev& C, const double R[3], int x, int y, int z) {
  double r[3];
  rel_pos(B, R, (double)x, (double)y, (double)z, r);
  double d2 = __dadd_rn(__dadd_rn(__dmul_rn(r[0], r[0]), __dmul_rn(r[1], r[1])),
                        __dmul_rn(r[2], r[2]));
  return d2 < __dmul_rn(C.a0, C.a0);
}

// Rigid-body velocity v + omega x r at displacement r from the centre.
__device__ inline void rigid_vel(const ColDev& C, const double r[3], double ub[3]) {
  ub[0] = C.vel[0] + (C.omega[1] * r[2] - C.omega[2] * r[1]);
  ub[1] = C.vel[1] + (C.omega[2] * r[0] - C.omega[0] * r[2]);
  ub[2] = C.vel[2] + (C.omega[0] * r[1] - C.omega[1] * r[0]);
}

// Conservative integer test, one axis: can the colloid (radius + 3 sites)
// reach [lo, lo+ext) along axis a in some periodic image?
__device__ inline bool axis_near(const BoxDev& B, const ColDev& C, const double R[3], int a, int lo, int ext) {
  const int ra = (int)ceil(C.a0) + 3;
  const int L = a == 0 ? B.nx : (a == 1 ? B.ny : B.nz);
  const int c = (int)floor(R[a]);
  int best = 1 << 30;
  for (int k = -1; k <= 1; k++) {
    const int cc = c + k * L;
    const int d = cc < lo ? lo - cc : (cc > lo + ext - 1 ? cc - (lo + ext - 1) : 0);
    best = d < best ? d : best;
  }
  return best <= ra;
}

// Can any node of the block [lo, lo+ext) (per axis) lie within two lattice
// spacings of the colloid's surface?  Blocks for which this is false have no
// solid node of it within reach of their stencils.
__device__ inline bool block_near(const BoxDev& B, const ColDev& C, const double R[3], int x0, int y0, int z0,
                                  int ex, int ey, int ez) {
  return axis_near(B, C, R, 0, x0, ex) && axis_near(B, C, R, 1, y0, ey) && axis_near(B, C, R, 2, z0, ez);
}

// Bit k set for each colloid k of the box (at buffer parity par) that can
// reach the block.
__device__ inline unsigned near_mask(const BoxDev& B, const ColDev* cols, int par, int x0, int y0, int z0, int ex,
                                     int ey, int ez) {
  unsigned m = 0u;
  for (int k = 0; k < B.ncol; k++) {
    const ColDev& C = cols[B.col0 + k];
    if (block_near(B, C, C.pos[par], x0, y0, z0, ex, ey, ez)) m |= 1u << k;
  }
  return m;
}

// 1 + the index of the colloid (among those in mask) that holds node
// (x, y, z), or 0 for a fluid node.
__device__ inline int solid_id(const BoxDev& B, const ColDev* cols, unsigned mask, int par, int x, int y, int z) {
  for (unsigned m = mask; m; m &= m - 1u) {
    const int k = __builtin_ctz(m);
    const ColDev& C = cols[B.col0 + k];
    if (inside(B, C, C.pos[par], x, y, z)) return k + 1;
  }
  return 0;
}

// ---------------------------------------------------------------------
// Q-tensor algebra.  Five stored components (xx, xy, xz, yy, yz).
// ---------------------------------------------------------------------

template <typename R>
struct M3 {
  R m[3][3];
};

template <typename R>
__device__ inline void full5(const R q5[5], R q[3][3]) {
  q[0][0] = q5[0]; q[0][1] = q5[1]; q[0][2] = q5[2];
  q[1][0] = q5[1]; q[1][1] = q5[3]; q[1][2] = q5[4];
  q[2][0] = q5[2]; q[2][1] = q5[4]; q[2][2] = -q5[0] - q5[3];
}

// Material constants in the arithmetic precision of a kernel.
template <typename R>
struct Mat {
  R A0, gamma, K, q0, xi, Gamma, tau, rho0, itau, fsrc;
  __device__ explicit Mat(const BoxDev& B)
      : A0((R)B.A0), gamma((R)B.gamma), K((R)B.K), q0((R)B.q0), xi((R)B.xi),
        Gamma((R)B.Gamma), tau((R)B.tau), rho0((R)B.rho0), itau((R)B.itau), fsrc((R)B.fsrc) {}
};

// 1/x: exact division in FP64; in FP32 the hardware reciprocal refined by
// one Newton step (within an ulp or two of the correctly rounded value).
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return r * (2.0f - x * r);
}

// Local stencil quantities at one node from its own Q and the six face
// neighbours: Q, central first derivatives d[g] = D0_g Q and the compact
// Laplacian, each as five stored components.
template <typename R>
struct Stencil {
  R q[5], d[3][5], lap[5];
};

template <typename R>
__device__ inline void stencil5(const R c5[5], const R xp[5], const R xm[5], const R yp[5], const R ym[5],
                                const R zp[5], const R zm[5], Stencil<R>& st) {
#pragma unroll
  for (int k = 0; k < 5; k++) {
    st.q[k] = c5[k];
    st.d[0][k] = (R)0.5 * (xp[k] - xm[k]);
    st.d[1][k] = (R)0.5 * (yp[k] - ym[k]);
    st.d[2][k] = (R)0.5 * (zp[k] - zm[k]);
    st.lap[k] = ((xp[k] + xm[k]) + (yp[k] + ym[k])) + (zp[k] + zm[k]) - (R)6 * c5[k];
  }
}

// Isotropic 27-point variant of the stencil (the alternative reading of
// "the same stencil", Sec. 2.2): D_g Q = 3 sum_i w_i c_ig Q(x + c_i) with the
// D3Q27 weights 2/27 (faces), 1/54 (edges), 1/216 (corners), whose second
// moment is 1/3, and the Laplacian (14 sum_faces + 3 sum_edges + sum_corners
// - 128 Q)/30.  q points at the node in component 0 of a Q box with
// component stride cs, row stride sy and plane stride sz.
template <typename R>
__device__ inline void stencil27(const R* q, int cs, int sy, int sz, Stencil<R>& st) {
#pragma unroll
  for (int k = 0; k < 5; k++) {
    const R* p = q + k * cs;
    R lap = (R)0, d0 = (R)0, d1 = (R)0, d2 = (R)0;
#pragma unroll
    for (int dz = -1; dz <= 1; dz++)
#pragma unroll
      for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++) {
          const int n = (dx != 0) + (dy != 0) + (dz != 0);
          if (n == 0) continue;
          const R v = p[dx + dy * sy + dz * sz];
          const R wl = n == 1 ? (R)14 : (n == 2 ? (R)3 : (R)1);
          const R wg = n == 1 ? (R)(3.0 * 2.0 / 27.0) : (n == 2 ? (R)(3.0 / 54.0) : (R)(3.0 / 216.0));
          lap += wl * v;
          if (dx) d0 += (dx > 0 ? wg : -wg) * v;
          if (dy) d1 += (dy > 0 ? wg : -wg) * v;
          if (dz) d2 += (dz > 0 ? wg : -wg) * v;
        }
    st.q[k] = p[0];
    st.d[0][k] = d0;
    st.d[1][k] = d1;
    st.d[2][k] = d2;
    st.lap[k] = (lap - (R)128 * p[0]) / (R)30;
  }
}

// Full contraction A:B of two traceless symmetric tensors in five components.
template <typename R>
__device__ inline R dot5(const R a[5], const R b[5]) {
  return (R)2 * (a[0] * b[0] + a[3] * b[3] + a[1] * b[1] + a[2] * b[2] + a[4] * b[4]) + a[0] * b[3] +
         a[3] * b[0];
}

// Molecular field H (Eq. 2 applied to Eq. 1): bulk part
// -A0(1-g/3)Q + A0 g (Q.Q - Tr(Q^2)/3 I) - A0 g Tr(Q^2) Q, plus K lap Q and,
// for a cholesteric, -2 K q0 (M + M^T) - 4 K q0^2 Q with M_ab = e_agd d_g Q_db.
// Also returns Q.Q (symmetric, 3x3) and Tr(Q^2) for the stress.
template <typename R, bool CHIRAL>
__device__ inline void mol_field(const Mat<R>& p, const Stencil<R>& st, R q[3][3], R q2[3][3], R& tr2,
                                 R M[3][3], R h[3][3]) {
  full5(st.q, q);
  for (int i = 0; i < 3; i++)
    for (int j = i; j < 3; j++) q2[i][j] = q2[j][i] = q[i][0] * q[0][j] + q[i][1] * q[1][j] + q[i][2] * q[2][j];
  tr2 = dot5(st.q, st.q);
  R lap[3][3];
  full5(st.lap, lap);
  const R A0 = p.A0, g = p.gamma, K = p.K, q0 = p.q0;
  R cq = -A0 * ((R)1 - g / (R)3) - A0 * g * tr2;
  if (CHIRAL) {
    R d[3][3][3];
    full5(st.d[0], d[0]); full5(st.d[1], d[1]); full5(st.d[2], d[2]);
    for (int b = 0; b < 3; b++) {
      M[0][b] = d[1][2][b] - d[2][1][b];
      M[1][b] = d[2][0][b] - d[0][2][b];
      M[2][b] = d[0][1][b] - d[1][0][b];
    }
    cq -= (R)4 * K * q0 * q0;
  }
  const R t3 = tr2 / (R)3;
  for (int i = 0; i < 3; i++)
    for (int j = i; j < 3; j++) {
      R v = cq * q[i][j] + A0 * g * (q2[i][j] - (i == j ? t3 : (R)0)) + K * lap[i][j];
      if (CHIRAL) v -= (R)2 * K * q0 * (M[i][j] + M[j][i]);
      h[i][j] = h[j][i] = v;
    }
}

// One-constant free-energy density f (Eq. 1 in the one-constant form that
// Sec. 2.1 states is equivalent to it):
// bulk + K/2 |dQ|^2 + 2 K q0 Q:M + 2 K q0^2 |Q|^2.
template <typename R, bool CHIRAL>
__device__ inline R energy_density(const Mat<R>& p, const Stencil<R>& st, const R q[3][3], const R q2[3][3],
                                   R tr2, const R M[3][3]) {
  R tr3 = (R)0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) tr3 += q[i][j] * q2[j][i];
  const R dd = dot5(st.d[0], st.d[0]) + dot5(st.d[1], st.d[1]) + dot5(st.d[2], st.d[2]);
  const R A0 = p.A0, g = p.gamma, K = p.K;
  R fe = (R)0.5 * A0 * ((R)1 - g / (R)3) * tr2 - A0 * g / (R)3 * tr3 + (R)0.25 * A0 * g * tr2 * tr2 +
         (R)0.5 * K * dd;
  if (CHIRAL) {
    R qm = (R)0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) qm += q[i][j] * M[i][j];
    fe += (R)2 * K * p.q0 * qm + (R)2 * K * p.q0 * p.q0 * tr2;
  }
  return fe;
}

// Stress of Eq. (4) without the fluid pressure rho c_s^2, column b only:
// P_ab = f d_ab + 2 xi (Q + I/3)_ab Q:H - (2 xi/3) H_ab - E_ab
//        + (1 - xi)(QH)_ab - (1 + xi)(QH)_ba,
// E_ab = K d_aQ:d_bQ + 2 K q0 e_bjk (d_aQ Q)_jk.
template <typename R, bool CHIRAL, int b>
__device__ inline void stress_col(const Mat<R>& p, const Stencil<R>& st, const R q[3][3], const R h[3][3], R fe,
                                  R out[3]) {
  R d[3][3][3];
  full5(st.d[0], d[0]); full5(st.d[1], d[1]); full5(st.d[2], d[2]);
  R trqh = (R)0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) trqh += q[i][j] * h[i][j];
  const R K = p.K, xi = p.xi;
  constexpr int b1 = b == 2 ? 0 : b + 1, b2 = b == 0 ? 2 : b - 1;
  for (int a = 0; a < 3; a++) {
    const R qh_ab = q[a][0] * h[0][b] + q[a][1] * h[1][b] + q[a][2] * h[2][b];
    const R qh_ba = q[b][0] * h[0][a] + q[b][1] * h[1][a] + q[b][2] * h[2][a];
    R E = K * dot5(st.d[a], st.d[b]);
    if (CHIRAL) {
      // (d_a Q Q)_{b1 b2} - (d_a Q Q)_{b2 b1}
      R ax = (R)0;
      for (int n = 0; n < 3; n++) ax += d[a][b1][n] * q[n][b2] - d[a][b2][n] * q[n][b1];
      E += (R)2 * K * p.q0 * ax;
    }
    out[a] = (a == b ? fe + (R)2 * xi * (q[a][b] + (R)1 / (R)3) * trqh : (R)2 * xi * q[a][b] * trqh) -
             (R)2 * xi / (R)3 * h[a][b] - E + ((R)1 - xi) * qh_ab - ((R)1 + xi) * qh_ba;
  }
}

// Co-rotation term of the material derivative (Eq. 2, Beris-Edwards form):
// S = (xi D + Om)(Q + I/3) + (Q + I/3)(xi D - Om) - 2 xi (Q + I/3) Q:W,
// W_ab = d_b u_a.  Returns the five stored components.
template <typename R>
__device__ inline void corotation(R xi, const R W[3][3], const R q5[5], R S5[5]) {
  R q[3][3], D[3][3], Om[3][3];
  full5(q5, q);
  R qw = (R)0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      D[i][j] = (R)0.5 * (W[i][j] + W[j][i]);
      Om[i][j] = (R)0.5 * (W[i][j] - W[j][i]);
      qw += q[i][j] * W[j][i];
    }
  const int I[5] = {0, 0, 0, 1, 1}, J[5] = {0, 1, 2, 1, 2};
  for (int k = 0; k < 5; k++) {
    const int a = I[k], b = J[k];
    R acc = (R)0;
    for (int g = 0; g < 3; g++) {
      const R Aga = q[g][b] + (g == b ? (R)1 / (R)3 : (R)0);
      const R Aag = q[a][g] + (a == g ? (R)1 / (R)3 : (R)0);
      acc += (xi * D[a][g] + Om[a][g]) * Aga + Aag * (xi * D[g][b] - Om[g][b]);
    }
    S5[k] = acc - (R)2 * xi * (q[a][b] + (a == b ? (R)1 / (R)3 : (R)0)) * qw;
  }
}

// One Jacobi rotation zeroing a[P][Q] (R the third index), applied to the
// eigenvector columns v.  The pivot is a template argument so that a and v
// stay in registers (runtime indices would put both arrays in scratch).
template <int P, int Q>
__device__ inline void jacobi_rot(double (&a)[3][3], double (&v)[3][3]) {
  constexpr int R = 3 - P - Q;
  const double apq = a[P][Q];
  const double th = (a[Q][Q] - a[P][P]) / (2.0 * apq);
  const double t = fabs(th) > 1e150 ? 0.5 / th : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
  const double arp = a[R][P], arq = a[R][Q];
  a[P][P] -= t * apq;
  a[Q][Q] += t * apq;
  a[P][Q] = a[Q][P] = 0.0;
  a[R][P] = a[P][R] = c * arp - s * arq;
  a[R][Q] = a[Q][R] = s * arp + c * arq;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const double vkp = v[k][P], vkq = v[k][Q];
    v[k][P] = c * vkp - s * vkq;
    v[k][Q] = s * vkp + c * vkq;
  }
}

// Principal axis of a symmetric 3x3 matrix (FP64): classical Jacobi, each
// rotation annihilating the largest off-diagonal entry, until the
// off-diagonal mass is below 1e-30 of the total; the eigenvector of the
// largest diagonal entry (lowest index on ties).
__device__ inline void principal_axis(const double A[3][3], double n[3]) {
  double a[3][3], v[3][3];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      a[i][j] = 0.5 * (A[i][j] + A[j][i]);
      v[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int it = 0; it < 100; it++) {
    double o01 = fabs(a[0][1]), o02 = fabs(a[0][2]), o12 = fabs(a[1][2]);
    double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) tot += a[i][j] * a[i][j];
    if (off == 0.0 || off <= 1e-30 * tot) break;
    if (o02 > o01 && o02 >= o12) jacobi_rot<0, 2>(a, v);
    else if (o12 > o01 && o12 > o02) jacobi_rot<1, 2>(a, v);
    else jacobi_rot<0, 1>(a, v);
  }
  double best = a[0][0];
  int k = 0;
  if (a[1][1] > best) { k = 1; best = a[1][1]; }
  if (a[2][2] > best) k = 2;
#pragma unroll
  for (int i = 0; i < 3; i++) n[i] = k == 0 ? v[i][0] : (k == 1 ? v[i][1] : v[i][2]);
}

// Anchoring target Q^0 = S0 (n0 n0 - I/3) at a boundary solid node
// (Sec. 2.2): n0 = outward normal (homeotropic) or the principal axis of
// the neighbouring Q projected on the tangent plane (planar), with the
// fallbacks s x z and s x x when the projection vanishes.
__device__ inline void anchor_target(const BoxDev& B, const ColDev& C, const double R[3], int x, int y, int z,
                                     const double qbar[3][3], double q0[3][3]) {
  double r[3], s[3], n0[3];
  rel_pos(B, R, (double)x, (double)y, (double)z, r);
  const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (rn < 1e-12) { s[0] = 0.0; s[1] = 0.0; s[2] = 1.0; }
  else { s[0] = r[0] / rn; s[1] = r[1] / rn; s[2] = r[2] / rn; }
  if (C.anchoring == 2) {
    double n[3];
    principal_axis(qbar, n);
    const double ns = n[0] * s[0] + n[1] * s[1] + n[2] * s[2];
    double t[3] = {n[0] - ns * s[0], n[1] - ns * s[1], n[2] - ns * s[2]};
    double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    if (tn < 1e-12) {  // s x z
      t[0] = s[1]; t[1] = -s[0]; t[2] = 0.0;
      tn = sqrt(t[0] * t[0] + t[1] * t[1]);
      if (tn < 1e-12) {  // s x x
        t[0] = 0.0; t[1] = s[2]; t[2] = -s[1];
        tn = sqrt(t[1] * t[1] + t[2] * t[2]);
      }
    }
    n0[0] = t[0] / tn; n0[1] = t[1] / tn; n0[2] = t[2] / tn;
  } else {
    n0[0] = s[0]; n0[1] = s[1]; n0[2] = s[2];
  }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) q0[a][b] = C.S0 * (n0[a] * n0[b] - (a == b ? 1.0 / 3.0 : 0.0));
}

}  // namespace lc
