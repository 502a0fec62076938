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

// One box of the batch.  Host and device share this layout; the colloid
// position is advanced on the device by the finalize kernel.
struct BoxDev {
  int nx, ny, nz, hydro;
  long long off;            // first site of the box in the concatenated arrays
  int tile_base, ntx, nty, ntz;          // fused-kernel tiles of this box
  int ghost_base, ghost_ext;             // ghost launch: thread range, bbox edge
  int event_base, event_ext;             // event launch: thread range, bbox edge
  int event_blk0, event_nblk;            // event partial-sum blocks of this box
  double tau, rho0, A0, gamma, K, q0, xi, Gamma;
  double body[3];
  int present, motion, anchoring, pad_;
  double pos[3], a0, vel[3], omega[3], S0, W;
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
__device__ inline bool inside(const BoxDev& B, const double R[3], int x, int y, int z) {
  double r[3];
  rel_pos(B, R, (double)x, (double)y, (double)z, r);
  double d2 = __dadd_rn(__dadd_rn(__dmul_rn(r[0], r[0]), __dmul_rn(r[1], r[1])),
                        __dmul_rn(r[2], r[2]));
  return d2 < __dmul_rn(B.a0, B.a0);
}

// Rigid-body velocity v + omega x r at displacement r from the centre.
__device__ inline void rigid_vel(const BoxDev& B, const double r[3], double ub[3]) {
  ub[0] = B.vel[0] + (B.omega[1] * r[2] - B.omega[2] * r[1]);
  ub[1] = B.vel[1] + (B.omega[2] * r[0] - B.omega[0] * r[2]);
  ub[2] = B.vel[2] + (B.omega[0] * r[1] - B.omega[1] * r[0]);
}

// Conservative integer test: can any node of the block [lo, lo+ext) (per
// axis) lie within two lattice spacings of the colloid surface?  Blocks for
// which this is false have no solid node within reach of their stencils.
__device__ inline bool block_near(const BoxDev& B, const double R[3], int x0, int y0, int z0,
                                  int ex, int ey, int ez) {
  if (!B.present) return false;
  const int ra = (int)ceil(B.a0) + 3;
  const int lo[3] = {x0, y0, z0}, ext[3] = {ex, ey, ez}, L[3] = {B.nx, B.ny, B.nz};
  for (int a = 0; a < 3; a++) {
    int c = (int)floor(R[a]);
    int best = 1 << 30;
    for (int k = -1; k <= 1; k++) {
      int cc = c + k * L[a];
      int d = cc < lo[a] ? lo[a] - cc : (cc > lo[a] + ext[a] - 1 ? cc - (lo[a] + ext[a] - 1) : 0);
      best = d < best ? d : best;
    }
    if (best > ra) return false;
  }
  return true;
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
  R A0, gamma, K, q0, xi, Gamma, tau, rho0;
  __device__ explicit Mat(const BoxDev& B)
      : A0((R)B.A0), gamma((R)B.gamma), K((R)B.K), q0((R)B.q0), xi((R)B.xi),
        Gamma((R)B.Gamma), tau((R)B.tau), rho0((R)B.rho0) {}
};

// Molecular field H (Eq. 2 applied to Eq. 1) and, if wanted, the stress P
// of Eq. (4) without the fluid pressure rho c_s^2, at one node from its own
// Q and the six face neighbours.  Central first derivatives, compact
// Laplacian.  Chiral terms: H gains -2 K q0 (M + M^T) - 4 K q0^2 Q with
// M_ab = e_agd d_g Q_db; P = f I + 2 xi (Q + I/3) Q:H - xi (H A + A H)
// - E + QH - HQ, E_ab = K d_aQ:d_bQ + 2 K q0 e_bjk (d_aQ Q)_jk, and f the
// one-constant free-energy density.
template <typename R, bool WANT_P>
__device__ inline void field_and_stress(const Mat<R>& p, const R c5[5], const R xp[5],
                                        const R xm[5], const R yp[5], const R ym[5],
                                        const R zp[5], const R zm[5], R H5[5], R P[9]) {
  R q[3][3], d[3][3][3], lap[3][3];
  full5(c5, q);
  {
    R a[3][3], b[3][3];
    full5(xp, a); full5(xm, b);
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) { d[0][i][j] = (R)0.5 * (a[i][j] - b[i][j]); lap[i][j] = a[i][j] + b[i][j]; }
    full5(yp, a); full5(ym, b);
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) { d[1][i][j] = (R)0.5 * (a[i][j] - b[i][j]); lap[i][j] += a[i][j] + b[i][j]; }
    full5(zp, a); full5(zm, b);
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        d[2][i][j] = (R)0.5 * (a[i][j] - b[i][j]);
        lap[i][j] += a[i][j] + b[i][j] - (R)6 * q[i][j];
      }
  }
  R q2[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) q2[i][j] = q[i][0] * q[0][j] + q[i][1] * q[1][j] + q[i][2] * q[2][j];
  const R tr2 = q2[0][0] + q2[1][1] + q2[2][2];
  // M_ab = e_agd d_g Q_db
  R M[3][3];
  for (int b = 0; b < 3; b++) {
    M[0][b] = d[1][2][b] - d[2][1][b];
    M[1][b] = d[2][0][b] - d[0][2][b];
    M[2][b] = d[0][1][b] - d[1][0][b];
  }
  const R A0 = p.A0, g = p.gamma, K = p.K, q0 = p.q0;
  const R cq = -A0 * ((R)1 - g / (R)3) - A0 * g * tr2 - (R)4 * K * q0 * q0;
  R h[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      h[i][j] = cq * q[i][j] + A0 * g * (q2[i][j] - (i == j ? tr2 / (R)3 : (R)0)) + K * lap[i][j] -
                (R)2 * K * q0 * (M[i][j] + M[j][i]);
  H5[0] = h[0][0]; H5[1] = h[0][1]; H5[2] = h[0][2]; H5[3] = h[1][1]; H5[4] = h[1][2];
  if (!WANT_P) return;
  // one-constant free-energy density
  R tr3 = (R)0, qm = (R)0, dd = (R)0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      tr3 += q[i][j] * q2[j][i];
      qm += q[i][j] * M[i][j];
    }
  R E1[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = a; b < 3; b++) {
      R s = (R)0;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) s += d[a][i][j] * d[b][i][j];
      E1[a][b] = E1[b][a] = s;
    }
  dd = E1[0][0] + E1[1][1] + E1[2][2];
  const R fe = (R)0.5 * A0 * ((R)1 - g / (R)3) * tr2 - A0 * g / (R)3 * tr3 +
               (R)0.25 * A0 * g * tr2 * tr2 + (R)0.5 * K * dd + (R)2 * K * q0 * qm +
               (R)2 * K * q0 * q0 * tr2;
  R qh[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) qh[i][j] = q[i][0] * h[0][j] + q[i][1] * h[1][j] + q[i][2] * h[2][j];
  const R trqh = qh[0][0] + qh[1][1] + qh[2][2];
  const R xi = p.xi;
  for (int a = 0; a < 3; a++) {
    // axial vector of the antisymmetric part of (d_a Q) Q
    R dq[3][3];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        dq[i][j] = d[a][i][0] * q[0][j] + d[a][i][1] * q[1][j] + d[a][i][2] * q[2][j];
    const R ax[3] = {dq[1][2] - dq[2][1], dq[2][0] - dq[0][2], dq[0][1] - dq[1][0]};
    for (int b = 0; b < 3; b++) {
      const R E = K * E1[a][b] + (R)2 * K * q0 * ax[b];
      P[3 * a + b] = (a == b ? fe : (R)0) + (R)2 * xi * (q[a][b] + (a == b ? (R)1 / (R)3 : (R)0)) * trqh -
                     (R)2 * xi / (R)3 * h[a][b] - E + ((R)1 - xi) * qh[a][b] - ((R)1 + xi) * qh[b][a];
    }
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

// Principal axis of a symmetric 3x3 matrix (FP64): classical Jacobi, each
// rotation annihilating the largest off-diagonal entry, until the
// off-diagonal mass is below 1e-30 of the total; the eigenvector of the
// largest diagonal entry (lowest index on ties).
__device__ inline void principal_axis(const double A[3][3], double n[3]) {
  double a[3][3], v[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      a[i][j] = 0.5 * (A[i][j] + A[j][i]);
      v[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int it = 0; it < 100; it++) {
    double o01 = fabs(a[0][1]), o02 = fabs(a[0][2]), o12 = fabs(a[1][2]);
    double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    double tot = 0.0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) tot += a[i][j] * a[i][j];
    if (off == 0.0 || off <= 1e-30 * tot) break;
    int p = 0, q = 1;
    if (o02 > o01 && o02 >= o12) { p = 0; q = 2; }
    else if (o12 > o01 && o12 > o02) { p = 1; q = 2; }
    const double apq = a[p][q];
    const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
    const double t = fabs(th) > 1e150 ? 0.5 / th
                                      : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
    const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
    const int r = 3 - p - q;
    const double arp = a[r][p], arq = a[r][q];
    a[p][p] -= t * apq;
    a[q][q] += t * apq;
    a[p][q] = a[q][p] = 0.0;
    a[r][p] = a[p][r] = c * arp - s * arq;
    a[r][q] = a[q][r] = s * arp + c * arq;
    for (int k = 0; k < 3; k++) {
      const double vkp = v[k][p], vkq = v[k][q];
      v[k][p] = c * vkp - s * vkq;
      v[k][q] = s * vkp + c * vkq;
    }
  }
  int k = 0;
  if (a[1][1] > a[k][k]) k = 1;
  if (a[2][2] > a[k][k]) k = 2;
  n[0] = v[0][k]; n[1] = v[1][k]; n[2] = v[2][k];
}

// Anchoring target Q^0 = S0 (n0 n0 - I/3) at a boundary solid node
// (Sec. 2.2): n0 = outward normal (homeotropic) or the principal axis of
// the neighbouring Q projected on the tangent plane (planar), with the
// fallbacks s x z and s x x when the projection vanishes.
__device__ inline void anchor_target(const BoxDev& B, const double R[3], int x, int y, int z,
                                     const double qbar[3][3], double q0[3][3]) {
  double r[3], s[3], n0[3];
  rel_pos(B, R, (double)x, (double)y, (double)z, r);
  const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (rn < 1e-12) { s[0] = 0.0; s[1] = 0.0; s[2] = 1.0; }
  else { s[0] = r[0] / rn; s[1] = r[1] / rn; s[2] = r[2] / rn; }
  if (B.anchoring == 2) {
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
    for (int b = 0; b < 3; b++) q0[a][b] = B.S0 * (n0[a] * n0[b] - (a == b ? 1.0 / 3.0 : 0.0));
}

}  // namespace lc
