// lc_march.hpp -- the fused step in z-marching form (FP32).
//
// Columns of TX x TY nodes march through the z planes of a work item with
// rolling LDS planes; the per-site arithmetic is that of the 3D-tile kernel
// (Sec. 2.1-2.2: H and P from the Q stencil, face divergence of P,
// Beris-Edwards update with upwind fluxes, BGK collision with Guo forcing,
// push streaming with bounce-back on links, colloid sums).
//
// The including file provides the architecture layer first (lds_sync,
// FieldBuf, keep_live: lc_arch.hpp on the device).
#pragma once

#include <type_traits>

#include "lc_kernels.hpp"
#include "lc_reduce.hpp"

#ifndef LC_ARCH_LAYER
#error "include the architecture layer (lc_arch.hpp) before lc_march.hpp"
#endif

namespace lc {

// LDS of one block of the z-marching kernel: rolling planes.
template <typename R, int TX, int TY>
struct MarchSmem {
  static constexpr int NT = TX * TY;
  static constexpr int QPX = TX + 4, QP = (TX + 4) * (TY + 4);   // Q plane, halo 2
  static constexpr int UPX = TX + 2, UP = (TX + 2) * (TY + 2);   // velocity plane, halo 1
  static constexpr int NRX = 2 * TY, NRY = 2 * TX;               // face rings of a plane
  static constexpr int PS = 6 * NT + 3 * (NRX + NRY);           // x and y stress columns of a plane
  R Q[5][5 * QP];
  unsigned char S[5][QP];
  R U[4][3 * UP];
  R P[2][PS];
  double red[2][(NT / 64) * 12];   // per-wave colloid sums of the current z group (two sets)
};

// Block = TX x TY columns marching through the z planes of one work item
// (whole groups of kGroup planes), one thread per column.  Each plane's stress is computed once per column (full at the
// columns, the x or y column on the four face rows around the tile); the
// z faces take their stress from the neighbouring planes' results held in
// registers.  Planes of Q (halo 2) and u (halo 1) are loaded one step ahead
// into registers and rotated through LDS, so one barrier per plane suffices.
template <typename R, int TX, int TY, int CZ, bool CHIRAL>
__device__ __forceinline__ void march_tile(const BoxDev& B, const int2 tt, const StepPtrs<R>& a,
                                           MarchSmem<R, TX, TY>& sm);

// Persistent form: block b works through its own list of items.
template <typename R, int TX, int TY, int CZ>
__global__ void __launch_bounds__(TX* TY)
    k_march(const BoxDev* __restrict__ boxes, const int2* __restrict__ items, const int* __restrict__ offs,
            StepPtrs<R> a) {
  __shared__ MarchSmem<R, TX, TY> sm;
  const int i0 = offs[blockIdx.x], i1 = offs[blockIdx.x + 1];
  for (int it = i0; it < i1; it++) {
    const int2 tt = items[it];
    const BoxDev& B = boxes[item_box(tt.x)];
    if (it > i0) lds_sync();   // the previous item's LDS reads are done
    if (B.q0 != 0.0) march_tile<R, TX, TY, CZ, true>(B, tt, a, sm);
    else march_tile<R, TX, TY, CZ, false>(B, tt, a, sm);
  }
}

template <typename R, int TX, int TY, int CZ, bool CHIRAL>
__device__ __forceinline__ void march_tile(const BoxDev& B, const int2 tt, const StepPtrs<R>& a,
                                           MarchSmem<R, TX, TY>& sm) {
  using SM = MarchSmem<R, TX, TY>;
  constexpr int NT = SM::NT, QPX = SM::QPX, QP = SM::QP, UPX = SM::UPX, UP = SM::UP;
  constexpr int NRX = SM::NRX, NRY = SM::NRY;
  constexpr int MQ = (QP + NT - 1) / NT, MU = (UP + NT - 1) / NT;
  constexpr int NR = NRX + NRY;

  const int nx = B.nx, ny = B.ny, nz = B.nz, hydro = B.hydro;
  const int nxy = nx * ny;
  const int cb = item_cb(tt.y), g0 = item_g0(tt.y), ng = item_ng(tt.x);
  const int ncb = B.ntx * B.nty;
  const int tix = cb % B.ntx, tiy = cb / B.ntx;
  const int x0 = tix * TX, y0 = tiy * TY, z0 = g0 * kGroup;
  const int zend = z0 + ng * kGroup < nz ? z0 + ng * kGroup : nz;
  const unsigned off = (unsigned)B.off;
  const long long NS = a.nsites;
  const FieldBuf bfin(a.fin, NS, 19), bfout(a.fout, NS, 19), bqin(a.Qin, NS, 5), bqout(a.Qout, NS, 5),
      buin(a.uin, NS, 3), buout(a.uout, NS, 3);
  // boxes on the marching kernel hold at most one colloid (the runtime sends
  // boxes with more to the 3D-tile kernel); the table has at least one entry
  const bool has = B.ncol > 0;
  const ColDev& C = a.cols[has ? B.col0 : 0];
  const double Rc[3] = {C.pos[a.par][0], C.pos[a.par][1], C.pos[a.par][2]};
  // nominal extent (whole groups): every group's own test (in k_post)
  // covers a subset of this range, so a group counted there was written here
  const bool near = has && block_near(B, C, Rc, x0 - 2, y0 - 2, z0 - 2, TX + 4, TY + 4, ng * kGroup + 4);
  const Mat<R> mp(B);
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool incol = gx < nx && gy < ny;

  auto wrapn = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };

  // this thread's elements of a halo plane: 2D offsets computed once
  int qo[MQ], qwx[MQ], qwy[MQ];
#pragma unroll
  for (int m = 0; m < MQ; m++) {
    const int e = tid + m * NT;
    const int ex = e % QPX, ey = e / QPX;
    qwx[m] = wrapn(x0 - 2 + ex, nx);
    qwy[m] = wrapn(y0 - 2 + ey, ny);
    qo[m] = qwx[m] + nx * qwy[m];
  }
  int uo[MU];
#pragma unroll
  for (int m = 0; m < MU; m++) {
    const int e = tid + m * NT;
    const int ex = e % UPX, ey = e / UPX;
    uo[m] = wrapn(x0 - 1 + ex, nx) + nx * wrapn(y0 - 1 + ey, ny);
  }
  R rq[MQ][5], ru[MU][3];
  auto fetch_q = [&](R (&dst)[MQ][5], int z) {
    const unsigned zo = off + (unsigned)(nxy * wrapn(z, nz));
#pragma unroll
    for (int m = 0; m < MQ; m++)
      if (m < MQ - 1 || tid + m * NT < QP)
#pragma unroll
        for (int c = 0; c < 5; c++) dst[m][c] = bqin.ld_nt(c, zo + (unsigned)qo[m]);
  };
  auto fetch_u = [&](R (&dst)[MU][3], int z) {
    const unsigned zo = off + (unsigned)(nxy * wrapn(z, nz));
#pragma unroll
    for (int m = 0; m < MU; m++)
      if (m < MU - 1 || tid + m * NT < UP)
#pragma unroll
        for (int c = 0; c < 3; c++) dst[m][c] = buin.ld_nt(c, zo + (unsigned)uo[m]);
  };
  auto store_q = [&](const R (&rq)[MQ][5], int slot, int z) {
    const int wz = wrapn(z, nz);
#pragma unroll
    for (int m = 0; m < MQ; m++) {
      const int e = tid + m * NT;
      if (m < MQ - 1 || e < QP) {
#pragma unroll
        for (int c = 0; c < 5; c++) sm.Q[slot][c * QP + e] = rq[m][c];
        sm.S[slot][e] = near ? (unsigned char)inside(B, C, Rc, qwx[m], qwy[m], wz) : (unsigned char)0;
      }
    }
  };
  auto store_u = [&](const R (&ru)[MU][3], int slot) {
#pragma unroll
    for (int m = 0; m < MU; m++) {
      const int e = tid + m * NT;
      if (m < MU - 1 || e < UP)
#pragma unroll
        for (int c = 0; c < 3; c++) sm.U[slot][c * UP + e] = ru[m][c];
    }
  };
  // rigid-body velocity at the solid nodes of a velocity plane (after the
  // plane's solid flags are in LDS)
  auto fix_u = [&](int uslot, int qslot, int z) {
    if (!near) return;
    const int wz = wrapn(z, nz);
    for (int e = tid; e < UP; e += NT) {
      const int ex = e % UPX, ey = e / UPX;
      if (!sm.S[qslot][(ey + 1) * QPX + ex + 1]) continue;
      double r[3], ub[3];
      rel_pos(B, Rc, (double)wrapn(x0 - 1 + ex, nx), (double)wrapn(y0 - 1 + ey, ny), (double)wz, r);
      rigid_vel(C, r, ub);
#pragma unroll
      for (int c = 0; c < 3; c++) sm.U[uslot][c * UP + e] = (R)ub[c];
    }
  };

  // Stress and field of plane p at the own column (full) and, if ring, on
  // the face rows (one column each).  Q slots of planes p-1, p, p+1.
  auto plane_stress = [&](int qm, int q0, int qp, int pslot, bool ring, R h5[5], R pz[3]) {
    const int ic = (ly + 2) * QPX + lx + 2;
    Stencil<R> st;
    {
      R c5[5], xp[5], xm[5], yp[5], ym[5], zp[5], zm[5];
#pragma unroll
      for (int c = 0; c < 5; c++) {
        const auto q = lds_at(sm.Q[q0], c * QP, QP, ic);
        c5[c] = q[0]; xp[c] = q[1]; xm[c] = q[-1]; yp[c] = q[QPX]; ym[c] = q[-QPX];
        zp[c] = sm.Q[qp][c * QP + ic]; zm[c] = sm.Q[qm][c * QP + ic];
      }
      stencil5(c5, xp, xm, yp, ym, zp, zm, st);
    }
    R q[3][3], q2[3][3], tr2, M[3][3], h[3][3];
    mol_field<R, CHIRAL>(mp, st, q, q2, tr2, M, h);
    h5[0] = h[0][0]; h5[1] = h[0][1]; h5[2] = h[0][2]; h5[3] = h[1][1]; h5[4] = h[1][2];
    if (hydro && !sm.S[q0][ic]) {
      const R fe = energy_density<R, CHIRAL>(mp, st, q, q2, tr2, M);
      R cxv[3], cyv[3];
      stress_col<R, CHIRAL, 0>(mp, st, q, h, fe, cxv);
      stress_col<R, CHIRAL, 1>(mp, st, q, h, fe, cyv);
      stress_col<R, CHIRAL, 2>(mp, st, q, h, fe, pz);
      if (ring) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
          sm.P[pslot][(2 * c) * NT + tid] = cxv[c];
          sm.P[pslot][(2 * c + 1) * NT + tid] = cyv[c];
        }
      }
    }
    if (hydro && ring && tid < NR) {
      // face rows: x faces (x = -1, TX) then y faces (y = -1, TY)
      int rx, ry, b;
      if (tid < NRX) { rx = tid < TY ? -1 : TX; ry = tid % TY; b = 0; }
      else { const int r = tid - NRX; ry = r < TX ? -1 : TY; rx = r % TX; b = 1; }
      const int ir = (ry + 2) * QPX + rx + 2;
      if (!sm.S[q0][ir]) {
        Stencil<R> sr;
        {
          R c5[5], xp[5], xm[5], yp[5], ym[5], zp[5], zm[5];
#pragma unroll
          for (int c = 0; c < 5; c++) {
            const auto qq = lds_at(sm.Q[q0], c * QP, QP, ir);
            c5[c] = qq[0]; xp[c] = qq[1]; xm[c] = qq[-1]; yp[c] = qq[QPX]; ym[c] = qq[-QPX];
            zp[c] = sm.Q[qp][c * QP + ir]; zm[c] = sm.Q[qm][c * QP + ir];
          }
          stencil5(c5, xp, xm, yp, ym, zp, zm, sr);
        }
        R rq3[3][3], rq2[3][3], rtr2, rM[3][3], rh[3][3], col[3];
        mol_field<R, CHIRAL>(mp, sr, rq3, rq2, rtr2, rM, rh);
        const R fe = energy_density<R, CHIRAL>(mp, sr, rq3, rq2, rtr2, rM);
        if (b == 0) stress_col<R, CHIRAL, 0>(mp, sr, rq3, rh, fe, col);
        else stress_col<R, CHIRAL, 1>(mp, sr, rq3, rh, fe, col);
        const int base = 6 * NT + (b == 0 ? 0 : 3 * NRX);
        const int nr = b == 0 ? NRX : NRY;
        const int idx = b == 0 ? tid : tid - NRX;
#pragma unroll
        for (int c = 0; c < 3; c++) sm.P[pslot][base + c * nr + idx] = col[c];
      }
    }
  };

  constexpr int NW = NT / 64;
  for (int e = tid; e < 2 * NW * 12; e += NT) (&sm.red[0][0])[e] = 0.0;
  // colloid sums of group g of this item (after the barrier that ends its
  // last plane): waves added in wave order, written to the group's slot, and
  // the set cleared for group g + 2 (at least one barrier later)
  auto flush = [&](int g) {
    if (near && tid < 12) {
      double* r = sm.red[g & 1];
      double t = 0.0;
      for (int w = 0; w < NW; w++) {
        t += r[w * 12 + tid];
        r[w * 12 + tid] = 0.0;
      }
      a.part[tid * a.nslot + C.slot_base + cb + (long long)ncb * (g0 + g)] = t;
    }
  };

  // populations of the own column, one plane ahead of their use
  R f[19];
  const unsigned gcol = off + (unsigned)(gx + nx * gy);
  auto fetch_f = [&](int z) {
    if (hydro && incol) {
      const unsigned gf = gcol + (unsigned)(nxy * z);
#pragma unroll
      for (int i = 0; i < 19; i++) f[i] = bfin.ld_nt(i, gf);
    }
  };
  fetch_f(z0);

  // prologue: Q planes z0-2 .. z0+2 in slots 0..4, u planes z0-1 .. z0+1
  // in slots 0..2, all requested before the first is stored
  {
    R pq[5][MQ][5], pu[3][MU][3];
#pragma unroll
    for (int k = 0; k < 5; k++) fetch_q(pq[k], z0 - 2 + k);
    if (hydro)
#pragma unroll
      for (int k = 0; k < 3; k++) fetch_u(pu[k], z0 - 1 + k);
#pragma unroll
    for (int k = 0; k < 5; k++) store_q(pq[k], k, z0 - 2 + k);
    if (hydro)
#pragma unroll
      for (int k = 0; k < 3; k++) store_u(pu[k], k);
  }
  lds_sync();
  if (hydro)
    for (int k = 0; k < 3; k++) fix_u(k, k + 1, z0 - 1 + k);
  R h_cur[5], h_nxt[5], pz_m[3] = {(R)0, (R)0, (R)0}, pz_c[3] = {(R)0, (R)0, (R)0},
                        pz_n[3] = {(R)0, (R)0, (R)0};
  {
    // Plane z0-1 needs only its z column, but it is computed exactly as the
    // loop computes every plane (face rows into the P slot that plane z0+1
    // overwrites next, the field kept live by keep_live): the compiler
    // fuses multiplies and adds by how their results are used, so a leaner
    // copy could round the z column differently and make the bits depend on
    // where work items start.
    R hdummy[5];
    plane_stress(0, 1, 2, 1, true, hdummy, pz_m);   // plane z0-1
    keep_live(hdummy);
    plane_stress(1, 2, 3, 0, true, h_cur, pz_c);    // plane z0
  }
  lds_sync();

  int qs_m1 = 1, qs_0 = 2, qs_p1 = 3, qs_p2 = 4, qs_free = 0;  // slots of planes k-1..k+2, k+3
  int us_m1 = 0, us_0 = 1, us_p1 = 2, us_free = 3;
  int ps_0 = 0;
  const int wv = tid >> 6;

  for (int k = z0; k < zend; k++) {
    const int gi = (k - z0) / kGroup;
    if (k > z0 && k - z0 == gi * kGroup) flush(gi - 1);
    double part[12];
#pragma unroll
    for (int c = 0; c < 12; c++) part[c] = 0.0;
    const int gz = k;
    const unsigned g = gcol + (unsigned)(nxy * gz);
    const bool more = k + 1 < zend;
    if (more) {
      fetch_q(rq, k + 3);
      if (hydro) fetch_u(ru, k + 2);
    }
    // stress of plane k+1
    plane_stress(qs_0, qs_p1, qs_p2, ps_0 ^ 1, true, h_nxt, pz_n);

    // own node of plane k
    const int ic = (ly + 2) * QPX + lx + 2;
    const int iu = (ly + 1) * UPX + lx + 1;
    const bool fluid = !sm.S[qs_0][ic];
    // the solid-aware update only where plane k's links can reach the colloid
    const bool pnear = near && block_near(B, C, Rc, x0 - 2, y0 - 2, k - 2, TX + 4, TY + 4, 5);
    auto update = [&](auto near_tag) {
      constexpr bool NEAR = decltype(near_tag)::value;
      R q5[5], dQ[5];
#pragma unroll
      for (int c = 0; c < 5; c++) {
        q5[c] = sm.Q[qs_0][c * QP + ic];
        dQ[c] = mp.Gamma * h_cur[c];
      }
      // solid flags of the 18 link neighbours
      bool sn[19];
#pragma unroll
      for (int i = 0; i < 19; i++) {
        const int sl = cz(i) > 0 ? qs_p1 : (cz(i) < 0 ? qs_m1 : qs_0);
        sn[i] = NEAR ? (bool)sm.S[sl][ic + cx(i) + cy(i) * QPX] : false;
      }
      R F[3] = {(R)0, (R)0, (R)0};
      // solid-link sums of this site: stress-face force and its torque about
      // r_site, bounce-back momentum
      double fps[3] = {0.0, 0.0, 0.0}, fts[3] = {0.0, 0.0, 0.0}, bbp[3] = {0.0, 0.0, 0.0};
      bool anys = false;
      if (NEAR) {
#pragma unroll
        for (int i = 1; i < 19; i++) anys = anys || sn[i];
      }
      if (hydro) {
        const auto Pp = lds_at(sm.P[ps_0], 0, SM::PS, 0);
        R Pc[3][3];   // own stress, [c][b]
#pragma unroll
        for (int c = 0; c < 3; c++) {
          Pc[c][0] = Pp[(2 * c) * NT + tid];
          Pc[c][1] = Pp[(2 * c + 1) * NT + tid];
          Pc[c][2] = pz_c[c];
        }
#pragma unroll
        for (int b = 0; b < 3; b++) {
          const bool sp = sn[2 * b + 1], sm_ = sn[2 * b + 2];
#pragma unroll
          for (int c = 0; c < 3; c++) {
            R pn, pmv;
            if (b == 0) {
              pn = lx + 1 < TX ? Pp[(2 * c) * NT + tid + 1] : Pp[6 * NT + c * NRX + TY + ly];
              pmv = lx > 0 ? Pp[(2 * c) * NT + tid - 1] : Pp[6 * NT + c * NRX + ly];
            } else if (b == 1) {
              pn = ly + 1 < TY ? Pp[(2 * c + 1) * NT + tid + TX] : Pp[6 * NT + 3 * NRX + c * NRY + TX + lx];
              pmv = ly > 0 ? Pp[(2 * c + 1) * NT + tid - TX] : Pp[6 * NT + 3 * NRX + c * NRY + lx];
            } else {
              pn = pz_n[c];
              pmv = pz_m[c];
            }
            const R pcv = Pc[c][b];
            const R pp = sp ? pcv : (R)0.5 * (pcv + pn);
            const R pm = sm_ ? pcv : (R)0.5 * (pcv + pmv);
            F[c] += pp - pm;
          }
          if (NEAR && (sp || sm_)) {
            // a face to a solid node with sign sg passes -sg P[:,b] to the
            // colloid at r_site + (sg/2) x_b; its torque about the centre
            // is r_site x ps - (1/2) x_b x P[:,b] for either sign
            const double nsg = (sp ? 1.0 : 0.0) - (sm_ ? 1.0 : 0.0);
            const double hc = 0.5 * ((sp ? 1.0 : 0.0) + (sm_ ? 1.0 : 0.0));
            const double p0 = (double)Pc[0][b], p1 = (double)Pc[1][b], p2 = (double)Pc[2][b];
            fps[0] -= nsg * p0; fps[1] -= nsg * p1; fps[2] -= nsg * p2;
            if (b == 0) { fts[1] += hc * p2; fts[2] -= hc * p1; }
            else if (b == 1) { fts[0] -= hc * p2; fts[2] += hc * p0; }
            else { fts[0] += hc * p1; fts[1] -= hc * p0; }
          }
        }
#pragma unroll
        for (int c = 0; c < 3; c++) F[c] += (R)B.body[c];

        // Beris-Edwards: velocity gradient, upwind fluxes, co-rotation
        R u0[3], W[3][3];
#pragma unroll
        for (int c = 0; c < 3; c++) u0[c] = sm.U[us_0][c * UP + iu];
#pragma unroll
        for (int b = 0; b < 3; b++) {
          R up[3], um[3];
#pragma unroll
          for (int c = 0; c < 3; c++) {
            if (b == 0) { up[c] = sm.U[us_0][c * UP + iu + 1]; um[c] = sm.U[us_0][c * UP + iu - 1]; }
            else if (b == 1) { up[c] = sm.U[us_0][c * UP + iu + UPX]; um[c] = sm.U[us_0][c * UP + iu - UPX]; }
            else { up[c] = sm.U[us_p1][c * UP + iu]; um[c] = sm.U[us_m1][c * UP + iu]; }
            W[c][b] = (R)0.5 * (up[c] - um[c]);
          }
          const bool fp = !sn[2 * b + 1], fm = !sn[2 * b + 2];
          const R ufp = (R)0.5 * (u0[b] + up[b]), ufm = (R)0.5 * (um[b] + u0[b]);
#pragma unroll
          for (int c = 0; c < 5; c++) {
            R qn_p, qn_m;
            if (b == 0) { qn_p = sm.Q[qs_0][c * QP + ic + 1]; qn_m = sm.Q[qs_0][c * QP + ic - 1]; }
            else if (b == 1) { qn_p = sm.Q[qs_0][c * QP + ic + QPX]; qn_m = sm.Q[qs_0][c * QP + ic - QPX]; }
            else { qn_p = sm.Q[qs_p1][c * QP + ic]; qn_m = sm.Q[qs_m1][c * QP + ic]; }
            const R phip = fp ? ufp * (ufp >= (R)0 ? q5[c] : qn_p) : (R)0;
            const R phim = fm ? ufm * (ufm >= (R)0 ? qn_m : q5[c]) : (R)0;
            dQ[c] -= phip - phim;
          }
        }
        R S5[5];
        corotation<R>(mp.xi, W, q5, S5);
#pragma unroll
        for (int c = 0; c < 5; c++) dQ[c] += S5[c];
      }
      R qn2 = (R)0;
#pragma unroll
      for (int c = 0; c < 5; c++) {
        const R v = q5[c] + dQ[c];
        bqout.st_nt(c, g, v);
        qn2 += v * v;
      }
      bool bad = !(qn2 < (R)100);
      if (hydro) {
        R rm1 = (R)0;
#pragma unroll
        for (int i = 0; i < 19; i++) rm1 += f[i];
        const R j[3] = {((f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10])) + ((f[11] - f[12]) + (f[13] - f[14])),
                        ((f[3] - f[4]) + (f[7] - f[8]) - (f[9] - f[10])) + ((f[15] - f[16]) + (f[17] - f[18])),
                        ((f[5] - f[6]) + (f[11] - f[12]) - (f[13] - f[14])) + ((f[15] - f[16]) - (f[17] - f[18]))};
        const R rho = (R)1 + rm1;
        const R irho = recip(rho);
        R u[3];
#pragma unroll
        for (int c = 0; c < 3; c++) u[c] = (j[c] + (R)0.5 * F[c]) * irho;
        const R usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const R uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        const R itau = mp.itau, fsrc = mp.fsrc;
        bad = bad || !(usq < (R)0.09);
        R fs[19];
        {
          const R w = (R)wgt(0);
          const R feq = w * rm1 + w * rho * ((R)-1.5 * usq);
          const R src = w * ((R)-3 * uF);
          fs[0] = f[0] - (f[0] - feq) * itau + fsrc * src;
        }
#pragma unroll
        for (int i = 1; i < 19; i += 2) {
          const R w = (R)wgt(i);
          const R cu = cdot(i, u);
          const R cF = cdot(i, F);
          const R even = w * rm1 + w * rho * ((R)4.5 * cu * cu - (R)1.5 * usq);
          const R odd = w * rho * (R)3 * cu;
          const R seven = w * ((R)9 * cu * cF - (R)3 * uF);
          const R sodd = w * (R)3 * cF;
          fs[i] = f[i] - (f[i] - (even + odd)) * itau + fsrc * (seven + sodd);
          fs[i + 1] = f[i + 1] - (f[i + 1] - (even - odd)) * itau + fsrc * (seven - sodd);
        }
        // the next plane's populations are requested before this plane's
        // stores (f is dead once fs is formed)
        if (more) fetch_f(k + 1);
        const int dxp = gx + 1 == nx ? 1 - nx : 1, dxm = gx == 0 ? nx - 1 : -1;
        const int dyp = gy + 1 == ny ? nx * (1 - ny) : nx, dym = gy == 0 ? nx * (ny - 1) : -nx;
        const int dzp = gz + 1 == nz ? nxy * (1 - nz) : nxy, dzm = gz == 0 ? nxy * (nz - 1) : -nxy;
        const int dxs[3] = {dxm, 0, dxp}, dys[3] = {dym, 0, dyp}, dzs[3] = {dzm, 0, dzp};
        // rigid-body velocity at this site: on a link of direction c its
        // projection equals that at the link midpoint, c.(w x c/2) = 0
        R ubs[3] = {(R)0, (R)0, (R)0};
        if (NEAR && anys) {
          double r[3], ub[3];
          rel_pos(B, Rc, (double)gx, (double)gy, (double)gz, r);
          rigid_vel(C, r, ub);
#pragma unroll
          for (int c = 0; c < 3; c++) ubs[c] = (R)ub[c];
        }
#pragma unroll
        for (int i = 0; i < 19; i++) {
          if (!NEAR || !sn[i]) {
            const unsigned gn = g + (unsigned)(dxs[cx(i) + 1] + dys[cy(i) + 1] + dzs[cz(i) + 1]);
            bfout.st(i, gn, fs[i]);
          } else {
            // link bounce-back with the moving-wall term; the link passes
            // (2 f_i - corr) c_i to the colloid at r_site + c_i/2, whose
            // torque about the centre is r_site x dp (c_i x c_i = 0)
            const R cub = cdot(i, ubs);
            const R corr = (R)(6.0 * wgt(i)) * (R)B.rho0 * cub;
            bfout.st_nt(opp(i), g, fs[i] - corr);
            const double m = 2.0 * ((double)fs[i] + wgt(i)) - (double)corr;
            if (cx(i)) bbp[0] += cx(i) > 0 ? m : -m;
            if (cy(i)) bbp[1] += cy(i) > 0 ? m : -m;
            if (cz(i)) bbp[2] += cz(i) > 0 ? m : -m;
          }
        }
#pragma unroll
        for (int c = 0; c < 3; c++) buout.st_nt(c, g, u[c]);
      }
      if (NEAR && anys) {
        double r[3];
        rel_pos(B, Rc, (double)gx, (double)gy, (double)gz, r);
        part[0] += bbp[0]; part[1] += bbp[1]; part[2] += bbp[2];
        part[6] += r[1] * bbp[2] - r[2] * bbp[1];
        part[7] += r[2] * bbp[0] - r[0] * bbp[2];
        part[8] += r[0] * bbp[1] - r[1] * bbp[0];
        part[3] += fps[0]; part[4] += fps[1]; part[5] += fps[2];
        part[9] += (r[1] * fps[2] - r[2] * fps[1]) + fts[0];
        part[10] += (r[2] * fps[0] - r[0] * fps[2]) + fts[1];
        part[11] += (r[0] * fps[1] - r[1] * fps[0]) + fts[2];
      }
      if (bad) atomicOr(a.flag, 1);
    };
    if (incol && fluid) {
      if (pnear) update(std::true_type{});
      else update(std::false_type{});
    }
    if (more && !(incol && fluid)) fetch_f(k + 1);
    if (pnear) {
      // wave sums in plane order into the wave's own slots (no barrier);
      // waves without a solid link this plane skip the reduction
      bool any = false;
#pragma unroll
      for (int c = 0; c < 12; c++) any = any || part[c] != 0.0;
      if (__any(any)) {
        const double v = WaveSums<12>::run(part);
        if (WaveSums<12>::writer()) sm.red[gi & 1][wv * 12 + WaveSums<12>::index()] += v;
      }
    }

    // rotate: planes k+3 (Q) and k+2 (u) enter the free slots
    if (more) {
      store_q(rq, qs_free, k + 3);
      if (hydro) store_u(ru, us_free);
    }
    lds_sync();
    if (more && hydro) {
      fix_u(us_free, qs_p2, k + 2);
      if (near) lds_sync();
    }
    const int qf = qs_m1;
    qs_m1 = qs_0; qs_0 = qs_p1; qs_p1 = qs_p2; qs_p2 = qs_free; qs_free = qf;
    const int uf = us_m1;
    us_m1 = us_0; us_0 = us_p1; us_p1 = us_free; us_free = uf;
    ps_0 ^= 1;
#pragma unroll
    for (int c = 0; c < 5; c++) h_cur[c] = h_nxt[c];
#pragma unroll
    for (int c = 0; c < 3; c++) { pz_m[c] = pz_c[c]; pz_c[c] = pz_n[c]; }
  }

  // the last plane's barrier has ordered every wave's sums of the last group
  flush((zend - 1 - z0) / kGroup);
  // far from the colloid every group's sums are zero: write them, so that
  // k_post can add all slots without repeating the geometry test
  if (has && !near && tid < 12)
    for (int g = 0; g < (zend - z0 + kGroup - 1) / kGroup; g++)
      a.part[tid * a.nslot + C.slot_base + cb + (long long)ncb * (g0 + g)] = 0.0;
}

}  // namespace lc
