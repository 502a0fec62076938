// lc_kernels.hip -- gfx950 kernels of the hybrid LB/FD step.
//
//   k_ghost     anchoring: Q at boundary solid nodes (Sec. 2.2, Q^0)
//   k_step      fused per-site pass: H and P from an LDS-staged Q halo,
//               force = discrete divergence of P over control-volume faces,
//               Beris-Edwards update of Q, BGK collision with Guo forcing,
//               push streaming with bounce-back on links, colloid force and
//               torque partial sums (Sec. 2.1-2.2)
//   k_post      after each step: moving-boundary events of a colloid with
//               prescribed motion, the next step's ghost Q, block sums of
//               the colloid force and torque, R += v; its first block per
//               box finishes the previous step (fixed-order sum of the block
//               sums, force history)
//   k_finish    the same finish, launched from the host for the last step
//   k_diag      free energy, mass, momentum, max|u| partials
//   k_defects   (3/2) lambda_max(Q) below a threshold
//
// Populations are stored shifted, f~ = f - w_i, which keeps FP32 rounding
// relative to the small deviations from rest.  Every array is
// structure-of-arrays [component][site] over the concatenation of all boxes.
#include <hip/hip_ext.h>

#include <type_traits>

#include "lc_kernels.hpp"
#include "lc_arch.hpp"
#include "lc_reduce.hpp"
#include "lc_march.hpp"

namespace lc {

// ---------------------------------------------------------------------
// fused step
// ---------------------------------------------------------------------

// Element idx of an array whose byte size fits in 32 bits: the byte offset
// is formed in 32 bits so that the access can use a scalar base address.
template <typename T>
__device__ inline const T* at32(const T* base, unsigned idx) {
  return (const T*)((const char*)base + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ inline T* at32(T* base, unsigned idx) {
  return (T*)((char*)base + idx * (unsigned)sizeof(T));
}

// Block = one TX x TY x TZ tile, one thread per node.  LDS holds Q with a
// halo of two nodes, solid flags, the velocity with a halo of one, the full
// stress P at the tile's nodes and, on the six face layers around the tile,
// only the column of P that the neighbouring face difference uses.
// Site offsets are 32-bit and added to per-component base pointers held in
// scalar registers.  Blocks whose stencils cannot reach the colloid take a
// path without any solid-node test.
// LDS of one block of the fused kernel.
template <typename R, int TX, int TY, int TZ>
struct StepSmem {
  static constexpr int NT = TX * TY * TZ;
  static constexpr int QN = (TX + 4) * (TY + 4) * (TZ + 4);
  static constexpr int PN = (TX + 2) * (TY + 2) * (TZ + 2);
  static constexpr int NF = 2 * (TX * TY + TY * TZ + TX * TZ);
  R Q[5 * QN];            // Q with a halo of two nodes
  R Pi[9 * NT];           // full stress at the tile's nodes
  R Ph[3 * NF];           // one column of the stress on the face layers
  R U[3 * PN];            // velocity with a halo of one node
  unsigned char S[QN];    // solid flags of the Q box
  double red[(NT / 64) * 12];
};

template <typename R, int TX, int TY, int TZ, bool CHIRAL>
__device__ __forceinline__ void step_tile(const BoxDev& B, const int2 tt, const StepPtrs<R>& a,
                                          StepSmem<R, TX, TY, TZ>& sm);

// One launch serves every box of the batch; each block takes the nematic or
// the cholesteric specialisation from its own box, so a box gives the same
// bits whether it runs alone or in a batch.
template <typename R, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX* TY* TZ)
    k_step(const BoxDev* __restrict__ boxes, const int2* __restrict__ tiles, StepPtrs<R> a) {
  const int2 tt = tiles[blockIdx.x];
  if (tt.x < 0) return;  // padding entry (whole block)
  const BoxDev& B = boxes[tt.x];
  __shared__ StepSmem<R, TX, TY, TZ> sm;
  if (B.q0 != 0.0) step_tile<R, TX, TY, TZ, true>(B, tt, a, sm);
  else step_tile<R, TX, TY, TZ, false>(B, tt, a, sm);
}

template <typename R, int TX, int TY, int TZ, bool CHIRAL>
__device__ __forceinline__ void step_tile(const BoxDev& B, const int2 tt, const StepPtrs<R>& a,
                                          StepSmem<R, TX, TY, TZ>& sm) {
  constexpr int NT = TX * TY * TZ;
  constexpr int QX = TX + 4, QY = TY + 4, QZ = TZ + 4, QN = QX * QY * QZ;
  constexpr int PX = TX + 2, PY = TY + 2, PZ = TZ + 2, PN = PX * PY * PZ;
  constexpr int NFZ = TX * TY, NFX = TY * TZ, NFY = TX * TZ, NF = 2 * (NFZ + NFX + NFY);
  constexpr int QSY = QX, QSZ = QX * QY;     // strides in the Q box
  constexpr int PSY = PX, PSZ = PX * PY;     // strides in the velocity box

  R* const sQ = sm.Q;
  R* const sPi = sm.Pi;
  R* const sPh = sm.Ph;
  R* const sU = sm.U;
  unsigned char* const sS = sm.S;
  double* const sred = sm.red;

  const int nx = B.nx, ny = B.ny, nz = B.nz, hydro = B.hydro;
  const int nxy = nx * ny;
  const int tix = tt.y % B.ntx, tiy = (tt.y / B.ntx) % B.nty, tiz = tt.y / (B.ntx * B.nty);
  const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * TZ;
  const unsigned off = (unsigned)B.off;
  const long long NS = a.nsites;
  // colloids that can reach the tile's stencils (bit k: colloid k of the box)
  const unsigned nmask = near_mask(B, a.cols, a.par, x0 - 2, y0 - 2, z0 - 2, TX + 4, TY + 4, TZ + 4);
  const bool near = nmask != 0u;
  // a single conditional correction wraps every halo coordinate
  const bool wide = nx >= TX + 2 && ny >= TY + 2 && nz >= TZ + 2;
  const Mat<R> mp(B);
  const int adv = B.adv;
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
  const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
  const bool inbox = gx < nx && gy < ny && gz < nz;
  const unsigned g = off + (unsigned)(gx + nx * gy + nxy * gz);

  auto wrap3 = [&](int& wx, int& wy, int& wz) {
    if (wide) {
      wx += wx < 0 ? nx : 0; wx -= wx >= nx ? nx : 0;
      wy += wy < 0 ? ny : 0; wy -= wy >= ny ? ny : 0;
      wz += wz < 0 ? nz : 0; wz -= wz >= nz ? nz : 0;
    } else {
      wx = wrapc(wx, nx); wy = wrapc(wy, ny); wz = wrapc(wz, nz);
    }
  };

  // populations of the own node, requested first so that their latency
  // overlaps the stencil phases
  R f[19];
  if (hydro && inbox) {
#pragma unroll
    for (int i = 0; i < 19; i++) f[i] = __builtin_nontemporal_load(at32(a.fin + i * NS, g));
  }

  // Phase 1: Q with a halo of two nodes, velocity with a halo of one.
  for (int s = tid; s < QN; s += NT) {
    const int qz = s / QSZ, rem = s - qz * QSZ, qy = rem / QX, qx = rem - qy * QX;
    int wx = x0 - 2 + qx, wy = y0 - 2 + qy, wz = z0 - 2 + qz;
    wrap3(wx, wy, wz);
    const unsigned gs = off + (unsigned)(wx + nx * wy + nxy * wz);
#pragma unroll
    for (int c = 0; c < 5; c++) sQ[c * QN + s] = *at32(a.Qin + c * NS, gs);
    sS[s] = near ? (unsigned char)solid_id(B, a.cols, nmask, a.par, wx, wy, wz) : (unsigned char)0;
  }
  if (hydro) {
    for (int s = tid; s < PN; s += NT) {
      const int uz = s / PSZ, rem = s - uz * PSZ, uy = rem / PX, ux = rem - uy * PX;
      int wx = x0 - 1 + ux, wy = y0 - 1 + uy, wz = z0 - 1 + uz;
      wrap3(wx, wy, wz);
      const unsigned gs = off + (unsigned)(wx + nx * wy + nxy * wz);
#pragma unroll
      for (int c = 0; c < 3; c++) sU[c * PN + s] = *at32(a.uin + c * NS, gs);
    }
  }
  lds_sync();

  // Phase 2a: own node: H (kept in registers) and the full stress.
  const int qc = (lz + 2) * QSZ + (ly + 2) * QSY + (lx + 2);
  const bool fluid = !sS[qc];
  R h5[5];
  const bool st27 = B.st27 != 0;
  {
    Stencil<R> st;
    if (st27) {
      stencil27(sQ + qc, QN, QSY, QSZ, st);
    } else {
      R c5[5], xp[5], xm[5], yp[5], ym[5], zp[5], zm[5];
#pragma unroll
      for (int c = 0; c < 5; c++) {
        const R* q = sQ + c * QN + qc;
        c5[c] = q[0]; xp[c] = q[1]; xm[c] = q[-1]; yp[c] = q[QSY]; ym[c] = q[-QSY];
        zp[c] = q[QSZ]; zm[c] = q[-QSZ];
      }
      stencil5(c5, xp, xm, yp, ym, zp, zm, st);
    }
    R q[3][3], q2[3][3], tr2, M[3][3], h[3][3];
    mol_field<R, CHIRAL>(mp, st, q, q2, tr2, M, h);
    h5[0] = h[0][0]; h5[1] = h[0][1]; h5[2] = h[0][2]; h5[3] = h[1][1]; h5[4] = h[1][2];
    if (hydro && fluid) {
      const R fe = energy_density<R, CHIRAL>(mp, st, q, q2, tr2, M);
      R col[3][3];
      stress_col<R, CHIRAL, 0>(mp, st, q, h, fe, col[0]);
      stress_col<R, CHIRAL, 1>(mp, st, q, h, fe, col[1]);
      stress_col<R, CHIRAL, 2>(mp, st, q, h, fe, col[2]);
#pragma unroll
      for (int b = 0; b < 3; b++)
#pragma unroll
        for (int c = 0; c < 3; c++) sPi[(3 * c + b) * NT + tid] = col[b][c];
    }
  }
  // Phase 2b: face layers: the one column of P each needs.
  if (hydro) {
    for (int hsite = tid; hsite < NF; hsite += NT) {
      int px, py, pz, b;
      int hh = hsite;
      if (hh < 2 * NFZ) {
        const int r = hh % NFZ;
        px = r % TX + 1; py = r / TX + 1; pz = hh < NFZ ? 0 : PZ - 1; b = 2;
      } else if ((hh -= 2 * NFZ) < 2 * NFX) {
        const int r = hh % NFX;
        py = r % TY + 1; pz = r / TY + 1; px = hh < NFX ? 0 : PX - 1; b = 0;
      } else {
        hh -= 2 * NFX;
        const int r = hh % NFY;
        px = r % TX + 1; pz = r / TX + 1; py = hh < NFY ? 0 : PY - 1; b = 1;
      }
      const int qh = (pz + 1) * QSZ + (py + 1) * QSY + (px + 1);
      if (near && sS[qh]) continue;
      Stencil<R> st;
      if (st27) {
        stencil27(sQ + qh, QN, QSY, QSZ, st);
      } else {
        R c5[5], xp[5], xm[5], yp[5], ym[5], zp[5], zm[5];
#pragma unroll
        for (int c = 0; c < 5; c++) {
          const R* q = sQ + c * QN + qh;
          c5[c] = q[0]; xp[c] = q[1]; xm[c] = q[-1]; yp[c] = q[QSY]; ym[c] = q[-QSY];
          zp[c] = q[QSZ]; zm[c] = q[-QSZ];
        }
        stencil5(c5, xp, xm, yp, ym, zp, zm, st);
      }
      R q[3][3], q2[3][3], tr2, M[3][3], h[3][3];
      mol_field<R, CHIRAL>(mp, st, q, q2, tr2, M, h);
      const R fe = energy_density<R, CHIRAL>(mp, st, q, q2, tr2, M);
      R col[3];
      if (b == 0) stress_col<R, CHIRAL, 0>(mp, st, q, h, fe, col);
      else if (b == 1) stress_col<R, CHIRAL, 1>(mp, st, q, h, fe, col);
      else stress_col<R, CHIRAL, 2>(mp, st, q, h, fe, col);
#pragma unroll
      for (int c = 0; c < 3; c++) sPh[c * NF + hsite] = col[c];
    }
    // rigid-body velocity at solid nodes of the velocity box
    if (near) {
      for (int s = tid; s < PN; s += NT) {
        const int uz = s / PSZ, rem = s - uz * PSZ, uy = rem / PX, ux = rem - uy * PX;
        const int id = sS[(uz + 1) * QSZ + (uy + 1) * QSY + (ux + 1)];
        if (!id) continue;
        int wx = x0 - 1 + ux, wy = y0 - 1 + uy, wz = z0 - 1 + uz;
        wrap3(wx, wy, wz);
        const ColDev& C = a.cols[B.col0 + id - 1];
        double r[3], ub[3];
        rel_pos(B, C.pos[a.par], (double)wx, (double)wy, (double)wz, r);
        rigid_vel(C, r, ub);
#pragma unroll
        for (int c = 0; c < 3; c++) sU[c * PN + s] = (R)ub[c];
      }
    }
  }
  lds_sync();

  // Phase 3: own node.
  const int pc = (lz + 1) * PSZ + (ly + 1) * PSY + (lx + 1);
  double part[12];
#pragma unroll
  for (int k = 0; k < 12; k++) part[k] = 0.0;
  int own = 0;   // 1 + colloid of this site's solid links (one by the separation of colloids)

  auto update = [&](auto near_tag) {
    constexpr bool NEAR = decltype(near_tag)::value;
    const int qst[3] = {1, QSY, QSZ}, pst[3] = {1, PSY, PSZ};
    R q5[5], dQ[5];
#pragma unroll
    for (int c = 0; c < 5; c++) {
      q5[c] = sQ[c * QN + qc];
      dQ[c] = mp.Gamma * h5[c];
    }
    R F[3] = {(R)0, (R)0, (R)0};
    bool solid_nb[19];
#pragma unroll
    for (int i = 0; i < 19; i++) {
      const int id = NEAR ? (int)sS[qc + cx(i) + cy(i) * QSY + cz(i) * QSZ] : 0;
      solid_nb[i] = id != 0;
      own = id > own ? id : own;
    }
    // solid-link sums of this site: stress-face force and its torque about
    // r_site, bounce-back momentum
    double fps[3] = {0.0, 0.0, 0.0}, fts[3] = {0.0, 0.0, 0.0}, bbp[3] = {0.0, 0.0, 0.0};
    bool anys = false;
    if (NEAR) {
#pragma unroll
      for (int i = 1; i < 19; i++) anys = anys || solid_nb[i];
    }
    if (hydro) {
      // force on the fluid: differences of P between opposite faces
      const int loc[3] = {lx, ly, lz}, ext[3] = {TX, TY, TZ}, ist[3] = {1, TX, TX * TY};
      // face-layer index of the neighbour across the + and - faces
      const int hp[3] = {2 * NFZ + NFX + ly + lz * TY, 2 * NFZ + 2 * NFX + NFY + lx + lz * TX, NFZ + lx + ly * TX};
      const int hm[3] = {2 * NFZ + ly + lz * TY, 2 * NFZ + 2 * NFX + lx + lz * TX, lx + ly * TX};
#pragma unroll
      for (int b = 0; b < 3; b++) {
        const bool sp = solid_nb[2 * b + 1], sm = solid_nb[2 * b + 2];
        const bool ip = loc[b] + 1 < ext[b], im = loc[b] > 0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
          const R pcv = sPi[(3 * c + b) * NT + tid];
          const R pn = ip ? sPi[(3 * c + b) * NT + tid + ist[b]] : sPh[c * NF + hp[b]];
          const R pmv = im ? sPi[(3 * c + b) * NT + tid - ist[b]] : sPh[c * NF + hm[b]];
          const R pp = sp ? pcv : (R)0.5 * (pcv + pn);
          const R pm = sm ? pcv : (R)0.5 * (pcv + pmv);
          F[c] += pp - pm;
        }
        // colloid force and torque from the solid-fluid faces: a face with
        // sign sg passes -sg P[:,b] at r_site + (sg/2) x_b, whose torque
        // about the centre is r_site x ps - (1/2) x_b x P[:,b]
        if (NEAR && (sp || sm)) {
          const double nsg = (sp ? 1.0 : 0.0) - (sm ? 1.0 : 0.0);
          const double hc = 0.5 * ((sp ? 1.0 : 0.0) + (sm ? 1.0 : 0.0));
          const double p0 = (double)sPi[(3 * 0 + b) * NT + tid], p1 = (double)sPi[(3 * 1 + b) * NT + tid],
                       p2 = (double)sPi[(3 * 2 + b) * NT + tid];
          fps[0] -= nsg * p0; fps[1] -= nsg * p1; fps[2] -= nsg * p2;
          if (b == 0) { fts[1] += hc * p2; fts[2] -= hc * p1; }
          else if (b == 1) { fts[0] -= hc * p2; fts[2] += hc * p0; }
          else { fts[0] += hc * p1; fts[1] -= hc * p0; }
        }
      }
#pragma unroll
      for (int c = 0; c < 3; c++) F[c] += (R)B.body[c];

      // Beris-Edwards: velocity gradient, upwind advective fluxes with zero
      // flux through solid faces, co-rotation
      R u0[3], W[3][3];
#pragma unroll
      for (int c = 0; c < 3; c++) u0[c] = sU[c * PN + pc];
#pragma unroll
      for (int b = 0; b < 3; b++) {
        R up[3], um[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
          up[c] = sU[c * PN + pc + pst[b]];
          um[c] = sU[c * PN + pc - pst[b]];
          W[c][b] = (R)0.5 * (up[c] - um[c]);
        }
        const bool fp = !solid_nb[2 * b + 1], fm = !solid_nb[2 * b + 2];
        const R ufp = (R)0.5 * (u0[b] + up[b]), ufm = (R)0.5 * (um[b] + u0[b]);
        if (adv == 1) {
#pragma unroll
          for (int c = 0; c < 5; c++) {
            const R phip = fp ? ufp * (ufp >= (R)0 ? q5[c] : sQ[c * QN + qc + qst[b]]) : (R)0;
            const R phim = fm ? ufm * (ufm >= (R)0 ? sQ[c * QN + qc - qst[b]] : q5[c]) : (R)0;
            dQ[c] -= phip - phim;
          }
        } else {
          // higher-order upwind face values; a face whose wider stencil
          // reaches a solid node takes the first-order value
          const int st = qst[b];
          auto face = [&](int lo, R uf, bool open, R phi[5]) {
            const int up = uf >= (R)0 ? lo : lo + st, dn = uf >= (R)0 ? lo + st : lo;
            const int upup = uf >= (R)0 ? lo - st : lo + 2 * st;
            const bool wide = !(NEAR && sS[upup]);
#pragma unroll
            for (int c = 0; c < 5; c++) {
              const R qu = sQ[c * QN + up];
              R qf = qu;
              if (wide) {
                const R quu = sQ[c * QN + upup];
                qf = adv == 2 ? ((R)3 * qu - quu) / (R)2 : ((R)2 * sQ[c * QN + dn] + (R)5 * qu - quu) / (R)6;
              }
              phi[c] = open ? uf * qf : (R)0;
            }
          };
          R phip[5], phim[5];
          face(qc, ufp, fp, phip);
          face(qc - st, ufm, fm, phim);
#pragma unroll
          for (int c = 0; c < 5; c++) dQ[c] -= phip[c] - phim[c];
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
      __builtin_nontemporal_store(v, at32(a.Qout + c * NS, g));
      qn2 += v * v;
    }
    bool bad = !(qn2 < (R)100);

    if (hydro) {
      // LB collision (BGK, Guo forcing with the half-force velocity); f holds
      // f - w_i, so rho = 1 + sum and sum(w_i c_i) = 0
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
        // the pair (i, i+1) has opposite velocities: shared even parts
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
      // push streaming: 32-bit offsets of the 26 neighbours
      const int dxp = gx + 1 == nx ? 1 - nx : 1, dxm = gx == 0 ? nx - 1 : -1;
      const int dyp = gy + 1 == ny ? nx * (1 - ny) : nx, dym = gy == 0 ? nx * (ny - 1) : -nx;
      const int dzp = gz + 1 == nz ? nxy * (1 - nz) : nxy, dzm = gz == 0 ? nxy * (nz - 1) : -nxy;
      const int dxs[3] = {dxm, 0, dxp}, dys[3] = {dym, 0, dyp}, dzs[3] = {dzm, 0, dzp};
      // rigid-body velocity at this site: on a link of direction c its
      // projection equals that at the link midpoint, c.(w x c/2) = 0
      R ubs[3] = {(R)0, (R)0, (R)0};
      if (NEAR && anys) {
        const ColDev& C = a.cols[B.col0 + own - 1];
        double r[3], ub[3];
        rel_pos(B, C.pos[a.par], (double)gx, (double)gy, (double)gz, r);
        rigid_vel(C, r, ub);
#pragma unroll
        for (int c = 0; c < 3; c++) ubs[c] = (R)ub[c];
      }
#pragma unroll
      for (int i = 0; i < 19; i++) {
        if (!NEAR || !solid_nb[i]) {
          const unsigned gn = g + (unsigned)(dxs[cx(i) + 1] + dys[cy(i) + 1] + dzs[cz(i) + 1]);
          *at32(a.fout + i * NS, gn) = fs[i];
        } else {
          // bounce-back on the link with the moving-wall correction; the
          // link passes (2 f_i - corr) c_i to the colloid at r_site + c_i/2,
          // whose torque about the centre is r_site x dp (c_i x c_i = 0)
          const R cub = cdot(i, ubs);
          const R corr = (R)(6.0 * wgt(i)) * (R)B.rho0 * cub;
          __builtin_nontemporal_store(fs[i] - corr, at32(a.fout + opp(i) * NS, g));
          const double m = 2.0 * ((double)fs[i] + wgt(i)) - (double)corr;
          if (cx(i)) bbp[0] += cx(i) > 0 ? m : -m;
          if (cy(i)) bbp[1] += cy(i) > 0 ? m : -m;
          if (cz(i)) bbp[2] += cz(i) > 0 ? m : -m;
        }
      }
#pragma unroll
      for (int c = 0; c < 3; c++) __builtin_nontemporal_store(u[c], at32(a.uout + c * NS, g));
    }
    if (NEAR && anys) {
      double r[3];
      rel_pos(B, a.cols[B.col0 + own - 1].pos[a.par], (double)gx, (double)gy, (double)gz, r);
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

  if (inbox && fluid) {
    if (near) update(std::true_type{});
    else update(std::false_type{});
  }

  // one slot per colloid of the box, every slot written each step (zeros
  // for colloids out of reach); a site's sums belong to its links' colloid
  for (int k = 0; k < B.ncol; k++) {
    double* out = a.part + a.cols[B.col0 + k].slot_base + tt.y;
    if ((nmask >> k) & 1u) {
      const bool mine = own == k + 1;
      double red[12];
#pragma unroll
      for (int c = 0; c < 12; c++) red[c] = mine ? part[c] : 0.0;
      block_sum<NT, 12>(red, sred, out, a.nslot);
      __syncthreads();   // sred serves the next colloid's sum
    } else if (tid < 12) {
      out[tid * a.nslot] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------
// ghost Q at boundary solid nodes
// ---------------------------------------------------------------------
template <typename R>
__device__ inline void load_full(const R* Q, long long NS, long long g, double q[3][3]) {
  const double xx = Q[g], xy = Q[NS + g], xz = Q[2 * NS + g], yy = Q[3 * NS + g], yz = Q[4 * NS + g];
  q[0][0] = xx; q[0][1] = xy; q[0][2] = xz;
  q[1][0] = xy; q[1][1] = yy; q[1][2] = yz;
  q[2][0] = xz; q[2][1] = yz; q[2][2] = -xx - yy;
}

__device__ inline long long site_of(const BoxDev& B, int x, int y, int z) {
  return B.off + x + (long long)B.nx * (y + (long long)B.ny * z);
}

// Q given to a node that the move Rold -> Rnew uncovers: the mean over its
// face neighbours that are fluid before and after the move, rounded to the
// storage precision.
template <typename R>
__device__ inline void exposed_q(const BoxDev& B, const ColDev& C, const double Rold[3], const double Rnew[3], int x,
                                 int y, int z, const R* Q, long long NS, double q5[5]) {
  const int nb[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  double qm[5] = {0, 0, 0, 0, 0};
  int nf = 0;
  for (int k = 0; k < 6; k++) {
    const int xn = wrapc(x + nb[k][0], B.nx), yn = wrapc(y + nb[k][1], B.ny), zn = wrapc(z + nb[k][2], B.nz);
    if (inside(B, C, Rold, xn, yn, zn) || inside(B, C, Rnew, xn, yn, zn)) continue;
    const long long gn = site_of(B, xn, yn, zn);
    for (int c = 0; c < 5; c++) qm[c] += (double)Q[c * NS + gn];
    nf++;
  }
  for (int c = 0; c < 5; c++) q5[c] = (double)(R)(nf ? qm[c] / nf : 0.0);
}

template <typename R>
__device__ inline void ghost_finish(const BoxDev& B, const ColDev& C, const double Rc[3], int x, int y, int z,
                                    double (&qbar)[3][3], int nf, R* __restrict__ Q, long long NS);

// Anchoring at node (x, y, z) for colloid C at Rc: if the node is solid
// with at least one fluid face neighbour, Q there becomes Q^0 (or its blend
// with the neighbours' mean for finite W).  When the colloid has just moved
// from Rold, neighbours it uncovered get their Q in this same pass, so their
// value is formed here by the same rule instead of being read.  Other
// colloids of the box stay out of reach (their surfaces are at least
// kColloidGap away), so only C is tested.
template <typename R>
__device__ inline void ghost_site(const BoxDev& B, const ColDev& C, const double Rold[3], const double Rc[3],
                                  bool moved, int x, int y, int z, R* __restrict__ Q, long long NS) {
  if (!inside(B, C, Rc, x, y, z)) return;
  double qbar[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  int nf = 0;
  if (B.st27) {
    // 27-point stencil: every solid node with a fluid node among its 26
    // neighbours, Qbar the mean of those (z, y, x order)
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          if (!(dx || dy || dz)) continue;
          const int xn = wrapc(x + dx, B.nx), yn = wrapc(y + dy, B.ny), zn = wrapc(z + dz, B.nz);
          if (inside(B, C, Rc, xn, yn, zn)) continue;
          double qq[3][3];
          if (moved && inside(B, C, Rold, xn, yn, zn)) {
            double q5[5];
            exposed_q<R>(B, C, Rold, Rc, xn, yn, zn, Q, NS, q5);
            qq[0][0] = q5[0]; qq[0][1] = q5[1]; qq[0][2] = q5[2];
            qq[1][0] = q5[1]; qq[1][1] = q5[3]; qq[1][2] = q5[4];
            qq[2][0] = q5[2]; qq[2][1] = q5[4]; qq[2][2] = -q5[0] - q5[3];
          } else {
            load_full(Q, NS, site_of(B, xn, yn, zn), qq);
          }
          for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) qbar[i][j] += qq[i][j];
          nf++;
        }
    ghost_finish<R>(B, C, Rc, x, y, z, qbar, nf, Q, NS);
    return;
  }
  const int nb[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  // all six neighbours are read at once (the loads overlap), then the fluid
  // ones are added in neighbour order
  double qn[6][3][3];
  bool fl[6];
#pragma unroll
  for (int k = 0; k < 6; k++) {
    const int xn = wrapc(x + nb[k][0], B.nx), yn = wrapc(y + nb[k][1], B.ny), zn = wrapc(z + nb[k][2], B.nz);
    load_full(Q, NS, site_of(B, xn, yn, zn), qn[k]);
    fl[k] = !inside(B, C, Rc, xn, yn, zn);
  }
  if (moved) {
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const int xn = wrapc(x + nb[k][0], B.nx), yn = wrapc(y + nb[k][1], B.ny), zn = wrapc(z + nb[k][2], B.nz);
      if (!fl[k] || !inside(B, C, Rold, xn, yn, zn)) continue;
      double q5[5];
      exposed_q<R>(B, C, Rold, Rc, xn, yn, zn, Q, NS, q5);
      qn[k][0][0] = q5[0]; qn[k][0][1] = q5[1]; qn[k][0][2] = q5[2];
      qn[k][1][0] = q5[1]; qn[k][1][1] = q5[3]; qn[k][1][2] = q5[4];
      qn[k][2][0] = q5[2]; qn[k][2][1] = q5[4]; qn[k][2][2] = -q5[0] - q5[3];
    }
  }
#pragma unroll
  for (int k = 0; k < 6; k++) {
    if (!fl[k]) continue;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) qbar[i][j] += qn[k][i][j];
    nf++;
  }
  ghost_finish<R>(B, C, Rc, x, y, z, qbar, nf, Q, NS);
}

// Ghost Q of a solid node from the sum qbar of its nf fluid neighbours:
// nothing for an interior node (nf = 0), else Q^0 (fixed anchoring), its
// blend with the neighbours' mean (finite W) or the mean (no anchoring).
template <typename R>
__device__ inline void ghost_finish(const BoxDev& B, const ColDev& C, const double Rc[3], int x, int y, int z,
                                    double (&qbar)[3][3], int nf, R* __restrict__ Q, long long NS) {
  if (nf == 0) return;  // interior solid node
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) qbar[i][j] /= nf;
  double qs[3][3];
  if (C.anchoring == 0) {
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) qs[i][j] = qbar[i][j];
  } else {
    double q0[3][3];
    anchor_target(B, C, Rc, x, y, z, qbar, q0);
    const bool fixed = isinf(C.W);
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        qs[i][j] = fixed ? q0[i][j] : (B.K * qbar[i][j] + C.W * q0[i][j]) / (B.K + C.W);
  }
  const long long g = site_of(B, x, y, z);
  Q[g] = (R)qs[0][0]; Q[NS + g] = (R)qs[0][1]; Q[2 * NS + g] = (R)qs[0][2];
  Q[3 * NS + g] = (R)qs[1][1]; Q[4 * NS + g] = (R)qs[1][2];
}

// Node l of the cube of edge E centred on floor(R), wrapped into the box.
__device__ inline void cube_site(const BoxDev& B, const double R[3], int E, long long l, int& x, int& y, int& z) {
  const int h = (E - 1) / 2;
  x = wrapc((int)floor(R[0]) - h + (int)(l % E), B.nx);
  y = wrapc((int)floor(R[1]) - h + (int)((l / E) % E), B.ny);
  z = wrapc((int)floor(R[2]) - h + (int)(l / ((long long)E * E)), B.nz);
}

// Stand-alone anchoring pass over one Q buffer (colloids at their current
// positions): one thread per ghost candidate of every colloid.
template <typename R>
__global__ void __launch_bounds__(256)
    k_ghost(const BoxDev* __restrict__ boxes, const ColDev* __restrict__ cols, int ncol, long long total,
            R* __restrict__ Q, long long NS, int par) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int k = 0;
  for (int j = 1; j < ncol; j++)
    if (t >= cols[j].ghost_base) k = j;
  const ColDev& C = cols[k];
  const BoxDev& B = boxes[C.box];
  const int E = C.ghost_ext;
  const long long l = t - C.ghost_base;
  if (l >= (long long)E * E * E) return;
  const double Rc[3] = {C.pos[par][0], C.pos[par][1], C.pos[par][2]};
  int x, y, z;
  cube_site(B, Rc, E, l, x, y, z);
  ghost_site<R>(B, C, Rc, Rc, false, x, y, z, Q, NS);
}

// ---------------------------------------------------------------------
// moving-boundary events (prescribed motion)
// ---------------------------------------------------------------------
__device__ inline void advanced_pos(const BoxDev& B, const ColDev& C, int par, double Rn[3]) {
  const int L[3] = {B.nx, B.ny, B.nz};
  for (int c = 0; c < 3; c++) {
    double r = __dadd_rn(C.pos[par][c], C.vel[c]);
    if (r >= L[c]) r = __dsub_rn(r, (double)L[c]);
    if (r < 0.0) r = __dadd_rn(r, (double)L[c]);
    Rn[c] = r;
  }
}

// Node (x, y, z) when colloid C moves Rc -> Rn: a node it uncovers gets
// fluid at rest in the wall frame and Q from its face neighbours; a node it
// covers gives its fluid momentum to the colloid.  p and the torque about
// Rn go to v[0..2] and v[6..8].  Other colloids are out of reach (gap).
template <typename R>
__device__ inline void event_site(const BoxDev& B, const ColDev& C, const double Rc[3], const double Rn[3], int x,
                                  int y, int z, const StepPtrs<R>& a, double v[12]) {
  const bool was = inside(B, C, Rc, x, y, z), now = inside(B, C, Rn, x, y, z);
  if (was == now) return;
  const long long NS = a.nsites;
  const long long g = site_of(B, x, y, z);
  double r[3], p[3] = {0, 0, 0};
  rel_pos(B, Rn, (double)x, (double)y, (double)z, r);
  if (was) {
    double ub[3];
    rigid_vel(C, r, ub);
    if (B.hydro) {
      const double usq = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
#pragma unroll
      for (int i = 0; i < 19; i++) {
        const double cu = cx(i) * ub[0] + cy(i) * ub[1] + cz(i) * ub[2];
        const double feq = wgt(i) * B.rho0 * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
        a.fout[i * NS + g] = (R)(feq - wgt(i));
        p[0] -= feq * cx(i); p[1] -= feq * cy(i); p[2] -= feq * cz(i);
      }
      for (int c = 0; c < 3; c++) a.uout[c * NS + g] = (R)ub[c];
    }
    double q5[5];
    exposed_q<R>(B, C, Rc, Rn, x, y, z, a.Qout, NS, q5);
    for (int c = 0; c < 5; c++) a.Qout[c * NS + g] = (R)q5[c];
  } else if (B.hydro) {
#pragma unroll
    for (int i = 0; i < 19; i++) {
      const double fi = (double)a.fout[i * NS + g] + wgt(i);
      p[0] += fi * cx(i); p[1] += fi * cy(i); p[2] += fi * cz(i);
    }
  }
  v[0] += p[0]; v[1] += p[1]; v[2] += p[2];
  v[6] += r[1] * p[2] - r[2] * p[1];
  v[7] += r[2] * p[0] - r[0] * p[2];
  v[8] += r[0] * p[1] - r[1] * p[0];
}

// ---------------------------------------------------------------------
// post-step: events, next step's ghost Q, colloid sums, history, R += v
// ---------------------------------------------------------------------
// Force, torque and history entry of one finished step of colloid g (table
// index): the block vectors of its post-step kernel added in block order
// (nt threads).  Every load (block vectors, step count, the pending flag
// when one is given) is issued before the first sum, so the finish costs one
// memory round trip; each thread still adds its vectors in increasing block
// order.  With a flag that reads zero nothing is written.
template <int NT>
__device__ inline void finish_colloid(ColDev& C, int g, const double* __restrict__ bpart,
                                      const double* __restrict__ fsum, double* __restrict__ force,
                                      double* __restrict__ hist, int cap, long long* __restrict__ count, double* sred,
                                      double* sres, const int* __restrict__ pend = nullptr) {
  constexpr int KB = 4;   // block vectors in flight per thread
  const bool go = pend == nullptr || *pend != 0;
  const long long n = count[g];
  const int nblk = C.post_nblk;
  const double* p0 = bpart + 12LL * C.post_blk0;
  double w[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k0 = 0; k0 < nblk; k0 += KB * NT) {
    double t[KB][12];
#pragma unroll
    for (int j = 0; j < KB; j++) {
      const int k = k0 + j * NT + (int)threadIdx.x;
      const double* p = p0 + 12LL * (k < nblk ? k : 0);
#pragma unroll
      for (int c = 0; c < 12; c++) t[j][c] = p[c];
    }
#pragma unroll
    for (int j = 0; j < KB; j++)
      if (k0 + j * NT + (int)threadIdx.x < nblk)
#pragma unroll
        for (int c = 0; c < 12; c++) w[c] += t[j][c];
  }
  block_sum<NT, 12>(w, sred, sres);
  __syncthreads();
  if (!go) return;
  // a free colloid: the link and stress sums were added before the move
  // (k_free); the block vectors hold the events' momentum, which also goes
  // to its velocity
  const bool free_motion = C.motion == 2;
  if (threadIdx.x < 12) {
    const double val = free_motion ? fsum[12 * g + threadIdx.x] + sres[threadIdx.x] : sres[threadIdx.x];
    force[12 * g + threadIdx.x] = val;
    hist[((long long)g * cap + (n % cap)) * 12 + threadIdx.x] = val;
  }
  if (threadIdx.x == 0) {
    if (free_motion)
      for (int k = 0; k < 3; k++) {
        C.vel[k] += sres[k] / C.mass;
        C.omega[k] += sres[6 + k] / C.inertia;
      }
    count[g] = n + 1;
  }
}

// Free colloids, one block per colloid of the table, after the fused
// kernel: the step's link and stress sums (all its slots, fixed order) into
// fsum, then vel += (F_bbl + F_stress + fext)/M, omega += (T_bbl + T_stress)/I
// and the next position pos[par ^ 1] = pos[par] + vel.
__global__ void __launch_bounds__(kFinishBlock)
    k_free(const BoxDev* __restrict__ boxes, ColDev* __restrict__ cols, const double* __restrict__ part,
           long long nslot, int par, double* __restrict__ fsum) {
  __shared__ double sred[(kFinishBlock / 64) * 12];
  __shared__ double sres[12];
  const int g = blockIdx.x;
  ColDev& C = cols[g];
  if (C.motion != 2) return;
  const BoxDev& B = boxes[C.box];
  const long long nt = (long long)B.ntx * B.nty * B.ntz;
  double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // two slots per thread in flight (more would spill at 1024 threads),
  // added in increasing slot order
  constexpr int KS = 2;
  for (long long k0 = 0; k0 < nt; k0 += KS * kFinishBlock) {
    double t[KS][12];
#pragma unroll
    for (int j = 0; j < KS; j++) {
      const long long k = k0 + j * kFinishBlock + threadIdx.x;
      const double* p = part + C.slot_base + (k < nt ? k : 0);
#pragma unroll
      for (int c = 0; c < 12; c++) t[j][c] = p[c * nslot];
    }
#pragma unroll
    for (int j = 0; j < KS; j++)
      if (k0 + j * kFinishBlock + threadIdx.x < nt)
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] += t[j][c];
  }
  block_sum<kFinishBlock, 12>(v, sred, sres);
  __syncthreads();
  if (threadIdx.x < 12) fsum[12 * g + threadIdx.x] = sres[threadIdx.x];
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; k++) {
      C.vel[k] += (sres[k] + sres[3 + k] + C.fext[k]) / C.mass;
      C.omega[k] += (sres[6 + k] + sres[9 + k]) / C.inertia;
    }
    double Rn[3];
    advanced_pos(B, C, par, Rn);
    C.pos[par ^ 1][0] = Rn[0]; C.pos[par ^ 1][1] = Rn[1]; C.pos[par ^ 1][2] = Rn[2];
  }
}

// Threads of colloid g, in three ranges: fused-kernel slot sums (kPostSlots
// consecutive slots each; every slot was written this step, zeros where the
// colloid is out of reach, so all are added), then one thread per event
// candidate, then one per ghost candidate.  Each thread has one role, so
// the roles' memory latencies overlap.  Each block adds its threads'
// 12-vectors (slot sums and event momenta) in thread order into its slot of
// this step's half of bpart.  The last block of a colloid has no such role:
// it finishes the previous step of the colloid if that is still pending
// (adding the previous half's block vectors in block order) while the
// others work, checks that the colloid started this step at least
// kColloidGap (surface to surface) from the box's other colloids, writes
// the next position and marks this step pending; the post-step kernel of the
// next step (or k_finish, from the host) finishes it.
template <typename R>
__global__ void __launch_bounds__(kPostBlock)
    k_post(const BoxDev* __restrict__ boxes, const int* __restrict__ owner, StepPtrs<R> a, double* __restrict__ bpart,
           int* __restrict__ pending, const double* __restrict__ fsum, double* __restrict__ force,
           double* __restrict__ hist, int cap, long long* __restrict__ count, int nblk_all) {
  __shared__ double sred[(kPostBlock / 64) * 12];
  __shared__ double sres[12];
  const int g = owner[blockIdx.x];   // the colloid this block serves
  ColDev& C = a.cols[g];
  const BoxDev& B = boxes[C.box];
  const int par = a.par;
  const bool finisher = (int)blockIdx.x == C.post_blk0 + C.post_nblk - 1;
  // the positions first: the finish below changes only a free colloid's
  // velocity, which the next position (already formed by k_free) does not use
  const double Rc[3] = {C.pos[par][0], C.pos[par][1], C.pos[par][2]};
  const bool free_motion = C.motion == 2;
  const bool moving = C.motion != 0;
  double Rn[3] = {Rc[0], Rc[1], Rc[2]};
  if (free_motion) {
    // k_free has moved it already
    Rn[0] = C.pos[par ^ 1][0]; Rn[1] = C.pos[par ^ 1][1]; Rn[2] = C.pos[par ^ 1][2];
  } else if (moving) {
    advanced_pos(B, C, par, Rn);
  }
  if (finisher) {
    finish_colloid<kPostBlock>(C, g, bpart + 12LL * nblk_all * (par ^ 1), fsum, force, hist, cap, count, sred, sres,
                               pending + g);
    __syncthreads();
  }
  long long l = (long long)((int)blockIdx.x - C.post_blk0) * kPostBlock + threadIdx.x;
  double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  {
    const long long nt = (long long)B.ntx * B.nty * B.ntz;
    const long long nst = free_motion ? 0 : (nt + kPostSlots - 1) / kPostSlots;
    const long long ne = moving ? (long long)C.event_ext * C.event_ext * C.event_ext : 0;
    const long long ng = (long long)C.ghost_ext * C.ghost_ext * C.ghost_ext;
    if (l < nst) {
      const long long k0 = l * kPostSlots;
      double t[kPostSlots][12];
#pragma unroll
      for (int j = 0; j < kPostSlots; j++) {
        const bool ok = k0 + j < nt;
        const double* p = a.part + C.slot_base + (ok ? k0 + j : 0);
#pragma unroll
        for (int c = 0; c < 12; c++) t[j][c] = ok ? p[c * a.nslot] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kPostSlots; j++)
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] += t[j][c];
    } else {
      l -= nst;
      int x, y, z;
      if (l < ne) {
        cube_site(B, Rc, C.event_ext, l, x, y, z);
        event_site<R>(B, C, Rc, Rn, x, y, z, a, v);
      } else if (l - ne < ng) {
        cube_site(B, Rn, C.ghost_ext, l - ne, x, y, z);
        ghost_site<R>(B, C, Rc, Rn, moving, x, y, z, a.Qout, a.nsites);
      }
    }
  }
  block_sum<kPostBlock, 12>(v, sred, bpart + 12LL * nblk_all * par + 12LL * blockIdx.x);
  if (finisher && threadIdx.x == 0) {
    for (int k = 0; k < B.ncol; k++) {
      const ColDev& D = a.cols[B.col0 + k];
      if (B.col0 + k == g) continue;
      double r[3];
      rel_pos(B, Rc, D.pos[par][0], D.pos[par][1], D.pos[par][2], r);
      if (sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) < C.a0 + D.a0 + kColloidGap) atomicOr(a.flag, 2);
    }
    C.pos[par ^ 1][0] = Rn[0]; C.pos[par ^ 1][1] = Rn[1]; C.pos[par ^ 1][2] = Rn[2];
    pending[g] = 1;
  }
}

// One block per colloid: finishes the pending step of buffer parity par.
__global__ void __launch_bounds__(kFinishBlock)
    k_finish(ColDev* __restrict__ cols, int par, int nblk_all, const double* __restrict__ bpart,
             int* __restrict__ pending, const double* __restrict__ fsum, double* __restrict__ force,
             double* __restrict__ hist, int cap, long long* __restrict__ count) {
  __shared__ double sred[(kFinishBlock / 64) * 12];
  __shared__ double sres[12];
  const int g = blockIdx.x;
  if (!pending[g]) return;
  finish_colloid<kFinishBlock>(cols[g], g, bpart + 12LL * nblk_all * par, fsum, force, hist, cap, count, sred, sres);
  if (threadIdx.x == 0) pending[g] = 0;
}

// ---------------------------------------------------------------------
// diagnostics and defects (off the time loop)
// ---------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256)
    k_diag(const BoxDev* __restrict__ boxes, int box, StepPtrs<R> a, double* out) {
  __shared__ double sred[4 * 6];
  const BoxDev& B = boxes[box];
  const long long NS = a.nsites;
  const long long nsite = (long long)B.nx * B.ny * B.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};
  if (t < nsite) {
    const int x = (int)(t % B.nx), y = (int)((t / B.nx) % B.ny), z = (int)(t / ((long long)B.nx * B.ny));
    const unsigned all = B.ncol >= 32 ? ~0u : (1u << B.ncol) - 1u;
    // 1 + the colloid holding the node, 0 for fluid
    auto sid = [&](int xx, int yy, int zz) {
      return solid_id(B, a.cols, all, a.par, wrapc(xx, B.nx), wrapc(yy, B.ny), wrapc(zz, B.nz));
    };
    auto solid = [&](int xx, int yy, int zz) { return sid(xx, yy, zz) != 0; };
    auto gidx = [&](int xx, int yy, int zz) {
      return B.off + wrapc(xx, B.nx) + (long long)B.nx * (wrapc(yy, B.ny) + (long long)B.ny * wrapc(zz, B.nz));
    };
    const bool sx = solid(x, y, z);
    const long long g = gidx(x, y, z);
    double q[3][3];
    load_full(a.Qin, NS, g, q);
    const double A0 = B.A0, gm = B.gamma, K = B.K, q0 = B.q0;
    if (!sx) {
      double d[3][3][3];
      if (B.st27) {
        // isotropic 27-point gradient (the stencil the box's field uses)
        for (int c = 0; c < 3; c++)
          for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) d[c][i][j] = 0.0;
        for (int dz = -1; dz <= 1; dz++)
          for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
              const int n = (dx != 0) + (dy != 0) + (dz != 0);
              if (n == 0) continue;
              const double wg = 3.0 * (n == 1 ? 2.0 / 27.0 : (n == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
              const int cc[3] = {dx, dy, dz};
              double qq[3][3];
              load_full(a.Qin, NS, gidx(x + dx, y + dy, z + dz), qq);
              for (int c = 0; c < 3; c++)
                for (int i = 0; i < 3; i++)
                  for (int j = 0; j < 3; j++) d[c][i][j] += wg * cc[c] * qq[i][j];
            }
      } else {
        const int e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int c = 0; c < 3; c++) {
          double qp[3][3], qm[3][3];
          load_full(a.Qin, NS, gidx(x + e[c][0], y + e[c][1], z + e[c][2]), qp);
          load_full(a.Qin, NS, gidx(x - e[c][0], y - e[c][1], z - e[c][2]), qm);
          for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) d[c][i][j] = 0.5 * (qp[i][j] - qm[i][j]);
        }
      }
      double tr2 = 0, tr3 = 0, chi = 0;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          tr2 += q[i][j] * q[i][j];
          for (int k = 0; k < 3; k++) tr3 += q[i][j] * q[j][k] * q[k][i];
        }
      for (int b = 0; b < 3; b++) {
        chi += q[0][b] * (d[1][2][b] - d[2][1][b]) + q[1][b] * (d[2][0][b] - d[0][2][b]) +
               q[2][b] * (d[0][1][b] - d[1][0][b]);
      }
      v[0] += 0.5 * A0 * (1.0 - gm / 3.0) * tr2 - A0 * gm / 3.0 * tr3 + 0.25 * A0 * gm * tr2 * tr2 +
              2.0 * K * q0 * chi + 2.0 * K * q0 * q0 * tr2;
      if (B.hydro) {
        for (int i = 0; i < 19; i++) {
          const double fi = (double)a.fin[i * NS + g] + wgt(i);
          v[1] += fi;
          v[2] += fi * cx(i); v[3] += fi * cy(i); v[4] += fi * cz(i);
        }
        double u2 = 0;
        for (int c = 0; c < 3; c++) u2 += (double)a.uin[c * NS + g] * (double)a.uin[c * NS + g];
        v[5] = sqrt(u2);
      }
    }
    for (int c = 0; c < 3; c++) {
      const int xn = x + (c == 0), yn = y + (c == 1), zn = z + (c == 2);
      const bool sn = solid(xn, yn, zn);
      if (sx && sn) continue;
      double qn[3][3], dd = 0;
      load_full(a.Qin, NS, gidx(xn, yn, zn), qn);
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) dd += (qn[i][j] - q[i][j]) * (qn[i][j] - q[i][j]);
      v[0] += 0.5 * K * dd;
      const int xs = sx ? x : xn, ys = sx ? y : yn, zs = sx ? z : zn;
      const ColDev* Cs = sx != sn ? &a.cols[B.col0 + sid(xs, ys, zs) - 1] : nullptr;
      if (Cs && Cs->anchoring != 0 && !isinf(Cs->W)) {
        // W/2 |Qs - Q^0|^2 at the solid end of the face
        const int nb[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        double qbar[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, qs[3][3], qz[3][3];
        int nf = 0;
        if (B.st27) {
          for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
              for (int dx = -1; dx <= 1; dx++) {
                if (!(dx || dy || dz) || solid(xs + dx, ys + dy, zs + dz)) continue;
                double qq[3][3];
                load_full(a.Qin, NS, gidx(xs + dx, ys + dy, zs + dz), qq);
                for (int i = 0; i < 3; i++)
                  for (int j = 0; j < 3; j++) qbar[i][j] += qq[i][j];
                nf++;
              }
        } else {
          for (int k = 0; k < 6; k++) {
            if (solid(xs + nb[k][0], ys + nb[k][1], zs + nb[k][2])) continue;
            double qq[3][3];
            load_full(a.Qin, NS, gidx(xs + nb[k][0], ys + nb[k][1], zs + nb[k][2]), qq);
            for (int i = 0; i < 3; i++)
              for (int j = 0; j < 3; j++) qbar[i][j] += qq[i][j];
            nf++;
          }
        }
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) qbar[i][j] /= nf;
        anchor_target(B, *Cs, Cs->pos[a.par], wrapc(xs, B.nx), wrapc(ys, B.ny), wrapc(zs, B.nz), qbar, qz);
        load_full(a.Qin, NS, gidx(xs, ys, zs), qs);
        double w2 = 0;
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) w2 += (qs[i][j] - qz[i][j]) * (qs[i][j] - qz[i][j]);
        v[0] += 0.5 * Cs->W * w2;
      }
    }
  }
  // max|u| is reduced as a max, the rest as sums
  __shared__ double smax[4];
  double m = v[5];
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
  v[5] = 0.0;
  block_sum<256, 6>(v, sred, out + 6LL * blockIdx.x);
  __syncthreads();
  if (threadIdx.x == 0) out[6LL * blockIdx.x + 5] = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
}

// Totals of the diagnostics partials of nb blocks (6 doubles each): thread
// c < 5 adds component c over the blocks in block order starting from zero,
// thread 5 takes the maximum of component 5 -- the order lc_get_diag uses
// on the host, so both give the same bits.
__global__ void __launch_bounds__(64)
    k_diag_total(const double* __restrict__ part, long long nb, double* __restrict__ out6) {
  const int c = threadIdx.x;
  if (c >= 6) return;
  double s = 0.0;
#pragma unroll 8
  for (long long k = 0; k < nb; k++) {
    const double v = part[6 * k + c];
    if (c < 5) s += v;
    else s = s < v ? v : s;
  }
  out6[c] = s;
}

// Largest eigenvalue of a symmetric traceless 3x3 matrix (trigonometric
// solution of the characteristic cubic).
__device__ inline double lambda_max(const double q[3][3]) {
  const double p2 = q[0][1] * q[0][1] + q[0][2] * q[0][2] + q[1][2] * q[1][2];
  const double p1 = q[0][0] * q[0][0] + q[1][1] * q[1][1] + q[2][2] * q[2][2] + 2.0 * p2;
  const double p = sqrt(p1 / 6.0);
  if (p < 1e-300) return 0.0;
  double bm[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) bm[i][j] = q[i][j] / p;
  double det = bm[0][0] * (bm[1][1] * bm[2][2] - bm[1][2] * bm[2][1]) -
               bm[0][1] * (bm[1][0] * bm[2][2] - bm[1][2] * bm[2][0]) +
               bm[0][2] * (bm[1][0] * bm[2][1] - bm[1][1] * bm[2][0]);
  double r = 0.5 * det;
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  return 2.0 * p * cos(acos(r) / 3.0);
}

template <typename R>
__global__ void __launch_bounds__(256)
    k_defects(const BoxDev* __restrict__ boxes, const ColDev* __restrict__ cols, int box, const R* __restrict__ Q,
              long long NS, double thr, unsigned char* __restrict__ mask, unsigned long long* __restrict__ count,
              int par) {
  const BoxDev& B = boxes[box];
  const long long nsite = (long long)B.nx * B.ny * B.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsite) return;
  const int x = (int)(t % B.nx), y = (int)((t / B.nx) % B.ny), z = (int)(t / ((long long)B.nx * B.ny));
  const unsigned all = (1u << B.ncol) - 1u;
  unsigned char m = 0;
  if (!solid_id(B, cols, all, par, x, y, z)) {
    double q[3][3];
    load_full(Q, NS, B.off + t, q);
    m = 1.5 * lambda_max(q) < thr;
  }
  mask[t] = m;
  if (m) atomicAdd(count, 1ULL);
}

// Solid map of one box: 1 + the colloid holding the node, 0 for fluid.
__global__ void __launch_bounds__(256)
    k_solid(const BoxDev* __restrict__ boxes, const ColDev* __restrict__ cols, int box, unsigned char* __restrict__ id,
            int par) {
  const BoxDev& B = boxes[box];
  const long long nsite = (long long)B.nx * B.ny * B.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsite) return;
  const int x = (int)(t % B.nx), y = (int)((t / B.nx) % B.ny), z = (int)(t / ((long long)B.nx * B.ny));
  id[t] = (unsigned char)solid_id(B, cols, (1u << B.ncol) - 1u, par, x, y, z);
}

template <typename R>
__global__ void __launch_bounds__(256) k_fill_f(R* f, long long NS, double rho0) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NS) return;
#pragma unroll
  for (int i = 0; i < 19; i++) f[i * NS + t] = (R)(wgt(i) * rho0 - wgt(i));
}

// ---------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------
// Launch with start/stop events carried by the dispatch itself when given
// (no separate event commands between the kernels of a step).
template <typename K, typename... Args>
void launch_ev(K kernel, unsigned nblk, unsigned nthr, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0 || e1) hipExtLaunchKernelGGL(kernel, dim3(nblk), dim3(nthr), 0, s, e0, e1, 0, args...);
  else hipLaunchKernelGGL(kernel, dim3(nblk), dim3(nthr), 0, s, args...);
}

template <typename R>
hipError_t launch_step(int tile, int nblk, const BoxDev* boxes, const int2* tiles, const int* offs,
                       const StepPtrs<R>& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
#define LC_TILE_CASE(ID, X, Y, Z, KIND)                                                             \
  case ID:                                                                                           \
    if constexpr (KIND == 0) launch_ev(k_step<R, X, Y, Z>, nblk, X * Y * Z, s, e0, e1, boxes, tiles, a); \
    else launch_ev(k_march<R, X, Y, Z>, nblk, X * Y, s, e0, e1, boxes, tiles, offs, a);                 \
    break;
  if constexpr (sizeof(R) == 4) {
    switch (tile) {
      LC_TILES_F32(LC_TILE_CASE)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (tile) {
      LC_TILES_F64(LC_TILE_CASE)
      default: return hipErrorInvalidValue;
    }
  }
#undef LC_TILE_CASE
  return hipGetLastError();
}

int march_blocks_per_cu(int tile) {
  int n = 0;
#define LC_OCC_CASE(ID, X, Y, Z, KIND)                                                           \
  case ID:                                                                                      \
    if constexpr (KIND == 1)                                                                     \
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_march<float, X, Y, Z>, X * Y, 0) != hipSuccess) n = 0; \
    break;
  switch (tile) {
    LC_TILES_F32(LC_OCC_CASE)
    default: break;
  }
#undef LC_OCC_CASE
  return n;
}

template <typename R>
hipError_t launch_ghost(const BoxDev* boxes, const ColDev* cols, int ncol, long long total, R* Q, long long NS, int par,
                        hipStream_t s) {
  if (total <= 0 || ncol <= 0) return hipSuccess;
  // small blocks: the few thousand boundary candidates spread over many CUs
  k_ghost<R><<<(unsigned)((total + 63) / 64), 64, 0, s>>>(boxes, cols, ncol, total, Q, NS, par);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_post(int nblk, const int* owner, const BoxDev* boxes, const StepPtrs<R>& a, double* bpart,
                       int* pending, const double* fsum, double* force, double* hist, int cap, long long* count,
                       hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  k_post<R><<<(unsigned)nblk, kPostBlock, 0, s>>>(boxes, owner, a, bpart, pending, fsum, force, hist, cap, count,
                                                  nblk);
  return hipGetLastError();
}

hipError_t launch_free(int ncol, const BoxDev* boxes, ColDev* cols, const double* part, long long nslot, int par,
                       double* fsum, hipStream_t s) {
  if (ncol <= 0) return hipSuccess;
  k_free<<<(unsigned)ncol, kFinishBlock, 0, s>>>(boxes, cols, part, nslot, par, fsum);
  return hipGetLastError();
}

hipError_t launch_finish(int ncol, int nblk, ColDev* cols, int par, const double* bpart, int* pending,
                         const double* fsum, double* force, double* hist, int cap, long long* count, hipStream_t s) {
  if (ncol <= 0) return hipSuccess;
  k_finish<<<(unsigned)ncol, kFinishBlock, 0, s>>>(cols, par, nblk, bpart, pending, fsum, force, hist, cap, count);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_diag(const BoxDev* boxes, int box, long long nsite, const StepPtrs<R>& a, double* out,
                       hipStream_t s) {
  k_diag<R><<<(unsigned)((nsite + 255) / 256), 256, 0, s>>>(boxes, box, a, out);
  return hipGetLastError();
}

hipError_t launch_diag_total(const double* part, long long nb, double* out6, hipStream_t s) {
  k_diag_total<<<1, 64, 0, s>>>(part, nb, out6);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_defects(const BoxDev* boxes, const ColDev* cols, int box, long long nsite, const R* Q, long long NS,
                          double thr,
                          unsigned char* mask, unsigned long long* count, int par, hipStream_t s) {
  k_defects<R><<<(unsigned)((nsite + 255) / 256), 256, 0, s>>>(boxes, cols, box, Q, NS, thr, mask, count, par);
  return hipGetLastError();
}

hipError_t launch_solid(const BoxDev* boxes, const ColDev* cols, int box, long long nsite, unsigned char* id, int par,
                        hipStream_t s) {
  k_solid<<<(unsigned)((nsite + 255) / 256), 256, 0, s>>>(boxes, cols, box, id, par);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fill(R* f, long long NS, double rho0, hipStream_t s) {
  k_fill_f<R><<<(unsigned)((NS + 255) / 256), 256, 0, s>>>(f, NS, rho0);
  return hipGetLastError();
}

#define LC_INST(R)                                                                                        \
  template hipError_t launch_step<R>(int, int, const BoxDev*, const int2*, const int*, const StepPtrs<R>&,   \
                                     hipStream_t, hipEvent_t, hipEvent_t);                                  \
  template hipError_t launch_ghost<R>(const BoxDev*, const ColDev*, int, long long, R*, long long, int,     \
                                      hipStream_t);                                                         \
  template hipError_t launch_post<R>(int, const int*, const BoxDev*, const StepPtrs<R>&, double*, int*,           \
                                     const double*,                                                         \
                                     double*, double*, int, long long*, hipStream_t);                        \
  template hipError_t launch_diag<R>(const BoxDev*, int, long long, const StepPtrs<R>&, double*, hipStream_t); \
  template hipError_t launch_defects<R>(const BoxDev*, const ColDev*, int, long long, const R*, long long, double, \
                                        unsigned char*, unsigned long long*, int, hipStream_t);             \
  template hipError_t launch_fill<R>(R*, long long, double, hipStream_t);
LC_INST(float)
LC_INST(double)

}  // namespace lc
