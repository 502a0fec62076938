/*
 * lco.c -- plain FP64 CPU oracle of the hybrid LB/FD step (see lco.h).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.
 *
 * The code follows the paper's equations in the paper's order and uses
 * plain loops over lattice sites.  Where the paper defers a detail to other
 * work, the reading taken is stated next to the code that implements it.
 * One time step (function step_once) is:
 *   1. ghost Q at boundary solid nodes: anchoring (Sec. 2.2, Eq. for Q^0)
 *   2. molecular field H (Eq. 1, Eq. 2) and stress P (Eq. 4) at fluid nodes
 *   3. force on the fluid = discrete divergence of P over control-volume
 *      faces, colloid force = sum of P.s over solid-fluid faces (Sec. 2.2,
 *      Eq. for F^coll)
 *   4. Beris-Edwards update of Q (Eq. 2) with co-rotation, zero advective
 *      flux through solid faces, lagged velocity u^{n-1} (Sec. 2.2)
 *   5. LB collision with the force, push streaming, bounce-back on links
 *      with the moving-wall correction; link momentum to the colloid
 *      (Sec. 2.2, BBL)
 *   6. for a freely moving colloid: velocity and position from the summed
 *      force (molecular-dynamics-like step, Sec. 2.2; reading in lco.h)
 *   7. moving-boundary events for a moving colloid (Sec. 2.2, last
 *      paragraph)
 */
#include "lco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19 velocity set and weights (rest 1/3, axis 1/18, diagonal 1/36). */
static const int CV[19][3] = {
  { 0, 0, 0},
  { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
  { 1, 1, 0}, {-1,-1, 0}, { 1,-1, 0}, {-1, 1, 0},
  { 1, 0, 1}, {-1, 0,-1}, { 1, 0,-1}, {-1, 0, 1},
  { 0, 1, 1}, { 0,-1,-1}, { 0, 1,-1}, { 0,-1, 1}};
static const double WT[19] = {
  1.0/3.0,
  1.0/18.0, 1.0/18.0, 1.0/18.0, 1.0/18.0, 1.0/18.0, 1.0/18.0,
  1.0/36.0, 1.0/36.0, 1.0/36.0, 1.0/36.0, 1.0/36.0, 1.0/36.0,
  1.0/36.0, 1.0/36.0, 1.0/36.0, 1.0/36.0, 1.0/36.0, 1.0/36.0};

static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

struct lco_sim {
  lco_params p;
  lco_colloid c[LCO_MAX_COLLOIDS];  /* the first ncol are present */
  int ncol;
  int err;                  /* a step found two colloids too close: stepping stops */
  long N;
  long nstep;
  double *f, *fn, *fstar;   /* 19N */
  double *Q, *Qn;           /* 5N  */
  double *Q0;               /* 5N, anchoring target at boundary solid nodes */
  double *u;                /* 3N, velocity of the previous collision */
  double *H, *P, *F;        /* 5N, 9N, 3N work */
  unsigned char *solid;     /* N: 0 fluid, k + 1 inside colloid k */
  double force[LCO_MAX_COLLOIDS][12];
};

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

static int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }

static long sidx(const lco_sim* s, int x, int y, int z) {
  return (long)wrapi(x, s->p.nx) +
         (long)s->p.nx * ((long)wrapi(y, s->p.ny) + (long)s->p.ny * wrapi(z, s->p.nz));
}

static void scoord(const lco_sim* s, long i, int* x, int* y, int* z) {
  *x = (int)(i % s->p.nx);
  *y = (int)((i / s->p.nx) % s->p.ny);
  *z = (int)(i / ((long)s->p.nx * s->p.ny));
}

/* minimum-image displacement along an axis of period L */
static double minimg(double d, int L) {
  if (d > 0.5 * L) d -= L;
  else if (d < -0.5 * L) d += L;
  return d;
}

static double eps3(int a, int b, int c) {
  if (a == b || b == c || a == c) return 0.0;
  /* even permutations of (0,1,2) */
  if ((a == 0 && b == 1) || (a == 1 && b == 2) || (a == 2 && b == 0)) return 1.0;
  return -1.0;
}

static void full_from5(const double* Q, long N, long i, double q[3][3]) {
  double xx = Q[0 * N + i], xy = Q[1 * N + i], xz = Q[2 * N + i];
  double yy = Q[3 * N + i], yz = Q[4 * N + i];
  q[0][0] = xx; q[0][1] = xy; q[0][2] = xz;
  q[1][0] = xy; q[1][1] = yy; q[1][2] = yz;
  q[2][0] = xz; q[2][1] = yz; q[2][2] = -xx - yy;
}

static void store5(double* Q, long N, long i, double q[3][3]) {
  Q[0 * N + i] = q[0][0]; Q[1 * N + i] = q[0][1]; Q[2 * N + i] = q[0][2];
  Q[3 * N + i] = q[1][1]; Q[4 * N + i] = q[1][2];
}

static double frob2(double a[3][3]) {
  double r = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) r += a[i][j] * a[i][j];
  return r;
}

/* displacement (minimum image) from the colloid centre R to a point */
static void rel_pos(const lco_sim* s, const double R[3], double px, double py, double pz,
                    double r[3]) {
  r[0] = minimg(px - R[0], s->p.nx);
  r[1] = minimg(py - R[1], s->p.ny);
  r[2] = minimg(pz - R[2], s->p.nz);
}

/* Solid/fluid assignment from the nominal radius and the position
 * (Sec. 2.2): a node is solid iff |x - R|^2 < a0^2 (distance exactly a0
 * counts as fluid). */
static int inside(const lco_sim* s, const lco_colloid* c, const double R[3], int x, int y, int z) {
  double r[3];
  rel_pos(s, R, x, y, z, r);
  return r[0] * r[0] + r[1] * r[1] + r[2] * r[2] < c->a0 * c->a0;
}

/* Colloid k of a solid node (solid[i] = k + 1). */
static const lco_colloid* owner(const lco_sim* s, long i) { return &s->c[s->solid[i] - 1]; }

/* rigid-body velocity v + omega x r (Sec. 2.2) */
static void rigid_vel(const lco_colloid* c, const double r[3], double ub[3]) {
  ub[0] = c->vel[0] + c->omega[1] * r[2] - c->omega[2] * r[1];
  ub[1] = c->vel[1] + c->omega[2] * r[0] - c->omega[0] * r[2];
  ub[2] = c->vel[2] + c->omega[0] * r[1] - c->omega[1] * r[0];
}

static void cross(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------ */
/* exposed pieces                                                       */
/* ------------------------------------------------------------------ */

void lco_lattice(int c[19][3], double w[19]) {
  for (int i = 0; i < 19; i++) {
    for (int a = 0; a < 3; a++) c[i][a] = CV[i][a];
    w[i] = WT[i];
  }
}

/* LB equilibrium, second order in u, weights w_i, c_s^2 = 1/3. */
void lco_feq(double rho, const double u[3], double feq[19]) {
  double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < 19; i++) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    feq[i] = WT[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
  }
}

/* Principal axis (eigenvector of the largest eigenvalue) of a symmetric
 * 3x3 matrix by cyclic Jacobi rotations in FP64.  Rotation planes are
 * visited in the fixed order (0,1), (0,2), (1,2); sweeps stop when the
 * off-diagonal norm falls below 1e-15 of the matrix norm.  Ties between
 * equal largest eigenvalues go to the lowest index. */
int lco_principal_axis(const double A9[9], double n[3], double* lam) {
  double a[3][3], v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) a[i][j] = 0.5 * (A9[3 * i + j] + A9[3 * j + i]);
  static const int PP[3] = {0, 0, 1}, QQ[3] = {1, 2, 2};
  for (int sweep = 0; sweep < 64; sweep++) {
    double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    double tot = frob2(a);
    if (off == 0.0 || off <= 1e-30 * tot) break;
    for (int k = 0; k < 3; k++) {
      int p = PP[k], q = QQ[k];
      if (a[p][q] == 0.0) continue;
      double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
      double t;
      if (fabs(theta) > 1e150) t = 0.5 / theta;
      else t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
      double apq = a[p][q];
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.0;
      for (int r = 0; r < 3; r++) {
        if (r == p || r == q) continue;
        double arp = a[r][p], arq = a[r][q];
        a[r][p] = a[p][r] = cs * arp - sn * arq;
        a[r][q] = a[q][r] = sn * arp + cs * arq;
      }
      for (int r = 0; r < 3; r++) {
        double vrp = v[r][p], vrq = v[r][q];
        v[r][p] = cs * vrp - sn * vrq;
        v[r][q] = sn * vrp + cs * vrq;
      }
    }
  }
  int k = 0;
  for (int i = 1; i < 3; i++)
    if (a[i][i] > a[k][k]) k = i;
  for (int r = 0; r < 3; r++) n[r] = v[r][k];
  if (lam) *lam = a[k][k];
  return LCO_OK;
}

/* Bulk part of the molecular field (Eq. 1 bulk terms into Eq. 2):
 * H = -A0(1-g/3)Q + A0 g (Q.Q - Tr(Q^2)/3 I) - A0 g Tr(Q^2) Q. */
static void bulk_field_full(const lco_params* p, double q[3][3], double h[3][3]) {
  double q2[3][3], tr2 = 0.0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double acc = 0.0;
      for (int g = 0; g < 3; g++) acc += q[a][g] * q[g][b];
      q2[a][b] = acc;
    }
  tr2 = q2[0][0] + q2[1][1] + q2[2][2];
  double A0 = p->A0, gm = p->gamma;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      h[a][b] = -A0 * (1.0 - gm / 3.0) * q[a][b] +
                A0 * gm * (q2[a][b] - (a == b ? tr2 / 3.0 : 0.0)) -
                A0 * gm * tr2 * q[a][b];
}

void lco_bulk_field(const lco_params* p, const double Q5[5], double H5[5]) {
  double q[3][3], h[3][3];
  full_from5(Q5, 1, 0, q);
  bulk_field_full(p, q, h);
  H5[0] = h[0][0]; H5[1] = h[0][1]; H5[2] = h[0][2]; H5[3] = h[1][1]; H5[4] = h[1][2];
}

/* Co-rotation term of the material derivative for rod-like molecules
 * (Eq. 2; the paper defers the form to Beris and Edwards):
 * S = (xi D + Om)(Q + I/3) + (Q + I/3)(xi D - Om) - 2 xi (Q + I/3) Tr(Q W),
 * with W_ab = d_b u_a, D = (W + W^T)/2, Om = (W - W^T)/2. */
static void corotation_full(double xi, double W[3][3], double q[3][3], double S[3][3]) {
  double D[3][3], Om[3][3], A[3][3];
  double trqw = 0.0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      D[a][b] = 0.5 * (W[a][b] + W[b][a]);
      Om[a][b] = 0.5 * (W[a][b] - W[b][a]);
      A[a][b] = q[a][b] + (a == b ? 1.0 / 3.0 : 0.0);
      trqw += q[a][b] * W[b][a];
    }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double acc = 0.0;
      for (int g = 0; g < 3; g++)
        acc += (xi * D[a][g] + Om[a][g]) * A[g][b] + A[a][g] * (xi * D[g][b] - Om[g][b]);
      S[a][b] = acc - 2.0 * xi * A[a][b] * trqw;
    }
}

void lco_corotation(double xi, const double W9[9], const double Q5[5], double S5[5]) {
  double W[3][3], q[3][3], S[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) W[a][b] = W9[3 * a + b];
  full_from5(Q5, 1, 0, q);
  corotation_full(xi, W, q, S);
  S5[0] = S[0][0]; S5[1] = S[0][1]; S5[2] = S[0][2]; S5[3] = S[1][1]; S5[4] = S[1][2];
}

void lco_single_site(const lco_params* p, const double W9[9], long nsteps, double Q5[5]) {
  double W[3][3], q[3][3], S[3][3], h[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) W[a][b] = W9[3 * a + b];
  for (long n = 0; n < nsteps; n++) {
    full_from5(Q5, 1, 0, q);
    corotation_full(p->xi, W, q, S);
    bulk_field_full(p, q, h);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) q[a][b] += S[a][b] + p->Gamma * h[a][b];
    store5(Q5, 1, 0, q);
  }
}

/* ------------------------------------------------------------------ */
/* creation, state access                                               */
/* ------------------------------------------------------------------ */

int lco_create(const lco_params* p, lco_sim** out) {
  if (!p || !out) return LCO_EINVAL;
  *out = NULL;
  if (p->nx < 4 || p->ny < 4 || p->nz < 4) return LCO_EINVAL;
  if (!(p->tau > 0.5) || !(p->rho0 > 0.0) || !(p->Gamma >= 0.0) || !(p->K >= 0.0))
    return LCO_EINVAL;
  if (p->advection < 0 || p->advection > 3) return LCO_EINVAL;
  if (p->stencil != 0 && p->stencil != 7 && p->stencil != 27) return LCO_EINVAL;
  lco_sim* s = (lco_sim*)calloc(1, sizeof(lco_sim));
  if (!s) return LCO_ENOMEM;
  s->p = *p;
  if (s->p.advection == 0) s->p.advection = 1;
  if (s->p.stencil == 0) s->p.stencil = 7;
  s->N = (long)p->nx * p->ny * p->nz;
  long N = s->N;
  s->f = (double*)calloc(19 * N, sizeof(double));
  s->fn = (double*)calloc(19 * N, sizeof(double));
  s->fstar = (double*)calloc(19 * N, sizeof(double));
  s->Q = (double*)calloc(5 * N, sizeof(double));
  s->Qn = (double*)calloc(5 * N, sizeof(double));
  s->Q0 = (double*)calloc(5 * N, sizeof(double));
  s->u = (double*)calloc(3 * N, sizeof(double));
  s->H = (double*)calloc(5 * N, sizeof(double));
  s->P = (double*)calloc(9 * N, sizeof(double));
  s->F = (double*)calloc(3 * N, sizeof(double));
  s->solid = (unsigned char*)calloc(N, 1);
  if (!s->f || !s->fn || !s->fstar || !s->Q || !s->Qn || !s->Q0 || !s->u || !s->H ||
      !s->P || !s->F || !s->solid) {
    lco_destroy(s);
    return LCO_ENOMEM;
  }
  for (int i = 0; i < 19; i++)
    for (long k = 0; k < N; k++) s->f[i * N + k] = WT[i] * p->rho0;
  *out = s;
  return LCO_OK;
}

void lco_destroy(lco_sim* s) {
  if (!s) return;
  free(s->f); free(s->fn); free(s->fstar); free(s->Q); free(s->Qn); free(s->Q0);
  free(s->u); free(s->H); free(s->P); free(s->F); free(s->solid);
  free(s);
}

static void classify(lco_sim* s) {
  long N = s->N;
  for (long i = 0; i < N; i++) {
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    s->solid[i] = 0;
    for (int k = 0; k < s->ncol && !s->solid[i]; k++)
      if (inside(s, &s->c[k], s->c[k].pos, x, y, z)) s->solid[i] = (unsigned char)(k + 1);
  }
}

/* solid nodes carry no fluid */
static void clear_solid_fluid(lco_sim* s) {
  long N = s->N;
  for (long i = 0; i < N; i++) {
    if (!s->solid[i]) continue;
    for (int k = 0; k < 19; k++) s->f[k * N + i] = 0.0;
    for (int a = 0; a < 3; a++) s->u[a * N + i] = 0.0;
  }
}

/* Minimum-image distance between two centres. */
static double centre_distance(const lco_sim* s, const double A[3], const double B[3]) {
  double r[3];
  rel_pos(s, A, B[0], B[1], B[2], r);
  return sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
}

/* Several colloids in one box must keep their surfaces at least
 * LCO_COLLOID_GAP lattice units apart (Introduction / Sec. 3.2 outlook:
 * interactions through the liquid crystal, no lubrication): then no fluid
 * node has links or faces to two colloids, and every ghost node's fluid
 * neighbours and every uncovered node's neighbours see one colloid only. */
static int separated(const lco_sim* s, int n, const lco_colloid* c) {
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++)
      if (centre_distance(s, c[i].pos, c[j].pos) < c[i].a0 + c[j].a0 + LCO_COLLOID_GAP) return 0;
  return 1;
}

int lco_set_colloids(lco_sim* s, int n, const lco_colloid* c) {
  if (!s || n < 0 || n > LCO_MAX_COLLOIDS || (n > 0 && !c)) return LCO_EINVAL;
  int Lmin = s->p.nx < s->p.ny ? s->p.nx : s->p.ny;
  if (s->p.nz < Lmin) Lmin = s->p.nz;
  lco_colloid v[LCO_MAX_COLLOIDS];
  memset(v, 0, sizeof(v));
  for (int k = 0; k < n; k++) {
    if (!c[k].present) return LCO_EINVAL;
    if (!(c[k].a0 > 1.0) || !(2.0 * c[k].a0 + 4.0 <= Lmin)) return LCO_EINVAL;
    if (c[k].anchoring < LCO_ANCHOR_NONE || c[k].anchoring > LCO_ANCHOR_PLANAR) return LCO_EINVAL;
    if (c[k].motion != LCO_FIXED && c[k].motion != LCO_PRESCRIBED && c[k].motion != LCO_FREE) return LCO_EINVAL;
    if (!(c[k].W >= 0.0)) return LCO_EINVAL;
    if (c[k].anchoring != LCO_ANCHOR_NONE && !(s->p.K + c[k].W > 0.0)) return LCO_EINVAL;
    v[k] = c[k];
    /* keep the centre inside [0, L) */
    int L[3] = {s->p.nx, s->p.ny, s->p.nz};
    for (int a = 0; a < 3; a++) {
      double r = fmod(v[k].pos[a], (double)L[a]);
      if (r < 0) r += L[a];
      v[k].pos[a] = r;
    }
  }
  if (!separated(s, n, v)) return LCO_EINVAL;
  for (int k = 0; k < n; k++) s->c[k] = v[k];
  s->ncol = n;
  memset(s->force, 0, sizeof(s->force));
  s->err = 0;
  classify(s);
  clear_solid_fluid(s);
  return LCO_OK;
}

int lco_set_colloid(lco_sim* s, const lco_colloid* c) {
  if (!s || !c) return LCO_EINVAL;
  return lco_set_colloids(s, c->present ? 1 : 0, c);
}

int lco_get_colloid(const lco_sim* s, lco_colloid* c) {
  if (!s || !c) return LCO_EINVAL;
  if (s->ncol > 0) *c = s->c[0];
  else memset(c, 0, sizeof(*c));
  return LCO_OK;
}

int lco_num_colloids(const lco_sim* s) { return s ? s->ncol : -1; }

int lco_get_colloids(const lco_sim* s, int n, lco_colloid* c) {
  if (!s || n < 0 || n > s->ncol || (n > 0 && !c)) return LCO_EINVAL;
  for (int k = 0; k < n; k++) c[k] = s->c[k];
  return LCO_OK;
}

int lco_set_Q(lco_sim* s, const double* Q5) {
  if (!s || !Q5) return LCO_EINVAL;
  memcpy(s->Q, Q5, sizeof(double) * 5 * s->N);
  return LCO_OK;
}

int lco_set_f(lco_sim* s, const double* f19) {
  if (!s || !f19) return LCO_EINVAL;
  memcpy(s->f, f19, sizeof(double) * 19 * s->N);
  clear_solid_fluid(s);
  return LCO_OK;
}

int lco_set_u(lco_sim* s, const double* u3) {
  if (!s || !u3) return LCO_EINVAL;
  memcpy(s->u, u3, sizeof(double) * 3 * s->N);
  clear_solid_fluid(s);
  return LCO_OK;
}

int lco_get_Q(const lco_sim* s, double* Q5) {
  if (!s || !Q5) return LCO_EINVAL;
  memcpy(Q5, s->Q, sizeof(double) * 5 * s->N);
  return LCO_OK;
}

int lco_get_f(const lco_sim* s, double* f19) {
  if (!s || !f19) return LCO_EINVAL;
  memcpy(f19, s->f, sizeof(double) * 19 * s->N);
  return LCO_OK;
}

int lco_get_u(const lco_sim* s, double* u3) {
  if (!s || !u3) return LCO_EINVAL;
  memcpy(u3, s->u, sizeof(double) * 3 * s->N);
  return LCO_OK;
}

int lco_get_solid(const lco_sim* s, unsigned char* solid) {
  if (!s || !solid) return LCO_EINVAL;
  memcpy(solid, s->solid, s->N);
  return LCO_OK;
}

int lco_get_force(const lco_sim* s, double out[12]) {
  if (!s || !out) return LCO_EINVAL;
  memcpy(out, s->force[0], sizeof(s->force[0]));
  return LCO_OK;
}

int lco_get_forces(const lco_sim* s, int n, double* out) {
  if (!s || n < 0 || n > s->ncol || (n > 0 && !out)) return LCO_EINVAL;
  memcpy(out, s->force, sizeof(double) * 12 * n);
  return LCO_OK;
}

long lco_get_nstep(const lco_sim* s) { return s ? s->nstep : -1; }

/* ------------------------------------------------------------------ */
/* step pieces                                                          */
/* ------------------------------------------------------------------ */

/* A solid node within reach of a fluid node's Q stencil: a fluid face
 * neighbour (7-point stencil) or a fluid node among its 26 neighbours
 * (27-point stencil). */
static int is_boundary_solid(const lco_sim* s, int x, int y, int z) {
  if (!s->solid[sidx(s, x, y, z)]) return 0;
  if (s->p.stencil == 27) {
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++)
          if ((dx || dy || dz) && !s->solid[sidx(s, x + dx, y + dy, z + dz)]) return 1;
    return 0;
  }
  static const int E[6][3] = {{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1}};
  for (int k = 0; k < 6; k++)
    if (!s->solid[sidx(s, x + E[k][0], y + E[k][1], z + E[k][2])]) return 1;
  return 0;
}

/* Surface director and target tensor Q^0 = S0 (n0 n0 - I/3) at a boundary
 * solid node (Sec. 2.2).  qbar is the mean Q of the fluid face neighbours;
 * homeotropic: n0 = s (local outward unit normal); planar: the principal
 * axis of qbar (the "existing director") projected onto the tangent plane
 * and normalised, with fallbacks s x z, then s x x when the projection
 * vanishes. */
static void anchoring_target(const lco_sim* s, const lco_colloid* c, int x, int y, int z,
                             double qbar[3][3], double q0[3][3]) {
  double r[3], sh[3];
  rel_pos(s, c->pos, x, y, z, r);
  double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (rn < 1e-12) { sh[0] = 0; sh[1] = 0; sh[2] = 1; }
  else { sh[0] = r[0] / rn; sh[1] = r[1] / rn; sh[2] = r[2] / rn; }
  double n0[3];
  if (c->anchoring == LCO_ANCHOR_PLANAR) {
    double A9[9], n[3];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) A9[3 * a + b] = qbar[a][b];
    lco_principal_axis(A9, n, NULL);
    double ns = n[0] * sh[0] + n[1] * sh[1] + n[2] * sh[2];
    double t[3] = {n[0] - ns * sh[0], n[1] - ns * sh[1], n[2] - ns * sh[2]};
    double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    if (tn < 1e-12) {
      double ez[3] = {0, 0, 1};
      cross(sh, ez, t);
      tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
      if (tn < 1e-12) {
        double ex[3] = {1, 0, 0};
        cross(sh, ex, t);
        tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
      }
    }
    for (int a = 0; a < 3; a++) n0[a] = t[a] / tn;
  } else {
    for (int a = 0; a < 3; a++) n0[a] = sh[a];
  }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      q0[a][b] = c->S0 * (n0[a] * n0[b] - (a == b ? 1.0 / 3.0 : 0.0));
}

/* Ghost Q at every boundary solid node, from the current Q at its fluid
 * face neighbours.  Fixed anchoring (W = inf) sets Q^0 itself, as in the
 * paper; a finite W blends (K qbar + W Q^0)/(K + W), the minimiser of
 * K/2|qbar - Qs|^2 + W/2|Qs - Q^0|^2; no anchoring copies qbar. */
static void ghost_all(lco_sim* s, double* Q) {
  if (!s->ncol) return;
  long N = s->N;
  static const int E[6][3] = {{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1}};
  #pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    if (!is_boundary_solid(s, x, y, z)) continue;
    double qbar[3][3] = {{0}}, qn[3][3], q0[3][3], qs[3][3];
    int nf = 0;
    if (s->p.stencil == 27) {
      /* the mean over the fluid nodes among the 26 neighbours */
      for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
          for (int dx = -1; dx <= 1; dx++) {
            if (!(dx || dy || dz)) continue;
            long j = sidx(s, x + dx, y + dy, z + dz);
            if (s->solid[j]) continue;
            full_from5(Q, N, j, qn);
            for (int a = 0; a < 3; a++)
              for (int b = 0; b < 3; b++) qbar[a][b] += qn[a][b];
            nf++;
          }
    } else {
      for (int k = 0; k < 6; k++) {
        long j = sidx(s, x + E[k][0], y + E[k][1], z + E[k][2]);
        if (s->solid[j]) continue;
        full_from5(Q, N, j, qn);
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) qbar[a][b] += qn[a][b];
        nf++;
      }
    }
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) qbar[a][b] /= nf;
    const lco_colloid* c = owner(s, i);
    if (c->anchoring == LCO_ANCHOR_NONE) {
      store5(Q, N, i, qbar);
      double z0[3][3] = {{0}};
      store5(s->Q0, N, i, z0);
      continue;
    }
    anchoring_target(s, c, x, y, z, qbar, q0);
    store5(s->Q0, N, i, q0);
    double K = s->p.K, W = c->W;
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++)
        qs[a][b] = isinf(W) ? q0[a][b] : (K * qbar[a][b] + W * q0[a][b]) / (K + W);
    store5(Q, N, i, qs);
  }
}

/* Central first derivatives D0_g Q and compact Laplacian at site (x,y,z);
 * solid neighbours contribute their ghost values (Sec. 2.2: the same
 * stencil everywhere in the fluid). */
static void stencil(const lco_sim* s, const double* Q, int x, int y, int z,
                    double q[3][3], double dq[3][3][3], double lap[3][3]) {
  long N = s->N;
  full_from5(Q, N, sidx(s, x, y, z), q);
  if (s->p.stencil == 27) {
    /* isotropic 27-point operators (the variant of the "same stencil"
     * reading): D_g Q = 3 sum_i w_i c_ig Q(x + c_i) with the D3Q27 weights
     * 2/27 (faces), 1/54 (edges), 1/216 (corners), whose second moment is
     * 1/3; Laplacian (14 sum_faces + 3 sum_edges + sum_corners - 128 Q)/30,
     * exact on quadratics with an isotropic leading error */
    for (int g = 0; g < 3; g++)
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) dq[g][a][b] = 0.0;
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) lap[a][b] = 0.0;
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          const int n = abs(dx) + abs(dy) + abs(dz);
          if (n == 0) continue;
          const double wg = n == 1 ? 2.0 / 27.0 : (n == 2 ? 1.0 / 54.0 : 1.0 / 216.0);
          const double wl = n == 1 ? 14.0 : (n == 2 ? 3.0 : 1.0);
          const int c[3] = {dx, dy, dz};
          double qn[3][3];
          full_from5(Q, N, sidx(s, x + dx, y + dy, z + dz), qn);
          for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
              lap[a][b] += wl * qn[a][b];
              for (int g = 0; g < 3; g++) dq[g][a][b] += 3.0 * wg * c[g] * qn[a][b];
            }
        }
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) lap[a][b] = (lap[a][b] - 128.0 * q[a][b]) / 30.0;
    return;
  }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) lap[a][b] = -6.0 * q[a][b];
  for (int g = 0; g < 3; g++) {
    int e[3] = {0, 0, 0};
    e[g] = 1;
    double qp[3][3], qm[3][3];
    full_from5(Q, N, sidx(s, x + e[0], y + e[1], z + e[2]), qp);
    full_from5(Q, N, sidx(s, x - e[0], y - e[1], z - e[2]), qm);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        dq[g][a][b] = 0.5 * (qp[a][b] - qm[a][b]);
        lap[a][b] += qp[a][b] + qm[a][b];
      }
  }
}

/* Molecular field H = -dF/dQ + Tr(dF/dQ) I / 3 for the free energy of
 * Eq. (1): bulk part plus K lap Q - 2 K q0 (e_agd d_g Q_db + e_bgd d_g Q_da)
 * - 4 K q0^2 Q. */
static void mol_field(const lco_params* p, double q[3][3], double dq[3][3][3],
                      double lap[3][3], double h[3][3]) {
  bulk_field_full(p, q, h);
  double K = p->K, q0 = p->q0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double chi = 0.0;
      for (int g = 0; g < 3; g++)
        for (int d = 0; d < 3; d++)
          chi += eps3(a, g, d) * dq[g][d][b] + eps3(b, g, d) * dq[g][d][a];
      h[a][b] += K * lap[a][b] - 2.0 * K * q0 * chi - 4.0 * K * q0 * q0 * q[a][b];
    }
}

/* Free-energy density of Eq. (1) in the one-constant form:
 * bulk + K/2 |dQ|^2 + 2 K q0 Q_ab e_agd d_g Q_db + 2 K q0^2 |Q|^2. */
static double bulk_energy(const lco_params* p, double q[3][3]) {
  double tr2 = frob2(q), tr3 = 0.0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      for (int g = 0; g < 3; g++) tr3 += q[a][b] * q[b][g] * q[g][a];
  return 0.5 * p->A0 * (1.0 - p->gamma / 3.0) * tr2 - p->A0 * p->gamma / 3.0 * tr3 +
         0.25 * p->A0 * p->gamma * tr2 * tr2;
}

static double chiral_cross(double q[3][3], double dq[3][3][3]) {
  double acc = 0.0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      for (int g = 0; g < 3; g++)
        for (int d = 0; d < 3; d++) acc += q[a][b] * eps3(a, g, d) * dq[g][d][b];
  return acc;
}

/* Stress of Eq. (4) without the fluid's own pressure rho c_s^2 (the LB
 * carries it); the isotropic pressure is read as P0 = rho c_s^2 - f,
 * f the free-energy density, so P gains +f I.  The Ericksen term uses
 * dF/d(d_b Q_gn) of the one-constant form: K d_b Q_gn + 2 K q0 e_mbg Q_mn. */
static void chem_stress(const lco_params* p, double q[3][3], double dq[3][3][3],
                        double h[3][3], double P[3][3]) {
  double K = p->K, q0 = p->q0, xi = p->xi;
  double fpt = bulk_energy(p, q);
  double dq2 = 0.0;
  for (int g = 0; g < 3; g++) dq2 += frob2(dq[g]);
  fpt += 0.5 * K * dq2 + 2.0 * K * q0 * chiral_cross(q, dq) + 2.0 * K * q0 * q0 * frob2(q);
  double trqh = 0.0, A[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      trqh += q[a][b] * h[a][b];
      A[a][b] = q[a][b] + (a == b ? 1.0 / 3.0 : 0.0);
    }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double ha = 0.0, ah = 0.0, qh = 0.0, hq = 0.0;
      for (int g = 0; g < 3; g++) {
        ha += h[a][g] * A[g][b];
        ah += A[a][g] * h[g][b];
        qh += q[a][g] * h[g][b];
        hq += h[a][g] * q[g][b];
      }
      double E = 0.0;
      for (int g = 0; g < 3; g++)
        for (int n = 0; n < 3; n++) {
          double dfd = K * dq[b][g][n];
          for (int m = 0; m < 3; m++) dfd += 2.0 * K * q0 * eps3(m, b, g) * q[m][n];
          E += dq[a][g][n] * dfd;
        }
      P[a][b] = (a == b ? fpt : 0.0) + 2.0 * xi * A[a][b] * trqh - xi * ha - xi * ah - E +
                qh - hq;
    }
}

/* H (and P if wanted) at every fluid node from Q with ghost values. */
static void compute_HP(lco_sim* s, const double* Q, int want_P) {
  long N = s->N;
  #pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) continue;
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    double q[3][3], dq[3][3][3], lap[3][3], h[3][3], P[3][3];
    stencil(s, Q, x, y, z, q, dq, lap);
    mol_field(&s->p, q, dq, lap, h);
    store5(s->H, N, i, h);
    if (want_P) {
      chem_stress(&s->p, q, dq, h, P);
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) s->P[(3 * a + b) * N + i] = P[a][b];
    }
  }
}

/* Force on the fluid: discrete divergence of P over the faces of each
 * control volume (Sec. 2.2).  The face value is the mean of the two nodes
 * between fluid nodes and the fluid node's own P at a solid-fluid face. */
static void compute_F(lco_sim* s) {
  long N = s->N;
  #pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) continue;
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    double F[3] = {0, 0, 0};
    for (int b = 0; b < 3; b++) {
      int e[3] = {0, 0, 0};
      e[b] = 1;
      long jp = sidx(s, x + e[0], y + e[1], z + e[2]);
      long jm = sidx(s, x - e[0], y - e[1], z - e[2]);
      for (int a = 0; a < 3; a++) {
        double pc = s->P[(3 * a + b) * N + i];
        double pp = s->solid[jp] ? pc : 0.5 * (pc + s->P[(3 * a + b) * N + jp]);
        double pm = s->solid[jm] ? pc : 0.5 * (pc + s->P[(3 * a + b) * N + jm]);
        F[a] += pp - pm;
      }
    }
    for (int a = 0; a < 3; a++) s->F[a * N + i] = F[a] + s->p.body_force[a];
  }
}

/* Colloid force and torque from the stress: the sum of P.s over the
 * solid-fluid control-volume faces (Sec. 2.2, F^coll = int P.s dS), with s
 * the outward colloid normal of the face.  Serial for a fixed order. */
static void colloid_stress(lco_sim* s, double Fs[][3], double Ts[][3]) {
  long N = s->N;
  for (int k = 0; k < LCO_MAX_COLLOIDS; k++)
    for (int a = 0; a < 3; a++) Fs[k][a] = Ts[k][a] = 0.0;
  if (!s->ncol) return;
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) continue;
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    for (int b = 0; b < 3; b++)
      for (int sg = 1; sg >= -1; sg -= 2) {
        int e[3] = {0, 0, 0};
        e[b] = sg;
        long j = sidx(s, x + e[0], y + e[1], z + e[2]);
        if (!s->solid[j]) continue;
        /* the solid node sits at x + sg e_b: outward colloid normal -sg e_b */
        double ps[3], r[3], t[3];
        const int k = s->solid[j] - 1;
        for (int a = 0; a < 3; a++) ps[a] = -sg * s->P[(3 * a + b) * N + i];
        rel_pos(s, s->c[k].pos, x + 0.5 * e[0], y + 0.5 * e[1], z + 0.5 * e[2], r);
        cross(r, ps, t);
        for (int a = 0; a < 3; a++) { Fs[k][a] += ps[a]; Ts[k][a] += t[a]; }
      }
  }
}

static void site_velocity(const lco_sim* s, int x, int y, int z, double u[3]) {
  long j = sidx(s, x, y, z);
  if (s->solid[j]) {
    double r[3];
    const lco_colloid* c = owner(s, j);
    rel_pos(s, c->pos, x, y, z, r);
    rigid_vel(c, r, u);
  } else {
    for (int a = 0; a < 3; a++) u[a] = s->u[a * s->N + j];
  }
}

/* Advective flux through the face between node (x,y,z) and its neighbour
 * at +e_b (Sec. 2.2): ubar Q_face with ubar the mean of the two nodes'
 * velocities and Q_face taken upwind; zero when either node is solid.
 * Orders of the upwind value: 1 the upwind node; 2 linear extrapolation
 * from the two upwind nodes, (3 Q_up - Q_upup)/2; 3 upwind-biased,
 * (2 Q_down + 5 Q_up - Q_upup)/6.  A face whose wider stencil reaches a
 * solid node takes the first-order value. */
static void face_flux(const lco_sim* s, int x, int y, int z, int b, double phi[3][3]) {
  long N = s->N;
  int e[3] = {0, 0, 0};
  e[b] = 1;
  for (int a = 0; a < 3; a++)
    for (int c = 0; c < 3; c++) phi[a][c] = 0.0;
  long j0 = sidx(s, x, y, z), j1 = sidx(s, x + e[0], y + e[1], z + e[2]);
  if (s->solid[j0] || s->solid[j1]) return;
  double u0[3], u1[3];
  site_velocity(s, x, y, z, u0);
  site_velocity(s, x + e[0], y + e[1], z + e[2], u1);
  double uf = 0.5 * (u0[b] + u1[b]);
  /* along the flow: upwind node, the one before it, the downwind node */
  long jup, jupup, jdown;
  if (uf >= 0.0) {
    jup = j0; jdown = j1; jupup = sidx(s, x - e[0], y - e[1], z - e[2]);
  } else {
    jup = j1; jdown = j0; jupup = sidx(s, x + 2 * e[0], y + 2 * e[1], z + 2 * e[2]);
  }
  int order = s->p.advection;
  if (order > 1 && s->solid[jupup]) order = 1;
  double qu[3][3], qd[3][3], quu[3][3], qf[3][3];
  full_from5(s->Q, N, jup, qu);
  if (order == 1) {
    for (int a = 0; a < 3; a++)
      for (int c = 0; c < 3; c++) qf[a][c] = qu[a][c];
  } else {
    full_from5(s->Q, N, jupup, quu);
    full_from5(s->Q, N, jdown, qd);
    for (int a = 0; a < 3; a++)
      for (int c = 0; c < 3; c++)
        qf[a][c] = order == 2 ? (3.0 * qu[a][c] - quu[a][c]) / 2.0
                              : (2.0 * qd[a][c] + 5.0 * qu[a][c] - quu[a][c]) / 6.0;
  }
  for (int a = 0; a < 3; a++)
    for (int c = 0; c < 3; c++) phi[a][c] = uf * qf[a][c];
}

/* Beris-Edwards update at fluid nodes, forward Euler with dt = 1:
 * Q^{n+1} = Q^n - div(u Q) + S(W, Q^n) + Gamma H^n.  Velocity gradient by
 * central differences with v + omega x r at solid nodes; advective fluxes
 * at control-volume faces, first-order upwind with the face velocity the
 * mean of the two nodes, zero through solid-fluid faces (Sec. 2.2). */
static void be_update(lco_sim* s) {
  long N = s->N;
  const int hydro = s->p.hydro;
  #pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) {
      for (int c = 0; c < 5; c++) s->Qn[c * N + i] = s->Q[c * N + i];
      continue;
    }
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    double q[3][3], h[3][3], dQ[3][3];
    full_from5(s->Q, N, i, q);
    full_from5(s->H, N, i, h);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) dQ[a][b] = s->p.Gamma * h[a][b];
    if (hydro) {
      double W[3][3], S[3][3], u0[3];
      site_velocity(s, x, y, z, u0);
      for (int b = 0; b < 3; b++) {
        int e[3] = {0, 0, 0};
        e[b] = 1;
        double up[3], um[3];
        site_velocity(s, x + e[0], y + e[1], z + e[2], up);
        site_velocity(s, x - e[0], y - e[1], z - e[2], um);
        for (int a = 0; a < 3; a++) W[a][b] = 0.5 * (up[a] - um[a]);
        /* advective fluxes through the + and - faces along b */
        double phip[3][3], phim[3][3];
        face_flux(s, x, y, z, b, phip);
        face_flux(s, x - e[0], y - e[1], z - e[2], b, phim);
        for (int a = 0; a < 3; a++)
          for (int c = 0; c < 3; c++) dQ[a][c] -= phip[a][c] - phim[a][c];
      }
      corotation_full(s->p.xi, W, q, S);
      for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) dQ[a][c] += S[a][c];
    }
    double qn[3][3];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) qn[a][b] = q[a][b] + dQ[a][b];
    store5(s->Qn, N, i, qn);
  }
}

/* LB collision at fluid nodes: BGK with the forcing of Guo et al.
 * (half-force velocity); the velocity is stored for the next Q update. */
static void lb_collide(lco_sim* s) {
  long N = s->N;
  const double tau = s->p.tau;
  #pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) continue;
    double rho = 0.0, j[3] = {0, 0, 0}, F[3], u[3], feq[19];
    for (int k = 0; k < 19; k++) {
      double fk = s->f[k * N + i];
      rho += fk;
      for (int a = 0; a < 3; a++) j[a] += fk * CV[k][a];
    }
    for (int a = 0; a < 3; a++) {
      F[a] = s->F[a * N + i];
      u[a] = (j[a] + 0.5 * F[a]) / rho;
    }
    lco_feq(rho, u, feq);
    for (int k = 0; k < 19; k++) {
      double cu = CV[k][0] * u[0] + CV[k][1] * u[1] + CV[k][2] * u[2];
      double cF = CV[k][0] * F[0] + CV[k][1] * F[1] + CV[k][2] * F[2];
      double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
      double src = WT[k] * (3.0 * (cF - uF) + 9.0 * cu * cF);
      double fk = s->f[k * N + i];
      s->fstar[k * N + i] = fk - (fk - feq[k]) / tau + (1.0 - 0.5 / tau) * src;
    }
    for (int a = 0; a < 3; a++) s->u[a * N + i] = u[a];
  }
}

/* Push streaming with bounce-back on links (Sec. 2.2): a population whose
 * link ends on a solid node is reflected back into the fluid node with the
 * moving-wall correction -6 w_i rho0 c_i.u_b, u_b the rigid-body velocity at
 * the link midpoint; the momentum (2 f*_i - 6 w_i rho0 c_i.u_b) c_i goes to
 * the colloid. */
static void lb_stream(lco_sim* s, double Fb[][3], double Tb[][3]) {
  long N = s->N;
  #pragma omp parallel for schedule(static)
  for (long k = 0; k < 19 * N; k++) s->fn[k] = 0.0;
  #pragma omp parallel for schedule(static)
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) continue;
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    for (int k = 0; k < 19; k++) {
      long j = sidx(s, x + CV[k][0], y + CV[k][1], z + CV[k][2]);
      double fs = s->fstar[k * N + i];
      if (!s->solid[j]) {
        s->fn[k * N + j] = fs;
      } else {
        double r[3], ub[3];
        const lco_colloid* c = owner(s, j);
        rel_pos(s, c->pos, x + 0.5 * CV[k][0], y + 0.5 * CV[k][1], z + 0.5 * CV[k][2], r);
        rigid_vel(c, r, ub);
        double cub = CV[k][0] * ub[0] + CV[k][1] * ub[1] + CV[k][2] * ub[2];
        s->fn[opposite(k) * N + i] = fs - 6.0 * WT[k] * s->p.rho0 * cub;
      }
    }
  }
  for (int c = 0; c < LCO_MAX_COLLOIDS; c++)
    for (int a = 0; a < 3; a++) Fb[c][a] = Tb[c][a] = 0.0;
  if (!s->ncol) return;
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) continue;
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    for (int k = 1; k < 19; k++) {
      long j = sidx(s, x + CV[k][0], y + CV[k][1], z + CV[k][2]);
      if (!s->solid[j]) continue;
      double r[3], ub[3], dp[3], t[3];
      const int ic = s->solid[j] - 1;
      rel_pos(s, s->c[ic].pos, x + 0.5 * CV[k][0], y + 0.5 * CV[k][1], z + 0.5 * CV[k][2], r);
      rigid_vel(&s->c[ic], r, ub);
      double cub = CV[k][0] * ub[0] + CV[k][1] * ub[1] + CV[k][2] * ub[2];
      double m = 2.0 * s->fstar[k * N + i] - 6.0 * WT[k] * s->p.rho0 * cub;
      for (int a = 0; a < 3; a++) dp[a] = m * CV[k][a];
      cross(r, dp, t);
      for (int a = 0; a < 3; a++) { Fb[ic][a] += dp[a]; Tb[ic][a] += t[a]; }
    }
  }
}

/* Moving-boundary events for a moving colloid (Sec. 2.2): the centre
 * advances by v (prescribed, or the velocity just updated), nodes are
 * reclassified, a node that becomes
 * fluid receives equilibrium populations at rho0 and the local rigid-body
 * velocity and, for Q, the mean over its face neighbours that held fluid
 * both before and after the move (zero if there is none); a node that
 * becomes solid is dropped.  The momentum of removed and added fluid goes
 * to the colloid (added to Fe, Te). */
static void events(lco_sim* s, double* Qn, double Fe[][3], double Te[][3]) {
  for (int k = 0; k < LCO_MAX_COLLOIDS; k++)
    for (int a = 0; a < 3; a++) Fe[k][a] = Te[k][a] = 0.0;
  int moving = 0;
  for (int k = 0; k < s->ncol; k++) moving |= s->c[k].motion != LCO_FIXED;
  if (!moving) return;
  long N = s->N;
  int L[3] = {s->p.nx, s->p.ny, s->p.nz};
  double Rn[LCO_MAX_COLLOIDS][3];
  for (int k = 0; k < s->ncol; k++)
    for (int a = 0; a < 3; a++) {
      Rn[k][a] = s->c[k].pos[a];
      if (s->c[k].motion == LCO_FIXED) continue;
      Rn[k][a] += s->c[k].vel[a];
      if (Rn[k][a] >= L[a]) Rn[k][a] -= L[a];
      if (Rn[k][a] < 0.0) Rn[k][a] += L[a];
    }
  unsigned char* nsolid = (unsigned char*)malloc(N);
  for (long i = 0; i < N; i++) {
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    nsolid[i] = 0;
    for (int k = 0; k < s->ncol && !nsolid[i]; k++)
      if (inside(s, &s->c[k], Rn[k], x, y, z)) nsolid[i] = (unsigned char)(k + 1);
  }
  static const int E[6][3] = {{1,0,0},{-1,0,0},{0,1,0},{0,-1,0},{0,0,1},{0,0,-1}};
  for (long i = 0; i < N; i++) {
    int was = s->solid[i], now = nsolid[i];
    if (was == now) continue;
    if (was && now) { s->err = 1; continue; }   /* from one colloid into another: excluded by the gap */
    const int k = (was ? was : now) - 1;
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    double r[3], p[3] = {0, 0, 0}, t[3];
    rel_pos(s, Rn[k], x, y, z, r);
    if (was && !now) {
      double ub[3], feq[19];
      rigid_vel(&s->c[k], r, ub);
      if (s->p.hydro) {
        lco_feq(s->p.rho0, ub, feq);
        for (int q = 0; q < 19; q++) {
          s->fn[q * N + i] = feq[q];
          for (int a = 0; a < 3; a++) p[a] -= feq[q] * CV[q][a];
        }
        for (int a = 0; a < 3; a++) s->u[a * N + i] = ub[a];
      }
      double qm[3][3] = {{0}}, qk[3][3];
      int nf = 0;
      for (int q = 0; q < 6; q++) {
        long j = sidx(s, x + E[q][0], y + E[q][1], z + E[q][2]);
        if (s->solid[j] || nsolid[j]) continue;
        full_from5(Qn, N, j, qk);
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) qm[a][b] += qk[a][b];
        nf++;
      }
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) qm[a][b] = nf ? qm[a][b] / nf : 0.0;
      store5(Qn, N, i, qm);
    } else {
      if (s->p.hydro) {
        for (int q = 0; q < 19; q++) {
          for (int a = 0; a < 3; a++) p[a] += s->fn[q * N + i] * CV[q][a];
          s->fn[q * N + i] = 0.0;
        }
        for (int a = 0; a < 3; a++) s->u[a * N + i] = 0.0;
      }
    }
    cross(r, p, t);
    for (int a = 0; a < 3; a++) { Fe[k][a] += p[a]; Te[k][a] += t[a]; }
  }
  memcpy(s->solid, nsolid, N);
  for (int k = 0; k < s->ncol; k++)
    for (int a = 0; a < 3; a++) s->c[k].pos[a] = Rn[k][a];
  free(nsolid);
}

/* One time step in the order: ghost Q; H, P and the force from Q^n;
 * Q^{n+1} with u^{n-1}; LB collision with F^n storing u^n; streaming with
 * bounce-back; colloid events. */
static void step_once(lco_sim* s) {
  double Fs[LCO_MAX_COLLOIDS][3], Ts[LCO_MAX_COLLOIDS][3], Fb[LCO_MAX_COLLOIDS][3],
      Tb[LCO_MAX_COLLOIDS][3], Fe[LCO_MAX_COLLOIDS][3], Te[LCO_MAX_COLLOIDS][3];
  for (int k = 0; k < LCO_MAX_COLLOIDS; k++)
    for (int a = 0; a < 3; a++) Fs[k][a] = Ts[k][a] = Fb[k][a] = Tb[k][a] = 0.0;
  ghost_all(s, s->Q);
  compute_HP(s, s->Q, s->p.hydro);
  if (s->p.hydro) {
    compute_F(s);
    colloid_stress(s, Fs, Ts);
  }
  be_update(s);
  if (s->p.hydro) {
    lb_collide(s);
    lb_stream(s, Fb, Tb);
  }
  double M[LCO_MAX_COLLOIDS] = {0}, I[LCO_MAX_COLLOIDS] = {0};
  for (int c = 0; c < s->ncol; c++) {
    lco_colloid* cc = &s->c[c];
    if (cc->motion != LCO_FREE) continue;
    const double rc = cc->rho_c > 0.0 ? cc->rho_c : s->p.rho0;
    const double a = cc->a0;
    M[c] = 4.0 / 3.0 * acos(-1.0) * a * a * a * rc;
    I[c] = 0.4 * M[c] * a * a;
    for (int k = 0; k < 3; k++) {
      cc->vel[k] += (Fb[c][k] + Fs[c][k] + cc->fext[k]) / M[c];
      cc->omega[k] += (Tb[c][k] + Ts[c][k]) / I[c];
    }
  }
  events(s, s->Qn, Fe, Te);
  for (int c = 0; c < s->ncol; c++) {
    lco_colloid* cc = &s->c[c];
    if (cc->motion != LCO_FREE) continue;
    for (int k = 0; k < 3; k++) {
      cc->vel[k] += Fe[c][k] / M[c];
      cc->omega[k] += Te[c][k] / I[c];
    }
  }
  double* t = s->Q; s->Q = s->Qn; s->Qn = t;
  if (s->p.hydro) { t = s->f; s->f = s->fn; s->fn = t; }
  memset(s->force, 0, sizeof(s->force));
  for (int c = 0; c < s->ncol; c++)
    for (int a = 0; a < 3; a++) {
      s->force[c][a] = Fb[c][a] + Fe[c][a];
      s->force[c][3 + a] = Fs[c][a];
      s->force[c][6 + a] = Tb[c][a] + Te[c][a];
      s->force[c][9 + a] = Ts[c][a];
    }
  s->nstep++;
}

/* A step may start only with every pair of colloids at least
 * LCO_COLLOID_GAP apart (surface to surface); otherwise the step is refused
 * and the simulation stops (LCO_ESTATE). */
int lco_step(lco_sim* s, int nsteps) {
  if (!s || nsteps < 0) return LCO_EINVAL;
  for (int n = 0; n < nsteps; n++) {
    if (s->err || !separated(s, s->ncol, s->c)) {
      s->err = 1;
      return LCO_ESTATE;
    }
    step_once(s);
  }
  return s->err ? LCO_ESTATE : LCO_OK;
}

int lco_ghost(lco_sim* s, double* Q5_out) {
  if (!s) return LCO_EINVAL;
  ghost_all(s, s->Q);
  if (Q5_out) memcpy(Q5_out, s->Q, sizeof(double) * 5 * s->N);
  return LCO_OK;
}

int lco_fields(lco_sim* s, double* H5, double* P9, double* F3) {
  if (!s) return LCO_EINVAL;
  ghost_all(s, s->Q);
  compute_HP(s, s->Q, 1);
  compute_F(s);
  if (H5) memcpy(H5, s->H, sizeof(double) * 5 * s->N);
  if (P9) memcpy(P9, s->P, sizeof(double) * 9 * s->N);
  if (F3) memcpy(F3, s->F, sizeof(double) * 3 * s->N);
  return LCO_OK;
}

/* Free energy of the discrete model:
 * F_d = sum over fluid nodes of [bulk + 2 K q0 Q:(e D0 Q) + 2 K q0^2 |Q|^2]
 *     + K/2 sum over lattice faces with at least one fluid end |dQ|^2
 *     + W/2 sum over solid-fluid faces |Qs - Q^0|^2 (finite W only).
 * Its gradient is -H where the lattice H is exact (no colloid, or q0 = 0
 * with fixed anchoring). */
static double free_energy(lco_sim* s) {
  long N = s->N;
  ghost_all(s, s->Q);
  long double Fd = 0.0L;   /* extended-precision accumulator */
  const double K = s->p.K, q0 = s->p.q0;

  for (long i = 0; i < N; i++) {
    int x, y, z;
    scoord(s, i, &x, &y, &z);
    if (!s->solid[i]) {
      double q[3][3], dq[3][3][3], lap[3][3];
      stencil(s, s->Q, x, y, z, q, dq, lap);
      Fd += bulk_energy(&s->p, q) + 2.0 * K * q0 * chiral_cross(q, dq) +
            2.0 * K * q0 * q0 * frob2(q);
    }
    double qa[3][3];
    full_from5(s->Q, N, i, qa);
    for (int b = 0; b < 3; b++) {
      int e[3] = {0, 0, 0};
      e[b] = 1;
      long j = sidx(s, x + e[0], y + e[1], z + e[2]);
      if (s->solid[i] && s->solid[j]) continue;
      double qb[3][3], d[3][3];
      full_from5(s->Q, N, j, qb);
      for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) d[a][c] = qb[a][c] - qa[a][c];
      Fd += 0.5 * K * frob2(d);
      if (!s->solid[i] != !s->solid[j]) {
        long js = s->solid[i] ? i : j;
        const lco_colloid* cl = owner(s, js);
        if (cl->anchoring == LCO_ANCHOR_NONE || isinf(cl->W)) continue;
        double qs[3][3], qz[3][3];
        full_from5(s->Q, N, js, qs);
        full_from5(s->Q0, N, js, qz);
        for (int a = 0; a < 3; a++)
          for (int c = 0; c < 3; c++) d[a][c] = qs[a][c] - qz[a][c];
        Fd += 0.5 * cl->W * frob2(d);
      }
    }
  }
  return (double)Fd;
}

int lco_get_diag(lco_sim* s, double out[6]) {
  if (!s || !out) return LCO_EINVAL;
  long N = s->N;
  out[0] = free_energy(s);
  /* extended-precision accumulators: sums of ~1e6 near-equal terms */
  long double mass = 0.0L, mom[3] = {0, 0, 0};
  double umax = 0.0;
  for (long i = 0; i < N; i++) {
    if (s->solid[i]) continue;
    for (int k = 0; k < 19; k++) {
      double fk = s->f[k * N + i];
      mass += fk;
      for (int a = 0; a < 3; a++) mom[a] += fk * CV[k][a];
    }
    double u2 = 0.0;
    for (int a = 0; a < 3; a++) u2 += s->u[a * N + i] * s->u[a * N + i];
    if (sqrt(u2) > umax) umax = sqrt(u2);
  }
  out[1] = (double)mass;
  out[2] = (double)mom[0]; out[3] = (double)mom[1]; out[4] = (double)mom[2];
  out[5] = umax;
  return LCO_OK;
}
