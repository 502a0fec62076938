/*
 * lco.h -- plain FP64 CPU oracle of the hybrid lattice-Boltzmann /
 * finite-difference step for colloids in a liquid crystal
 * (Lintuvuori, Marenduzzo, Stratford, Cates, "Colloids in liquid crystals:
 * a lattice Boltzmann study", Soft Matter 2011).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the definition of "correct"
 * against which the HIP library is checked.  It shares no code, header,
 * table or helper with the HIP path.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.
 *
 * Conventions (all FP64, lattice units dx = dt = 1):
 *   - site index  s = x + nx*(y + ny*z), periodic in all three axes;
 *   - arrays are structure-of-arrays [component][z][y][x];
 *   - Q is stored as five components (xx, xy, xz, yy, yz), Qzz = -Qxx-Qyy
 *     (traceless symmetric, Sec. 2.1);
 *   - D3Q19 order: 0 rest; 1..6 = +x -x +y -y +z -z; 7..18 = (+1,+1,0),
 *     (-1,-1,0), (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1), (+1,0,-1),
 *     (-1,0,+1), (0,+1,+1), (0,-1,-1), (0,+1,-1), (0,-1,+1): opposite
 *     directions are adjacent pairs.
 *   - colloid force layout (12 doubles): F_bbl[3], F_stress[3], T_bbl[3],
 *     T_stress[3]; momentum exchanged by moving-boundary events is added to
 *     F_bbl / T_bbl.
 */
#ifndef LCO_H
#define LCO_H

#ifdef __cplusplus
extern "C" {
#endif

enum { LCO_OK = 0, LCO_EINVAL = 1, LCO_ENOMEM = 2, LCO_ESTATE = 5 };
enum { LCO_ANCHOR_NONE = 0, LCO_ANCHOR_NORMAL = 1, LCO_ANCHOR_PLANAR = 2 };
enum { LCO_FIXED = 0, LCO_PRESCRIBED = 1, LCO_FREE = 2 };
/* Colloids per box, and the least surface-to-surface distance two of them
 * may have at the start of a step (no lubrication; then no fluid node has
 * links or faces to two colloids). */
enum { LCO_MAX_COLLOIDS = 16 };
#define LCO_COLLOID_GAP 3.0

typedef struct lco_params {
  int nx, ny, nz;
  int hydro;              /* 1: full coupled step; 0: u = 0, dQ/dt = Gamma H */
  double tau;             /* BGK relaxation time, viscosity (tau - 1/2)/3 */
  double rho0;            /* reference density (initial fluid, BBL, new fluid) */
  double A0, gamma, K, q0, xi, Gamma;   /* Eq. (1), Eq. (2), Eq. (4) */
  double body_force[3];   /* uniform force density on fluid nodes */
  /* Variants of two readings of Sec. 2.2 (0 selects the default):
   * advection: order of the upwind face values of the advective flux,
   *   1 (first order, default), 2 (second-order upwind: linear
   *   extrapolation from the two upwind nodes), 3 (third-order
   *   upwind-biased: two upwind nodes and the downwind one); a face whose
   *   wider stencil reaches a solid node uses first order;
   * stencil: finite-difference stencil of the Q derivatives, 7 (central
   *   first derivatives and compact Laplacian, default) or 27 (isotropic
   *   27-point gradient and Laplacian; ghost Q then goes to every solid node
   *   with a fluid node among its 26 neighbours, from their mean). */
  int advection;
  int stencil;
} lco_params;

typedef struct lco_colloid {
  int present;            /* 0: no colloid in the box */
  int motion;             /* LCO_FIXED, LCO_PRESCRIBED (R += v every step) or
                             LCO_FREE (v and omega follow the force, below) */
  int anchoring;          /* LCO_ANCHOR_NONE / NORMAL / PLANAR (Sec. 2.2) */
  int pad_;
  double pos[3];          /* centre R */
  double a0;              /* nominal radius (Sec. 2.2) */
  double vel[3];          /* v */
  double omega[3];        /* angular velocity */
  double S0;              /* surface order of Eq. for Q^0 (Sec. 2.2) */
  double W;               /* anchoring strength; +inf = fixed Q^0 */
  /* LCO_FREE only.  The paper updates the particle velocity from the summed
   * link and stress force, and the position from the velocity, in a
   * molecular-dynamics-like step without giving it; the reading taken is
   * explicit Euler at the end of each step:
   *   V += (F + fext)/M, omega += T/I with M = 4/3 pi a0^3 rho_c and
   *   I = 2/5 M a0^2, then R += V (the new V), then the moving-boundary
   *   events of the move (with the new V, omega), whose momentum is added
   *   to V and omega as well (F, T: the step's link and stress sums). */
  double fext[3];         /* constant external force on the colloid */
  double rho_c;           /* colloid density; <= 0 means rho0 */
} lco_colloid;

typedef struct lco_sim lco_sim;

int  lco_create(const lco_params* p, lco_sim** out);
void lco_destroy(lco_sim* s);
/* Colloids of the box.  lco_set_colloids replaces them with n (0..16), all
 * present and pairwise at least LCO_COLLOID_GAP apart surface to surface
 * (else LCO_EINVAL); lco_set_colloid sets the one colloid c (none if
 * c->present is 0).  Getters: colloid 0, the number, the first n. */
int  lco_set_colloids(lco_sim* s, int n, const lco_colloid* c);
int  lco_set_colloid(lco_sim* s, const lco_colloid* c);
int  lco_get_colloid(const lco_sim* s, lco_colloid* c);
int  lco_num_colloids(const lco_sim* s);
int  lco_get_colloids(const lco_sim* s, int n, lco_colloid* c);
int  lco_set_Q(lco_sim* s, const double* Q5);      /* 5*N */
int  lco_set_f(lco_sim* s, const double* f19);     /* 19*N, pre-collision */
int  lco_set_u(lco_sim* s, const double* u3);      /* 3*N lagged velocity */
int  lco_get_Q(const lco_sim* s, double* Q5);
int  lco_get_f(const lco_sim* s, double* f19);
int  lco_get_u(const lco_sim* s, double* u3);
int  lco_get_solid(const lco_sim* s, unsigned char* solid);
/* LCO_ESTATE: a step would start with two colloids closer than the gap
 * (the simulation then stays stopped). */
int  lco_step(lco_sim* s, int nsteps);
/* Force and torque of the last step, 12 doubles per colloid: colloid 0 /
 * the first n colloids. */
int  lco_get_force(const lco_sim* s, double out[12]);
int  lco_get_forces(const lco_sim* s, int n, double* out);
long lco_get_nstep(const lco_sim* s);
/* F_d, mass, momentum[3], max|u|  (Q ghost values refreshed first) */
int  lco_get_diag(lco_sim* s, double out[6]);

/* Pieces exposed for the pins (all refresh ghost Q from the current Q). */
int  lco_fields(lco_sim* s, double* H5, double* P9, double* F3);
int  lco_ghost(lco_sim* s, double* Q5_out);        /* Q with ghost values */
void lco_bulk_field(const lco_params* p, const double Q5[5], double H5[5]);
void lco_corotation(double xi, const double W9[9], const double Q5[5], double S5[5]);
void lco_feq(double rho, const double u[3], double feq[19]);
void lco_lattice(int c[19][3], double w[19]);
int  lco_principal_axis(const double A9[9], double n[3], double* lam);
/* single-site Beris-Edwards integration under a fixed velocity gradient
 * W9 (row-major W_ab = d_b u_a), bulk field only; Q5 is updated in place */
void lco_single_site(const lco_params* p, const double W9[9], long nsteps, double Q5[5]);

#ifdef __cplusplus
}
#endif
#endif
