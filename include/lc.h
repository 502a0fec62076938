/*
 * lc.h -- C ABI of the MI355X (gfx950) library for the hybrid lattice
 * Boltzmann / finite-difference time step of Lintuvuori, Marenduzzo,
 * Stratford and Cates, "Colloids in liquid crystals: a lattice Boltzmann
 * study" (Soft Matter 2011).
 *
 * One step couples D3Q19 collide-and-stream for the fluid (Sec. 2.1,
 * Navier-Stokes equation; Sec. 2.2, bounce-back on links) to a
 * finite-difference Beris-Edwards update of the Q tensor (Eq. 1 free
 * energy, Eq. 2 dynamics, Eq. 4 stress) around colloids with normal or
 * planar anchoring (Sec. 2.2, equation for Q^0): one per box, or several
 * (the colloid-colloid interactions of the paper's outlook, Introduction and
 * Sec. 3.2).
 *
 * Conventions shared by every call
 *  - Return value: LC_OK (0) or a positive lc_status code.  Nothing throws
 *    across the ABI; lc_last_error(ctx) returns a message for the last
 *    failure on that context (NULL ctx: the last failure of lc_create*).
 *  - Lattice units dx = dt = 1.  Box b has nx*ny*nz sites, periodic in all
 *    axes; site index s = x + nx*(y + ny*z).
 *  - Host arrays are FP64, structure-of-arrays [component][z][y][x], x
 *    fastest.  Q has 5 components (xx, xy, xz, yy, yz), Qzz = -Qxx-Qyy.
 *  - D3Q19 order: 0 rest; 1..6 = +x -x +y -y +z -z; 7..18 = (+1,+1,0),
 *    (-1,-1,0), (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1), (+1,0,-1),
 *    (-1,0,+1), (0,+1,+1), (0,-1,-1), (0,+1,-1), (0,-1,+1).
 *  - The context is opaque and owned by the library.  Caller arrays are
 *    copied in or out during the call and never retained.
 *  - All device work is queued on the HIP stream given at creation (NULL =
 *    the default stream).  lc_step is asynchronous; getters synchronise the
 *    stream.  Use one context from one host thread at a time.
 *  - Device state: f (19 populations) and Q (5) are double-buffered, the
 *    velocity u of the last collision (3) too.  Sizes are given by
 *    lc_buffer_bytes; the library allocates them with hipMalloc unless the
 *    caller binds its own device memory with lc_bind_buffers.
 */
#ifndef LC_H
#define LC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lc_status {
  LC_OK = 0,
  LC_EINVAL = 1,     /* bad argument or parameter */
  LC_ENOMEM = 2,     /* device or host allocation failed */
  LC_EDEVICE = 3,    /* a HIP call failed */
  LC_ENUMERIC = 4,   /* a step produced a non-finite value or |u| >= 0.3 */
  LC_ESTATE = 5      /* call not valid in the current state, or two colloids
                        started a step closer than LC_COLLOID_GAP */
} lc_status;

enum { LC_FP32 = 0, LC_FP64 = 1 };
enum { LC_ANCHOR_NONE = 0, LC_ANCHOR_NORMAL = 1, LC_ANCHOR_PLANAR = 2 };
enum { LC_FIXED = 0, LC_PRESCRIBED = 1, LC_FREE = 2 };

/* Per-box parameters.  Material constants follow Eq. (1), Eq. (2) and
 * Eq. (4): A0, gamma (bulk), K (one elastic constant), q0 = 2 pi / pitch,
 * xi (flow aligning), Gamma (rotational diffusion).  tau is the BGK
 * relaxation time (viscosity (tau - 1/2)/3), rho0 the reference density.
 * hydro = 0 switches the fluid off (u = 0, dQ/dt = Gamma H).  precision
 * must be equal in all boxes of a context.  body_force is a uniform force
 * density on fluid nodes (zero for the paper's runs). */
typedef struct lc_params {
  int nx, ny, nz;
  int precision;          /* LC_FP32 or LC_FP64 */
  int hydro;
  int pad_;
  double tau, rho0;
  double A0, gamma, K, q0, xi, Gamma;
  double body_force[3];
  /* Variants of two readings of Sec. 2.2 (0 selects the default; both need
   * a 3D-tile shape of the fused kernel, which a context with a variant box
   * gets by default):
   * advection: order of the upwind face values of the advective flux of Q:
   *   1 first order (default), 2 second-order upwind (3 Q_up - Q_upup)/2,
   *   3 third-order upwind-biased (2 Q_down + 5 Q_up - Q_upup)/6; a face whose
   *   wider stencil reaches a solid node takes the first-order value;
   * stencil: 7 (central first derivatives and compact Laplacian, default)
   *   or 27 (isotropic 27-point gradient and Laplacian; ghost Q then goes to
   *   every solid node with a fluid node among its 26 neighbours, from the
   *   mean of those). */
  int advection;
  int stencil;
} lc_params;

/* One spherical colloid (Sec. 2.2): nodes with |x - R|^2 < a0^2 are solid.
 * motion LC_FIXED keeps R; LC_PRESCRIBED advances R by vel every step with
 * the moving-boundary events of Sec. 2.2; LC_FREE lets vel and omega follow
 * the force (the paper's molecular-dynamics-like step, which it does not
 * spell out; the reading taken is explicit Euler at the end of each step:
 * vel += (F_bbl + F_stress + fext)/M, omega += (T_bbl + T_stress)/I with
 * M = 4/3 pi a0^3 rho_c and I = 2/5 M a0^2, then R += vel (the new vel),
 * then the events of that move, whose momentum is added to vel and omega
 * too).  Anchoring sets Q at boundary
 * solid nodes to Q^0 = S0 (n0 n0 - I/3) with n0 the surface normal (NORMAL)
 * or the projection of the neighbouring director on the tangent plane
 * (PLANAR); W = +INFINITY is the paper's fixed value, a finite W blends
 * (K Qbar + W Q^0)/(K + W) with Qbar the mean of the fluid face
 * neighbours; NONE copies Qbar. */
typedef struct lc_colloid {
  int present;            /* 0: no colloid in the box */
  int motion;             /* LC_FIXED or LC_PRESCRIBED */
  int anchoring;          /* LC_ANCHOR_* */
  int pad_;
  double pos[3];
  double a0;
  double vel[3];
  double omega[3];
  double S0;
  double W;
  double fext[3];         /* LC_FREE: constant external force on the colloid */
  double rho_c;           /* LC_FREE: colloid density (<= 0: the fluid's rho0) */
} lc_colloid;

/* Diagnostics of one box: discrete free energy (bulk + chiral terms at
 * fluid nodes, K/2 |dQ|^2 over faces with a fluid end, W/2 |Qs - Q^0|^2
 * over solid-fluid faces), fluid mass and momentum of the pre-collision
 * populations, and max |u| of the last collision. */
typedef struct lc_diag {
  double free_energy;
  double mass;
  double momentum[3];
  double umax;
} lc_diag;

typedef struct lc_ctx lc_ctx;

/* Create a context for one box / for nbox independent boxes stepped
 * together (p points to nbox parameter sets).  The fluid starts at rest,
 * f = w_i rho0; Q = 0 until lc_set_Q; no colloid until lc_set_colloid.
 * hip_stream is a hipStream_t (or NULL).  Box edges must be >= 8. */
int lc_create(const lc_params* p, void* hip_stream, lc_ctx** out);
int lc_create_batch(int nbox, const lc_params* p, void* hip_stream, lc_ctx** out);
void lc_destroy(lc_ctx* ctx);
const char* lc_last_error(const lc_ctx* ctx);

/* Device buffer sizes in bytes: out[0] = one f buffer (19 x sites),
 * out[1] = one Q buffer (5 x sites), out[2] = one u buffer (3 x sites),
 * for all boxes together, in the context's precision. */
int lc_buffer_bytes(const lc_ctx* ctx, size_t out[3]);
/* Use caller-owned device memory (e.g. torch tensors) for the two f, two Q
 * and two u buffers; the library frees its own copies and copies their
 * current contents over.  The caller keeps the memory alive until
 * lc_destroy.  Pointers must be 256-byte aligned. */
int lc_bind_buffers(lc_ctx* ctx, void* f0, void* f1, void* Q0, void* Q1, void* u0, void* u1);

/* Colloids of box `box` (Sec. 2.2).  A box holds 0 to LC_MAX_COLLOIDS
 * colloids whose surfaces are at least LC_COLLOID_GAP lattice units apart
 * (minimum image) at the start of every step: then no fluid node has links
 * or faces to two colloids (no lubrication).  A step that starts with two
 * colloids closer than that stops the context: the next getter returns
 * LC_ESTATE.  Each colloid is rejected if it does not fit (2 a0 + 4 > min box
 * edge) or a0 <= 1.  A box with several colloids runs on a 3D-tile shape (a
 * context on a marching shape is moved to the first 3D tile).
 *  lc_set_colloids: replaces the box's colloids with c[0..n-1] (all with
 *    present = 1); colloid k keeps its force history if the box had a k-th
 *    colloid before.  On an error the box keeps its colloids.
 *  lc_set_colloid:  the one colloid c, or none if c->present is 0.
 *  lc_num_colloids: the box's number of colloids (-1 on a bad box).
 *  lc_get_colloids: the first n colloids, at their current positions (and a
 *    free colloid's current velocities); lc_get_colloid: colloid 0, or
 *    present = 0 if there is none. */
#define LC_MAX_COLLOIDS 16
#define LC_COLLOID_GAP 3.0
int lc_set_colloids(lc_ctx* ctx, int box, int n, const lc_colloid* c);
int lc_set_colloid(lc_ctx* ctx, int box, const lc_colloid* c);
int lc_num_colloids(lc_ctx* ctx, int box);
int lc_get_colloids(lc_ctx* ctx, int box, int n, lc_colloid* c);
int lc_get_colloid(lc_ctx* ctx, int box, lc_colloid* c);

/* Whole-box field transfers (FP64 host arrays, see conventions). */
int lc_set_Q(lc_ctx* ctx, int box, const double* Q5);
int lc_set_f(lc_ctx* ctx, int box, const double* f19);
int lc_set_u(lc_ctx* ctx, int box, const double* u3);
int lc_get_Q(lc_ctx* ctx, int box, double* Q5);
int lc_get_f(lc_ctx* ctx, int box, double* f19);   /* pre-collision f^n */
int lc_get_u(lc_ctx* ctx, int box, double* u3);    /* velocity of the last collision */

/* Checkpoint and restart (the paper describes none; this is a plain save of
 * the evolving state).  The state holds both buffers of f, Q and u bit for
 * bit in the context's precision (a step leaves solid nodes untouched, so
 * the second buffer is kept too), every colloid at its current position,
 * the step count, the last-step forces and the force-history rings.  Material parameters are not part of it: a context takes its own
 * lc_params.  A context created with the same lc_params (and precision)
 * that is given the state continues exactly as the saved one would have:
 * every later getter returns the same bits.
 * The format is the library's own: a header (magic "LCSTATE2", version,
 * precision, box count, sites, step count, colloid count), one record per
 * box (shape, colloid count), one per colloid (history count, colloid),
 * then raw arrays in native byte order.
 *  lc_state_bytes: the size of this context's state in bytes.
 *  lc_get_state:   writes the state into caller-owned host memory buf of
 *                  `bytes` >= lc_state_bytes; synchronises the stream;
 *                  LC_ENUMERIC if a step was flagged.
 *  lc_set_state:   reads a state written by lc_get_state (its colloids
 *                  replace the context's).  LC_EINVAL if buf is NULL or
 *                  short, or its precision, box count, box shapes or
 *                  colloids do not fit this context; the context is then
 *                  unchanged.  Clears the error flags. */
int lc_state_bytes(const lc_ctx* ctx, size_t* out);
int lc_get_state(lc_ctx* ctx, void* buf, size_t bytes);
int lc_set_state(lc_ctx* ctx, const void* buf, size_t bytes);

/* Advance every box by nsteps steps.  Each step: one fused pass per site
 * (molecular field H, stress P, force = discrete divergence of P,
 * Beris-Edwards update of Q, LB collision with that force, push streaming
 * with bounce-back on links and the colloid's force/torque sums), then the
 * moving-boundary events, the ghost Q at boundary solid nodes (anchoring)
 * of the new Q for the next step, and the colloid update.  Before the first
 * step after a change from the host the ghost Q are formed once.
 * Asynchronous; replays a captured HIP graph when graphs are enabled. */
int lc_step(lc_ctx* ctx, int nsteps);
int lc_sync(lc_ctx* ctx);       /* wait for the stream; LC_ENUMERIC if flagged */
/* Capture the step graph now (graphs on and none captured for the current
 * layout), so that the next lc_step does not pay for the capture.  Queues
 * no work; a no-op when graphs are off or already captured. */
int lc_prepare(lc_ctx* ctx);
long lc_get_nstep(lc_ctx* ctx); /* steps taken (host count) */

/* Colloid force and torque of the last step: F_bbl[3], F_stress[3],
 * T_bbl[3], T_stress[3] (Sec. 2.2: link momentum from bounce-back;
 * F^coll = sum of P.s over solid-fluid faces), torques about the colloid's
 * centre.  Momentum of fluid removed or added by moving-boundary events is
 * included in F_bbl and T_bbl.  lc_get_colloid_force: colloid k of the box;
 * lc_get_force: colloid 0 (zeros for a box without colloids). */
int lc_get_colloid_force(lc_ctx* ctx, int box, int k, double out[12]);
int lc_get_force(lc_ctx* ctx, int box, double out[12]);
/* The last nsteps forces (oldest first), 12 doubles each, of colloid k /
 * colloid 0 (zeros for a box without colloids); nsteps must not exceed the
 * steps the colloid has taken (lc_get_force_history: the context's steps)
 * nor the history capacity (lc_history_capacity). */
int lc_get_colloid_force_history(lc_ctx* ctx, int box, int k, int nsteps, double* out);
int lc_get_force_history(lc_ctx* ctx, int box, int nsteps, double* out);
int lc_history_capacity(const lc_ctx* ctx);

/* Solid map of a box from the library's own sphere test (Sec. 2.2):
 * id[s] = 1 + the index of the colloid holding site s, 0 at fluid sites
 * (caller-owned, nx*ny*nz bytes, x fastest).  Synchronises the stream. */
int lc_get_solid(lc_ctx* ctx, int box, unsigned char* id);

int lc_get_diag(lc_ctx* ctx, int box, lc_diag* out);

/* lc_get_diag for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same summation order, so the same bits, but the
 * per-block partials and totals live in a static device array of 1 MiB per
 * GPU, held until the process ends, instead of memory the context
 * allocates; the call allocates nothing.  Boxes of more than 5,591,040
 * sites (21,840 blocks of 256) do not fit: LC_EINVAL with a message.  Every
 * call on one GPU uses that GPU's one array, so calls that overlap on one
 * GPU (several host threads, or contexts on different streams) race and
 * must be serialised by the caller.  Synchronises the context's stream. */
int lc_get_diag_noalloc(lc_ctx* ctx, int box, lc_diag* out);

/* Defect sites (Sec. 3.1 footnote: order-parameter isosurface): mask[s] = 1
 * where a fluid site has (3/2) lambda_max(Q) < threshold; count_out gets
 * the number of such sites.  mask may be NULL. */
int lc_defects(lc_ctx* ctx, int box, double threshold, unsigned char* mask, long* count_out);

/* Execution controls.  Tile shapes are the fused kernel's block shapes:
 * every shape does the same per-site arithmetic, and results of different
 * shapes agree to rounding (the stress sums are grouped differently).  For
 * one shape the bits do not depend on how a box's planes are split into
 * work items, on the other boxes of the context or on graphs.
 * lc_num_tiles / lc_tile_shape list the shapes for the context's
 * precision, lc_set_tile picks one.  Graphs capture repeated steps in a
 * HIP graph (default on). */
int lc_num_tiles(const lc_ctx* ctx);
int lc_tile_shape(const lc_ctx* ctx, int id, int out[3]);
int lc_set_tile(lc_ctx* ctx, int id);
int lc_get_tile(const lc_ctx* ctx);
int lc_use_graph(lc_ctx* ctx, int enable);

/* Launch geometry of the fused kernel for the current tile: blocks per
 * step and threads per block. */
int lc_launch_info(const lc_ctx* ctx, long out[2]);

/* Run nsteps steps without graphs, with start/stop HIP events carried by
 * fused-kernel dispatches (hipExtLaunchKernel: no separate event commands
 * between the kernels) and events on the context's stream around the whole
 * run.  A dispatch that carries events adds about 6 us between kernels on
 * MI355X, so only every s-th dispatch does, s = ceil(nsteps / 64): at most
 * 64 timed dispatches spread evenly over the run.  out[0] = mean
 * fused-kernel time of the timed dispatches (ms), out[1] = mean time per
 * step (ms), out[2] = total (ms).  Synchronises the stream. */
int lc_time_kernel(lc_ctx* ctx, int nsteps, double out[3]);

#ifdef __cplusplus
}
#endif
#endif
