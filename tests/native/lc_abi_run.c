/*
 * lc_abi_run.c -- drives the library through include/lc.h alone (plain C,
 * no HIP code, no Python): contexts in both precisions, one and several
 * colloids, the variants, batches, tile changes, graphs on and off,
 * checkpoints, diagnostics, defects, the allocation-free diagnostics call,
 * timing, and the documented error returns.  Exits 0 when every check
 * holds; prints the failing check otherwise.
 *
 * Built by tests/test_native_gpu.py against liblc.so; built with clang's
 * address and undefined-behaviour sanitizers against liblc_hostsan.so (the
 * library's host code instrumented the same way) it runs the library's
 * host code under those sanitizers without preloading anything.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lc.h"

#define LC_TEST_PI 3.14159265358979323846

static int failures = 0;

#define CHECK(cond, ...)                                       \
  do {                                                         \
    if (!(cond)) {                                             \
      fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);     \
      fprintf(stderr, __VA_ARGS__);                            \
      fprintf(stderr, "\n");                                   \
      failures++;                                              \
    }                                                          \
  } while (0)

#define OK(call, ctx)                                                                               \
  do {                                                                                              \
    int rc_ = (call);                                                                               \
    if (rc_ != LC_OK) {                                                                             \
      fprintf(stderr, "FAIL %s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #call, rc_,                 \
              lc_last_error(ctx) ? lc_last_error(ctx) : "");                                        \
      exit(1);                                                                                      \
    }                                                                                               \
  } while (0)

static lc_params material(int n, int precision, double q0) {
  lc_params p;
  memset(&p, 0, sizeof(p));
  p.nx = p.ny = p.nz = n;
  p.precision = precision;
  p.hydro = 1;
  p.tau = 1.0;
  p.rho0 = 1.0;
  p.A0 = 0.01;
  p.gamma = 3.0;
  p.K = 0.01;
  p.q0 = q0;
  p.xi = 0.7;
  p.Gamma = 0.5;
  return p;
}

static lc_colloid colloid(double x, double y, double z, double a0, int motion, int anchoring) {
  lc_colloid c;
  memset(&c, 0, sizeof(c));
  c.present = 1;
  c.motion = motion;
  c.anchoring = anchoring;
  c.pos[0] = x;
  c.pos[1] = y;
  c.pos[2] = z;
  c.a0 = a0;
  c.S0 = 0.5;
  c.W = INFINITY;
  return c;
}

/* uniaxial Q = S (n n - I/3) with a director tilted along z by angle k z */
static double* helix(int nx, int ny, int nz, double S, double k) {
  const long N = (long)nx * ny * nz;
  double* Q = (double*)malloc(sizeof(double) * 5 * N);
  for (int z = 0; z < nz; z++)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        const long s = x + (long)nx * (y + (long)ny * z);
        const double n[3] = {cos(k * z) * 0.9, sin(k * z) * 0.9, 0.43588989435406733};
        Q[0 * N + s] = S * (n[0] * n[0] - 1.0 / 3.0);
        Q[1 * N + s] = S * n[0] * n[1];
        Q[2 * N + s] = S * n[0] * n[2];
        Q[3 * N + s] = S * (n[1] * n[1] - 1.0 / 3.0);
        Q[4 * N + s] = S * n[1] * n[2];
      }
  return Q;
}

static int all_finite(const double* a, long n) {
  for (long i = 0; i < n; i++)
    if (!isfinite(a[i])) return 0;
  return 1;
}

/* One box, one colloid: stepping, getters, diagnostics, checkpoint. */
static void single_box(int precision) {
  const int n = 32;
  const long N = (long)n * n * n;
  lc_params p = material(n, precision, 2 * LC_TEST_PI / 16);
  lc_ctx* c = NULL;
  OK(lc_create(&p, NULL, &c), NULL);
  lc_colloid k = colloid(15.3, 16.2, 15.8, 5.0, LC_PRESCRIBED, LC_ANCHOR_NORMAL);
  k.vel[0] = 0.02;
  k.W = 0.02;
  OK(lc_set_colloid(c, 0, &k), c);
  double* Q0 = helix(n, n, n, 0.3, 2 * LC_TEST_PI / 16);
  OK(lc_set_Q(c, 0, Q0), c);
  OK(lc_prepare(c), c);
  OK(lc_step(c, 20), c);
  OK(lc_sync(c), c);
  CHECK(lc_get_nstep(c) == 20, "nstep %ld", lc_get_nstep(c));

  double* Q = (double*)malloc(sizeof(double) * 5 * N);
  double* f = (double*)malloc(sizeof(double) * 19 * N);
  double* u = (double*)malloc(sizeof(double) * 3 * N);
  OK(lc_get_Q(c, 0, Q), c);
  OK(lc_get_f(c, 0, f), c);
  OK(lc_get_u(c, 0, u), c);
  CHECK(all_finite(Q, 5 * N) && all_finite(f, 19 * N) && all_finite(u, 3 * N), "non-finite field");

  double F[12], H[20 * 12];
  OK(lc_get_force(c, 0, F), c);
  OK(lc_get_force_history(c, 0, 20, H), c);
  CHECK(memcmp(F, H + 19 * 12, sizeof(F)) == 0, "last history entry differs from the force");
  CHECK(lc_get_force_history(c, 0, 21, H) == LC_EINVAL, "history beyond the steps taken accepted");

  lc_diag d1, d2;
  OK(lc_get_diag(c, 0, &d1), c);
  OK(lc_get_diag_noalloc(c, 0, &d2), c);
  CHECK(memcmp(&d1, &d2, sizeof(d1)) == 0, "noalloc diagnostics differ");
  CHECK(d1.mass > 0.9 * N && d1.mass < N, "mass %g", d1.mass);

  unsigned char* solid = (unsigned char*)malloc(N);
  OK(lc_get_solid(c, 0, solid), c);
  long ns = 0;
  for (long s = 0; s < N; s++) ns += solid[s] != 0;
  CHECK(ns > 400 && ns < 600, "solid nodes %ld for a0 = 5", ns);
  long ndef = -1;
  OK(lc_defects(c, 0, 0.2, solid, &ndef), c);
  CHECK(ndef >= 0 && ndef < N, "defects %ld", ndef);

  /* checkpoint: a second context continues bit for bit */
  size_t bytes = 0;
  OK(lc_state_bytes(c, &bytes), c);
  void* st = malloc(bytes);
  OK(lc_get_state(c, st, bytes), c);
  lc_ctx* c2 = NULL;
  OK(lc_create(&p, NULL, &c2), NULL);
  CHECK(lc_set_state(c2, st, bytes - 1) == LC_EINVAL, "short state accepted");
  OK(lc_set_state(c2, st, bytes), c2);
  OK(lc_step(c, 7), c);
  OK(lc_step(c2, 7), c2);
  double* Q2 = (double*)malloc(sizeof(double) * 5 * N);
  OK(lc_get_Q(c, 0, Q), c);
  OK(lc_get_Q(c2, 0, Q2), c2);
  CHECK(memcmp(Q, Q2, sizeof(double) * 5 * N) == 0, "restarted context differs");

  /* graphs off, then timing */
  OK(lc_use_graph(c, 0), c);
  OK(lc_step(c, 3), c);
  double t[3];
  OK(lc_time_kernel(c, 8, t), c);
  CHECK(t[0] > 0 && t[1] >= t[0] && t[2] > 0, "times %g %g %g", t[0], t[1], t[2]);
  long li[2];
  OK(lc_launch_info(c, li), c);
  CHECK(li[0] > 0 && li[1] > 0, "launch info %ld %ld", li[0], li[1]);

  /* error returns */
  CHECK(lc_get_Q(c, 1, Q) == LC_EINVAL, "box 1 of a one-box context accepted");
  CHECK(lc_get_Q(c, 0, NULL) == LC_EINVAL, "NULL array accepted");
  CHECK(lc_step(c, -1) == LC_EINVAL, "negative step count accepted");
  lc_colloid big = colloid(16, 16, 16, 15.0, LC_FIXED, LC_ANCHOR_NORMAL);
  CHECK(lc_set_colloid(c, 0, &big) == LC_EINVAL, "colloid larger than the box accepted");
  CHECK(lc_last_error(c) != NULL, "no message after an error");

  free(st);
  free(Q0);
  free(Q);
  free(Q2);
  free(f);
  free(u);
  free(solid);
  lc_destroy(c2);
  lc_destroy(c);
}

/* Several colloids with the variants (3D tile), free motion. */
static void colloids_and_variants(int precision) {
  const int n = 24;
  lc_params p = material(n, precision, 0.15);
  p.advection = 3;
  p.stencil = 27;
  lc_ctx* c = NULL;
  OK(lc_create(&p, NULL, &c), NULL);
  lc_colloid k[3] = {colloid(6.3, 7.1, 5.8, 3.2, LC_PRESCRIBED, LC_ANCHOR_PLANAR),
                     colloid(16.6, 15.2, 17.4, 4.4, LC_FREE, LC_ANCHOR_NORMAL),
                     colloid(5.5, 18.3, 16.9, 2.7, LC_FIXED, LC_ANCHOR_NONE)};
  k[0].vel[0] = 0.05;
  k[0].W = 0.02;
  k[1].fext[2] = 1e-3;
  OK(lc_set_colloids(c, 0, 3, k), c);
  CHECK(lc_num_colloids(c, 0) == 3, "colloid count %d", lc_num_colloids(c, 0));
  double* Q0 = helix(n, n, n, 0.3, 0.15);
  OK(lc_set_Q(c, 0, Q0), c);
  OK(lc_step(c, 12), c);
  lc_colloid out[3];
  OK(lc_get_colloids(c, 0, 3, out), c);
  CHECK(fabs(out[0].pos[0] - (6.3 + 12 * 0.05)) < 1e-9, "prescribed position %g", out[0].pos[0]);
  double F[12];
  for (int j = 0; j < 3; j++) {
    OK(lc_get_colloid_force(c, 0, j, F), c);
    CHECK(all_finite(F, 12), "force of colloid %d", j);
  }
  /* too close: refused, the box keeps its colloids */
  lc_colloid close2[2] = {colloid(8, 8, 8, 3.0, LC_FIXED, LC_ANCHOR_NORMAL),
                          colloid(16.5, 8, 8, 3.0, LC_FIXED, LC_ANCHOR_NORMAL)};
  CHECK(lc_set_colloids(c, 0, 2, close2) == LC_EINVAL, "colloids 2.5 apart accepted");
  CHECK(lc_num_colloids(c, 0) == 3, "refused set changed the colloids");
  CHECK(lc_set_colloids(c, 0, LC_MAX_COLLOIDS + 1, close2) == LC_EINVAL, "17 colloids accepted");
  OK(lc_sync(c), c);
  free(Q0);
  lc_destroy(c);
}

/* A batch of three boxes on every tile shape. */
static void batch_tiles(void) {
  lc_params p[3] = {material(24, LC_FP32, 0.0), material(20, LC_FP32, 0.2), material(28, LC_FP32, 0.15)};
  p[1].ny = 16;
  lc_ctx* c = NULL;
  OK(lc_create_batch(3, p, NULL, &c), NULL);
  lc_colloid k = colloid(10.2, 9.7, 10.4, 4.0, LC_FIXED, LC_ANCHOR_PLANAR);
  OK(lc_set_colloid(c, 2, &k), c);
  for (int b = 0; b < 3; b++) {
    double* Q0 = helix(p[b].nx, p[b].ny, p[b].nz, 0.3, 0.2);
    OK(lc_set_Q(c, b, Q0), c);
    free(Q0);
  }
  const int nt = lc_num_tiles(c);
  CHECK(nt >= 2, "tiles %d", nt);
  int used = 0;
  for (int t = 0; t < nt; t++) {
    int shape[3];
    OK(lc_tile_shape(c, t, shape), c);
    if (lc_set_tile(c, t) != LC_OK) continue;   /* a shape the boxes cannot use */
    CHECK(lc_get_tile(c) == t, "tile %d not taken", t);
    OK(lc_step(c, 2), c);
    OK(lc_sync(c), c);
    used++;
  }
  CHECK(used >= 2, "only %d tile shapes ran", used);
  CHECK(lc_set_tile(c, nt) == LC_EINVAL, "tile id beyond the table accepted");
  lc_destroy(c);
}

int main(void) {
  printf("single box fp32\n");
  fflush(stdout);
  single_box(LC_FP32);
  printf("single box fp64\n");
  fflush(stdout);
  single_box(LC_FP64);
  printf("colloids and variants fp64\n");
  fflush(stdout);
  colloids_and_variants(LC_FP64);
  printf("colloids and variants fp32\n");
  fflush(stdout);
  colloids_and_variants(LC_FP32);
  printf("batch on every tile\n");
  fflush(stdout);
  batch_tiles();
  lc_params bad = material(4, LC_FP32, 0.0);
  lc_ctx* c = NULL;
  CHECK(lc_create(&bad, NULL, &c) == LC_EINVAL && c == NULL, "4^3 box accepted");
  CHECK(lc_last_error(NULL) != NULL, "no message after a failed create");
  printf("%s (%d failed checks)\n", failures ? "FAILED" : "ok", failures);
  fflush(stdout);
  fflush(stderr);
  /* Leave without the HIP runtime's exit handlers (every context is
   * destroyed by now): under the address sanitizer, its allocator's
   * bookkeeping of device memory trips over the runtime's own teardown. */
  _Exit(failures ? 1 : 0);
}
