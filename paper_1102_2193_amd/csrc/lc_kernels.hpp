// lc_kernels.hpp -- launch interface between the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "lc_dev.hpp"

namespace lc {

// Device pointers of one step: inputs at time n, outputs at n+1.
template <typename R>
struct StepPtrs {
  const R* fin;
  R* fout;
  const R* Qin;
  R* Qout;
  const R* uin;
  R* uout;
  long long nsites;   // component stride (all boxes)
  double* part;       // colloid partial sums, component-major: part[c * nslot + slot],
                      // per colloid one slot per 3D tile or per (column block, z group)
                      // of its box (ColDev::slot_base + tile)
  long long nslot;
  int* flag;          // bit 0: a non-finite value or |u| >= 0.3; bit 1: two colloids too close
  int par;            // buffer parity of the step (slot of ColDev::pos)
  ColDev* cols;       // colloid table (every box's colloids, box by box)
};

// Block shapes of the fused kernel, per precision: (id, TX, TY, TZ, kind).
// kind 0: 3D tile of TX x TY x TZ nodes; kind 1: TX x TY columns marching
// through TZ planes.
#define LC_TILES_F32(X)  \
  X(0, 32, 8, 16, 1)     \
  X(1, 32, 8, 8, 1)      \
  X(2, 32, 8, 32, 1)     \
  X(3, 64, 4, 16, 1)     \
  X(4, 16, 16, 16, 1)    \
  X(5, 32, 16, 8, 1)     \
  X(6, 16, 8, 2, 0)      \
  X(7, 32, 16, 16, 1)    \
  X(8, 64, 8, 8, 1)
// FP64 (the verification precision) uses the 3D-tile form only.
#define LC_TILES_F64(X)  \
  X(0, 8, 4, 4, 0)       \
  X(1, 16, 4, 2, 0)

// Marching kernel work items.  The z extent of a box is cut into groups of
// kGroup planes; the colloid sums are kept per (column block, group), so they
// do not depend on how groups are bundled into work items.  A work item is
// the int2 (box | ng << 16, cb | g0 << 16): box, number of groups ng, column
// block cb (x fastest) and first group g0.  Limits: box, cb < 2^16;
// g0, ng < 2^15.  Padding items have x = -1.
constexpr int kGroup = 1;
// Threads per block of the post-step kernel; every box has its own whole
// blocks (one box per block).
constexpr int kPostBlock = 64;
// Colloid slots added by one post-step thread; threads of the per-box
// finishing kernel.
constexpr int kPostSlots = 4;
constexpr int kFinishBlock = 1024;
constexpr int kMaxBoxes = 1 << 16, kMaxColBlocks = 1 << 16, kMaxGroups = 1 << 15;
__host__ __device__ inline int2 march_item(int box, int cb, int g0, int ng) {
  return make_int2(box | (ng << 16), cb | (g0 << 16));
}
__host__ __device__ inline int item_box(int x) { return x & 0xffff; }
__host__ __device__ inline int item_ng(int x) { return x >> 16; }
__host__ __device__ inline int item_cb(int y) { return y & 0xffff; }
__host__ __device__ inline int item_g0(int y) { return y >> 16; }

// One launch of the fused kernel.  3D tiles: one block per entry of
// `tiles`.  Marching shapes: `nblk` persistent blocks, block b taking the
// work items tiles[offs[b]] .. tiles[offs[b+1]-1] in order.  e0/e1 (may be
// null): events recorded when the kernel starts and ends.
template <typename R>
hipError_t launch_step(int tile, int nblk, const BoxDev* boxes, const int2* tiles, const int* offs,
                       const StepPtrs<R>& a, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Resident blocks per compute unit of FP32 marching shape `tile` (0 if the
// shape is not a marching one).
int march_blocks_per_cu(int tile);
// Anchoring pass: ghost Q at the boundary solid nodes of the Q buffer
// (before the first step and after any change made from the host), for the
// colloids at pos[par].
template <typename R>
hipError_t launch_ghost(const BoxDev* boxes, const ColDev* cols, int ncol, long long total, R* Q, long long NS, int par,
                        hipStream_t s);
// After the fused kernel, per colloid of the table: moving-boundary events,
// the next step's ghost Q, per-block sums of the fused kernel's colloid
// slots and the event momenta (nblk blocks, 12 doubles each, into bpart +
// 12 * nblk * a.par), a check of the gap to the box's other colloids (flag
// bit 1) and the next position pos[a.par ^ 1].  The last block of each
// colloid first finishes the colloid's previous step if pending[colloid] is
// set (its block sums are in the other half of bpart): force, force
// history, count; then marks this step pending.  A free colloid's slots were
// added by launch_free (fsum), which also moved it; its block sums then hold
// only the event momenta.
// owner[blk] = the colloid (table index) post-step block blk serves.
template <typename R>
hipError_t launch_post(int nblk, const int* owner, const BoxDev* boxes, const StepPtrs<R>& a, double* bpart,
                       int* pending, const double* fsum, double* force, double* hist, int cap, long long* count,
                       hipStream_t s);
// Free colloids (one block per colloid of the table, others untouched): the
// step's slot sums into fsum [12 per colloid], the velocity update and the
// next position.
hipError_t launch_free(int ncol, const BoxDev* boxes, ColDev* cols, const double* part, long long nslot, int par,
                       double* fsum, hipStream_t s);
// Finish a pending step of buffer parity par (one block per colloid;
// colloids with pending[k] == 0 are left alone); a free colloid also
// receives the events' momentum.
hipError_t launch_finish(int ncol, int nblk, ColDev* cols, int par, const double* bpart, int* pending,
                         const double* fsum, double* force, double* hist, int cap, long long* count, hipStream_t s);
template <typename R>
hipError_t launch_diag(const BoxDev* boxes, int box, long long nsite, const StepPtrs<R>& a, double* out,
                       hipStream_t s);
// Totals of nb diagnostics partials (6 doubles each, as written by
// launch_diag) into out6: sums of components 0..4 in block order, maximum of
// component 5.
hipError_t launch_diag_total(const double* part, long long nb, double* out6, hipStream_t s);
template <typename R>
hipError_t launch_defects(const BoxDev* boxes, const ColDev* cols, int box, long long nsite, const R* Q, long long NS,
                          double thr, unsigned char* mask, unsigned long long* count, int par, hipStream_t s);
// Solid map of box `box`: id[site] = 1 + the colloid holding it, 0 for fluid.
hipError_t launch_solid(const BoxDev* boxes, const ColDev* cols, int box, long long nsite, unsigned char* id, int par,
                        hipStream_t s);
template <typename R>
hipError_t launch_fill(R* f, long long NS, double rho0, hipStream_t s);

}  // namespace lc
