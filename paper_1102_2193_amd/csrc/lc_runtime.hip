// lc_runtime.hip -- host runtime behind the C ABI of include/lc.h: box
// layout, tile work lists, the per-step launch sequence, HIP graph capture
// of repeated steps, transfers and diagnostics.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "../../include/lc.h"
#include "lc_internal.hpp"
#include "lc_kernels.hpp"

using lc::BoxDev;
using lc::ColDev;

namespace {

struct TileShape {
  int x, y, z, kind;   // kind 1: x*y columns marching through z planes
};

#define LC_SHAPE(ID, X, Y, Z, KIND) {X, Y, Z, KIND},
const TileShape kTilesF32[] = {LC_TILES_F32(LC_SHAPE)};
const TileShape kTilesF64[] = {LC_TILES_F64(LC_SHAPE)};
#undef LC_SHAPE
const int kNumF32 = sizeof(kTilesF32) / sizeof(kTilesF32[0]);
const int kNumF64 = sizeof(kTilesF64) / sizeof(kTilesF64[0]);

const int kHistCap = 8192;     // force history ring (steps)
const int kGraphSteps = 16;    // steps per captured graph (even)
const int kTimedDispatches = 64;  // most fused-kernel dispatches lc_time_kernel times
const int kXcd = 8;            // accelerator complex dies on MI355X

std::string g_create_error;

// Diagnostics without allocation (lc_get_diag_noalloc): the partials of the
// diagnostics kernel, 6 doubles per block of 256 sites, and the six totals
// live in one static device array per GPU.
constexpr long long kNoallocDiagBlocks = 21840;   // boxes of up to 5,591,040 sites
constexpr long long kNoallocTotals = 6 * kNoallocDiagBlocks;
constexpr long long kScratchDoubles = kNoallocTotals + 8;   // 1.0 MiB
constexpr int kMaxDevices = 64;

}  // namespace

// Scratch of lc_get_diag_noalloc (sizes above).  Each GPU the library runs
// on holds its own copy until the process ends.  In host code this name is
// not a device address: kernels and copies take the per-device address that
// scratch_address() obtains with hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

struct lc_ctx {
  int nbox = 0;
  int dev = 0;                  // device current at creation
  double* scratch_dev = nullptr;  // that device's address of the static scratch
  std::string scratch_err;        // why scratch_dev is null
  int prec = LC_FP32;
  size_t esz = 4;
  std::vector<lc_params> prm;
  std::vector<std::vector<lc_colloid>> col;   // per box, its colloids
  std::vector<BoxDev> hb;       // host copy of the descriptors
  std::vector<ColDev> hc;       // host copy of the colloid table (box by box)
  int ncol = 0;                 // colloids in all boxes (entries of the table)
  long long nsites = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* f[2] = {nullptr, nullptr};
  void* Q[2] = {nullptr, nullptr};
  void* u[2] = {nullptr, nullptr};
  bool own_buf = true;
  int cur = 0;                  // buffer index holding time n
  BoxDev* dbox = nullptr;
  ColDev* dcol = nullptr;       // colloid table (at least one entry allocated)
  size_t dcol_cap = 0;
  int tile = 0;
  int nblk = 0;                 // fused-kernel blocks (incl. XCD padding)
  int ntile = 0;                // real tiles
  long long nslot = 1;          // colloid slots of the fused kernel (>= 1)
  int2* dtiles = nullptr;
  int* doffs = nullptr;         // marching shapes: item range of each persistent block
  double* dpart = nullptr;      // 12 per tile
  long long ghost_total = 0;
  int npost = 0;                // blocks of the post-step kernel
  double* dbpart = nullptr;     // 12 per post-step block, one half per buffer parity
  int* dpostmap = nullptr;      // per post-step block, the colloid it serves
  size_t dbpart_cap = 0;
  int* dpending = nullptr;      // per colloid: a step whose force sums are not yet added
  double* dfsum = nullptr;      // 12 per colloid: link and stress sums of a free colloid's step
  bool maybe_pending = false;   // a step ran since the last finish from the host
  bool ghost_fresh = false;     // ghost Q of buffer cur matches the colloids
  double* dforce = nullptr;     // 12 per colloid
  double* dhist = nullptr;      // colloids * kHistCap * 12
  long long* dcount = nullptr;  // steps per colloid on the device
  int col_cap = 0;              // colloids the per-colloid arrays above hold
  std::vector<int> colbase;     // per box, its first entry of the colloid table
  int* dflag = nullptr;
  double* ddiag = nullptr;
  size_t ddiag_cap = 0;
  long nstep = 0;
  bool any_colloid = false, any_moving = false, any_free = false;
  bool use_graph = true;
  bool graph_ok = false;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  std::string err;
};

namespace {

int fail(lc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                             \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, LC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

const TileShape& tile_shape(const lc_ctx* c, int id) {
  return c->prec == LC_FP32 ? kTilesF32[id] : kTilesF64[id];
}
int num_tiles(const lc_ctx* c) { return c->prec == LC_FP32 ? kNumF32 : kNumF64; }

long long box_sites(const lc_params& p) { return (long long)p.nx * p.ny * p.nz; }

void destroy_graph(lc_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->graph_ok = false;
}

// Read the device copy of the colloid table back (positions, and a free
// colloid's velocities, change on the device) before the host rewrites it.
int pull_boxes(lc_ctx* c) {
  if (c->ncol == 0) return LC_OK;
  HIPCHK(c, hipMemcpyAsync(c->hc.data(), c->dcol, sizeof(ColDev) * c->ncol, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (const ColDev& C : c->hc) {
    const int k = (int)(&C - c->hc.data()) - c->colbase[C.box];
    lc_colloid& h = c->col[C.box][k];
    for (int a = 0; a < 3; a++) {
      h.pos[a] = C.pos[c->cur][a];
      h.vel[a] = C.vel[a];       // a free colloid's change on the device
      h.omega[a] = C.omega[a];
    }
  }
  return LC_OK;
}

int first_3d_tile(const lc_ctx* c) {
  for (int t = 0; t < num_tiles(c); t++)
    if (tile_shape(c, t).kind == 0) return t;
  return 0;
}

// Contexts whose boxes hold several colloids, higher-order advection or the
// 27-point stencil run on the 3D-tile kernel only.
bool needs_3d(const lc_ctx* c) {
  for (int b = 0; b < c->nbox; b++) {
    const BoxDev& B = c->hb[b];
    if (B.adv != 1 || B.st27 || c->col[b].size() > 1) return true;
  }
  return false;
}

// Can the colloid (radius + 3 + margin) reach the block [lo, lo + ext) in any
// periodic image?  The integer test of the kernels, widened by `margin`
// sites; used only to decide how work is cut, never what is computed.
const int kMargin = 2;       // sites of colloid motion covered between layouts
// Cost model of marching work, in plane-times of the solid-free path: a
// fixed start per work item (prologue loads and stresses) plus one per
// plane; where the colloid can reach, 1.43 per plane, and 1.95 where the
// column block's own rectangle of the plane holds solid nodes (fitted to
// per-block clocks of the 128^3 drag case: 5.3, 7.6 and 10.3 us per plane,
// 12 us for each further item a block starts).
const double kItemStart = 2.3, kNearPlaneCost = 1.43, kSolidPlaneCost = 1.95;
const int kMaxPiecesPerBlock = 3;

// Does the rectangle [x0, x0 + ex) x [y0, y0 + ey) of plane z hold a lattice
// node inside the colloid (any periodic image)?  The lattice node nearest to
// the centre is found axis by axis; only the schedule's cost uses it.
bool host_solid_rect(const lc_params& p, const lc_colloid& k, int x0, int y0, int ex, int ey, int z) {
  if (!k.present) return false;
  const int lo[3] = {x0, y0, z}, hi[3] = {x0 + ex - 1, y0 + ey - 1, z}, L[3] = {p.nx, p.ny, p.nz};
  double d2 = 0.0;
  for (int a = 0; a < 3; a++) {
    double best = 1e300;
    for (int m = -1; m <= 1; m++) {
      const double c = k.pos[a] + m * L[a];
      double q = floor(c + 0.5);
      q = q < lo[a] ? lo[a] : (q > hi[a] ? hi[a] : q);
      const double e = (q - c) * (q - c);
      best = e < best ? e : best;
    }
    d2 += best;
  }
  return d2 < k.a0 * k.a0;
}

bool host_near(const lc_params& p, const lc_colloid& k, int x0, int y0, int z0, int ex, int ey, int ez,
               int margin) {
  if (!k.present) return false;
  const int ra = (int)ceil(k.a0) + 3 + margin;
  const int lo[3] = {x0, y0, z0}, ext[3] = {ex, ey, ez}, L[3] = {p.nx, p.ny, p.nz};
  for (int a = 0; a < 3; a++) {
    const int cc = (int)floor(k.pos[a]);
    int best = 1 << 30;
    for (int m = -1; m <= 1; m++) {
      const int q = cc + m * L[a];
      const int d = q < lo[a] ? lo[a] - q : (q > lo[a] + ext[a] - 1 ? q - (lo[a] + ext[a] - 1) : 0);
      best = d < best ? d : best;
    }
    if (best > ra) return false;
  }
  return true;
}

// Persistent-block schedule of the marching kernel.  The z groups of every
// column block, taken in spatial order (box, column block, z), carry an
// estimated cost: one plane-time per plane, kNearPlaneCost where the
// colloid can reach, kSolidPlaneCost where the block's rectangle of the plane
// holds solid nodes, plus kItemStart for each work item (run of groups of
// one column block) a block starts.  Each column block's run is cut into
// pieces of equal cost, the piece counts apportioned over the resident
// blocks, and the pieces dealt out die by die (below).  Every (box, column
// block, group) is checked to be covered exactly once.
int march_schedule(lc_ctx* c, const TileShape& T, int slots, std::vector<int2>& order, std::vector<int>& offs) {
  struct Grp {
    int b, cb, g;
    double cost;
  };
  std::vector<Grp> grp;
  for (int b = 0; b < c->nbox; b++) {
    const BoxDev& B = c->hb[b];
    const lc_params& p = c->prm[b];
    lc_colloid none;
    memset(&none, 0, sizeof(none));
    // marching boxes hold at most one colloid
    const lc_colloid& k = c->col[b].empty() ? none : c->col[b][0];
    const int ncb = B.ntx * B.nty;
    for (int cb = 0; cb < ncb; cb++) {
      const int x0 = (cb % B.ntx) * T.x, y0 = (cb / B.ntx) * T.y;
      for (int g = 0; g < B.ntz; g++) {
        const bool nr =
            host_near(p, k, x0 - 2, y0 - 2, g * lc::kGroup - 2, T.x + 4, T.y + 4, lc::kGroup + 4, kMargin);
        double cost = 0.0;
        for (int z = g * lc::kGroup; z < (g + 1) * lc::kGroup && z < B.nz; z++)
          cost += !nr ? 1.0 : (host_solid_rect(p, k, x0, y0, T.x, T.y, z) ? kSolidPlaneCost : kNearPlaneCost);
        grp.push_back({b, cb, g, cost});
      }
    }
  }
  // Pieces: every column block's run of groups is cut on its own into n
  // pieces of about equal cost (so the pieces of uniform column blocks start
  // at the same planes and neighbouring blocks march side by side); the n
  // are apportioned greedily, one more piece at a time to the column block
  // with the most expensive pieces, until the blocks are used up.
  struct Col {
    size_t first, last;   // group index range [first, last)
    double cost;          // sum of group costs
    int n;
  };
  std::vector<Col> cols;
  for (size_t i = 0; i < grp.size();) {
    size_t j = i;
    double cost = 0.0;
    while (j < grp.size() && grp[j].b == grp[i].b && grp[j].cb == grp[i].cb) cost += grp[j++].cost;
    cols.push_back({i, j, cost, 1});
    i = j;
  }
  auto piece = [](const Col& k) { return k.cost / k.n + kItemStart; };
  struct Piece {
    size_t first, last;
    double cost;
  };
  // One plan for `target` pieces in all: returns the largest estimated
  // load of a block and fills bins.
  auto plan = [&](int target, std::vector<std::vector<int2>>& bins) -> double {
    std::vector<Col> cs = cols;
    if ((int)cs.size() <= target) {
      typedef std::pair<double, int> P;   // (piece cost, column)
      std::priority_queue<P> heap;
      for (int q = 0; q < (int)cs.size(); q++) heap.push(P(piece(cs[q]), q));
      for (int used = (int)cs.size(); used < target && !heap.empty(); used++) {
        const int q = heap.top().second;
        heap.pop();
        if (cs[q].n >= (int)(cs[q].last - cs[q].first)) continue;   // one group per piece already
        cs[q].n++;
        heap.push(P(piece(cs[q]), q));
      }
    }
    std::vector<Piece> pieces;
    for (const Col& k : cs) {
      double acc = 0.0;
      int made = 0;
      size_t start = k.first;
      for (size_t g = k.first; g < k.last; g++) {
        // a new piece starts where the cumulative cost first reaches made/n
        if (g > k.first && made < k.n && acc >= k.cost * made / k.n - 1e-9) {
          pieces.push_back({start, g, 0.0});
          start = g;
        }
        if (g == k.first || g == start) made++;
        acc += grp[g].cost;
      }
      pieces.push_back({start, k.last, 0.0});
    }
    for (Piece& pc : pieces) {
      pc.cost = kItemStart;
      for (size_t g = pc.first; g < pc.last; g++) pc.cost += grp[g].cost;
    }
    // Pieces ordered by (box, first plane, column block); the q-th goes to
    // block (q / per_die) + 8 (q % per_die), so each die takes every column
    // block of a slab of planes and the halo rows its blocks share with
    // their x and y neighbours pass through the same L2.  With more pieces
    // than blocks, a die's pieces go longest first to its least loaded block.
    std::stable_sort(pieces.begin(), pieces.end(), [&](const Piece& u, const Piece& v) {
      const Grp& a = grp[u.first];
      const Grp& b = grp[v.first];
      if (a.b != b.b) return a.b < b.b;
      if (a.g != b.g) return a.g < b.g;
      return a.cb < b.cb;
    });
    const int per_die = slots / kXcd;
    const int np = (int)pieces.size();
    bins.assign(slots, std::vector<int2>());
    std::vector<double> load(slots, 0.0);
    const int per_die_pieces = (np + kXcd - 1) / kXcd;
    for (int d = 0; d < kXcd; d++) {
      const int q0 = std::min(np, d * per_die_pieces), q1 = std::min(np, (d + 1) * per_die_pieces);
      std::vector<int> idx;
      for (int q = q0; q < q1; q++) idx.push_back(q);
      if ((int)idx.size() > per_die)
        std::stable_sort(idx.begin(), idx.end(), [&](int u, int v) { return pieces[u].cost > pieces[v].cost; });
      for (int t = 0; t < (int)idx.size(); t++) {
        int j = t;
        if (t >= per_die) {
          j = 0;
          for (int m = 1; m < per_die; m++)
            if (load[d + kXcd * m] < load[d + kXcd * j]) j = m;
        }
        const int blk = d + kXcd * j;
        const Piece& pc = pieces[idx[t]];
        load[blk] += pc.cost;
        size_t i = pc.first;
        while (i < pc.last) {
          size_t e = std::min(pc.last, i + (size_t)(lc::kMaxGroups - 1));
          bins[blk].push_back(lc::march_item(grp[i].b, grp[i].cb, grp[i].g, (int)(e - i)));
          i = e;
        }
      }
    }
    return *std::max_element(load.begin(), load.end());
  };
  // One, two or three pieces per resident block: more pieces spread the
  // colloid's expensive planes over more blocks but each adds an item start;
  // the plan with the smallest estimated largest load wins (fewer pieces on
  // a tie within 1%).
  std::vector<std::vector<int2>> bins, trial;
  double best = plan(slots, bins);
  for (int k = 2; k <= kMaxPiecesPerBlock; k++) {
    const double m = plan(slots * k, trial);
    if (m < best * 0.99) {
      best = m;
      bins.swap(trial);
    }
  }
  // coverage: every (box, column block, group) exactly once
  long long total = 0;
  for (int b = 0; b < c->nbox; b++) total += (long long)c->hb[b].ntx * c->hb[b].nty * c->hb[b].ntz;
  std::vector<unsigned char> seen((size_t)total, 0);
  for (const auto& bn : bins)
    for (const int2& it : bn) {
      const int b = lc::item_box(it.x), ng = lc::item_ng(it.x), cb = lc::item_cb(it.y), g0 = lc::item_g0(it.y);
      if (b >= c->nbox) return fail(c, LC_EINVAL, "internal: bad marching work item");
      const BoxDev& B = c->hb[b];
      if (ng < 1 || cb >= B.ntx * B.nty || g0 + ng > B.ntz)
        return fail(c, LC_EINVAL, "internal: bad marching work item");
      for (int g = g0; g < g0 + ng; g++) {
        unsigned char& sn = seen[(size_t)B.tile_base + cb + (size_t)B.ntx * B.nty * g];
        if (sn++) return fail(c, LC_EINVAL, "internal: overlapping marching work items");
      }
    }
  for (unsigned char sn : seen)
    if (!sn) return fail(c, LC_EINVAL, "internal: marching work items leave a gap");
  order.clear();
  offs.assign(1, 0);
  for (const auto& bn : bins) {
    for (const int2& it : bn) order.push_back(it);
    offs.push_back((int)order.size());
  }
  if (order.empty()) order.push_back(make_int2(-1, 0));
  return LC_OK;
}

// Rebuild descriptors, tile list and launch ranges for the current tile
// shape and colloids; upload.
//
// Marching kernel: each column block's z groups are bundled into work items
// of the shape's plane count, except where the colloid can reach, where
// every group is an item of its own (the solid-aware path costs about twice
// as much per plane).  Those short items go first in the launch, spread over
// the dies, so that the hardware's in-order dispatch starts them at once and
// fills the remaining time with the long items.
// Finish the last step from the host if its colloid sums are still pending
// (the next step's post-step kernel would otherwise do it).
int flush(lc_ctx* c) {
  if (!c->maybe_pending) return LC_OK;
  if (c->ncol > 0)
    HIPCHK(c, lc::launch_finish(c->ncol, c->npost, c->dcol, c->cur ^ 1, c->dbpart, c->dpending, c->dfsum, c->dforce,
                                c->dhist, kHistCap, c->dcount, c->stream));
  c->maybe_pending = false;
  return LC_OK;
}

// The marching kernel addresses each population array through one buffer
// resource with 32-bit component offsets: 19 x sites x 4 bytes must stay
// below 4 GiB.
bool march_fits(const lc_ctx* c) { return 19.0 * 4.0 * (double)c->nsites < 4294967296.0; }

// The per-colloid device arrays (last force, history ring, step count,
// pending flag, free-motion sums) for a new colloid table whose box b
// starts at entry base[b] (total entries): colloid k of box b keeps its
// entries across layouts; colloids a box gains start empty.  The caller has
// flushed any pending step.
int resize_colloid_arrays(lc_ctx* c, const std::vector<int>& base, int total) {
  const int cap = std::max(1, total);
  if (c->col_cap == cap && c->colbase == base) return LC_OK;
  double *force = nullptr, *hist = nullptr, *fsum = nullptr;
  long long* count = nullptr;
  int* pend = nullptr;
  const size_t hrow = (size_t)kHistCap * 12;
  auto bail = [&](hipError_t e) {
    for (void* p : {(void*)force, (void*)hist, (void*)fsum, (void*)count, (void*)pend}) (void)hipFree(p);
    return fail(c, LC_ENOMEM, std::string("per-colloid arrays: ") + hipGetErrorString(e));
  };
  hipError_t e = hipMalloc(&force, sizeof(double) * 12 * cap);
  if (e == hipSuccess) e = hipMalloc(&hist, sizeof(double) * hrow * cap);
  if (e == hipSuccess) e = hipMalloc(&fsum, sizeof(double) * 12 * cap);
  if (e == hipSuccess) e = hipMalloc(&count, sizeof(long long) * cap);
  if (e == hipSuccess) e = hipMalloc(&pend, sizeof(int) * cap);
  if (e != hipSuccess) return bail(e);
  HIPCHK(c, hipMemsetAsync(force, 0, sizeof(double) * 12 * cap, c->stream));
  HIPCHK(c, hipMemsetAsync(hist, 0, sizeof(double) * hrow * cap, c->stream));
  HIPCHK(c, hipMemsetAsync(fsum, 0, sizeof(double) * 12 * cap, c->stream));
  HIPCHK(c, hipMemsetAsync(count, 0, sizeof(long long) * cap, c->stream));
  HIPCHK(c, hipMemsetAsync(pend, 0, sizeof(int) * cap, c->stream));
  if (c->col_cap > 0 && !c->colbase.empty()) {
    for (int b = 0; b < c->nbox; b++) {
      const int on = (b + 1 < c->nbox ? c->colbase[b + 1] : c->ncol) - c->colbase[b];
      const int nn = (b + 1 < c->nbox ? base[b + 1] : total) - base[b];
      const int m = std::min(on, nn);
      if (m <= 0) continue;
      const size_t o = c->colbase[b], n = base[b];
      HIPCHK(c, hipMemcpyAsync(force + 12 * n, c->dforce + 12 * o, sizeof(double) * 12 * m, hipMemcpyDeviceToDevice,
                               c->stream));
      HIPCHK(c, hipMemcpyAsync(hist + hrow * n, c->dhist + hrow * o, sizeof(double) * hrow * m,
                               hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(fsum + 12 * n, c->dfsum + 12 * o, sizeof(double) * 12 * m, hipMemcpyDeviceToDevice,
                               c->stream));
      HIPCHK(c, hipMemcpyAsync(count + n, c->dcount + o, sizeof(long long) * m, hipMemcpyDeviceToDevice, c->stream));
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  (void)hipFree(c->dforce);
  (void)hipFree(c->dhist);
  (void)hipFree(c->dfsum);
  (void)hipFree(c->dcount);
  (void)hipFree(c->dpending);
  c->dforce = force; c->dhist = hist; c->dfsum = fsum; c->dcount = count; c->dpending = pend;
  c->col_cap = cap;
  return LC_OK;
}

int layout(lc_ctx* c) {
  {
    int rc = flush(c);   // the block sums of a pending step follow the old layout
    if (rc != LC_OK) return rc;
  }
  const TileShape& T = tile_shape(c, c->tile);
  long long tb = 0, gb = 0, sb = 0;
  int pblk = 0, total = 0;
  c->any_colloid = c->any_moving = c->any_free = false;
  std::vector<int2> tiles;
  std::vector<int> base(c->nbox, 0);
  std::vector<ColDev> table;
  if (T.kind == 1 && c->nbox > lc::kMaxBoxes) return fail(c, LC_EINVAL, "too many boxes for the marching kernel");
  if (T.kind == 1 && !march_fits(c))
    return fail(c, LC_EINVAL, "context too large for the marching kernel (19 x sites x 4 bytes >= 4 GiB); use a 3D tile");
  if (T.kind == 1 && needs_3d(c))
    return fail(c, LC_EINVAL,
                "the marching kernel has one colloid per box, first-order advection and the 7-point stencil only; "
                "use a 3D tile");
  for (int b = 0; b < c->nbox; b++) {
    BoxDev& B = c->hb[b];
    const lc_params& p = c->prm[b];
    B.ntx = (p.nx + T.x - 1) / T.x;
    B.nty = (p.ny + T.y - 1) / T.y;
    B.tile_base = (int)tb;
    if (T.kind == 1) {
      const int ngz = (p.nz + lc::kGroup - 1) / lc::kGroup;
      const int ncb = B.ntx * B.nty;
      if (ncb > lc::kMaxColBlocks || ngz > lc::kMaxGroups)
        return fail(c, LC_EINVAL, "box too large for the marching kernel's work items");
      B.ntz = ngz;
      tb += (long long)ncb * ngz;
    } else {
      B.ntz = (p.nz + T.z - 1) / T.z;
      const int nt = B.ntx * B.nty * B.ntz;
      for (int t = 0; t < nt; t++) tiles.push_back(make_int2(b, t));
      tb += nt;
    }
    const long long nt = (long long)B.ntx * B.nty * B.ntz;   // slots per colloid of this box
    base[b] = total;
    B.col0 = total;
    B.ncol = (int)c->col[b].size();
    for (const lc_colloid& k : c->col[b]) {
      ColDev C;
      memset(&C, 0, sizeof(C));
      C.box = b;
      C.motion = k.motion;
      C.anchoring = k.anchoring;
      for (int a = 0; a < 3; a++) {
        C.pos[0][a] = C.pos[1][a] = k.pos[a];
        C.vel[a] = k.vel[a];
        C.omega[a] = k.omega[a];
        C.fext[a] = k.fext[a];
      }
      C.a0 = k.a0;
      C.S0 = k.S0;
      C.W = k.W;
      const double rc = k.rho_c > 0.0 ? k.rho_c : p.rho0;
      C.mass = 4.0 / 3.0 * acos(-1.0) * k.a0 * k.a0 * k.a0 * rc;
      C.inertia = 0.4 * C.mass * k.a0 * k.a0;
      C.slot_base = (int)sb;
      sb += nt;
      const int ca = (int)ceil(k.a0);
      C.ghost_ext = 2 * ca + 3;
      C.ghost_base = (int)gb;
      gb += (long long)C.ghost_ext * C.ghost_ext * C.ghost_ext;
      const bool moving = k.motion != LC_FIXED;
      C.event_ext = moving ? 2 * ca + 5 : 0;
      // post-step threads: slot sums (kPostSlots slots each), one per event
      // candidate, one per ghost candidate, then one more block that only
      // finishes the previous step (a free colloid's slots are added before
      // the post-step kernel)
      const long long nst = k.motion != LC_FREE ? (nt + lc::kPostSlots - 1) / lc::kPostSlots : 0;
      const long long ne = (long long)C.event_ext * C.event_ext * C.event_ext;
      const long long ng = (long long)C.ghost_ext * C.ghost_ext * C.ghost_ext;
      C.post_blk0 = pblk;
      C.post_nblk = (int)((nst + ne + ng + lc::kPostBlock - 1) / lc::kPostBlock) + 1;
      if ((long long)pblk + C.post_nblk > (1LL << 30)) return fail(c, LC_EINVAL, "too many post-step blocks");
      pblk += C.post_nblk;
      c->any_colloid = true;
      c->any_moving |= moving;
      c->any_free |= k.motion == LC_FREE;
      table.push_back(C);
      total++;
    }
  }
  if (tb > (1LL << 30)) return fail(c, LC_EINVAL, "too many tiles");
  if (sb > (1LL << 30)) return fail(c, LC_EINVAL, "too many colloid slots");
  {
    int rc = resize_colloid_arrays(c, base, total);
    if (rc != LC_OK) return rc;
  }
  c->colbase = base;
  c->ncol = total;
  c->hc = table;
  c->ntile = (int)tb;
  c->nslot = std::max<long long>(1, sb);
  c->ghost_total = gb;
  c->npost = pblk;
  c->ghost_fresh = false;
  std::vector<int2> order;
  std::vector<int> offs;
  if (T.kind == 1) {
    int dev = 0, cus = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = std::max(1, lc::march_blocks_per_cu(c->tile));
    const int slots = std::max(1, cus * per_cu / kXcd) * kXcd;
    const int rc = march_schedule(c, T, slots, order, offs);
    if (rc != LC_OK) return rc;
    c->nblk = slots;
  } else {
    // One block per tile; workgroup i, which runs on die i % 8, takes the
    // contiguous chunk (i % 8) of the spatial list (L2 locality).
    const int nt = (int)tiles.size();
    const int per = (nt + kXcd - 1) / kXcd;
    c->nblk = per * kXcd;
    order.assign(c->nblk, make_int2(-1, 0));
    for (int i = 0; i < per * kXcd; i++) {
      const int s = (i % kXcd) * per + i / kXcd;
      if (s < nt) order[i] = tiles[s];
    }
  }
  if (c->dtiles) (void)hipFree(c->dtiles);
  if (c->doffs) (void)hipFree(c->doffs);
  if (c->dpart) (void)hipFree(c->dpart);
  c->dtiles = nullptr;
  c->doffs = nullptr;
  c->dpart = nullptr;
  HIPCHK(c, hipMalloc(&c->dtiles, sizeof(int2) * order.size()));
  if (!offs.empty()) {
    HIPCHK(c, hipMalloc(&c->doffs, sizeof(int) * offs.size()));
    HIPCHK(c, hipMemcpyAsync(c->doffs, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipMalloc(&c->dpart, sizeof(double) * 12 * c->nslot));
  HIPCHK(c, hipMemsetAsync(c->dpart, 0, sizeof(double) * 12 * c->nslot, c->stream));
  if ((size_t)pblk * 24 > c->dbpart_cap) {
    if (c->dbpart) (void)hipFree(c->dbpart);
    if (c->dpostmap) (void)hipFree(c->dpostmap);
    c->dbpart = nullptr;
    c->dpostmap = nullptr;
    c->dbpart_cap = std::max<size_t>(24, (size_t)pblk * 24);
    HIPCHK(c, hipMalloc(&c->dbpart, sizeof(double) * c->dbpart_cap));
    HIPCHK(c, hipMalloc(&c->dpostmap, sizeof(int) * (c->dbpart_cap / 24)));
  }
  if (pblk > 0) {
    std::vector<int> owner((size_t)pblk);
    for (int g = 0; g < total; g++)
      for (int k = 0; k < table[g].post_nblk; k++) owner[(size_t)table[g].post_blk0 + k] = g;
    HIPCHK(c, hipMemcpyAsync(c->dpostmap, owner.data(), sizeof(int) * pblk, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  // the colloid table (a zeroed entry when there is none: the marching
  // kernel reads entry 0 of a box without colloids but uses nothing of it)
  if ((size_t)std::max(1, total) > c->dcol_cap) {
    if (c->dcol) (void)hipFree(c->dcol);
    c->dcol = nullptr;
    c->dcol_cap = (size_t)std::max(1, total);
    HIPCHK(c, hipMalloc(&c->dcol, sizeof(ColDev) * c->dcol_cap));
  }
  if (total > 0) {
    HIPCHK(c, hipMemcpyAsync(c->dcol, c->hc.data(), sizeof(ColDev) * total, hipMemcpyHostToDevice, c->stream));
  } else {
    HIPCHK(c, hipMemsetAsync(c->dcol, 0, sizeof(ColDev), c->stream));
  }
  HIPCHK(c, hipMemcpyAsync(c->dtiles, order.data(), sizeof(int2) * order.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->dbox, c->hb.data(), sizeof(BoxDev) * c->nbox, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  destroy_graph(c);
  return LC_OK;
}

template <typename R>
lc::StepPtrs<R> ptrs(lc_ctx* c, int from) {
  lc::StepPtrs<R> a;
  a.fin = (const R*)c->f[from];
  a.fout = (R*)c->f[1 - from];
  a.Qin = (const R*)c->Q[from];
  a.Qout = (R*)c->Q[1 - from];
  a.uin = (const R*)c->u[from];
  a.uout = (R*)c->u[1 - from];
  a.nsites = c->nsites;
  a.part = c->dpart;
  a.nslot = c->nslot;
  a.flag = c->dflag;
  a.par = from;
  a.cols = c->dcol;
  return a;
}

// One step from buffer `from`: the fused kernel, then the post-step kernel
// (events, the ghost Q of the new buffer, colloid sums, R += v).  The ghost
// Q of `from` must be current (ghost_pass).
template <typename R>
hipError_t enqueue_step(lc_ctx* c, int from, hipEvent_t k0 = nullptr, hipEvent_t k1 = nullptr) {
  hipError_t e;
  lc::StepPtrs<R> a = ptrs<R>(c, from);
  e = lc::launch_step<R>(c->tile, c->nblk, c->dbox, c->dtiles, c->doffs, a, c->stream, k0, k1);
  if (e != hipSuccess || c->ncol == 0) return e;
  c->maybe_pending = true;
  // a free colloid is moved by its own force: the slot sums come first, and
  // the step is finished at once (the next step reads the velocity)
  if (c->any_free &&
      (e = lc::launch_free(c->ncol, c->dbox, c->dcol, a.part, a.nslot, a.par, c->dfsum, c->stream)) != hipSuccess)
    return e;
  e = lc::launch_post<R>(c->npost, c->dpostmap, c->dbox, a, c->dbpart, c->dpending, c->dfsum, c->dforce, c->dhist,
                         kHistCap, c->dcount, c->stream);
  if (e != hipSuccess || !c->any_free) return e;
  return lc::launch_finish(c->ncol, c->npost, c->dcol, a.par, c->dbpart, c->dpending, c->dfsum, c->dforce, c->dhist,
                           kHistCap, c->dcount, c->stream);
}

hipError_t enqueue(lc_ctx* c, int from, hipEvent_t k0 = nullptr, hipEvent_t k1 = nullptr) {
  return c->prec == LC_FP32 ? enqueue_step<float>(c, from, k0, k1) : enqueue_step<double>(c, from, k0, k1);
}

// Anchoring pass over buffer cur, needed once after anything changed Q or
// a colloid from the host; every step then leaves the new buffer current.
int ghost_pass(lc_ctx* c) {
  if (c->ghost_fresh) return LC_OK;
  if (c->any_colloid) {
    hipError_t e = c->prec == LC_FP32
                       ? lc::launch_ghost<float>(c->dbox, c->dcol, c->ncol, c->ghost_total, (float*)c->Q[c->cur],
                                                 c->nsites, c->cur, c->stream)
                       : lc::launch_ghost<double>(c->dbox, c->dcol, c->ncol, c->ghost_total, (double*)c->Q[c->cur],
                                                  c->nsites, c->cur, c->stream);
    HIPCHK(c, e);
  }
  c->ghost_fresh = true;
  return LC_OK;
}

int build_graph(lc_ctx* c) {
  destroy_graph(c);
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < kGraphSteps && e == hipSuccess; k++) e = enqueue(c, k & 1);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, LC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  HIPCHK(c, e2);
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
  c->graph_ok = true;
  return LC_OK;
}

int check_box(lc_ctx* c, int box) {
  if (!c) return LC_EINVAL;
  if (box < 0 || box >= c->nbox) return fail(c, LC_EINVAL, "box index out of range");
  return LC_OK;
}

int validate_params(const lc_params& p, std::string& why) {
  if (p.nx < 8 || p.ny < 8 || p.nz < 8) { why = "box edges must be >= 8"; return LC_EINVAL; }
  if ((long long)p.nx * p.ny * p.nz > (1LL << 31)) { why = "box too large"; return LC_EINVAL; }
  if (p.precision != LC_FP32 && p.precision != LC_FP64) { why = "precision must be LC_FP32 or LC_FP64"; return LC_EINVAL; }
  if (!(p.tau > 0.5)) { why = "tau must exceed 1/2"; return LC_EINVAL; }
  if (!(p.rho0 > 0.0)) { why = "rho0 must be positive"; return LC_EINVAL; }
  if (!(p.Gamma >= 0.0) || !(p.K >= 0.0)) { why = "Gamma and K must be >= 0"; return LC_EINVAL; }
  if (p.advection < 0 || p.advection > 3) { why = "advection order must be 1, 2 or 3 (0: 1)"; return LC_EINVAL; }
  if (p.stencil != 0 && p.stencil != 7 && p.stencil != 27) { why = "stencil must be 7 or 27 (0: 7)"; return LC_EINVAL; }
  if (!isfinite(p.A0) || !isfinite(p.gamma) || !isfinite(p.q0) || !isfinite(p.xi)) {
    why = "non-finite material parameter";
    return LC_EINVAL;
  }
  return LC_OK;
}

// host <-> device conversion of one box's field
template <typename R>
int put_field(lc_ctx* c, void* dev, int box, int ncomp, const double* src, double shift_w) {
  const long long n = box_sites(c->prm[box]);
  std::vector<R> tmp((size_t)n);
  for (int k = 0; k < ncomp; k++) {
    const double sh = shift_w != 0.0 ? lc::wgt(k) : 0.0;
    for (long long i = 0; i < n; i++) tmp[i] = (R)(src[k * n + i] - sh);
    HIPCHK(c, hipMemcpyAsync((R*)dev + k * c->nsites + c->hb[box].off, tmp.data(), sizeof(R) * n,
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return LC_OK;
}

template <typename R>
int get_field(lc_ctx* c, const void* dev, int box, int ncomp, double* dst, double shift_w) {
  const long long n = box_sites(c->prm[box]);
  std::vector<R> tmp((size_t)n);
  for (int k = 0; k < ncomp; k++) {
    HIPCHK(c, hipMemcpyAsync(tmp.data(), (const R*)dev + k * c->nsites + c->hb[box].off, sizeof(R) * n,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double sh = shift_w != 0.0 ? lc::wgt(k) : 0.0;
    for (long long i = 0; i < n; i++) dst[k * n + i] = (double)tmp[i] + sh;
  }
  return LC_OK;
}

int put(lc_ctx* c, void* dev, int box, int ncomp, const double* src, bool shift) {
  c->ghost_fresh = false;
  return c->prec == LC_FP32 ? put_field<float>(c, dev, box, ncomp, src, shift ? 1.0 : 0.0)
                            : put_field<double>(c, dev, box, ncomp, src, shift ? 1.0 : 0.0);
}
int get(lc_ctx* c, const void* dev, int box, int ncomp, double* dst, bool shift) {
  return c->prec == LC_FP32 ? get_field<float>(c, dev, box, ncomp, dst, shift ? 1.0 : 0.0)
                            : get_field<double>(c, dev, box, ncomp, dst, shift ? 1.0 : 0.0);
}

// Validate a colloid for a box; v gets it with the centre wrapped into the box.
int check_colloid(const lc_params& p, const lc_colloid& k, lc_colloid& v, std::string& why) {
  v = k;
  if (!v.present) return LC_OK;
  const int Lmin = std::min(p.nx, std::min(p.ny, p.nz));
  if (!(v.a0 > 1.0) || !(2.0 * v.a0 + 4.0 <= Lmin)) { why = "colloid radius does not fit the box"; return LC_EINVAL; }
  if (v.anchoring < LC_ANCHOR_NONE || v.anchoring > LC_ANCHOR_PLANAR) { why = "bad anchoring"; return LC_EINVAL; }
  if (v.motion != LC_FIXED && v.motion != LC_PRESCRIBED && v.motion != LC_FREE) { why = "bad motion"; return LC_EINVAL; }
  if (!isfinite(v.fext[0]) || !isfinite(v.fext[1]) || !isfinite(v.fext[2]) || !isfinite(v.rho_c)) {
    why = "external force and colloid density must be finite";
    return LC_EINVAL;
  }
  if (!(v.W >= 0.0)) { why = "W must be >= 0"; return LC_EINVAL; }
  if (v.anchoring != LC_ANCHOR_NONE && !(p.K + v.W > 0.0)) { why = "K + W must be positive"; return LC_EINVAL; }
  for (int a = 0; a < 3; a++)
    if (!isfinite(v.pos[a]) || !isfinite(v.vel[a]) || !isfinite(v.omega[a]) || fabs(v.vel[a]) >= 1.0) {
      why = "colloid position/velocity must be finite, |v| < 1";
      return LC_EINVAL;
    }
  const int L[3] = {p.nx, p.ny, p.nz};
  for (int a = 0; a < 3; a++) {
    double r = fmod(v.pos[a], (double)L[a]);
    if (r < 0) r += L[a];
    v.pos[a] = r;
  }
  return LC_OK;
}

// n colloids for one box: each valid, present, and every pair at least
// kColloidGap apart surface to surface (minimum image); v gets them with
// the centres wrapped into the box.
int check_colloids(const lc_params& p, int n, const lc_colloid* k, std::vector<lc_colloid>& v, std::string& why) {
  if (n < 0 || n > lc::kMaxColloids) {
    why = "a box holds 0 to " + std::to_string(lc::kMaxColloids) + " colloids";
    return LC_EINVAL;
  }
  v.assign(n, lc_colloid());
  for (int i = 0; i < n; i++) {
    if (!k[i].present) { why = "colloid " + std::to_string(i) + " is not marked present"; return LC_EINVAL; }
    if (check_colloid(p, k[i], v[i], why) != LC_OK) return LC_EINVAL;
  }
  const int L[3] = {p.nx, p.ny, p.nz};
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++) {
      double d2 = 0.0;
      for (int a = 0; a < 3; a++) {
        double d = v[j].pos[a] - v[i].pos[a];
        if (d > 0.5 * L[a]) d -= L[a];
        else if (d < -0.5 * L[a]) d += L[a];
        d2 += d * d;
      }
      if (sqrt(d2) < v[i].a0 + v[j].a0 + lc::kColloidGap) {
        why = "colloids " + std::to_string(i) + " and " + std::to_string(j) + " are closer than " +
              std::to_string(lc::kColloidGap) + " lattice units (surface to surface)";
        return LC_EINVAL;
      }
    }
  return LC_OK;
}

int check_flag(lc_ctx* c) {
  int flag = 0;
  HIPCHK(c, hipMemcpyAsync(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (flag & 2)
    return fail(c, LC_ESTATE, "two colloids of a box started a step closer than 3 lattice units (surface to surface)");
  if (flag) return fail(c, LC_ENUMERIC, "a step produced a non-finite value or |u| >= 0.3");
  return LC_OK;
}

}  // namespace

int lc_internal_q_view(lc_ctx* c, int box, LcQView* out) {
  int rc = check_box(c, box);
  if (rc) return rc;
  out->Q = c->Q[c->cur];
  c->ghost_fresh = false;   // the caller writes Q
  out->nsites = c->nsites;
  out->off = c->hb[box].off;
  out->prec = c->prec;
  out->nx = c->prm[box].nx;
  out->ny = c->prm[box].ny;
  out->nz = c->prm[box].nz;
  out->stream = c->stream;
  return LC_OK;
}

extern "C" {

int lc_create(const lc_params* p, void* hip_stream, lc_ctx** out) {
  return lc_create_batch(1, p, hip_stream, out);
}

int lc_create_batch(int nbox, const lc_params* p, void* hip_stream, lc_ctx** out) {
  if (!out) return fail(nullptr, LC_EINVAL, "out is NULL");
  *out = nullptr;
  if (nbox < 1 || !p) return fail(nullptr, LC_EINVAL, "need at least one box");
  for (int b = 0; b < nbox; b++) {
    std::string why;
    if (validate_params(p[b], why) != LC_OK) return fail(nullptr, LC_EINVAL, "box " + std::to_string(b) + ": " + why);
    if (p[b].precision != p[0].precision) return fail(nullptr, LC_EINVAL, "all boxes must share one precision");
  }
  lc_ctx* c = new lc_ctx();
  c->nbox = nbox;
  c->prec = p[0].precision;
  c->esz = c->prec == LC_FP32 ? 4 : 8;
  c->prm.assign(p, p + nbox);
  c->col.assign(nbox, std::vector<lc_colloid>());
  c->hb.assign(nbox, BoxDev());
  long long off = 0;
  for (int b = 0; b < nbox; b++) {
    BoxDev& B = c->hb[b];
    memset(&B, 0, sizeof(B));
    const lc_params& q = p[b];
    B.nx = q.nx; B.ny = q.ny; B.nz = q.nz; B.hydro = q.hydro ? 1 : 0;
    B.off = off;
    // keep every box 64-site aligned for coalesced access
    off += (box_sites(q) + 63) / 64 * 64;
    B.tau = q.tau; B.rho0 = q.rho0; B.A0 = q.A0; B.gamma = q.gamma; B.K = q.K; B.q0 = q.q0;
    B.xi = q.xi; B.Gamma = q.Gamma;
    B.itau = 1.0 / q.tau;
    B.fsrc = 1.0 - 0.5 / q.tau;
    for (int a = 0; a < 3; a++) B.body[a] = q.body_force[a];
    B.adv = q.advection ? q.advection : 1;
    B.st27 = q.stencil == 27 ? 1 : 0;
  }
  c->nsites = off;
  // kernels address each component with 32-bit byte offsets
  if ((double)off * (c->prec == LC_FP32 ? 4.0 : 8.0) >= 4294967296.0) {
    delete c;
    return fail(nullptr, LC_EINVAL, "too many lattice sites for one context (32-bit offsets)");
  }
  int rc = LC_OK;
  auto bail = [&](int code, const std::string& m) {
    g_create_error = m;
    lc_destroy(c);
    return code;
  };
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(LC_EDEVICE, "hipStreamCreate failed");
    c->own_stream = true;
  }
  const size_t nf = 19 * c->nsites * c->esz, nq = 5 * c->nsites * c->esz, nu = 3 * c->nsites * c->esz;
  for (int k = 0; k < 2; k++) {
    hipError_t e = hipMalloc(&c->f[k], nf);
    if (e == hipSuccess) e = hipMalloc(&c->Q[k], nq);
    if (e == hipSuccess) e = hipMalloc(&c->u[k], nu);
    if (e != hipSuccess)
      return bail(LC_ENOMEM, std::string("device allocation of the fields failed: ") + hipGetErrorString(e));
  }
  if (hipMalloc(&c->dbox, sizeof(BoxDev) * nbox) != hipSuccess || hipMalloc(&c->dflag, sizeof(int)) != hipSuccess)
    return bail(LC_ENOMEM, "device allocation failed");
  {
    // the device the fields were allocated on (current), and its copy of the
    // static scratch
    // static scratch (only lc_get_diag_noalloc needs it: a failure here is
    // reported by that call)
    hipError_t e = hipGetDevice(&c->dev);
    if (e == hipSuccess) e = scratch_address(c->dev, &c->scratch_dev);
    if (e != hipSuccess) {
      c->scratch_dev = nullptr;
      c->scratch_err = std::string("device / static scratch address: ") + hipGetErrorString(e);
    }
  }
  {
    hipError_t e = hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream);
    for (int k = 0; k < 2 && e == hipSuccess; k++) {
      e = hipMemsetAsync(c->Q[k], 0, nq, c->stream);
      if (e == hipSuccess) e = hipMemsetAsync(c->u[k], 0, nu, c->stream);
    }
    if (e != hipSuccess) return bail(LC_EDEVICE, std::string("init: ") + hipGetErrorString(e));
  }
  // f = w_i rho0 everywhere (stored shifted by w_i)
  for (int k = 0; k < 2; k++) {
    // per-box rho0: fill with box 0's value, then fix boxes that differ
    hipError_t e = c->prec == LC_FP32 ? lc::launch_fill<float>((float*)c->f[k], c->nsites, p[0].rho0, c->stream)
                                      : lc::launch_fill<double>((double*)c->f[k], c->nsites, p[0].rho0, c->stream);
    if (e != hipSuccess) return bail(LC_EDEVICE, std::string("init: ") + hipGetErrorString(e));
  }
  if (!march_fits(c) || needs_3d(c)) {   // default to the first 3D-tile shape
    for (int t = 0; t < num_tiles(c); t++)
      if (tile_shape(c, t).kind == 0) {
        c->tile = t;
        break;
      }
  } else if (c->prec == LC_FP32) {
    // default: the marching shape measured fastest on 128^3 boxes (32 x 16
    // columns, groups of 8 planes); lc_set_tile or a tuner picks others
    for (int t = 0; t < num_tiles(c); t++) {
      const TileShape& T = tile_shape(c, t);
      if (T.kind == 1 && T.x == 32 && T.y == 16 && T.z == 8) {
        c->tile = t;
        break;
      }
    }
  }
  rc = layout(c);
  if (rc != LC_OK) return bail(rc, c->err);
  for (int b = 0; b < nbox; b++) {
    if (p[b].rho0 != p[0].rho0) {
      std::vector<double> f0((size_t)19 * box_sites(p[b]));
      for (int i = 0; i < 19; i++)
        for (long long s = 0; s < box_sites(p[b]); s++) f0[i * box_sites(p[b]) + s] = lc::wgt(i) * p[b].rho0;
      if ((rc = lc_set_f(c, b, f0.data())) != LC_OK) return bail(rc, c->err);
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(LC_EDEVICE, "initialisation failed");
  *out = c;
  return LC_OK;
}

void lc_destroy(lc_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  destroy_graph(c);
  if (c->own_buf)
    for (int k = 0; k < 2; k++) {
      if (c->f[k]) (void)hipFree(c->f[k]);
      if (c->Q[k]) (void)hipFree(c->Q[k]);
      if (c->u[k]) (void)hipFree(c->u[k]);
    }
  void* bufs[] = {c->dbox,  c->dtiles, c->doffs, c->dpart,  c->dbpart, c->dpending, c->dfsum,
                  c->dforce, c->dhist,  c->dcount, c->dflag,  c->ddiag,  c->dcol, c->dpostmap};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* lc_last_error(const lc_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int lc_buffer_bytes(const lc_ctx* c, size_t out[3]) {
  if (!c || !out) return LC_EINVAL;
  out[0] = 19 * c->nsites * c->esz;
  out[1] = 5 * c->nsites * c->esz;
  out[2] = 3 * c->nsites * c->esz;
  return LC_OK;
}

int lc_bind_buffers(lc_ctx* c, void* f0, void* f1, void* Q0, void* Q1, void* u0, void* u1) {
  if (!c) return LC_EINVAL;
  void* nf[2] = {f0, f1};
  void* nq[2] = {Q0, Q1};
  void* nu[2] = {u0, u1};
  for (int k = 0; k < 2; k++)
    if (!nf[k] || !nq[k] || !nu[k] || ((uintptr_t)nf[k] | (uintptr_t)nq[k] | (uintptr_t)nu[k]) % 256)
      return fail(c, LC_EINVAL, "buffers must be non-NULL and 256-byte aligned");
  size_t sz[3];
  lc_buffer_bytes(c, sz);
  for (int k = 0; k < 2; k++) {
    HIPCHK(c, hipMemcpyAsync(nf[k], c->f[k], sz[0], hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(nq[k], c->Q[k], sz[1], hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(nu[k], c->u[k], sz[2], hipMemcpyDeviceToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->own_buf)
    for (int k = 0; k < 2; k++) {
      (void)hipFree(c->f[k]);
      (void)hipFree(c->Q[k]);
      (void)hipFree(c->u[k]);
    }
  for (int k = 0; k < 2; k++) {
    c->f[k] = nf[k];
    c->Q[k] = nq[k];
    c->u[k] = nu[k];
  }
  c->own_buf = false;
  destroy_graph(c);
  return LC_OK;
}

int lc_set_colloids(lc_ctx* c, int box, int n, const lc_colloid* k) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (n > 0 && !k) return fail(c, LC_EINVAL, "colloids are NULL");
  std::vector<lc_colloid> v;
  std::string why;
  if (check_colloids(c->prm[box], n, k, v, why) != LC_OK) return fail(c, LC_EINVAL, why);
  if ((rc = pull_boxes(c)) != LC_OK) return rc;
  const std::vector<lc_colloid> old = c->col[box];
  const int old_tile = c->tile;
  c->col[box] = v;
  // several colloids in a box need the 3D-tile kernel
  if (needs_3d(c) && tile_shape(c, c->tile).kind == 1) c->tile = first_3d_tile(c);
  rc = layout(c);
  if (rc != LC_OK) {   // keep the previous colloids
    const std::string e = c->err;
    c->col[box] = old;
    c->tile = old_tile;
    layout(c);
    c->err = e;
  }
  return rc;
}

int lc_set_colloid(lc_ctx* c, int box, const lc_colloid* k) {
  if (!c) return LC_EINVAL;
  if (!k) return fail(c, LC_EINVAL, "colloid is NULL");
  return lc_set_colloids(c, box, k->present ? 1 : 0, k);
}

int lc_num_colloids(lc_ctx* c, int box) {
  if (check_box(c, box)) return -1;
  return (int)c->col[box].size();
}

int lc_get_colloids(lc_ctx* c, int box, int n, lc_colloid* k) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (n < 0 || n > (int)c->col[box].size() || (n > 0 && !k))
    return fail(c, LC_EINVAL, "n exceeds the box's colloids, or out is NULL");
  if ((rc = pull_boxes(c)) != LC_OK) return rc;
  for (int i = 0; i < n; i++) k[i] = c->col[box][i];
  return LC_OK;
}

int lc_get_colloid(lc_ctx* c, int box, lc_colloid* k) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!k) return fail(c, LC_EINVAL, "colloid is NULL");
  if (c->col[box].empty()) {
    memset(k, 0, sizeof(*k));
    return LC_OK;
  }
  return lc_get_colloids(c, box, 1, k);
}

int lc_set_Q(lc_ctx* c, int box, const double* Q5) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!Q5) return fail(c, LC_EINVAL, "Q is NULL");
  return put(c, c->Q[c->cur], box, 5, Q5, false);
}
int lc_set_f(lc_ctx* c, int box, const double* f19) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!f19) return fail(c, LC_EINVAL, "f is NULL");
  return put(c, c->f[c->cur], box, 19, f19, true);
}
int lc_set_u(lc_ctx* c, int box, const double* u3) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!u3) return fail(c, LC_EINVAL, "u is NULL");
  return put(c, c->u[c->cur], box, 3, u3, false);
}
int lc_get_Q(lc_ctx* c, int box, double* Q5) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!Q5) return fail(c, LC_EINVAL, "Q is NULL");
  if ((rc = check_flag(c)) != LC_OK) return rc;
  return get(c, c->Q[c->cur], box, 5, Q5, false);
}
int lc_get_f(lc_ctx* c, int box, double* f19) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!f19) return fail(c, LC_EINVAL, "f is NULL");
  if ((rc = check_flag(c)) != LC_OK) return rc;
  return get(c, c->f[c->cur], box, 19, f19, true);
}
int lc_get_u(lc_ctx* c, int box, double* u3) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!u3) return fail(c, LC_EINVAL, "u is NULL");
  if ((rc = check_flag(c)) != LC_OK) return rc;
  return get(c, c->u[c->cur], box, 3, u3, false);
}

// Checkpoint layout: header, one record per box, the last-step forces,
// the force-history rings, then f, Q and u raw in the context's precision
// (the buffer of time n first, then the other one), native byte order.
struct StateHeader {
  char magic[8];
  int version, precision, nbox, hist_cap;
  long long nsites, nstep;
  int ncol, pad_;      // colloids in all boxes
};
struct StateBox {
  int nx, ny, nz, ncol;
};
struct StateCol {
  long long count;     // steps recorded in this colloid's history ring
  lc_colloid col;
};
const char kStateMagic[8] = {'L', 'C', 'S', 'T', 'A', 'T', 'E', '2'};
const int kStateVersion = 2;

size_t state_bytes_for(const lc_ctx* c, int ncol) {
  size_t sz[3];
  lc_buffer_bytes(c, sz);
  return sizeof(StateHeader) + sizeof(StateBox) * c->nbox + sizeof(StateCol) * ncol + sizeof(double) * 12 * ncol +
         sizeof(double) * 12 * (size_t)kHistCap * ncol + 2 * (sz[0] + sz[1] + sz[2]);
}

size_t state_bytes(const lc_ctx* c) { return state_bytes_for(c, c->ncol); }

int lc_state_bytes(const lc_ctx* c, size_t* out) {
  if (!c || !out) return LC_EINVAL;
  *out = state_bytes(c);
  return LC_OK;
}

int lc_get_state(lc_ctx* c, void* buf, size_t bytes) {
  if (!c) return LC_EINVAL;
  if (!buf || bytes < state_bytes(c)) return fail(c, LC_EINVAL, "state buffer is NULL or smaller than lc_state_bytes");
  int rc = check_flag(c);
  if (rc) return rc;
  if ((rc = flush(c)) != LC_OK) return rc;
  if ((rc = pull_boxes(c)) != LC_OK) return rc;
  char* p = (char*)buf;
  StateHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, kStateMagic, 8);
  h.version = kStateVersion;
  h.precision = c->prec;
  h.nbox = c->nbox;
  h.hist_cap = kHistCap;
  h.nsites = c->nsites;
  h.nstep = c->nstep;
  h.ncol = c->ncol;
  memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  std::vector<long long> cnt(std::max(1, c->ncol));
  if (c->ncol > 0) {
    HIPCHK(c, hipMemcpyAsync(cnt.data(), c->dcount, sizeof(long long) * c->ncol, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  for (int b = 0; b < c->nbox; b++) {
    StateBox r;
    memset(&r, 0, sizeof(r));
    r.nx = c->prm[b].nx; r.ny = c->prm[b].ny; r.nz = c->prm[b].nz;
    r.ncol = (int)c->col[b].size();
    memcpy(p, &r, sizeof(r));
    p += sizeof(r);
  }
  for (int b = 0; b < c->nbox; b++)
    for (size_t k = 0; k < c->col[b].size(); k++) {
      StateCol r;
      memset(&r, 0, sizeof(r));
      r.count = cnt[c->colbase[b] + k];
      r.col = c->col[b][k];
      memcpy(p, &r, sizeof(r));
      p += sizeof(r);
    }
  size_t sz[3];
  lc_buffer_bytes(c, sz);
  const size_t nforce = sizeof(double) * 12 * c->ncol, nhist = sizeof(double) * 12 * (size_t)kHistCap * c->ncol;
  if (c->ncol > 0) {
    HIPCHK(c, hipMemcpyAsync(p, c->dforce, nforce, hipMemcpyDeviceToHost, c->stream));
    p += nforce;
    HIPCHK(c, hipMemcpyAsync(p, c->dhist, nhist, hipMemcpyDeviceToHost, c->stream));
    p += nhist;
  }
  void* const* fld[3] = {c->f, c->Q, c->u};
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 2; j++) {
      HIPCHK(c, hipMemcpyAsync(p, fld[k][c->cur ^ j], sz[k], hipMemcpyDeviceToHost, c->stream));
      p += sz[k];
    }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

int lc_set_state(lc_ctx* c, const void* buf, size_t bytes) {
  if (!c) return LC_EINVAL;
  if (!buf || bytes < sizeof(StateHeader)) return fail(c, LC_EINVAL, "state buffer is NULL or too small");
  const char* p = (const char*)buf;
  StateHeader h;
  memcpy(&h, p, sizeof(h));
  p += sizeof(h);
  if (memcmp(h.magic, kStateMagic, 8) != 0 || h.version != kStateVersion)
    return fail(c, LC_EINVAL, "not a state written by lc_get_state (magic or version)");
  if (h.precision != c->prec || h.nbox != c->nbox || h.nsites != c->nsites || h.hist_cap != kHistCap)
    return fail(c, LC_EINVAL, "state precision, box count or size does not match the context");
  if (h.nstep < 0 || h.ncol < 0 || h.ncol > lc::kMaxColloids * c->nbox)
    return fail(c, LC_EINVAL, "bad step or colloid count in the state");
  if (bytes < state_bytes_for(c, h.ncol)) return fail(c, LC_EINVAL, "state buffer is smaller than the state it holds");
  // validate everything before changing the context
  std::vector<int> nb(c->nbox);
  int total = 0;
  for (int b = 0; b < c->nbox; b++) {
    StateBox r;
    memcpy(&r, p, sizeof(r));
    p += sizeof(r);
    if (r.nx != c->prm[b].nx || r.ny != c->prm[b].ny || r.nz != c->prm[b].nz)
      return fail(c, LC_EINVAL, "box " + std::to_string(b) + " of the state has another shape");
    if (r.ncol < 0 || r.ncol > lc::kMaxColloids) return fail(c, LC_EINVAL, "bad colloid count in the state");
    nb[b] = r.ncol;
    total += r.ncol;
  }
  if (total != h.ncol) return fail(c, LC_EINVAL, "colloid counts of the state do not add up");
  std::vector<long long> cnt(std::max(1, total));
  std::vector<std::vector<lc_colloid>> col(c->nbox);
  for (int b = 0, g = 0; b < c->nbox; b++) {
    std::vector<lc_colloid> raw(nb[b]);
    for (int k = 0; k < nb[b]; k++, g++) {
      StateCol r;
      memcpy(&r, p, sizeof(r));
      p += sizeof(r);
      if (r.count < 0) return fail(c, LC_EINVAL, "negative history count in the state");
      cnt[g] = r.count;
      raw[k] = r.col;
    }
    std::string why;
    if (check_colloids(c->prm[b], nb[b], raw.data(), col[b], why) != LC_OK)
      return fail(c, LC_EINVAL, "box " + std::to_string(b) + " of the state: " + why);
  }
  int frc = flush(c);   // a pending step of this context must not land in the restored history
  if (frc != LC_OK) return frc;
  if ((frc = pull_boxes(c)) != LC_OK) return frc;
  const std::vector<std::vector<lc_colloid>> old = c->col;
  const int old_tile = c->tile;
  c->col = col;
  if (needs_3d(c) && tile_shape(c, c->tile).kind == 1) c->tile = first_3d_tile(c);
  int rc = layout(c);
  if (rc != LC_OK) {
    const std::string e = c->err;
    c->col = old;
    c->tile = old_tile;
    layout(c);
    c->err = e;
    return rc;
  }
  size_t sz[3];
  lc_buffer_bytes(c, sz);
  const size_t nforce = sizeof(double) * 12 * total, nhist = sizeof(double) * 12 * (size_t)kHistCap * total;
  if (total > 0) {
    HIPCHK(c, hipMemsetAsync(c->dpending, 0, sizeof(int) * total, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dcount, cnt.data(), sizeof(long long) * total, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dforce, p, nforce, hipMemcpyHostToDevice, c->stream));
    p += nforce;
    HIPCHK(c, hipMemcpyAsync(c->dhist, p, nhist, hipMemcpyHostToDevice, c->stream));
    p += nhist;
  }
  void* const* fld[3] = {c->f, c->Q, c->u};
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 2; j++) {
      HIPCHK(c, hipMemcpyAsync(fld[k][c->cur ^ j], p, sz[k], hipMemcpyHostToDevice, c->stream));
      p += sz[k];
    }
  HIPCHK(c, hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->nstep = (long)h.nstep;
  return LC_OK;
}

int lc_step(lc_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return LC_EINVAL;
  int left = nsteps;
  if (nsteps > 0) {
    int rc = ghost_pass(c);
    if (rc != LC_OK) return rc;
  }
  auto eager = [&]() -> int {
    hipError_t e = enqueue(c, c->cur);
    if (e != hipSuccess) return fail(c, LC_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    c->cur ^= 1;
    c->nstep++;
    left--;
    return LC_OK;
  };
  int rc;
  if (c->use_graph && left >= kGraphSteps + (c->cur ? 1 : 0)) {
    if (c->cur == 1 && (rc = eager()) != LC_OK) return rc;
    if (!c->graph_ok && (rc = build_graph(c)) != LC_OK) return rc;
    while (left >= kGraphSteps) {
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      c->nstep += kGraphSteps;
      left -= kGraphSteps;
    }
    // the replayed graph's last step is finished by the next step or, for
    // the getters, by flush (the flag is set on the host, not by the capture)
    c->maybe_pending = true;
  }
  while (left > 0)
    if ((rc = eager()) != LC_OK) return rc;
  return LC_OK;
}

int lc_prepare(lc_ctx* c) {
  if (!c) return LC_EINVAL;
  if (!c->use_graph || c->graph_ok) return LC_OK;
  return build_graph(c);
}

int lc_sync(lc_ctx* c) {
  if (!c) return LC_EINVAL;
  return check_flag(c);
}

long lc_get_nstep(lc_ctx* c) { return c ? c->nstep : -1; }

int lc_get_colloid_force(lc_ctx* c, int box, int k, double out[12]) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!out) return fail(c, LC_EINVAL, "out is NULL");
  if (k < 0 || k >= (int)c->col[box].size()) return fail(c, LC_EINVAL, "colloid index out of range");
  if ((rc = flush(c)) != LC_OK) return rc;
  HIPCHK(c, hipMemcpyAsync(out, c->dforce + 12 * (c->colbase[box] + k), sizeof(double) * 12, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LC_OK;
}

int lc_get_force(lc_ctx* c, int box, double out[12]) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!out) return fail(c, LC_EINVAL, "out is NULL");
  if (c->col[box].empty()) {
    for (int i = 0; i < 12; i++) out[i] = 0.0;
    return LC_OK;
  }
  return lc_get_colloid_force(c, box, 0, out);
}

int lc_history_capacity(const lc_ctx* c) { return c ? kHistCap : 0; }

int lc_get_colloid_force_history(lc_ctx* c, int box, int k, int nsteps, double* out) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (k < 0 || k >= (int)c->col[box].size()) return fail(c, LC_EINVAL, "colloid index out of range");
  if (!out || nsteps < 0 || nsteps > kHistCap)
    return fail(c, LC_EINVAL, "nsteps exceeds the history capacity, or out is NULL");
  if ((rc = flush(c)) != LC_OK) return rc;
  const int g = c->colbase[box] + k;
  long long cnt = 0;
  HIPCHK(c, hipMemcpyAsync(&cnt, c->dcount + g, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (nsteps > cnt) return fail(c, LC_EINVAL, "nsteps exceeds the steps this colloid has taken");
  std::vector<double> h((size_t)kHistCap * 12);
  HIPCHK(c, hipMemcpyAsync(h.data(), c->dhist + (size_t)g * kHistCap * 12, sizeof(double) * h.size(),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int j = 0; j < nsteps; j++) {
    const long long n = cnt - nsteps + j;
    memcpy(out + 12 * j, h.data() + 12 * (n % kHistCap), sizeof(double) * 12);
  }
  return LC_OK;
}

int lc_get_force_history(lc_ctx* c, int box, int nsteps, double* out) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!out || nsteps < 0 || nsteps > kHistCap || nsteps > c->nstep)
    return fail(c, LC_EINVAL, "nsteps exceeds the steps taken or the history capacity");
  if (c->col[box].empty()) {   // no colloid: no force
    for (long j = 0; j < 12L * nsteps; j++) out[j] = 0.0;
    return LC_OK;
  }
  return lc_get_colloid_force_history(c, box, 0, nsteps, out);
}

int lc_get_solid(lc_ctx* c, int box, unsigned char* id) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!id) return fail(c, LC_EINVAL, "out is NULL");
  const long long n = box_sites(c->prm[box]);
  unsigned char* d = nullptr;
  HIPCHK(c, hipMalloc(&d, n));
  hipError_t e = lc::launch_solid(c->dbox, c->dcol, box, n, d, c->cur, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(id, d, n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  HIPCHK(c, e);
  return LC_OK;
}

int lc_get_diag(lc_ctx* c, int box, lc_diag* out) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!out) return fail(c, LC_EINVAL, "out is NULL");
  if ((rc = check_flag(c)) != LC_OK) return rc;
  const long long n = box_sites(c->prm[box]);
  const long long nb = (n + 255) / 256;
  if ((size_t)(6 * nb) > c->ddiag_cap) {
    if (c->ddiag) (void)hipFree(c->ddiag);
    c->ddiag = nullptr;
    c->ddiag_cap = 6 * nb;
    HIPCHK(c, hipMalloc(&c->ddiag, sizeof(double) * c->ddiag_cap));
  }
  hipError_t e = hipSuccess;
  if (c->prec == LC_FP32) {
    lc::StepPtrs<float> a = ptrs<float>(c, c->cur);
    if (c->any_colloid)
      e = lc::launch_ghost<float>(c->dbox, c->dcol, c->ncol, c->ghost_total, (float*)c->Q[c->cur], c->nsites, c->cur,
                                  c->stream);
    if (e == hipSuccess) e = lc::launch_diag<float>(c->dbox, box, n, a, c->ddiag, c->stream);
  } else {
    lc::StepPtrs<double> a = ptrs<double>(c, c->cur);
    if (c->any_colloid)
      e = lc::launch_ghost<double>(c->dbox, c->dcol, c->ncol, c->ghost_total, (double*)c->Q[c->cur], c->nsites,
                                   c->cur, c->stream);
    if (e == hipSuccess) e = lc::launch_diag<double>(c->dbox, box, n, a, c->ddiag, c->stream);
  }
  HIPCHK(c, e);
  std::vector<double> h((size_t)(6 * nb));
  HIPCHK(c, hipMemcpyAsync(h.data(), c->ddiag, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memset(out, 0, sizeof(*out));
  for (long long k = 0; k < nb; k++) {
    out->free_energy += h[6 * k + 0];
    out->mass += h[6 * k + 1];
    for (int a = 0; a < 3; a++) out->momentum[a] += h[6 * k + 2 + a];
    out->umax = std::max(out->umax, h[6 * k + 5]);
  }
  return LC_OK;
}

int lc_get_diag_noalloc(lc_ctx* c, int box, lc_diag* out) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if (!out) return fail(c, LC_EINVAL, "out is NULL");
  const long long n = box_sites(c->prm[box]);
  const long long nb = (n + 255) / 256;
  if (nb > kNoallocDiagBlocks)
    return fail(c, LC_EINVAL, "box of " + std::to_string(n) + " sites exceeds the static diagnostics scratch (at most " +
                                  std::to_string(kNoallocDiagBlocks * 256) + " sites); use lc_get_diag");
  if (!c->scratch_dev) return fail(c, LC_EDEVICE, c->scratch_err);
  if ((rc = check_flag(c)) != LC_OK) return rc;
  hipError_t e;
  if (c->prec == LC_FP32) {
    lc::StepPtrs<float> a = ptrs<float>(c, c->cur);
    if (c->any_colloid &&
        (e = lc::launch_ghost<float>(c->dbox, c->dcol, c->ncol, c->ghost_total, (float*)c->Q[c->cur], c->nsites, c->cur,
                                     c->stream)) != hipSuccess)
      return fail(c, LC_EDEVICE, std::string("ghost launch: ") + hipGetErrorString(e));
    e = lc::launch_diag<float>(c->dbox, box, n, a, c->scratch_dev, c->stream);
  } else {
    lc::StepPtrs<double> a = ptrs<double>(c, c->cur);
    if (c->any_colloid &&
        (e = lc::launch_ghost<double>(c->dbox, c->dcol, c->ncol, c->ghost_total, (double*)c->Q[c->cur], c->nsites, c->cur,
                                      c->stream)) != hipSuccess)
      return fail(c, LC_EDEVICE, std::string("ghost launch: ") + hipGetErrorString(e));
    e = lc::launch_diag<double>(c->dbox, box, n, a, c->scratch_dev, c->stream);
  }
  HIPCHK(c, e);
  HIPCHK(c, lc::launch_diag_total(c->scratch_dev, nb, c->scratch_dev + kNoallocTotals, c->stream));
  double tot[6];
  HIPCHK(c, hipMemcpyAsync(tot, c->scratch_dev + kNoallocTotals, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out->free_energy = tot[0];
  out->mass = tot[1];
  for (int a = 0; a < 3; a++) out->momentum[a] = tot[2 + a];
  out->umax = tot[5];
  return LC_OK;
}

int lc_defects(lc_ctx* c, int box, double threshold, unsigned char* mask, long* count_out) {
  int rc = check_box(c, box);
  if (rc) return rc;
  if ((rc = check_flag(c)) != LC_OK) return rc;
  const long long n = box_sites(c->prm[box]);
  unsigned char* dm = nullptr;
  unsigned long long* dc = nullptr;
  HIPCHK(c, hipMalloc(&dm, n));
  if (hipMalloc(&dc, sizeof(unsigned long long)) != hipSuccess) {
    (void)hipFree(dm);
    return fail(c, LC_ENOMEM, "hipMalloc failed");
  }
  hipError_t e = hipMemsetAsync(dc, 0, sizeof(unsigned long long), c->stream);
  if (e == hipSuccess)
    e = c->prec == LC_FP32
            ? lc::launch_defects<float>(c->dbox, c->dcol, box, n, (const float*)c->Q[c->cur], c->nsites, threshold,
                                        dm, dc, c->cur, c->stream)
            : lc::launch_defects<double>(c->dbox, c->dcol, box, n, (const double*)c->Q[c->cur], c->nsites, threshold,
                                         dm, dc, c->cur, c->stream);
  unsigned long long cnt = 0;
  if (e == hipSuccess) {
    if (mask) e = hipMemcpyAsync(mask, dm, n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, dc, sizeof(cnt), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  (void)hipFree(dm);
  (void)hipFree(dc);
  HIPCHK(c, e);
  if (count_out) *count_out = (long)cnt;
  return LC_OK;
}

int lc_num_tiles(const lc_ctx* c) { return c ? num_tiles(c) : 0; }

int lc_tile_shape(const lc_ctx* c, int id, int out[3]) {
  if (!c || !out || id < 0 || id >= num_tiles(c)) return LC_EINVAL;
  const TileShape& t = tile_shape(c, id);
  out[0] = t.x;
  out[1] = t.y;
  out[2] = t.z;
  return LC_OK;
}

int lc_set_tile(lc_ctx* c, int id) {
  if (!c) return LC_EINVAL;
  if (id < 0 || id >= num_tiles(c)) return fail(c, LC_EINVAL, "tile id out of range");
  if (id == c->tile) return LC_OK;
  int rc = pull_boxes(c);
  if (rc) return rc;
  const int old = c->tile;
  c->tile = id;
  rc = layout(c);
  if (rc != LC_OK) {   // keep the context on its previous shape
    const std::string why = c->err;
    c->tile = old;
    layout(c);
    c->err = why;
  }
  return rc;
}

int lc_get_tile(const lc_ctx* c) { return c ? c->tile : -1; }

int lc_use_graph(lc_ctx* c, int enable) {
  if (!c) return LC_EINVAL;
  c->use_graph = enable != 0;
  return LC_OK;
}

int lc_launch_info(const lc_ctx* c, long out[2]) {
  if (!c || !out) return LC_EINVAL;
  const TileShape& t = tile_shape(c, c->tile);
  out[0] = c->nblk;
  out[1] = t.kind ? (long)t.x * t.y : (long)t.x * t.y * t.z;
  return LC_OK;
}

int lc_time_kernel(lc_ctx* c, int nsteps, double out[3]) {
  if (!c || !out || nsteps < 1) return LC_EINVAL;
  int rc = ghost_pass(c);
  if (rc != LC_OK) return rc;
  // every stride-th dispatch carries the events (the last of each run of
  // stride), at most kTimedDispatches over the run
  const int stride = (nsteps + kTimedDispatches - 1) / kTimedDispatches;
  const int nt = nsteps / stride;
  std::vector<hipEvent_t> ev(2 * nt + 2);
  for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
  HIPCHK(c, hipEventRecord(ev[2 * nt], c->stream));
  for (int k = 0; k < nsteps; k++) {
    const bool timed = (k + 1) % stride == 0;
    const int j = (k + 1) / stride - 1;
    hipError_t e = timed ? enqueue(c, c->cur, ev[2 * j], ev[2 * j + 1]) : enqueue(c, c->cur);
    if (e != hipSuccess) return fail(c, LC_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    c->cur ^= 1;
    c->nstep++;
  }
  HIPCHK(c, hipEventRecord(ev[2 * nt + 1], c->stream));
  HIPCHK(c, hipEventSynchronize(ev[2 * nt + 1]));
  double ks = 0.0;
  for (int j = 0; j < nt; j++) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
    ks += ms;
  }
  float tot = 0.f;
  HIPCHK(c, hipEventElapsedTime(&tot, ev[2 * nt], ev[2 * nt + 1]));
  for (auto& e : ev) (void)hipEventDestroy(e);
  out[0] = ks / nt;
  out[1] = tot / nsteps;
  out[2] = tot;
  return check_flag(c);
}

}  // extern "C"
