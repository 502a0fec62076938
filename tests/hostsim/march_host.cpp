// CPU run of the marching kernel's own source (paper_1102_2193_amd/csrc/
// lc_march.hpp) over one box for one step, with the architecture layer of
// this directory: every global access checked against its array and its
// 32-bit byte offset, every LDS read made through a component pointer
// checked against that component, every direct LDS subscript checked by the
// compiler's bounds sanitizer, LDS filled with 0xff bytes before each
// block, stores counted per element.  Test infrastructure only: it shares
// the kernel's code, not the oracle's, and the test compares its results
// with the oracle.
//
// build:  clang++ -std=c++17 -pthread -ffp-contract=off -DHOSTSIM_TX=32 -DHOSTSIM_TY=16
//         -I tests/hostsim -I paper_1102_2193_amd/csrc march_host.cpp (+ a sanitizer)
// usage: march_host <case dir> <out dir> <TX> <TY> <f32|f64> <planes per item> <items per block>
//   case dir: params.txt (key value lines), f.bin (19 x N, stored form f - w),
//             Q.bin (5 x N, ghost values at solid nodes), u.bin (3 x N); doubles
//   out dir:  f.bin, Q.bin, u.bin (NaN where not written), stores_f.bin,
//             stores_Q.bin, stores_u.bin (uint8 counts), force.bin (12 sums of
//             the colloid slots, slot order), report.txt
#include "lc_arch.hpp"
#include "lc_march.hpp"

#include <pthread.h>
#include <time.h>

#include <cstdarg>
#include <limits>
#include <memory>
#include <vector>

extern "C" char __start_hostsim_lds[], __stop_hostsim_lds[];

namespace hostsim {

thread_local dim3 thread_idx, block_idx;

void fail(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "march_host: ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
  std::fflush(stderr);
  std::abort();
}

constexpr int kWaitSeconds = 60;

// Generation-counting rendezvous of `live` threads; a thread that finishes
// the kernel leaves the count, as a finished wave leaves the hardware
// barrier.  Plain pthreads (the C library is what the sanitizers intercept).
struct Rendezvous {
  pthread_mutex_t m = PTHREAD_MUTEX_INITIALIZER;
  pthread_cond_t cv = PTHREAD_COND_INITIALIZER;
  int live = 0, arrived = 0;
  long long gen = 0;
  ~Rendezvous() {
    pthread_mutex_destroy(&m);
    pthread_cond_destroy(&cv);
  }
  void release() {
    arrived = 0;
    gen++;
    pthread_cond_broadcast(&cv);
  }
  void arrive(const char* what) {
    pthread_mutex_lock(&m);
    const long long g = gen;
    if (++arrived == live) {
      release();
      pthread_mutex_unlock(&m);
      return;
    }
    timespec until;
    clock_gettime(CLOCK_REALTIME, &until);
    until.tv_sec += kWaitSeconds;
    while (gen == g)
      if (pthread_cond_timedwait(&cv, &m, &until) != 0 && gen == g)
        fail("%s: %d of %d threads arrived (thread %u block %u)", what, arrived, live, thread_idx.x, block_idx.x);
    pthread_mutex_unlock(&m);
  }
  void leave() {
    pthread_mutex_lock(&m);
    live--;
    if (arrived > 0 && arrived == live) release();
    pthread_mutex_unlock(&m);
  }
};

struct Wave {
  Rendezvous rv;
  uint64_t word[64];
};

struct Block {
  Rendezvous rv;
  std::vector<std::unique_ptr<Wave>> waves;
};
Block* g_block = nullptr;

void block_barrier(const char* what) { g_block->rv.arrive(what); }

void wave_gather(uint64_t mine, uint64_t all[64], const char* what) {
  Wave& w = *g_block->waves[thread_idx.x >> 6];
  w.word[thread_idx.x & 63] = mine;
  w.rv.arrive(what);
  std::memcpy(all, w.word, sizeof(w.word));
  w.rv.arrive(what);
}

std::vector<ArrayInfo> g_arrays;
const ArrayInfo& array_info(const void* base) {
  for (const ArrayInfo& a : g_arrays)
    if (a.base == base) return a;
  fail("FieldBuf over an unknown array %p", base);
}

// Runs fn() as a block of nt threads.
template <typename F>
void run_block(unsigned nt, unsigned blk, F& fn) {
  Block b;
  b.rv.live = (int)nt;
  for (unsigned w = 0; w < nt / 64; w++) {
    b.waves.emplace_back(new Wave);
    b.waves.back()->rv.live = 64;
  }
  g_block = &b;
  std::memset(__start_hostsim_lds, 0xff, (size_t)(__stop_hostsim_lds - __start_hostsim_lds));
  struct Arg {
    F* fn;
    Block* b;
    unsigned t, blk;
  };
  std::vector<Arg> args(nt);
  std::vector<pthread_t> th(nt);
  pthread_attr_t attr;
  pthread_attr_init(&attr);
  pthread_attr_setstacksize(&attr, 4 << 20);
  for (unsigned t = 0; t < nt; t++) {
    args[t] = Arg{&fn, &b, t, blk};
    auto body = [](void* p) -> void* {
      Arg& a = *(Arg*)p;
      thread_idx.x = a.t;
      block_idx.x = a.blk;
      (*a.fn)();
      a.b->waves[a.t >> 6]->rv.leave();
      a.b->rv.leave();
      return nullptr;
    };
    if (pthread_create(&th[t], &attr, body, &args[t]) != 0) fail("pthread_create failed for thread %u", t);
  }
  for (unsigned t = 0; t < nt; t++) pthread_join(th[t], nullptr);
  pthread_attr_destroy(&attr);
  g_block = nullptr;
}

}  // namespace hostsim

namespace {

using hostsim::fail;

// params.txt: "key value" lines
struct Params {
  struct KV {
    char k[32];
    double v;
  };
  std::vector<KV> kv;
  double operator()(const char* k) const {
    for (const KV& e : kv)
      if (!std::strcmp(e.k, k)) return e.v;
    fail("params: %s missing", k);
  }
  double at(const char* k, int i) const {
    char name[40];
    std::snprintf(name, sizeof(name), "%s%d", k, i);
    return (*this)(name);
  }
};

const char* path(const char* dir, const char* name) {
  static thread_local char buf[4096];
  std::snprintf(buf, sizeof(buf), "%s/%s", dir, name);
  return buf;
}

Params read_params(const char* dir) {
  FILE* f = std::fopen(path(dir, "params.txt"), "r");
  if (!f) fail("cannot read %s/params.txt", dir);
  Params p;
  Params::KV e;
  while (std::fscanf(f, "%31s %lf", e.k, &e.v) == 2) p.kv.push_back(e);
  std::fclose(f);
  return p;
}

std::vector<double> read_doubles(const char* dir, const char* name, size_t n) {
  std::vector<double> v(n);
  FILE* f = std::fopen(path(dir, name), "rb");
  if (!f || std::fread(v.data(), sizeof(double), n, f) != n) fail("cannot read %zu doubles from %s/%s", n, dir, name);
  std::fclose(f);
  return v;
}

void write_bytes(const char* dir, const char* name, const void* p, size_t n) {
  FILE* f = std::fopen(path(dir, name), "wb");
  if (!f || std::fwrite(p, 1, n, f) != n) fail("cannot write %s/%s", dir, name);
  std::fclose(f);
}

template <typename R, int TX, int TY, int CZ>
int run(const Params& get, const char* dir, const char* out, int planes, int per_block) {
  using lc::BoxDev;
  using lc::ColDev;
  BoxDev B;
  std::memset(&B, 0, sizeof(B));
  B.nx = (int)get("nx"); B.ny = (int)get("ny"); B.nz = (int)get("nz");
  B.hydro = (int)get("hydro");
  B.off = 0;
  B.tile_base = 0;
  B.ntx = (B.nx + TX - 1) / TX;
  B.nty = (B.ny + TY - 1) / TY;
  B.ntz = (B.nz + lc::kGroup - 1) / lc::kGroup;
  B.tau = get("tau"); B.rho0 = get("rho0"); B.A0 = get("A0"); B.gamma = get("gamma"); B.K = get("K");
  B.q0 = get("q0"); B.xi = get("xi"); B.Gamma = get("Gamma");
  B.itau = 1.0 / B.tau;
  B.fsrc = 1.0 - 0.5 / B.tau;
  B.body[0] = get("body0"); B.body[1] = get("body1"); B.body[2] = get("body2");
  B.adv = 1;
  B.st27 = 0;
  B.col0 = 0;
  B.ncol = (int)get("ncol");
  const long long N = (long long)B.nx * B.ny * B.nz;
  const int ncb = B.ntx * B.nty;
  const long long nslot = (long long)ncb * B.ntz;

  ColDev C;
  std::memset(&C, 0, sizeof(C));
  if (B.ncol) {
    C.box = 0;
    C.motion = (int)get("motion");
    C.anchoring = (int)get("anchoring");
    for (int k = 0; k < 3; k++) {
      C.pos[0][k] = C.pos[1][k] = get.at("pos", k);
      C.vel[k] = get.at("vel", k);
      C.omega[k] = get.at("omega", k);
    }
    C.a0 = get("a0");
    C.S0 = get("S0");
    C.W = get("W");
    C.slot_base = 0;
  }

  std::vector<R> fin(19 * N), Qin(5 * N), uin(3 * N), fout(19 * N), Qout(5 * N), uout(3 * N);
  {
    const auto f = read_doubles(dir, "f.bin", 19 * N), Q = read_doubles(dir, "Q.bin", 5 * N),
               u = read_doubles(dir, "u.bin", 3 * N);
    for (long long i = 0; i < 19 * N; i++) fin[i] = (R)f[i];
    for (long long i = 0; i < 5 * N; i++) Qin[i] = (R)Q[i];
    for (long long i = 0; i < 3 * N; i++) uin[i] = (R)u[i];
  }
  const R nan = std::numeric_limits<R>::quiet_NaN();
  std::fill(fout.begin(), fout.end(), nan);
  std::fill(Qout.begin(), Qout.end(), nan);
  std::fill(uout.begin(), uout.end(), nan);
  std::unique_ptr<std::atomic<unsigned char>[]> sf(new std::atomic<unsigned char>[19 * N]),
      sq(new std::atomic<unsigned char>[5 * N]), su(new std::atomic<unsigned char>[3 * N]);
  for (long long i = 0; i < 19 * N; i++) sf[i] = 0;
  for (long long i = 0; i < 5 * N; i++) sq[i] = 0;
  for (long long i = 0; i < 3 * N; i++) su[i] = 0;
  const int es = (int)sizeof(R);
  hostsim::g_arrays = {{"fin", fin.data(), N, 19, es, nullptr},       {"Qin", Qin.data(), N, 5, es, nullptr},
                       {"uin", uin.data(), N, 3, es, nullptr},        {"fout", fout.data(), N, 19, es, sf.get()},
                       {"Qout", Qout.data(), N, 5, es, sq.get()},     {"uout", uout.data(), N, 3, es, su.get()}};

  // colloid slots, NaN until written; a separate allocation, so the
  // address sanitizer sees any write beyond it
  std::unique_ptr<double[]> part(new double[12 * nslot]);
  for (long long i = 0; i < 12 * nslot; i++) part[i] = std::numeric_limits<double>::quiet_NaN();
  int flag = 0;
  std::unique_ptr<ColDev[]> cols(new ColDev[1]);
  cols[0] = C;
  std::unique_ptr<BoxDev[]> boxes(new BoxDev[1]);
  boxes[0] = B;

  lc::StepPtrs<R> a;
  a.fin = fin.data(); a.fout = fout.data();
  a.Qin = Qin.data(); a.Qout = Qout.data();
  a.uin = uin.data(); a.uout = uout.data();
  a.nsites = N;
  a.part = part.get();
  a.nslot = nslot;
  a.flag = &flag;
  a.par = 0;
  a.cols = cols.get();

  // work items: each column block's groups cut into runs of `planes`
  std::vector<int2> items;
  for (int cb = 0; cb < ncb; cb++)
    for (int g = 0; g < B.ntz; g += planes) items.push_back(lc::march_item(0, cb, g, std::min(planes, B.ntz - g)));
  std::vector<int> offs(1, 0);
  while (offs.back() < (int)items.size()) offs.push_back(std::min((int)items.size(), offs.back() + per_block));
  const int nblk = (int)offs.size() - 1;
  std::unique_ptr<int2[]> ditems(new int2[items.size()]);
  std::copy(items.begin(), items.end(), ditems.get());
  std::unique_ptr<int[]> doffs(new int[offs.size()]);
  std::copy(offs.begin(), offs.end(), doffs.get());

  auto kernel = [&] { lc::k_march<R, TX, TY, CZ>(boxes.get(), ditems.get(), doffs.get(), a); };
  for (int b = 0; b < nblk; b++) hostsim::run_block(TX * TY, (unsigned)b, kernel);

  // results
  auto dump = [&](const char* name, const std::vector<R>& v) {
    std::vector<double> d(v.begin(), v.end());
    write_bytes(out, name, d.data(), d.size() * sizeof(double));
  };
  dump("f.bin", fout);
  dump("Q.bin", Qout);
  dump("u.bin", uout);
  auto dumpc = [&](const char* name, const std::atomic<unsigned char>* s, long long n) {
    std::vector<unsigned char> c(n);
    for (long long i = 0; i < n; i++) c[i] = s[i].load();
    write_bytes(out, name, c.data(), c.size());
  };
  dumpc("stores_f.bin", sf.get(), 19 * N);
  dumpc("stores_Q.bin", sq.get(), 5 * N);
  dumpc("stores_u.bin", su.get(), 3 * N);
  double force[12] = {0};
  long long unwritten = 0;
  if (B.ncol)
    for (int c = 0; c < 12; c++)
      for (long long s = 0; s < nslot; s++) {
        const double v = part[c * nslot + s];
        if (std::isnan(v)) unwritten++;
        else force[c] += v;
      }
  write_bytes(out, "force.bin", force, sizeof(force));
  FILE* rep = std::fopen(path(out, "report.txt"), "w");
  if (!rep) fail("cannot write %s/report.txt", out);
  std::fprintf(rep, "lds_bytes %zu\nlds_section_bytes %lld\nblocks %d\nitems %zu\nslots %lld\nslots_unwritten %lld\nflag %d\n",
               sizeof(lc::MarchSmem<R, TX, TY>), (long long)(__stop_hostsim_lds - __start_hostsim_lds), nblk,
               items.size(), nslot, unwritten, flag);
  std::fclose(rep);
  return 0;
}

// One marching shape per build (-DHOSTSIM_TX=.. -DHOSTSIM_TY=..; the plane
// count CZ of a shape only sizes the work items the runtime makes, which
// this driver makes itself), so the sanitizer builds compile in parallel.
template <typename R>
int dispatch(int tx, int ty, const Params& p, const char* dir, const char* out, int planes, int per_block) {
  if (tx == HOSTSIM_TX && ty == HOSTSIM_TY) return run<R, HOSTSIM_TX, HOSTSIM_TY, 8>(p, dir, out, planes, per_block);
  fail("this build runs the %d x %d shape, not %d x %d", HOSTSIM_TX, HOSTSIM_TY, tx, ty);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 8) fail("usage: march_host <case dir> <out dir> <TX> <TY> <f32|f64> <planes> <items per block>");
  const char *dir = argv[1], *out = argv[2], *prec = argv[5];
  const int tx = std::atoi(argv[3]), ty = std::atoi(argv[4]), planes = std::atoi(argv[6]), per = std::atoi(argv[7]);
  if (planes < 1 || per < 1) fail("planes and items per block must be positive");
  const Params p = read_params(dir);
  if (!std::strcmp(prec, "f32")) return dispatch<float>(tx, ty, p, dir, out, planes, per);
  if (!std::strcmp(prec, "f64")) return dispatch<double>(tx, ty, p, dir, out, planes, per);
  fail("precision %s", prec);
}
