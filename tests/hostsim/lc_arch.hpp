// Host version of the marching kernel's architecture layer (the names of
// paper_1102_2193_amd/csrc/lc_arch.hpp), with every access checked.
// Test infrastructure only.
//
//   lds_sync   block rendezvous;
//   FieldBuf   any element type (FP32 or FP64); each load and store checks
//              the component and site against the array, forms the byte
//              offset in 32 bits as the device does and checks it against
//              the resource's range, and counts the stores per element;
//   lds_at     a pointer object whose reads check the component range;
//   keep_live  nothing.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>

#define LC_ARCH_LAYER 1

namespace hostsim {

// A device array known to the driver: name, size and a store count per
// element (null for inputs).
struct ArrayInfo {
  const char* name;
  const void* base;
  long long ns;
  int ncomp;
  int esize;
  std::atomic<unsigned char>* stores;
};
const ArrayInfo& array_info(const void* base);

}  // namespace hostsim

namespace lc {

inline void lds_sync() { hostsim::block_barrier("lds_sync"); }

struct FieldBuf {
  const hostsim::ArrayInfo* a;
  char* p;
  unsigned nrec;   // range of the resource in bytes, formed as on the device
  unsigned cs;     // bytes between components
  template <typename T>
  FieldBuf(const T* ptr, long long ns, int ncomp)
      : a(&hostsim::array_info(ptr)),
        p((char*)ptr),
        nrec((unsigned)ncomp * (unsigned)ns * (unsigned)sizeof(T)),
        cs((unsigned)ns * (unsigned)sizeof(T)) {
    if (a->ns != ns || a->ncomp != ncomp || a->esize != (int)sizeof(T))
      hostsim::fail("FieldBuf %s: made with ns %lld ncomp %d, array has ns %lld ncomp %d", a->name, ns, ncomp, a->ns,
                    a->ncomp);
    if ((unsigned long long)ncomp * (unsigned long long)ns * sizeof(T) >= (1ull << 32))
      hostsim::fail("FieldBuf %s: %d x %lld elements do not fit a 32-bit range", a->name, ncomp, ns);
  }
  // byte offset of (c, s) exactly as the device forms it (32-bit unsigned)
  unsigned byte(int c, unsigned s, const char* op) const {
    if (c < 0 || c >= a->ncomp || (long long)s >= a->ns)
      hostsim::fail("%s %s: component %d site %u outside %d x %lld (thread %u block %u)", op, a->name, c, s, a->ncomp,
                    a->ns, threadIdx.x, blockIdx.x);
    const unsigned off = s * (unsigned)a->esize + (unsigned)c * cs;
    const unsigned long long want = (unsigned long long)s * a->esize + (unsigned long long)c * a->ns * a->esize;
    if (off != want || off >= nrec) hostsim::fail("%s %s: byte offset %u (want %llu) range %u", op, a->name, off, want, nrec);
    return off;
  }
  struct Val {
    const char* q;
    int esize;
    operator float() const {
      if (esize == 4) { float v; std::memcpy(&v, q, 4); return v; }
      double v; std::memcpy(&v, q, 8); return (float)v;
    }
    operator double() const {
      if (esize == 8) { double v; std::memcpy(&v, q, 8); return v; }
      float v; std::memcpy(&v, q, 4); return (double)v;
    }
  };
  Val ld(int c, unsigned s) const { return Val{p + byte(c, s, "load"), a->esize}; }
  Val ld_nt(int c, unsigned s) const { return ld(c, s); }
  template <typename V>
  void st(int c, unsigned s, V v) const {
    const unsigned off = byte(c, s, "store");
    if (!a->stores) hostsim::fail("store into input array %s", a->name);
    if (a->esize == 4) { const float x = (float)v; std::memcpy(p + off, &x, 4); }
    else { const double x = (double)v; std::memcpy(p + off, &x, 8); }
    a->stores[off / a->esize].fetch_add(1, std::memory_order_relaxed);
  }
  template <typename V>
  void st_nt(int c, unsigned s, V v) const { st(c, s, v); }
};

template <typename T>
struct LdsRow {
  const T* row;
  int n_all, lo, n, off;
  const T& operator[](int i) const {
    const int k = lo + off + i;
    if (off + i < 0 || off + i >= n || k < 0 || k >= n_all)
      hostsim::fail("LDS read at %d outside component [%d, %d) of a %d-element row (thread %u block %u)", k, lo,
                    lo + n, n_all, threadIdx.x, blockIdx.x);
    return row[k];
  }
};
template <typename T, int N>
LdsRow<T> lds_at(const T (&row)[N], int lo, int n, int off) {
  return LdsRow<T>{row, N, lo, n, off};
}

template <typename R>
inline void keep_live(const R (&)[5]) {}

}  // namespace lc
