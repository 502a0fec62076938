// lc_arch.hpp -- the few gfx950-specific operations of the marching kernel:
// an LDS-only barrier, FP32 field arrays addressed through one buffer
// resource each, a pointer into one component of an LDS array, and a
// register keep-alive.  Everything else in the kernel is plain C++ over
// these, so a host build that supplies its own versions of exactly these
// names (with bounds checks) runs the kernel's index arithmetic unchanged.
#pragma once

#include <hip/hip_runtime.h>

#define LC_ARCH_LAYER 1

namespace lc {

// Barrier that orders LDS only: global loads issued before it stay in
// flight (the populations are requested at kernel entry).
__device__ inline void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// FP32 field array [component][site] addressed through one buffer resource:
// component c of site s is at byte s*4 (per lane) + c*stride (scalar
// offset).  One 128-bit resource per array replaces a 64-bit base address
// per component, which the marching kernel cannot keep in scalar registers.
// The range is the whole array (ncomp x ns floats), so no access is
// clamped.  FP32 only: the marching kernel exists in FP32 alone.
struct FieldBuf {
  __amdgpu_buffer_rsrc_t r;
  unsigned cs;   // bytes between components
  __device__ FieldBuf(const float* p, long long ns, int ncomp)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)((unsigned)ncomp * (unsigned)ns * 4u),
                                            0x00020000)),
        cs((unsigned)ns * 4u) {}
  // Scalar offset of component c.  The empty asm hides the stride from the
  // optimiser at each access, so the product is formed by one scalar
  // multiply next to its load or store; left visible, all eighteen products
  // are hoisted out of the plane loop, overflow the scalar registers and come
  // back through vector-lane reloads (a vector instruction plus a wait
  // before each access).
  __device__ unsigned co(int c) const {
    if (c == 0) return 0u;
    unsigned k = cs;
    asm volatile("" : "+s"(k));
    return (unsigned)c * k;
  }
  // aux 2 = non-temporal (streamed once)
  __device__ float ld(int c, unsigned s) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, s * 4u, co(c), 0));
  }
  __device__ float ld_nt(int c, unsigned s) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, s * 4u, co(c), 2));
  }
  __device__ void st(int c, unsigned s, float v) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, s * 4u, co(c), 0);
  }
  __device__ void st_nt(int c, unsigned s, float v) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, s * 4u, co(c), 2);
  }
};

// Element `off` of LDS component [lo, lo + n) of an array: the reads made
// through the pointer stay within that component (n is checked only by the
// host version of this layer).
template <typename T, int N>
__device__ inline const T* lds_at(const T (&row)[N], int lo, [[maybe_unused]] int n, int off) {
  return row + lo + off;
}

// Keeps five values live in vector registers (their computation cannot be
// dropped or rescheduled as dead code).
template <typename R>
__device__ inline void keep_live(const R (&v)[5]) {
  asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]));
}

}  // namespace lc
