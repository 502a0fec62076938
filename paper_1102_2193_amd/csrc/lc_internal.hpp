// lc_internal.hpp -- library-internal access to a context's current Q
// buffer (used by the warm start to write its prediction on the device).
#pragma once

#include <hip/hip_runtime.h>

struct lc_ctx;

struct LcQView {
  void* Q;               // current Q buffer [5][nsites]
  long long nsites;      // component stride
  long long off;         // first site of the box
  int prec;              // LC_FP32 / LC_FP64
  int nx, ny, nz;
  hipStream_t stream;
};

int lc_internal_q_view(lc_ctx* c, int box, LcQView* out);
