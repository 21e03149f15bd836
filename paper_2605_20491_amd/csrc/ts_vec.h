// Launchers of the FP64 vector kernels (vec.hip).
#pragma once

#include "ts_internal.h"

namespace ts {

struct StencilArgs {
  int d = 0;
  int64_t N = 0;
  int64_t n[TS_MAX_D] = {};
  int64_t stride[TS_MAX_D] = {};
  double ih2[TS_MAX_D] = {};
  const double* f[TS_MAX_D] = {};  // device samples of f_k
  const double* V2 = nullptr;
  double s = 0.0;
  const double* u = nullptr;
  double* out = nullptr;
};

hipError_t launch_stencil(const StencilArgs& a, hipStream_t st);

}  // namespace ts
