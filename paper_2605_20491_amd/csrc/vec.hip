// HBM-bound FP64 kernels around the separable apply: the non-separable
// operator by its stencil (paper eq. (general_system)), and the reductions
// and vector updates of PCG and iterative refinement.
#include "ts_internal.h"
#include "ts_vec.h"

namespace ts {
namespace {

// out = (sum_k h_k^-2 (2u - u_{-e_k} - u_{+e_k}) + (sum_k f_k[j_k] + V2 + s) u), zero ghosts.
__global__ __launch_bounds__(256) void k_stencil(StencilArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const double u0 = a.u[i];
  double diag = a.s + (a.V2 ? a.V2[i] : 0.0);
  double acc = 0.0;
  int64_t rem = i;
  for (int k = a.d - 1; k >= 0; --k) {
    const int64_t nk = a.n[k];
    const int64_t j = rem % nk;
    rem /= nk;
    diag += a.f[k][j];
    const int64_t st = a.stride[k];
    const double lo = (j > 0) ? a.u[i - st] : 0.0;
    const double hi = (j + 1 < nk) ? a.u[i + st] : 0.0;
    acc += a.ih2[k] * (2.0 * u0 - lo - hi);
  }
  a.out[i] = acc + diag * u0;
}

}  // namespace

hipError_t launch_stencil(const StencilArgs& a, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  int64_t blocks = (a.N + 255) / 256;
  hipLaunchKernelGGL(k_stencil, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace ts
