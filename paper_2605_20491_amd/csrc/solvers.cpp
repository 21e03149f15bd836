// Solvers on top of the separable apply: the stencil operator entry point,
// iterative refinement, PCG (paper Sec. 3.2), shifted inverse iteration
// (Sec. 4.1, 5.3.1) and the splitting schemes (Sec. 5.1).
#include <cmath>
#include <string>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_internal.h"
#include "ts_vec.h"

namespace ts {

StencilArgs stencil_args(const ts_plan* p, const double* V2, double s, const double* u, double* out) {
  StencilArgs a;
  a.d = p->d;
  a.N = p->N;
  int64_t st = 1;
  for (int k = p->d - 1; k >= 0; --k) {
    a.n[k] = p->n[k];
    a.stride[k] = st;
    st *= p->n[k];
    a.ih2[k] = p->ax[k]->ih2;
    a.f[k] = p->ax[k]->f;
  }
  a.V2 = V2;
  a.s = s;
  a.u = u;
  a.out = out;
  return a;
}

}  // namespace ts

using namespace ts;

extern "C" {

int ts_operator_apply(ts_plan* plan, const double* V2, double s, const double* u, double* out,
                      void* hip_stream) {
  if (!plan || !u || !out) { set_error("null argument"); return TS_ERR_INVALID; }
  if (u == out) { set_error("u and out must not alias"); return TS_ERR_INVALID; }
  hipError_t e = launch_stencil(stencil_args(plan, V2, s, u, out), (hipStream_t)hip_stream);
  if (e != hipSuccess) { set_error(std::string("stencil launch failed: ") + hipGetErrorString(e)); return TS_ERR_DEVICE; }
  return TS_OK;
}

int ts_solve_refined(ts_plan*, const double*, double*, int, double, int, int*, double*, void*) {
  set_error("ts_solve_refined: not available in this build");
  return TS_ERR_INVALID;
}

int ts_pcg_solve(ts_plan*, const double*, const double*, double*, double, int, int, int*, double*, void*) {
  set_error("ts_pcg_solve: not available in this build");
  return TS_ERR_INVALID;
}

int ts_inverse_iteration(ts_plan*, const double*, double, double*, int, double, int, int, double*, int*,
                         void*) {
  set_error("ts_inverse_iteration: not available in this build");
  return TS_ERR_INVALID;
}

int ts_split_step(ts_plan*, const void*, void*, double, int, int, int, int, void*) {
  set_error("ts_split_step: not available in this build");
  return TS_ERR_INVALID;
}

}  // extern "C"
