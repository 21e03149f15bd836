// Apply drivers shared by the C ABI and the solvers.
#pragma once

#include "ts_internal.h"

namespace ts {

struct ApplyParams {
  const void* in = nullptr;
  void* out = nullptr;
  void* work = nullptr;
  DT tin = DT::F64, tout = DT::F64;
  int prec = 0;
  bool cplx = false;
  Epi epi = Epi::Inv;
  double shift = 0.0;
  const int* skip = nullptr;
};

int run_apply(ts_plan* p, const ApplyParams& ap, hipStream_t st);
int plan_workspace(ts_plan* p, size_t bytes, void** out);

// u = (H1 + shift)^{-1} b.  work: N*8 bytes of scratch, or null for the plan's.
// skip: optional device flag; when set, every kernel of the apply returns at once.
int apply_inverse_impl(ts_plan* p, double shift, const void* b, void* u, int dtype, int prec,
                       hipStream_t st, void* work, const int* skip);
// psi_out = exp(-i tau H1) psi_in.  work: N*16 bytes or null.
int apply_exp_impl(ts_plan* p, double tau, const void* in, void* out, int dtype, int prec,
                   hipStream_t st, void* work);

// Optional pointwise potential factors around one propagator apply (in place,
// psi_in == psi_out): psi <- e^{-i th_post V2} e^{-i tau H1} e^{-i th_pre V2} psi.
struct Phases {
  const void* V2 = nullptr;
  bool pre = false, post = false;
  double th_pre = 0.0, th_post = 0.0;
};
int apply_exp_phased(ts_plan* p, double tau, void* psi, int dtype, int prec, const Phases& ph,
                     hipStream_t st, void* work);

}  // namespace ts
