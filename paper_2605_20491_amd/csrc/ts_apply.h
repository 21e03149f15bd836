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
  const double2* phase = nullptr;  // Exp: tables Ep | Er | es of the scaling axis
  bool sym = false;                // use the plan's orthogonal (solver) factors
  bool in_rounded = false;         // BF16 of FP64 data: out already holds the input rounded to BF16
  bool in_folded = false;          // ... and folded along the axes bf16_fold_axes lists
  bool accumulate = false;         // out += the result (BF16 of FP64 data, see bf16_accumulate_ok)
};

int run_apply(ts_plan* p, const ApplyParams& ap, hipStream_t st);

// Scratch bytes of one apply in each context slot.
size_t need_inverse(const ts_plan* p, int slot);
size_t need_exp(const ts_plan* p, int slot);

// u = (H1 + shift)^{-1} b with the context's scratch.  skip: optional device
// flag; when set, every kernel of the apply returns at once.  sym: apply the
// symmetric form's inverse (the solvers' variables; differs from the public
// apply only for SEM plans).
int apply_inverse_impl(ts_plan* p, double shift, const void* b, void* u, int dtype, int prec,
                       hipStream_t st, ExecCtx& c, const int* skip, bool sym = false, bool in_rounded = false,
                       bool in_folded = false, bool accumulate = false);

// Whether a BF16 inverse apply of FP64 data `in` -> `out` (N values) starts
// with the streaming input sweep into `out`, which a producer of `in` may
// write itself instead (apply_inverse_impl's in_rounded).
bool bf16_sweep_applies(const ts_plan* p, const void* in, const void* out);
// The axes along which a BF16 inverse apply of FP64 data in -> out folds its
// input (the symmetric axes whose forward pass can read folded data), as the
// arguments of that fold (X = in, Y = out, fastest axis first); false if none.
bool bf16_fold_axes(const ts_plan* p, const void* in, void* out, bool sym, ButterflyArgs& b);
// Whether a BF16 inverse apply of FP64 data in -> out can add its result to
// out (apply_inverse_impl's accumulate): the last pass must run on the
// 256 x 256 tiles, and N % 8 == 0 places the workspace's two halves on
// 16-byte boundaries.
bool bf16_accumulate_ok(const ts_plan* p, const void* in, const void* out, bool sym);
// psi_out = exp(-i tau H1) psi_in.
int apply_exp_impl(ts_plan* p, double tau, const void* in, void* out, int dtype, int prec,
                   hipStream_t st, ExecCtx& c);

// Optional pointwise potential factors around one propagator apply (in place,
// psi_in == psi_out): psi <- e^{-i th_post V2} e^{-i tau H1} e^{-i th_pre V2} psi.
struct Phases {
  const void* V2 = nullptr;
  bool pre = false, post = false;
  double th_pre = 0.0, th_post = 0.0;
};
int apply_exp_phased(ts_plan* p, double tau, void* psi, int dtype, int prec, const Phases& ph,
                     hipStream_t st, ExecCtx& c);

// Solvers (solvers.cpp) on an explicit context.
int pcg_run(ts_plan* p, const double* V2, double s_op, double s_pc, const double* f, double* x,
            double rtol, int maxit, int prec, int* iters, double* relres, hipStream_t st, ExecCtx& c,
            bool scale_io = true);
int refine_run(ts_plan* p, const double* f, double* u, int inner, double rtol, int maxit, int* iters,
               double* relres, hipStream_t st, ExecCtx& c);
int split_run(ts_plan* p, const void* V2, void* psi, double dt, int nsteps, int scheme, int dtype, int prec,
              hipStream_t st, ExecCtx& c);
int qhop_run(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int M, bool magnus2, int dtype,
             int prec, hipStream_t st, ExecCtx& c);
int invit_run(ts_plan* plan, const double* V2, double shift, double* u, int steps, double lam_tol,
              double pcg_rtol, int maxit, int precond, double* lam_hist, int* pcg_iters, int* steps_done,
              hipStream_t st);
size_t need_solver(const ts_plan* p, int nvec);
// Device bytes of a plan's factors and tables (its scratch not included).
size_t plan_device_bytes(const ts_plan* p);

}  // namespace ts
