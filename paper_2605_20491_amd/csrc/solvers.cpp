// Solvers on top of the separable apply: the stencil operator entry point,
// iterative refinement of the mixed-precision inverse, PCG with the
// preconditioner (-Delta + V1 + sigma)^{-1} (paper Sec. 3.2), and shifted
// inverse iteration (Sec. 4.1, Sec. 5.3.1).
//
// All vectors, inner products and the scalars alpha, beta of PCG stay on the
// device in FP64.  The host enqueues iterations in chunks and polls a pinned
// copy of the scalar block one chunk behind; once the device sets its `done`
// flag every later kernel of the chunk returns at once, so the iterate is the
// one that met the tolerance.
#include <cmath>
#include <cstring>
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

namespace {

// Layout of the plan's solver buffer: a fixed header (two partial arrays and
// the scalar block) followed by nvec FP64 vectors of N; callers asking for
// different nvec see the same header.
struct SolverBufs {
  double* vec[5] = {};
  double* partial = nullptr;
  double* partial2 = nullptr;
  SolverScalars* sc = nullptr;
  SolverScalars* host = nullptr;  // pinned
};

int solver_buffers(ts_plan* p, int nvec, SolverBufs& b) {
  std::lock_guard<std::mutex> g(p->mu);
  const size_t vbytes = round_up((int64_t)(sizeof(double) * p->N), 256);
  const size_t header = round_up((int64_t)(2 * sizeof(double) * kRedBlocks + sizeof(SolverScalars)), 256);
  const size_t need = header + vbytes * nvec;
  if (p->solver_bytes < need) {
    if (p->solver) {
      hipDeviceSynchronize();
      hipFree(p->solver);
      p->solver = nullptr;
      p->solver_bytes = 0;
    }
    if (hipMalloc(&p->solver, need) != hipSuccess) {
      p->solver = nullptr;
      set_error("solver buffer allocation of " + std::to_string(need) + " bytes failed");
      return TS_ERR_NOMEM;
    }
    p->solver_bytes = need;
  }
  if (!p->solver_host) {
    if (hipHostMalloc(&p->solver_host, sizeof(SolverScalars), hipHostMallocDefault) != hipSuccess) {
      p->solver_host = nullptr;
      set_error("pinned host allocation failed");
      return TS_ERR_NOMEM;
    }
  }
  char* base = (char*)p->solver;
  b.partial = (double*)base;
  b.partial2 = b.partial + kRedBlocks;
  b.sc = (SolverScalars*)(b.partial2 + kRedBlocks);
  for (int i = 0; i < nvec; ++i) b.vec[i] = (double*)(base + header + vbytes * i);
  b.host = (SolverScalars*)p->solver_host;
  return TS_OK;
}

#define TS_TRY(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) {                                                           \
      set_error(std::string(#expr " failed: ") + hipGetErrorString(_e));              \
      return TS_ERR_DEVICE;                                                           \
    }                                                                                 \
  } while (0)

#define TS_RC(expr)          \
  do {                       \
    int _rc = (expr);        \
    if (_rc) return _rc;     \
  } while (0)

// Reset the scalar block from the pinned host mirror.
hipError_t reset_scalars(const SolverBufs& b, double tol2, hipStream_t st) {
  hipError_t e = hipStreamSynchronize(st);  // the host mirror may still be the target of a copy
  if (e != hipSuccess) return e;
  std::memset(b.host, 0, sizeof(SolverScalars));
  b.host->tol2 = tol2;
  return hipMemcpyAsync(b.sc, b.host, sizeof(SolverScalars), hipMemcpyHostToDevice, st);
}

hipError_t read_scalars(const SolverBufs& b, SolverScalars* out, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(b.host, b.sc, sizeof(SolverScalars), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) std::memcpy(out, b.host, sizeof(SolverScalars));
  return e;
}

int status_code(const SolverScalars& s) {
  switch (s.status) {
    case 1: set_error("PCG breakdown: <p, A p> <= 0"); return TS_ERR_BREAKDOWN;
    case 2: set_error("non-finite value in a residual or inner product"); return TS_ERR_NONFINITE;
    case 3: set_error("iteration limit reached"); return TS_ERR_NOCONV;
    default: return TS_OK;
  }
}

}  // namespace

// PCG for (H1 + V2 + s_op) x = f with preconditioner (H1 + s_pc)^{-1} in `prec`.
// x: in initial guess, out solution.  b: solver buffers with 4 vectors.
int pcg_run(ts_plan* p, const double* V2, double s_op, double s_pc, const double* f, double* x,
            double rtol, int maxit, int prec, int* iters, double* relres, hipStream_t st) {
  SolverBufs b;
  TS_RC(solver_buffers(p, 4, b));
  double *r = b.vec[0], *z = b.vec[1], *pp = b.vec[2], *q = b.vec[3];
  const int64_t N = p->N;
  const int flexible = prec != TS_PREC_FP64;
  const int* done = &b.sc->done;
  TS_TRY(reset_scalars(b, rtol * rtol, st));
  // r = f - A x ; ||r||^2, ||f||^2
  StencilArgs sa = stencil_args(p, V2, s_op, x, r);
  sa.mode = StOut::FminusAx;
  sa.rhs = f;
  sa.dot = StDot::OutdotOut;
  sa.partial = b.partial;
  TS_TRY(launch_stencil(sa, st));
  TS_TRY(launch_dot(f, f, N, b.partial2, nullptr, nullptr, nullptr, st));
  TS_TRY(launch_scalar(ScalarStep::InitRR, b.sc, b.partial, b.partial2, flexible, maxit, st));
  // z = M^{-1} r ; rz ; p = z
  TS_RC(apply_inverse_impl(p, s_pc, r, z, TS_F64, prec, st, nullptr, done));
  TS_TRY(launch_dot(r, z, N, b.partial, nullptr, nullptr, done, st));
  TS_TRY(launch_scalar(ScalarStep::InitRZ, b.sc, b.partial, nullptr, flexible, maxit, st));
  TS_TRY(hipMemcpyAsync(pp, z, sizeof(double) * N, hipMemcpyDeviceToDevice, st));

  StencilArgs sq = stencil_args(p, V2, s_op, pp, q);
  sq.dot = StDot::UdotOut;
  sq.partial = b.partial;
  sq.skip = done;
  const int chunk = N >= (int64_t(1) << 24) ? 2 : 8;
  hipEvent_t ev = nullptr;
  TS_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  SolverScalars snap{};
  int enq = 0;
  bool pending = false, finished = false;
  while (!finished) {
    if (enq < maxit) {
      for (int c = 0; c < chunk && enq < maxit; ++c, ++enq) {
        TS_TRY(launch_stencil(sq, st));
        TS_TRY(launch_scalar(ScalarStep::Alpha, b.sc, b.partial, nullptr, flexible, maxit, st));
        TS_TRY(launch_cg_update(x, r, pp, q, N, b.sc, b.partial, done, st));
        TS_TRY(launch_scalar(ScalarStep::RR, b.sc, b.partial, nullptr, flexible, maxit, st));
        TS_RC(apply_inverse_impl(p, s_pc, r, z, TS_F64, prec, st, nullptr, done));
        TS_TRY(launch_dot(z, r, N, b.partial, flexible ? q : nullptr, flexible ? b.partial2 : nullptr, done, st));
        TS_TRY(launch_scalar(ScalarStep::Beta, b.sc, b.partial, flexible ? b.partial2 : nullptr, flexible,
                             maxit, st));
        TS_TRY(launch_xpby(z, pp, N, b.sc, done, st));
      }
    }
    // poll the previous chunk's snapshot while this chunk runs
    if (pending) {
      TS_TRY(hipEventSynchronize(ev));
      std::memcpy(&snap, b.host, sizeof(snap));
      if (snap.done) finished = true;
    }
    if (!finished) {
      if (enq >= maxit && pending) {
        // every iteration is queued and the device has decided: read the final state below
        finished = true;
      } else {
        TS_TRY(hipMemcpyAsync(b.host, b.sc, sizeof(SolverScalars), hipMemcpyDeviceToHost, st));
        TS_TRY(hipEventRecord(ev, st));
        pending = true;
      }
    }
  }
  hipEventDestroy(ev);
  SolverScalars fin{};
  TS_TRY(read_scalars(b, &fin, st));
  // true residual ||f - A x|| / ||f||
  TS_TRY(launch_stencil(sa, st));
  TS_TRY(launch_scalar(ScalarStep::SetRR, b.sc, b.partial, nullptr, flexible, maxit, st));
  SolverScalars tr{};
  TS_TRY(read_scalars(b, &tr, st));
  if (iters) *iters = fin.iters;
  if (relres) *relres = fin.ff > 0 ? std::sqrt(tr.rr / fin.ff) : 0.0;
  if (!fin.done) {
    set_error("iteration limit reached");
    return TS_ERR_NOCONV;
  }
  return status_code(fin);
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

int ts_pcg_solve(ts_plan* plan, const double* V2, const double* f, double* u, double rtol, int maxit,
                 int precond, int* iters, double* relres, void* hip_stream) {
  if (!plan || !f || !u) { set_error("null argument"); return TS_ERR_INVALID; }
  if (!(rtol > 0.0) || maxit < 1) { set_error("rtol must be > 0 and maxit >= 1"); return TS_ERR_INVALID; }
  if (precond < TS_PREC_FP64 || precond > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  return pcg_run(plan, V2, plan->sigma, plan->sigma, f, u, rtol, maxit, precond, iters, relres,
                 (hipStream_t)hip_stream);
}

int ts_solve_refined(ts_plan* plan, const double* f, double* u, int inner, double rtol, int maxit,
                     int* iters, double* relres, void* hip_stream) {
  if (!plan || !f || !u) { set_error("null argument"); return TS_ERR_INVALID; }
  if (!(rtol > 0.0) || maxit < 1) { set_error("rtol must be > 0 and maxit >= 1"); return TS_ERR_INVALID; }
  if (inner < TS_PREC_FP64 || inner > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  hipStream_t st = (hipStream_t)hip_stream;
  SolverBufs b;
  TS_RC(solver_buffers(plan, 2, b));
  double *r = b.vec[0], *dlt = b.vec[1];
  const int64_t N = plan->N;
  TS_TRY(reset_scalars(b, rtol * rtol, st));
  // ||f||^2 into ff via InitRR with r = f
  TS_TRY(hipMemcpyAsync(r, f, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
  TS_TRY(launch_dot(f, f, N, b.partial, nullptr, nullptr, nullptr, st));
  TS_TRY(launch_scalar(ScalarStep::InitRR, b.sc, b.partial, b.partial, 0, maxit, st));
  SolverScalars s0{};
  TS_TRY(read_scalars(b, &s0, st));
  const double ff = s0.ff;
  if (ff == 0.0) {
    TS_TRY(hipMemsetAsync(u, 0, sizeof(double) * N, st));
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return TS_OK;
  }
  StencilArgs sa = stencil_args(plan, nullptr, plan->sigma, u, r);
  sa.mode = StOut::FminusAx;
  sa.rhs = f;
  sa.dot = StDot::OutdotOut;
  sa.partial = b.partial;
  double prev = ff, rr = ff;
  int slow = 0, it = 0;
  // first sweep from u = 0: u = M^{-1} f
  TS_RC(apply_inverse_impl(plan, plan->sigma, f, u, TS_F64, inner, st, nullptr, nullptr));
  for (it = 1;; ++it) {
    TS_TRY(launch_stencil(sa, st));
    TS_TRY(launch_scalar(ScalarStep::SetRR, b.sc, b.partial, nullptr, 0, maxit, st));
    SolverScalars s{};
    TS_TRY(read_scalars(b, &s, st));
    rr = s.rr;
    if (!std::isfinite(rr)) { set_error("non-finite residual"); return TS_ERR_NONFINITE; }
    if (rr <= rtol * rtol * ff) break;
    if (rr > 0.81 * prev) ++slow;  // contraction factor above 0.9
    prev = rr;
    if (it >= maxit) break;
    if (slow >= 2) {
      // Richardson stalls: finish with flexible CG on the same operator,
      // warm-started from the current u
      int cg_it = 0;
      double cg_res = 0.0;
      int rc = pcg_run(plan, nullptr, plan->sigma, plan->sigma, f, u, rtol, maxit - it, inner, &cg_it, &cg_res, st);
      if (iters) *iters = it + cg_it;
      if (relres) *relres = cg_res;
      return rc;
    }
    TS_RC(apply_inverse_impl(plan, plan->sigma, r, dlt, TS_F64, inner, st, nullptr, nullptr));
    TS_TRY(launch_axpy1(u, dlt, N, nullptr, st));
  }
  if (iters) *iters = it;
  if (relres) *relres = std::sqrt(rr / ff);
  if (rr > rtol * rtol * ff) { set_error("refinement did not reach rtol"); return TS_ERR_NOCONV; }
  return TS_OK;
}

int ts_inverse_iteration(ts_plan* plan, const double* V2, double shift, double* u, int steps,
                         double pcg_rtol, int maxit, int precond, double* lam_hist, int* pcg_iters,
                         void* hip_stream) {
  if (!plan || !u || steps < 0) { set_error("bad argument"); return TS_ERR_INVALID; }
  if (!std::isfinite(shift) || !(pcg_rtol > 0.0) || maxit < 1) { set_error("bad argument"); return TS_ERR_INVALID; }
  if (!(plan->lam_min - shift > 0.0)) {
    set_error("shift must lie below lambda_min(H1) for the preconditioner (H1 - shift)^{-1}");
    return TS_ERR_NOT_SPD;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t N = plan->N;
  // w (the PCG iterate, warm start) lives in its own buffer; PCG uses 4 more
  double* w = nullptr;
  if (hipMalloc(&w, sizeof(double) * N) != hipSuccess) { set_error("allocation failed"); return TS_ERR_NOMEM; }
  struct Free { double* p; ~Free() { hipFree(p); } } guard{w};
  SolverBufs b;
  TS_RC(solver_buffers(plan, 5, b));
  double* Hu = b.vec[4];
  auto rayleigh = [&](double* lam) -> int {
    // ||u||^2 -> aux0, u <- u / ||u||, lambda = u^T H u (s = 0)
    TS_TRY(reset_scalars(b, 0.0, st));
    TS_TRY(launch_dot(u, u, N, b.partial, nullptr, nullptr, nullptr, st));
    TS_TRY(launch_scalar(ScalarStep::SetAux0, b.sc, b.partial, nullptr, 0, 1, st));
    TS_TRY(launch_scale_invnorm(u, u, N, b.sc, st));
    StencilArgs s = stencil_args(plan, V2, 0.0, u, Hu);
    s.dot = StDot::UdotOut;
    s.partial = b.partial;
    TS_TRY(launch_stencil(s, st));
    TS_TRY(launch_scalar(ScalarStep::SetAux0, b.sc, b.partial, nullptr, 0, 1, st));
    SolverScalars sv{};
    TS_TRY(read_scalars(b, &sv, st));
    *lam = sv.aux[0];
    return TS_OK;
  };
  double lam = 0.0;
  TS_RC(rayleigh(&lam));
  if (lam_hist) lam_hist[0] = lam;
  TS_TRY(hipMemsetAsync(w, 0, sizeof(double) * N, st));
  for (int k = 0; k < steps; ++k) {
    int it = 0;
    double rr = 0.0;
    int rc = pcg_run(plan, V2, -shift, -shift, u, w, pcg_rtol, maxit, precond, &it, &rr, st);
    if (pcg_iters) pcg_iters[k] = it;
    if (rc) return rc;
    TS_TRY(hipMemcpyAsync(u, w, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    TS_RC(rayleigh(&lam));
    if (lam_hist) lam_hist[k + 1] = lam;
  }
  TS_TRY(hipStreamSynchronize(st));
  return TS_OK;
}

}  // extern "C"
