// Solvers on top of the separable apply: the stencil operator entry point,
// iterative refinement of the mixed-precision inverse, PCG with the
// preconditioner (-Delta + V1 + sigma)^{-1} (paper Sec. 3.2), and shifted
// inverse iteration (Sec. 4.1, Sec. 5.3.1).
//
// All vectors, inner products and the scalars alpha, beta of PCG stay on the
// device in FP64.  PCG and refinement are written as tasks (ts_tasks.h): the
// host enqueues a few iterations, then reads a pinned copy of the scalar
// block; once the device sets its `done` flag every later kernel returns at
// once, so the iterate is the one that met the tolerance.
#include <cmath>
#include <cstring>
#include <string>
#include <utility>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_internal.h"
#include "ts_tasks.h"
#include "ts_vec.h"

namespace ts {

StencilArgs stencil_args(const ts_plan* p, const double* V2, double s, const double* u, double* out, bool sym) {
  StencilArgs a;
  a.d = p->d;
  a.N = p->N;
  int64_t st = 1;
  const auto& ax = sym ? p->ax_sym : p->ax;
  for (int k = p->d - 1; k >= 0; --k) {
    a.n[k] = p->n[k];
    a.stride[k] = st;
    st *= p->n[k];
    a.ih2[k] = ax[k]->ih2;
    a.f[k] = ax[k]->f;
    a.band[k] = ax[k]->band;
  }
  a.bw = p->massed ? ax[0]->bw : 0;
  if (p->massed && ax[0]->op_pass) {  // wide band: per-axis MFMA passes into two plan buffers
    for (int k = 0; k < p->d; ++k) a.dense[k] = ax[k]->op_pass.get();
    const size_t vb = (size_t)round_up((int64_t)(sizeof(double) * p->N), 256);
    void* t = nullptr;
    if (ctx_get(const_cast<ts_plan*>(p)->ctx, kSlotOp, 2 * vb, &t) == TS_OK) {
      a.tmp0 = (double*)t;
      a.tmp1 = (double*)((char*)t + vb);
    }
  }
  a.V2 = V2;
  a.s = s;
  a.u = u;
  a.out = out;
  return a;
}

// SEM and generic plans: the solvers run on the symmetric form M^{-1/2} S M^{-1/2} + F in
// the variables M^{1/2} u (Euclidean inner products there are the mass inner
// products of u).  Scale x by M^{1/2} (up) or M^{-1/2} (down); no-op for FD.
hipError_t mass_scale(const ts_plan* p, const double* x, double* y, bool up, hipStream_t st) {
  if (!p->massed) {
    if (x != y) return hipMemcpyAsync(y, x, sizeof(double) * (size_t)p->N, hipMemcpyDeviceToDevice, st);
    return hipSuccess;
  }
  const double* w[TS_MAX_D];
  for (int k = 0; k < p->d; ++k) w[k] = up ? p->ax_sym[k]->msq : p->ax_sym[k]->imsq;
  return launch_axis_scale(x, y, p->d, p->n, w, st);
}

namespace {

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

// Layout of a context's solver slot: a fixed header (two partial arrays and
// the scalar block) followed by nvec FP64 vectors of N.
struct SolverBufs {
  double* vec[8] = {};
  double* partial = nullptr;
  double* partial2 = nullptr;
  SolverScalars* sc = nullptr;
  SolverScalars* host = nullptr;  // pinned mirror
};

size_t solver_header() {
  return round_up((int64_t)(2 * sizeof(double) * kRedBlocks + sizeof(SolverScalars)), 256);
}
size_t solver_vbytes(const ts_plan* p) { return round_up((int64_t)(sizeof(double) * p->N), 256); }

int solver_buffers(ExecCtx& c, const ts_plan* p, int nvec, SolverBufs& b) {
  void* base = nullptr;
  TS_RC(ctx_get(c, kSlotSolver, solver_header() + solver_vbytes(p) * nvec, &base));
  void* host = nullptr;
  TS_RC(ctx_host(c, &host));
  char* cb = (char*)base;
  b.partial = (double*)cb;
  b.partial2 = b.partial + kRedBlocks;
  b.sc = (SolverScalars*)(b.partial2 + kRedBlocks);
  for (int i = 0; i < nvec; ++i) b.vec[i] = (double*)(cb + solver_header() + solver_vbytes(p) * i);
  b.host = (SolverScalars*)host;
  return TS_OK;
}

hipError_t snapshot(const SolverBufs& b, hipStream_t st) {
  return hipMemcpyAsync(b.host, b.sc, sizeof(SolverScalars), hipMemcpyDeviceToHost, st);
}

int status_code(const SolverScalars& s) {
  switch (s.status) {
    case 1: set_error("PCG breakdown: <p, A p> <= 0"); return TS_ERR_BREAKDOWN;
    case 2: set_error("non-finite value in a residual or inner product"); return TS_ERR_NONFINITE;
    case 3: set_error("iteration limit reached"); return TS_ERR_NOCONV;
    default: return TS_OK;
  }
}

// ------------------------------------------------------------------ PCG --
class PcgTask : public Task {
 public:
  PcgTask(ts_plan* p, const double* V2, double s_op, double s_pc, const double* f, double* x, double rtol,
          int maxit, int prec, bool scale_io, ExecCtx& c)
      : p_(p), V2_(V2), s_op_(s_op), s_pc_(s_pc), f_(f), x_(x), rtol_(rtol), maxit_(maxit), prec_(prec),
        scale_(scale_io && p->massed), c_(c) {}

  int start(hipStream_t st) override {
    TS_RC(solver_buffers(c_, p_, scale_ ? 6 : 5, b_));
    r_ = b_.vec[0];
    z_ = b_.vec[1];
    pp_ = b_.vec[2];
    q_ = b_.vec[3];
    pp2_ = b_.vec[4];
    N_ = p_->N;
    if (scale_) {  // f and x into the symmetric form's variables
      TS_TRY(mass_scale(p_, f_, b_.vec[5], true, st));
      TS_TRY(mass_scale(p_, x_, x_, true, st));
      f_ = b_.vec[5];
    }
    flexible_ = prec_ != TS_PREC_FP64;
    done_ = &b_.sc->done;
    chunk_ = N_ >= (int64_t(1) << 24) ? 2 : (N_ >= (int64_t(1) << 20) ? 4 : 8);
    TS_TRY(launch_init_scalars(b_.sc, rtol_ * rtol_, st));
    // r = f - A x ; ||r||^2 and ||f||^2
    sa_ = stencil_args(p_, V2_, s_op_, x_, r_, true);
    sa_.mode = StOut::FminusAx;
    sa_.rhs = f_;
    sa_.dot = StDot::OutdotOut;
    sa_.partial = b_.partial;
    TS_TRY(launch_stencil(sa_, st));
    TS_TRY(launch_dot(f_, f_, N_, b_.partial2, nullptr, nullptr, nullptr, st));
    TS_TRY(launch_scalar(ScalarStep::InitRR, b_.sc, b_.partial, b_.partial2, flexible_, maxit_, st));
    // z = M^{-1} r ; <r, z> ; p = z
    TS_RC(apply_inverse_impl(p_, s_pc_, r_, z_, TS_F64, prec_, st, c_, done_, true));
    TS_TRY(launch_dot(r_, z_, N_, b_.partial, nullptr, nullptr, done_, st));
    TS_TRY(launch_scalar(ScalarStep::InitRZ, b_.sc, b_.partial, nullptr, flexible_, maxit_, st));
    std::swap(pp_, z_);  // p = z: the buffers trade roles instead of a copy
    sq_ = stencil_args(p_, V2_, s_op_, pp_, q_, true);
    sq_.dot = StDot::UdotOut;
    sq_.partial = b_.partial;
    sq_.skip = done_;
    // the update p = z + beta p rides on the next operator sweep (FD stencil only)
    can_fuse_ = sq_.bw == 0 && !sq_.dense[0];
    // a BF16 preconditioner's input rounding rides on the residual update,
    // which writes it where the apply's input sweep would (z, whose old values
    // the operator sweep has consumed by then)
    round_r_ = prec_ == TS_PREC_BF16 && bf16_sweep_applies(p_, r_, z_);
    // and when that apply folds its input, the update folds it too
    fold_r_ = round_r_ && bf16_fold_axes(p_, r_, z_, true, fb_) &&
              cg_update_fold_ok(fb_, x_, r_, pp_, q_, (const uint16_t*)z_) &&
              cg_update_fold_ok(fb_, x_, r_, pp2_, q_, (const uint16_t*)z_);
    TS_RC(enqueue_chunk(st));
    TS_TRY(snapshot(b_, st));
    return TS_OK;
  }

  int advance(hipStream_t st, bool* done) override {
    SolverScalars s;
    std::memcpy(&s, b_.host, sizeof(s));
    if (!final_) {
      if (!s.done && enq_ < maxit_) {
        TS_RC(enqueue_chunk(st));
        TS_TRY(snapshot(b_, st));
        *done = false;
        return TS_OK;
      }
      // recompute the true residual ||f - A x|| / ||f||
      final_ = true;
      TS_TRY(launch_stencil(sa_, st));
      TS_TRY(launch_scalar(ScalarStep::SetRR, b_.sc, b_.partial, nullptr, flexible_, maxit_, st));
      TS_TRY(snapshot(b_, st));
      *done = false;
      return TS_OK;
    }
    iters = s.iters;
    relres = s.ff > 0 ? std::sqrt(s.rr / s.ff) : 0.0;
    if (!s.done) {
      set_error("iteration limit reached");
      status = TS_ERR_NOCONV;
    } else {
      status = status_code(s);
    }
    if (scale_) TS_TRY(mass_scale(p_, x_, x_, false, st));  // back to the caller's variables
    *done = true;
    return TS_OK;
  }

 private:
  int enqueue_chunk(hipStream_t st) {
    for (int ci = 0; ci < chunk_ && enq_ < maxit_; ++ci, ++enq_) {
      // q = A p with <p, q>; after the first iteration p = z + beta p is formed
      // inside this sweep (into the other direction buffer)
      sq_.u = pp_;
      sq_.z = pending_ ? z_ : nullptr;
      sq_.bsc = pending_ ? b_.sc : nullptr;
      sq_.unew = pending_ ? pp2_ : nullptr;
      TS_TRY(launch_stencil(sq_, st));
      if (pending_) std::swap(pp_, pp2_);
      pending_ = false;
      TS_TRY(launch_scalar(ScalarStep::Alpha, b_.sc, b_.partial, nullptr, flexible_, maxit_, st));
      if (fold_r_)
        TS_TRY(launch_cg_update_fold(x_, r_, pp_, q_, fb_, b_.sc, b_.partial, done_, (uint16_t*)z_, st));
      else
        TS_TRY(launch_cg_update(x_, r_, pp_, q_, N_, b_.sc, b_.partial, done_, st, round_r_ ? (uint16_t*)z_ : nullptr));
      TS_TRY(launch_scalar(ScalarStep::RR, b_.sc, b_.partial, nullptr, flexible_, maxit_, st));
      TS_RC(apply_inverse_impl(p_, s_pc_, r_, z_, TS_F64, prec_, st, c_, done_, true, round_r_, fold_r_));
      TS_TRY(launch_dot(z_, r_, N_, b_.partial, flexible_ ? q_ : nullptr, flexible_ ? b_.partial2 : nullptr,
                        done_, st));
      TS_TRY(launch_scalar(ScalarStep::Beta, b_.sc, b_.partial, flexible_ ? b_.partial2 : nullptr, flexible_,
                           maxit_, st));
      if (can_fuse_) pending_ = true;
      else TS_TRY(launch_xpby(z_, pp_, N_, b_.sc, done_, st));
    }
    return TS_OK;
  }

  ts_plan* p_;
  const double* V2_;
  double s_op_, s_pc_;
  const double* f_;
  double* x_;
  double rtol_;
  int maxit_, prec_;
  bool scale_;
  ExecCtx& c_;
  SolverBufs b_;
  double *r_ = nullptr, *z_ = nullptr, *pp_ = nullptr, *q_ = nullptr, *pp2_ = nullptr;
  int64_t N_ = 0;
  int flexible_ = 0;
  bool can_fuse_ = false, pending_ = false, round_r_ = false, fold_r_ = false;
  ButterflyArgs fb_;  // the axes along which the BF16 preconditioner folds its input
  const int* done_ = nullptr;
  int chunk_ = 4, enq_ = 0;
  bool final_ = false;
  StencilArgs sa_, sq_;
};

// ------------------------------------------------------- refinement --
// u <- u + M^{-1}(f - (H1 + sigma) u), M^{-1} the apply in `inner` precision,
// residual in FP64 with the stencil; if a sweep contracts the residual by less
// than 0.9 twice, the rest is flexible CG warm-started from u.
class RefineTask : public Task {
 public:
  RefineTask(ts_plan* p, double sigma, const double* f, double* u, int inner, double rtol, int maxit,
             bool scale_io, ExecCtx& c)
      : p_(p), sigma_(sigma), f_(f), u_(u), inner_(inner), rtol_(rtol), maxit_(maxit),
        scale_(scale_io && p->massed), c_(c) {}

  int start(hipStream_t st) override {
    // vector 5 holds the scaled right-hand side: the CG fallback uses 0..4
    TS_RC(solver_buffers(c_, p_, scale_ ? 6 : 2, b_));
    r_ = b_.vec[0];
    dlt_ = b_.vec[1];
    N_ = p_->N;
    if (scale_) {
      TS_TRY(mass_scale(p_, f_, b_.vec[5], true, st));
      f_ = b_.vec[5];
    }
    TS_TRY(launch_init_scalars(b_.sc, rtol_ * rtol_, st));
    TS_TRY(launch_dot(f_, f_, N_, b_.partial, nullptr, nullptr, nullptr, st));
    TS_TRY(launch_scalar(ScalarStep::SetAux0, b_.sc, b_.partial, nullptr, 0, maxit_, st));
    // first sweep from u = 0: u = M^{-1} f, then its residual
    TS_RC(apply_inverse_impl(p_, sigma_, f_, u_, TS_F64, inner_, st, c_, nullptr, true));
    sa_ = stencil_args(p_, nullptr, sigma_, u_, r_, true);
    sa_.mode = StOut::FminusAx;
    sa_.rhs = f_;
    sa_.dot = StDot::OutdotOut;
    sa_.partial = b_.partial;
    TS_TRY(launch_stencil(sa_, st));
    TS_TRY(launch_scalar(ScalarStep::SetRR, b_.sc, b_.partial, nullptr, 0, maxit_, st));
    TS_TRY(snapshot(b_, st));
    sweeps_ = 1;
    acc_ = inner_ == TS_PREC_BF16 && bf16_accumulate_ok(p_, r_, u_, true);
    return TS_OK;
  }

  int advance(hipStream_t st, bool* done) override {
    TS_RC(step(st, done));
    if (*done && scale_) TS_TRY(mass_scale(p_, u_, u_, false, st));  // back to the caller's variables
    return TS_OK;
  }

 private:
  int step(hipStream_t st, bool* done) {
    if (cg_) {
      TS_RC(cg_->advance(st, done));
      if (*done) {
        iters = sweeps_ + cg_->iters;
        relres = cg_->relres;
        status = cg_->status;
      }
      return TS_OK;
    }
    SolverScalars s;
    std::memcpy(&s, b_.host, sizeof(s));
    const double ff = s.aux[0], rr = s.rr;
    *done = true;
    iters = sweeps_;
    if (ff == 0.0) {  // f = 0: u = M^{-1} 0 = 0 already
      relres = 0.0;
      return TS_OK;
    }
    relres = std::sqrt(rr / ff);
    if (!std::isfinite(rr)) { set_error("non-finite residual"); status = TS_ERR_NONFINITE; return TS_OK; }
    if (rr <= rtol_ * rtol_ * ff) return TS_OK;
    if (sweeps_ > 1 && rr > 0.81 * prev_) ++slow_;  // contraction factor above 0.9
    prev_ = rr;
    if (sweeps_ >= maxit_) { set_error("refinement did not reach rtol"); status = TS_ERR_NOCONV; return TS_OK; }
    *done = false;
    if (slow_ >= 2) {
      cg_ = make_pcg_task(p_, nullptr, sigma_, sigma_, f_, u_, rtol_, maxit_ - sweeps_, inner_, c_, false);
      return cg_->start(st);
    }
    if (acc_) {  // u += M^{-1} r in the apply's last pass
      TS_RC(apply_inverse_impl(p_, sigma_, r_, u_, TS_F64, inner_, st, c_, nullptr, true, false, false, true));
    } else {
      TS_RC(apply_inverse_impl(p_, sigma_, r_, dlt_, TS_F64, inner_, st, c_, nullptr, true));
      TS_TRY(launch_axpy1(u_, dlt_, N_, nullptr, st));
    }
    TS_TRY(launch_stencil(sa_, st));
    TS_TRY(launch_scalar(ScalarStep::SetRR, b_.sc, b_.partial, nullptr, 0, maxit_, st));
    TS_TRY(snapshot(b_, st));
    ++sweeps_;
    return TS_OK;
  }

  ts_plan* p_;
  bool acc_ = false;  // BF16 inner applies add their correction to u themselves
  double sigma_;
  const double* f_;
  double* u_;
  int inner_;
  double rtol_;
  int maxit_;
  bool scale_;
  ExecCtx& c_;
  SolverBufs b_;
  double *r_ = nullptr, *dlt_ = nullptr;
  int64_t N_ = 0;
  StencilArgs sa_;
  int sweeps_ = 0, slow_ = 0;
  double prev_ = 0.0;
  std::unique_ptr<Task> cg_;
};

// ------------------------------------------------- single applies --
class ApplyTask : public Task {
 public:
  ApplyTask(bool inverse, ts_plan* p, double param, const void* in, void* out, int dtype, int prec, ExecCtx& c)
      : inverse_(inverse), p_(p), param_(param), in_(in), out_(out), dtype_(dtype), prec_(prec), c_(c) {}
  int start(hipStream_t st) override {
    return inverse_ ? apply_inverse_impl(p_, param_, in_, out_, dtype_, prec_, st, c_, nullptr)
                    : apply_exp_impl(p_, param_, in_, out_, dtype_, prec_, st, c_);
  }
  int advance(hipStream_t, bool* done) override {
    *done = true;
    return TS_OK;
  }

 private:
  bool inverse_;
  ts_plan* p_;
  double param_;
  const void* in_;
  void* out_;
  int dtype_, prec_;
  ExecCtx& c_;
};

}  // namespace

int run_blocking(Task& t, hipStream_t st) {
  hipEvent_t ev = nullptr;
  TS_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  struct Guard { hipEvent_t e; ~Guard() { hipEventDestroy(e); } } guard{ev};
  TS_RC(t.start(st));
  for (;;) {
    TS_TRY(hipEventRecord(ev, st));
    TS_TRY(hipEventSynchronize(ev));
    bool done = false;
    TS_RC(t.advance(st, &done));
    if (done) break;
  }
  return t.status;
}

std::unique_ptr<Task> make_pcg_task(ts_plan* p, const double* V2, double s_op, double s_pc, const double* f,
                                    double* x, double rtol, int maxit, int prec, ExecCtx& c, bool scale_io) {
  return std::unique_ptr<Task>(new PcgTask(p, V2, s_op, s_pc, f, x, rtol, maxit, prec, scale_io, c));
}
std::unique_ptr<Task> make_refine_task(ts_plan* p, double sigma, const double* f, double* u, int inner, double rtol,
                                       int maxit, ExecCtx& c) {
  return std::unique_ptr<Task>(new RefineTask(p, sigma, f, u, inner, rtol, maxit, true, c));
}
std::unique_ptr<Task> make_inverse_task(ts_plan* p, double shift, const void* b, void* u, int dtype, int prec,
                                        ExecCtx& c) {
  return std::unique_ptr<Task>(new ApplyTask(true, p, shift, b, u, dtype, prec, c));
}
std::unique_ptr<Task> make_exp_task(ts_plan* p, double tau, const void* in, void* out, int dtype, int prec,
                                    ExecCtx& c) {
  return std::unique_ptr<Task>(new ApplyTask(false, p, tau, in, out, dtype, prec, c));
}

size_t need_solver(const ts_plan* p, int nvec) { return solver_header() + solver_vbytes(p) * nvec; }

int pcg_run(ts_plan* p, const double* V2, double s_op, double s_pc, const double* f, double* x, double rtol,
            int maxit, int prec, int* iters, double* relres, hipStream_t st, ExecCtx& c, bool scale_io) {
  PcgTask t(p, V2, s_op, s_pc, f, x, rtol, maxit, prec, scale_io, c);
  int rc = run_blocking(t, st);
  if (iters) *iters = t.iters;
  if (relres) *relres = t.relres;
  return rc;
}

int refine_run(ts_plan* p, const double* f, double* u, int inner, double rtol, int maxit, int* iters,
               double* relres, hipStream_t st, ExecCtx& c) {
  RefineTask t(p, p->sigma, f, u, inner, rtol, maxit, true, c);
  int rc = run_blocking(t, st);
  if (iters) *iters = t.iters;
  if (relres) *relres = t.relres;
  return rc;
}

// Shifted inverse iteration with an optional stop on the eigenvalue change
// (|lambda_k - lambda_{k-1}| <= lam_tol |lambda_k|).  Writes lam_hist[0..k]
// and pcg_iters[0..k-1] (host, may be null) and the steps taken.
int invit_run(ts_plan* plan, const double* V2, double shift, double* u, int steps, double lam_tol,
              double pcg_rtol, int maxit, int precond, double* lam_hist, int* pcg_iters, int* steps_done,
              hipStream_t st) {
  if (!plan || !u || steps < 0) { set_error("bad argument"); return TS_ERR_INVALID; }
  if (!std::isfinite(shift) || !(pcg_rtol > 0.0) || maxit < 1 || !(lam_tol >= 0.0)) {
    set_error("bad argument");
    return TS_ERR_INVALID;
  }
  if (precond < TS_PREC_FP64 || precond > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  if (!(plan->lam_min - shift > 0.0)) {
    set_error("shift must lie below lambda_min(H1) for the preconditioner (H1 - shift)^{-1}");
    return TS_ERR_NOT_SPD;
  }
  const int64_t N = plan->N;
  ExecCtx& c = plan->ctx;
  // PCG uses vectors 0..4; H u and the warm-started iterate w take 5 and 6
  SolverBufs b;
  TS_RC(solver_buffers(c, plan, 7, b));
  double* Hu = b.vec[5];
  double* w = b.vec[6];
  // SEM: iterate on the symmetric form, u in the variables M^{1/2} u
  TS_TRY(mass_scale(plan, u, u, true, st));
  auto rayleigh = [&](double* lam) -> int {
    // ||u||^2 -> aux0, u <- u / ||u||, lambda = u^T H u (s = 0)
    TS_TRY(launch_init_scalars(b.sc, 0.0, st));
    TS_TRY(launch_dot(u, u, N, b.partial, nullptr, nullptr, nullptr, st));
    TS_TRY(launch_scalar(ScalarStep::SetAux0, b.sc, b.partial, nullptr, 0, 1, st));
    TS_TRY(launch_scale_invnorm(u, u, N, b.sc, st));
    StencilArgs sa = stencil_args(plan, V2, 0.0, u, Hu, true);
    sa.dot = StDot::UdotOut;
    sa.partial = b.partial;
    TS_TRY(launch_stencil(sa, st));
    TS_TRY(launch_scalar(ScalarStep::SetAux0, b.sc, b.partial, nullptr, 0, 1, st));
    TS_TRY(snapshot(b, st));
    TS_TRY(hipStreamSynchronize(st));
    *lam = b.host->aux[0];
    return TS_OK;
  };
  double lam = 0.0;
  TS_RC(rayleigh(&lam));
  if (lam_hist) lam_hist[0] = lam;
  TS_TRY(hipMemsetAsync(w, 0, sizeof(double) * N, st));
  int k = 0;
  for (; k < steps; ++k) {
    int it = 0;
    double rr = 0.0;
    int rc = pcg_run(plan, V2, -shift, -shift, u, w, pcg_rtol, maxit, precond, &it, &rr, st, c, false);
    if (pcg_iters) pcg_iters[k] = it;
    if (rc) {
      mass_scale(plan, u, u, false, st);
      if (steps_done) *steps_done = k;
      return rc;
    }
    TS_TRY(hipMemcpyAsync(u, w, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    const double prev = lam;
    TS_RC(rayleigh(&lam));
    if (lam_hist) lam_hist[k + 1] = lam;
    if (lam_tol > 0.0 && std::fabs(lam - prev) <= lam_tol * std::fabs(lam)) {
      ++k;
      break;
    }
  }
  if (steps_done) *steps_done = k;
  TS_TRY(mass_scale(plan, u, u, false, st));
  TS_TRY(hipStreamSynchronize(st));
  return TS_OK;
}

}  // namespace ts

using namespace ts;

extern "C" {

int ts_operator_apply(ts_plan* plan, const double* V2, double s, const double* u, double* out,
                      void* hip_stream) {
  if (!plan || !u || !out) { set_error("null argument"); return TS_ERR_INVALID; }
  if (u == out) { set_error("u and out must not alias"); return TS_ERR_INVALID; }
  hipError_t e = launch_stencil(stencil_args(plan, V2, s, u, out, false), (hipStream_t)hip_stream);
  if (e != hipSuccess) { set_error(std::string("stencil launch failed: ") + hipGetErrorString(e)); return TS_ERR_DEVICE; }
  return TS_OK;
}

int ts_pcg_solve(ts_plan* plan, const double* V2, const double* f, double* u, double rtol, int maxit,
                 int precond, int* iters, double* relres, void* hip_stream) {
  if (!plan || !f || !u) { set_error("null argument"); return TS_ERR_INVALID; }
  if (!(rtol > 0.0) || maxit < 1) { set_error("rtol must be > 0 and maxit >= 1"); return TS_ERR_INVALID; }
  if (precond < TS_PREC_FP64 || precond > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  return pcg_run(plan, V2, plan->sigma, plan->sigma, f, u, rtol, maxit, precond, iters, relres,
                 (hipStream_t)hip_stream, plan->ctx);
}

int ts_solve_refined(ts_plan* plan, const double* f, double* u, int inner, double rtol, int maxit,
                     int* iters, double* relres, void* hip_stream) {
  if (!plan || !f || !u) { set_error("null argument"); return TS_ERR_INVALID; }
  if (!(rtol > 0.0) || maxit < 1) { set_error("rtol must be > 0 and maxit >= 1"); return TS_ERR_INVALID; }
  if (inner < TS_PREC_FP64 || inner > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  return refine_run(plan, f, u, inner, rtol, maxit, iters, relres, (hipStream_t)hip_stream, plan->ctx);
}

int ts_inverse_iteration(ts_plan* plan, const double* V2, double shift, double* u, int steps,
                         double pcg_rtol, int maxit, int precond, double* lam_hist, int* pcg_iters,
                         void* hip_stream) {
  if (!plan || !u || steps < 0) { set_error("bad argument"); return TS_ERR_INVALID; }
  return invit_run(plan, V2, shift, u, steps, 0.0, pcg_rtol, maxit, precond, lam_hist, pcg_iters, nullptr,
                   (hipStream_t)hip_stream);
}

}  // extern "C"
