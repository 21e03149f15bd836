// GPE ground state (paper Sec. 4.2-4.3) by Riemannian gradient flows on the
// L^2 unit sphere, eq. (riemannian_update):
//   u <- (u - tau R(u)) / ||u - tau R(u)||,
//   R(u) = G^{-1} E'(u) - [(u, G^{-1} E'(u)) / (u, G^{-1} u)] G^{-1} u,
// E'(u) = (-Delta + V + beta u^2) u, with the metric operator
//   modified H^1 flow (eq. (h1_metric)): G = -Delta + alpha, two applies of
//     the separable inverse per step;
//   a_u flow (eq. (au_metric)): G = -Delta + V + beta u^2, so G^{-1} E'(u) = u
//     and G^{-1} u is one PCG solve preconditioned with (-Delta + V1)^{-1}.
// Inner products are the grid's L^2 sums (weights prod_k m_k).  The energy
// eq. (gpe_energy) and the eigenvalue come from the fused operator kernel:
// E = (u, E'(u))/2 - beta (u^4, 1)/4, lambda = (u, E'(u)).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_gpe.h"
#include "ts_internal.h"
#include "ts_vec.h"

namespace ts {
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

GpeGrid gpe_grid(const ts_plan* p) {
  GpeGrid g;
  g.d = p->d;
  g.N = p->N;
  int64_t st = 1;
  for (int k = p->d - 1; k >= 0; --k) {
    const AxisFactor& F = *p->ax[k];
    g.n[k] = p->n[k];
    g.stride[k] = st;
    st *= p->n[k];
    g.mass[k] = F.mass;
    g.f[k] = F.f;
    g.ih2[k] = F.ih2;
    g.band[k] = F.band;
  }
  g.bw = p->massed ? p->ax[0]->bw : 0;
  return g;
}

// E'(u) and its two sums; plans with dense per-axis operators first form
// (sum_k B_k + F) u by the MFMA passes of the operator apply.
int gpe_op(const ts_plan* p, GpeOpArgs& op, double* Hu, hipStream_t st) {
  if (Hu) {
    StencilArgs sa = stencil_args(p, nullptr, 0.0, op.u, Hu, false);
    sa.skip = op.skip;
    TS_TRY(launch_stencil(sa, st));
    op.Hu = Hu;
  }
  TS_TRY(launch_gpe_op(op, st));
  return TS_OK;
}

// Device buffers of one flow call, released on scope exit.
struct GpeBufs {
  std::vector<void*> ptrs;
  void* host = nullptr;
  ~GpeBufs() {
    for (void* q : ptrs) hipFree(q);
    if (host) hipHostFree(host);
  }
  template <class T>
  int get(size_t count, T** out) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * count) != hipSuccess) {
      set_error("GPE scratch allocation failed");
      return TS_ERR_NOMEM;
    }
    ptrs.push_back(q);
    *out = (T*)q;
    return TS_OK;
  }
};

int check_common(ts_plan* p, double beta, double tau, double* u, int maxit, double tol) {
  if (!p || !u) { set_error("null argument"); return TS_ERR_INVALID; }
  if (!(beta >= 0.0) || !std::isfinite(beta)) { set_error("beta must be finite and >= 0"); return TS_ERR_INVALID; }
  if (!(tau > 0.0) || !std::isfinite(tau)) { set_error("tau must be positive"); return TS_ERR_INVALID; }
  if (maxit < 0 || !(tol >= 0.0)) { set_error("bad maxit or tol"); return TS_ERR_INVALID; }
  return TS_OK;
}

int finish(const GpeScalars& s, double* energy_hist, const double* hist_dev, int* iters, double* eigenvalue,
           double* energy, hipStream_t st) {
  if (iters) *iters = s.iters;
  if (eigenvalue) *eigenvalue = s.lam;
  if (energy) *energy = s.E;
  if (energy_hist)
    TS_TRY(hipMemcpyAsync(energy_hist, hist_dev, sizeof(double) * (size_t)(s.iters + 1), hipMemcpyDeviceToHost, st));
  TS_TRY(hipStreamSynchronize(st));
  if (s.status == 2) { set_error("non-finite value in the flow"); return TS_ERR_NONFINITE; }
  if (s.status == 3) { set_error("iteration limit reached"); return TS_ERR_NOCONV; }
  return TS_OK;
}

}  // namespace

int gpe_h1_flow(ts_plan* p, const double* V, double beta, double alpha, double tau, double* u, int maxit,
                double tol, double* energy_hist, int* iters, double* eigenvalue, double* energy, hipStream_t st) {
  TS_RC(check_common(p, beta, tau, u, maxit, tol));
  if (!(alpha + p->lam_min > 0.0)) { set_error("-Delta + alpha must be positive definite"); return TS_ERR_NOT_SPD; }
  const int64_t N = p->N;
  GpeBufs B;
  double *Ep, *g, *gu, *part, *part2, *hist, *Hu = nullptr;
  GpeScalars* sc;
  TS_RC(B.get(N, &Ep));
  if (p->ax[0]->op_pass) TS_RC(B.get(N, &Hu));
  TS_RC(B.get(N, &g));
  TS_RC(B.get(N, &gu));
  TS_RC(B.get(kRedBlocks, &part));
  TS_RC(B.get(kRedBlocks, &part2));
  TS_RC(B.get((size_t)maxit + 1, &hist));
  TS_RC(B.get(1, &sc));
  if (hipHostMalloc(&B.host, sizeof(GpeScalars), hipHostMallocDefault) != hipSuccess) {
    set_error("pinned allocation failed");
    return TS_ERR_NOMEM;
  }
  GpeScalars* hs = (GpeScalars*)B.host;
  const GpeGrid G = gpe_grid(p);
  const int* done = &sc->done;
  TS_TRY(launch_gpe_init(sc, beta, tol, maxit, st));
  // normalise the start in L^2
  TS_TRY(launch_wdot2(G, u, u, u, part, part2, nullptr, st));
  TS_TRY(launch_gpe_scalar(GpeStep::Norm, sc, part, nullptr, nullptr, st));
  TS_TRY(launch_gpe_normalize(u, N, sc, nullptr, st));
  GpeOpArgs op;
  op.grid = G;
  op.V2 = V;
  op.beta = beta;
  op.u = u;
  op.out = Ep;
  op.partial = part;
  op.partial2 = part2;
  op.skip = done;
  auto step = [&]() -> int {
    TS_RC(gpe_op(p, op, Hu, st));
    TS_TRY(launch_gpe_scalar(GpeStep::Energy, sc, part, part2, hist, st));
    TS_RC(apply_inverse_impl(p, alpha, Ep, g, TS_F64, TS_PREC_FP64, st, p->ctx, done));
    TS_RC(apply_inverse_impl(p, alpha, u, gu, TS_F64, TS_PREC_FP64, st, p->ctx, done));
    TS_TRY(launch_wdot2(G, u, g, gu, part, part2, done, st));
    TS_TRY(launch_gpe_scalar(GpeStep::Coef, sc, part, part2, nullptr, st));
    TS_TRY(launch_gpe_update(G, u, g, gu, tau, sc, part, done, st));
    TS_TRY(launch_gpe_scalar(GpeStep::Norm, sc, part, nullptr, nullptr, st));
    TS_TRY(launch_gpe_normalize(u, N, sc, done, st));
    return TS_OK;
  };
  // chunks of steps between host polls; the device flag ends the work early
  const int chunk = N >= (int64_t(1) << 24) ? 4 : 16;
  int enq = 0;
  GpeScalars s;
  for (;;) {
    for (int i = 0; i < chunk && enq <= maxit; ++i, ++enq) TS_RC(step());
    TS_TRY(hipMemcpyAsync(hs, sc, sizeof(GpeScalars), hipMemcpyDeviceToHost, st));
    TS_TRY(hipStreamSynchronize(st));
    std::memcpy(&s, hs, sizeof(s));
    if (s.done || enq > maxit) break;
  }
  if (!s.done) { s.status = 3; }
  return finish(s, energy_hist, hist, iters, eigenvalue, energy, st);
}

int gpe_au_flow(ts_plan* p, const double* V2, double beta, double tau, double* u, int maxit, double tol,
                double pcg_rtol, int pcg_maxit, int precond, double* energy_hist, int* iters, int* linear_its,
                double* eigenvalue, double* energy, hipStream_t st) {
  TS_RC(check_common(p, beta, tau, u, maxit, tol));
  if (!(p->lam_min > 0.0)) { set_error("-Delta + V1 must be positive definite"); return TS_ERR_NOT_SPD; }
  if (!(pcg_rtol > 0.0) || pcg_maxit < 1) { set_error("bad PCG tolerance or limit"); return TS_ERR_INVALID; }
  const int64_t N = p->N;
  GpeBufs B;
  double *Ep, *z, *W, *part, *part2, *hist, *Hu = nullptr;
  GpeScalars* sc;
  TS_RC(B.get(N, &Ep));
  if (p->ax[0]->op_pass) TS_RC(B.get(N, &Hu));
  TS_RC(B.get(N, &z));
  TS_RC(B.get(N, &W));
  TS_RC(B.get(kRedBlocks, &part));
  TS_RC(B.get(kRedBlocks, &part2));
  TS_RC(B.get((size_t)maxit + 1, &hist));
  TS_RC(B.get(1, &sc));
  if (hipHostMalloc(&B.host, sizeof(GpeScalars), hipHostMallocDefault) != hipSuccess) {
    set_error("pinned allocation failed");
    return TS_ERR_NOMEM;
  }
  GpeScalars* hs = (GpeScalars*)B.host;
  const GpeGrid G = gpe_grid(p);
  const int* done = &sc->done;
  TS_TRY(launch_gpe_init(sc, beta, tol, maxit, st));
  TS_TRY(launch_wdot2(G, u, u, u, part, part2, nullptr, st));
  TS_TRY(launch_gpe_scalar(GpeStep::Norm, sc, part, nullptr, nullptr, st));
  TS_TRY(launch_gpe_normalize(u, N, sc, nullptr, st));
  TS_TRY(hipMemsetAsync(z, 0, sizeof(double) * (size_t)N, st));
  GpeOpArgs op;
  op.grid = G;
  op.V2 = V2;
  op.beta = beta;
  op.u = u;
  op.out = Ep;
  op.partial = part;
  op.partial2 = part2;
  op.skip = done;
  int total_its = 0;
  GpeScalars s;
  for (int k = 0; k <= maxit; ++k) {
    TS_RC(gpe_op(p, op, Hu, st));
    TS_TRY(launch_gpe_scalar(GpeStep::Energy, sc, part, part2, hist, st));
    TS_TRY(hipMemcpyAsync(hs, sc, sizeof(GpeScalars), hipMemcpyDeviceToHost, st));
    TS_TRY(hipStreamSynchronize(st));
    std::memcpy(&s, hs, sizeof(s));
    if (s.done) break;
    // z = G_u^{-1} u, warm-started from the previous z
    TS_TRY(launch_gpe_potential(V2, u, beta, W, N, st));
    int its = 0;
    double rr = 0.0;
    int rc = pcg_run(p, W, 0.0, 0.0, u, z, pcg_rtol, pcg_maxit, precond, &its, &rr, st, p->ctx);
    total_its += its;
    if (rc) return rc;
    TS_TRY(launch_wdot2(G, u, z, u, part, part2, done, st));
    TS_TRY(launch_gpe_scalar(GpeStep::CoefInv, sc, part, part2, nullptr, st));
    TS_TRY(launch_gpe_update(G, u, u, z, tau, sc, part, done, st));
    TS_TRY(launch_gpe_scalar(GpeStep::Norm, sc, part, nullptr, nullptr, st));
    TS_TRY(launch_gpe_normalize(u, N, sc, done, st));
  }
  if (linear_its) *linear_its = total_its;
  return finish(s, energy_hist, hist, iters, eigenvalue, energy, st);
}

}  // namespace ts

using namespace ts;

extern "C" {

int ts_gpe_h1_flow(ts_plan* plan, const double* V, double beta, double alpha, double tau, double* u, int maxit,
                   double tol, double* energy_hist, int* iters, double* eigenvalue, double* energy,
                   void* hip_stream) {
  return gpe_h1_flow(plan, V, beta, alpha, tau, u, maxit, tol, energy_hist, iters, eigenvalue, energy,
                     (hipStream_t)hip_stream);
}

int ts_gpe_au_flow(ts_plan* plan, const double* V2, double beta, double tau, double* u, int maxit, double tol,
                   double pcg_rtol, int pcg_maxit, int precond, double* energy_hist, int* iters,
                   int* linear_iters, double* eigenvalue, double* energy, void* hip_stream) {
  if (precond < TS_PREC_FP64 || precond > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  return gpe_au_flow(plan, V2, beta, tau, u, maxit, tol, pcg_rtol, pcg_maxit, precond, energy_hist, iters,
                     linear_iters, eigenvalue, energy, (hipStream_t)hip_stream);
}

}  // extern "C"
