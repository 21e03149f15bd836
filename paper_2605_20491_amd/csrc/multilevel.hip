// Multi-level shifted inverse iteration (paper Sec. 5.3.1, Table
// tab:multilevel): solve on a coarse grid, carry the eigenvector to the next
// finer grid by tensor-product linear interpolation, continue there.
//
// The interpolation runs one axis at a time: a pass maps X viewed as
// [P][n_c][R] to [P][n_f][R] with two taps per fine node,
//   y[p, i, r] = w_lo[i] x[p, lo[i], r] + w_hi[i] x[p, hi[i], r],
// lo/hi = -1 standing for the Dirichlet zero outside the coarse nodes.  Each
// pass is one read and one write of the data (HBM-bound).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_internal.h"

namespace ts {
namespace {

constexpr int kThreads = 256;

struct AxisTaps {
  const int* lo;
  const int* hi;
  const double* wlo;
  const double* whi;
};

__global__ __launch_bounds__(kThreads) void k_interp_axis(const double* x, double* y, int64_t P, int64_t nc,
                                                         int64_t nf, int64_t R, AxisTaps t) {
  const int64_t total = P * nf * R;
  for (int64_t idx = blockIdx.x * (int64_t)kThreads + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kThreads) {
    const int64_t r = idx % R;
    const int64_t q = idx / R;
    const int64_t i = q % nf;
    const int64_t p = q / nf;
    const int lo = t.lo[i], hi = t.hi[i];
    double v = 0.0;
    if (lo >= 0) v += t.wlo[i] * x[(p * nc + lo) * R + r];
    if (hi >= 0) v += t.whi[i] * x[(p * nc + hi) * R + r];
    y[idx] = v;
  }
}

// out[idx] = prod_k v_k[i_k]
__global__ __launch_bounds__(kThreads) void k_outer(double* out, int d, int64_t N, const int64_t* n,
                                                   const double* const* v) {
  for (int64_t idx = blockIdx.x * (int64_t)kThreads + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * kThreads) {
    double s = 1.0;
    int64_t rem = idx;
    for (int k = d - 1; k >= 0; --k) {
      s *= v[k][rem % n[k]];
      rem /= n[k];
    }
    out[idx] = s;
  }
}

// Device buffers released on scope exit.
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* q : ptrs) hipFree(q);
  }
  template <class T>
  T* get(size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) return nullptr;
    ptrs.push_back(q);
    return (T*)q;
  }
};

// Fine node xf in the augmented coarse node list (-L, xc..., L): the coarse
// indices of the bracketing nodes (-1 at the boundary) and linear weights.
void axis_taps(const std::vector<double>& xc, const std::vector<double>& xf, double L, std::vector<int>& lo,
               std::vector<int>& hi, std::vector<double>& wlo, std::vector<double>& whi) {
  const int64_t nc = (int64_t)xc.size(), nf = (int64_t)xf.size();
  lo.resize(nf);
  hi.resize(nf);
  wlo.resize(nf);
  whi.resize(nf);
  for (int64_t i = 0; i < nf; ++i) {
    const double x = std::min(std::max(xf[i], -L), L);
    // first coarse node >= x
    const int64_t j = std::lower_bound(xc.begin(), xc.end(), x) - xc.begin();
    const double a = j == 0 ? -L : xc[j - 1];
    const double b = j == nc ? L : xc[j];
    const double t = b > a ? (x - a) / (b - a) : 0.0;
    lo[i] = (int)(j - 1);  // -1: the zero at -L
    hi[i] = j == nc ? -1 : (int)j;
    wlo[i] = 1.0 - t;
    whi[i] = t;
  }
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

inline unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 1 << 20); }

}  // namespace

int interpolate_run(const ts_plan* c, const ts_plan* f, const double* uc, double* uf, hipStream_t st) {
  if (!c || !f || !uc || !uf) { set_error("null argument"); return TS_ERR_INVALID; }
  if (c->d != f->d) { set_error("plans differ in dimension"); return TS_ERR_INVALID; }
  if (!(c->L > 0.0) || !(f->L > 0.0)) { set_error("interpolation needs FD or SEM plans (nodes on [-L, L])"); return TS_ERR_INVALID; }
  if (std::fabs(c->L - f->L) > 1e-12 * c->L) { set_error("plans differ in L"); return TS_ERR_INVALID; }
  const int d = c->d;
  Scratch S;
  // intermediate shapes: axes 0..k-1 fine, k..d-1 coarse; two ping-pong buffers
  int64_t maxN = 0;
  {
    int64_t cur = c->N;
    for (int k = 0; k < d; ++k) {
      cur = cur / c->n[k] * f->n[k];
      maxN = std::max(maxN, cur);
    }
  }
  double* buf[2] = {S.get<double>((size_t)maxN), S.get<double>((size_t)maxN)};
  if (!buf[0] || !buf[1]) { set_error("interpolation scratch allocation failed"); return TS_ERR_NOMEM; }
  std::vector<int64_t> shape(c->n, c->n + d);
  const double* src = uc;
  for (int k = 0; k < d; ++k) {
    std::vector<int> lo, hi;
    std::vector<double> wlo, whi;
    axis_taps(c->ax[k]->x_h, f->ax[k]->x_h, c->L, lo, hi, wlo, whi);
    const int64_t nf = f->n[k];
    int* dlo = S.get<int>(nf);
    int* dhi = S.get<int>(nf);
    double* dwl = S.get<double>(nf);
    double* dwh = S.get<double>(nf);
    if (!dlo || !dhi || !dwl || !dwh) { set_error("interpolation table allocation failed"); return TS_ERR_NOMEM; }
    TS_TRY(hipMemcpyAsync(dlo, lo.data(), sizeof(int) * nf, hipMemcpyHostToDevice, st));
    TS_TRY(hipMemcpyAsync(dhi, hi.data(), sizeof(int) * nf, hipMemcpyHostToDevice, st));
    TS_TRY(hipMemcpyAsync(dwl, wlo.data(), sizeof(double) * nf, hipMemcpyHostToDevice, st));
    TS_TRY(hipMemcpyAsync(dwh, whi.data(), sizeof(double) * nf, hipMemcpyHostToDevice, st));
    int64_t P = 1, R = 1;
    for (int m = 0; m < k; ++m) P *= shape[m];
    for (int m = k + 1; m < d; ++m) R *= shape[m];
    double* dst = (k == d - 1) ? uf : buf[k % 2];
    AxisTaps t{dlo, dhi, dwl, dwh};
    hipLaunchKernelGGL(k_interp_axis, dim3(grid_for(P * nf * R)), dim3(kThreads), 0, st, src, dst, P, shape[k], nf,
                       R, t);
    TS_TRY(hipGetLastError());
    shape[k] = nf;
    src = dst;
  }
  // the tables are freed on return: wait for the passes that read them
  TS_TRY(hipStreamSynchronize(st));
  return TS_OK;
}

// Separable ground state of H1 (column 0 of each axis's T), unit L^2 norm
// taken later by the inverse iteration's normalisation.
int separable_ground_state(const ts_plan* p, double* u, hipStream_t st) {
  Scratch S;
  std::vector<const double*> vptr(p->d);
  for (int k = 0; k < p->d; ++k) {
    const AxisFactor& F = *p->ax[k];
    std::vector<double> v(F.n);
    for (int64_t i = 0; i < F.n; ++i) {
      const double q = F.Q_h[(size_t)(i * F.n)];
      v[i] = p->massed ? q / std::sqrt(F.m_h[i]) : q;
    }
    double* dv = S.get<double>(F.n);
    if (!dv) { set_error("allocation failed"); return TS_ERR_NOMEM; }
    TS_TRY(hipMemcpyAsync(dv, v.data(), sizeof(double) * F.n, hipMemcpyHostToDevice, st));
    vptr[k] = dv;
  }
  const double** dptrs = S.get<const double*>(p->d);
  int64_t* dn = S.get<int64_t>(p->d);
  if (!dptrs || !dn) { set_error("allocation failed"); return TS_ERR_NOMEM; }
  TS_TRY(hipMemcpyAsync(dptrs, vptr.data(), sizeof(double*) * p->d, hipMemcpyHostToDevice, st));
  TS_TRY(hipMemcpyAsync(dn, p->n, sizeof(int64_t) * p->d, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_outer, dim3(grid_for(p->N)), dim3(kThreads), 0, st, u, p->d, p->N, dn, dptrs);
  TS_TRY(hipGetLastError());
  TS_TRY(hipStreamSynchronize(st));
  return TS_OK;
}

}  // namespace ts

using namespace ts;

extern "C" {

int ts_interpolate(const ts_plan* coarse, const ts_plan* fine, const double* uc, double* uf, void* hip_stream) {
  return interpolate_run(coarse, fine, uc, uf, (hipStream_t)hip_stream);
}

int ts_separable_ground_state(const ts_plan* plan, double* u, void* hip_stream) {
  if (!plan || !u) { set_error("null argument"); return TS_ERR_INVALID; }
  return separable_ground_state(plan, u, (hipStream_t)hip_stream);
}

int ts_multilevel_inverse_iteration(int nlevels, ts_plan* const* plans, const double* const* V2,
                                    const double* shifts, double* u, int max_steps, double lam_tol,
                                    double pcg_rtol, int pcg_maxit, int precond, double* lam_levels,
                                    int* steps, int* pcg_iters, void* hip_stream) {
  if (nlevels < 1 || !plans || !shifts || !u) { set_error("bad argument"); return TS_ERR_INVALID; }
  for (int l = 0; l < nlevels; ++l)
    if (!plans[l]) { set_error("null plan"); return TS_ERR_INVALID; }
  hipStream_t st = (hipStream_t)hip_stream;
  Scratch S;
  // level vectors: the finest level iterates in the caller's u
  std::vector<double*> lv(nlevels);
  for (int l = 0; l < nlevels; ++l) {
    lv[l] = (l == nlevels - 1) ? u : S.get<double>((size_t)plans[l]->N);
    if (!lv[l]) { set_error("level vector allocation failed"); return TS_ERR_NOMEM; }
  }
  TS_RC(separable_ground_state(plans[0], lv[0], st));
  for (int l = 0; l < nlevels; ++l) {
    if (l > 0) TS_RC(interpolate_run(plans[l - 1], plans[l], lv[l - 1], lv[l], st));
    std::vector<double> hist((size_t)max_steps + 1);
    std::vector<int> its((size_t)std::max(max_steps, 1));
    int done = 0;
    int rc = invit_run(plans[l], V2 ? V2[l] : nullptr, shifts[l], lv[l], max_steps, lam_tol, pcg_rtol, pcg_maxit,
                       precond, hist.data(), its.data(), &done, st);
    if (steps) steps[l] = done;
    if (pcg_iters) {
      int sum = 0;
      for (int k = 0; k < done; ++k) sum += its[k];
      pcg_iters[l] = sum;
    }
    if (lam_levels) lam_levels[l] = hist[done];
    if (rc) return rc;
  }
  return TS_OK;
}

}  // extern "C"
