// Kernels of the GPE ground-state flows (paper Sec. 4.2-4.3): the nonlinear
// operator E'(u) = (A + V2 + beta u^2) u fused with the two L^2 sums that give
// the energy and the eigenvalue, mass-weighted inner products, the Riemannian
// update, and the one-block scalar steps that keep every decision on the
// device.  The L^2 weight of a grid point is prod_k m_k(i_k), from the
// per-axis weights of the plan (FD: h; SEM: the lumped Gauss-Lobatto mass).
#include <cmath>

#include "ts_gpe.h"
#include "ts_reduce.h"
#include "ts_vec.h"

namespace ts {
namespace {

// Decode idx into per-axis coordinates (axis d-1 fastest) and return the
// point's L^2 weight.
__device__ __forceinline__ double point_weight(const GpeGrid& g, int64_t idx, int64_t* c) {
  double w = 1.0;
  int64_t rem = idx;
  for (int k = g.d - 1; k >= 0; --k) {
    const int64_t i = rem % g.n[k];
    rem /= g.n[k];
    c[k] = i;
    w *= g.mass[k][i];
  }
  return w;
}

__global__ __launch_bounds__(RT) void k_gpe_op(GpeOpArgs a) {
  if (a.skip && *a.skip) {
    if (threadIdx.x == 0) {
      a.partial[blockIdx.x] = 0.0;
      a.partial2[blockIdx.x] = 0.0;
    }
    return;
  }
  const GpeGrid& g = a.grid;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)RT + threadIdx.x; idx < g.N; idx += (int64_t)gridDim.x * RT) {
    int64_t c[TS_MAX_D];
    const double w = point_weight(g, idx, c);
    const double uc = a.u[idx];
    double acc = 0.0, diag = a.V2 ? a.V2[idx] : 0.0;
    if (a.Hu) acc = a.Hu[idx];
    for (int k = 0; k < g.d && !a.Hu; ++k) {
      const int64_t i = c[k], nk = g.n[k], st = g.stride[k];
      diag += g.f[k][i];
      if (g.bw == 0) {  // FD: h^-2 (2u - u_lo - u_hi), zero ghosts
        const double lo = i > 0 ? a.u[idx - st] : 0.0;
        const double hi = i + 1 < nk ? a.u[idx + st] : 0.0;
        acc += g.ih2[k] * (2.0 * uc - lo - hi);
      } else {          // SEM: band of M^{-1} S
        const int wd = 2 * g.bw + 1;
        const double* row = g.band[k] + i * wd;
        for (int t = 0; t < wd; ++t) {
          const int64_t j = i - g.bw + t;
          if (j >= 0 && j < nk) acc += row[t] * a.u[idx + (j - i) * st];
        }
      }
    }
    const double v = acc + (diag + a.beta * uc * uc) * uc;
    a.out[idx] = v;
    s1 += w * uc * v;
    const double u2 = uc * uc;
    s2 += w * u2 * u2;
  }
  const double t1 = block_sum(s1);
  const double t2 = block_sum(s2);
  if (threadIdx.x == 0) {
    a.partial[blockIdx.x] = t1;
    a.partial2[blockIdx.x] = t2;
  }
}

// partial = sum w x y, partial2 = sum w x z
__global__ __launch_bounds__(RT) void k_wdot2(GpeGrid g, const double* x, const double* y, const double* z,
                                              double* partial, double* partial2, const int* skip) {
  if (skip && *skip) {
    if (threadIdx.x == 0) {
      partial[blockIdx.x] = 0.0;
      partial2[blockIdx.x] = 0.0;
    }
    return;
  }
  double s1 = 0.0, s2 = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)RT + threadIdx.x; idx < g.N; idx += (int64_t)gridDim.x * RT) {
    int64_t c[TS_MAX_D];
    const double w = point_weight(g, idx, c);
    const double xi = x[idx];
    s1 += w * xi * y[idx];
    s2 += w * xi * z[idx];
  }
  const double t1 = block_sum(s1);
  const double t2 = block_sum(s2);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = t1;
    partial2[blockIdx.x] = t2;
  }
}

// u <- u - tau (g - c gu) with c from the scalar block; partial = sum w u^2.
// g may alias u (a_u flow: the metric gradient is u itself).
__global__ __launch_bounds__(RT) void k_gpe_update(GpeGrid g, double* u, const double* gr, const double* gu,
                                                   double tau, const GpeScalars* sc, double* partial,
                                                   const int* skip) {
  if (skip && *skip) {
    if (threadIdx.x == 0) partial[blockIdx.x] = 0.0;
    return;
  }
  const double cf = sc->c;
  double s = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)RT + threadIdx.x; idx < g.N; idx += (int64_t)gridDim.x * RT) {
    int64_t c[TS_MAX_D];
    const double w = point_weight(g, idx, c);
    const double v = u[idx] - tau * (gr[idx] - cf * gu[idx]);
    u[idx] = v;
    s += w * v * v;
  }
  const double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// u <- u / sqrt(sc->nrm2)
__global__ __launch_bounds__(RT) void k_gpe_normalize(double* u, int64_t N, const GpeScalars* sc, const int* skip) {
  if (skip && *skip) return;
  const double inv = 1.0 / sqrt(sc->nrm2);
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < N; i += (int64_t)gridDim.x * RT) u[i] *= inv;
}

// W = V2 + beta u^2 (the a_u metric's potential for PCG)
__global__ __launch_bounds__(RT) void k_gpe_potential(const double* V2, const double* u, double beta, double* W,
                                                      int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < N; i += (int64_t)gridDim.x * RT) {
    const double ui = u[i];
    W[i] = (V2 ? V2[i] : 0.0) + beta * ui * ui;
  }
}

__global__ __launch_bounds__(RT) void k_gpe_scalar(int what, GpeScalars* sc, const double* partial,
                                                   const double* partial2, double* hist) {
  const double a = sum_partials(partial, kRedBlocks);
  const double b = partial2 ? sum_partials(partial2, kRedBlocks) : 0.0;
  if (threadIdx.x != 0) return;
  if (sc->done) return;
  switch (what) {
    case (int)GpeStep::Energy: {
      // a = (u, E'(u)), b = (u^4, 1):  E = a/2 - beta b/4  (eq. (gpe_energy)), lambda = a
      const double E = 0.5 * a - 0.25 * sc->beta * b;
      sc->lam = a;
      if (!isfinite(E)) { sc->status = 2; sc->done = 1; break; }
      if (hist) hist[sc->iters] = E;
      if (sc->tol > 0.0 && sc->iters > 0 && fabs(E - sc->E) <= sc->tol * fabs(E)) sc->done = 1;
      else if (sc->iters >= sc->maxit) { sc->status = 3; sc->done = 1; }
      sc->E = E;
      if (!sc->done) sc->iters += 1;
      break;
    }
    case (int)GpeStep::Coef:     // c = (u, G^{-1} E') / (u, G^{-1} u)
      sc->c = a / b;
      if (!isfinite(sc->c)) { sc->status = 2; sc->done = 1; }
      break;
    case (int)GpeStep::CoefInv:  // c = (u, u) / (u, z)
      sc->c = b / a;
      if (!isfinite(sc->c)) { sc->status = 2; sc->done = 1; }
      break;
    case (int)GpeStep::Norm:
      sc->nrm2 = a;
      if (!(a > 0.0) || !isfinite(a)) { sc->status = 2; sc->done = 1; }
      break;
  }
}

__global__ void k_gpe_init(GpeScalars* sc, double beta, double tol, int maxit) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    GpeScalars z = {};
    z.beta = beta;
    z.tol = tol;
    z.maxit = maxit;
    *sc = z;
  }
}

inline unsigned stream_grid(int64_t n) { return (unsigned)std::min<int64_t>((n + RT - 1) / RT, 1 << 20); }

}  // namespace

hipError_t launch_gpe_op(const GpeOpArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_gpe_op, dim3(kRedBlocks), dim3(RT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_wdot2(const GpeGrid& g, const double* x, const double* y, const double* z, double* partial,
                        double* partial2, const int* skip, hipStream_t st) {
  hipLaunchKernelGGL(k_wdot2, dim3(kRedBlocks), dim3(RT), 0, st, g, x, y, z, partial, partial2, skip);
  return hipGetLastError();
}

hipError_t launch_gpe_update(const GpeGrid& g, double* u, const double* gr, const double* gu, double tau,
                             const GpeScalars* sc, double* partial, const int* skip, hipStream_t st) {
  hipLaunchKernelGGL(k_gpe_update, dim3(kRedBlocks), dim3(RT), 0, st, g, u, gr, gu, tau, sc, partial, skip);
  return hipGetLastError();
}

hipError_t launch_gpe_normalize(double* u, int64_t N, const GpeScalars* sc, const int* skip, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gpe_normalize, dim3(stream_grid(N)), dim3(RT), 0, st, u, N, sc, skip);
  return hipGetLastError();
}

hipError_t launch_gpe_potential(const double* V2, const double* u, double beta, double* W, int64_t N,
                                hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gpe_potential, dim3(stream_grid(N)), dim3(RT), 0, st, V2, u, beta, W, N);
  return hipGetLastError();
}

hipError_t launch_gpe_scalar(GpeStep what, GpeScalars* sc, const double* partial, const double* partial2,
                             double* hist, hipStream_t st) {
  hipLaunchKernelGGL(k_gpe_scalar, dim3(1), dim3(RT), 0, st, (int)what, sc, partial, partial2, hist);
  return hipGetLastError();
}

hipError_t launch_gpe_init(GpeScalars* sc, double beta, double tol, int maxit, hipStream_t st) {
  hipLaunchKernelGGL(k_gpe_init, dim3(1), dim3(64), 0, st, sc, beta, tol, maxit);
  return hipGetLastError();
}

}  // namespace ts
