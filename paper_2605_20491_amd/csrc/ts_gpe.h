// GPE ground-state flows (gpe_kernels.hip kernels, gpe.cpp drivers).
#pragma once

#include "ts_internal.h"

namespace ts {

// Grid description shared by the GPE kernels: extents, strides, the per-axis
// L^2 weights, and the operator A of the plan (FD stencil or SEM band) with
// its separable potential samples f_k.
struct GpeGrid {
  int d = 0;
  int64_t N = 0;
  int64_t n[TS_MAX_D] = {};
  int64_t stride[TS_MAX_D] = {};
  const double* mass[TS_MAX_D] = {};
  const double* f[TS_MAX_D] = {};
  double ih2[TS_MAX_D] = {};
  int bw = 0;
  const double* band[TS_MAX_D] = {};
};

struct GpeOpArgs {
  GpeGrid grid;
  const double* V2 = nullptr;  // grid potential added to the plan's, may be null
  double beta = 0.0;
  const double* u = nullptr;
  double* out = nullptr;       // (A + V2 + beta u^2) u
  double* partial = nullptr;   // [kRedBlocks] shares of (u, out)
  double* partial2 = nullptr;  // [kRedBlocks] shares of (u^4, 1)
  const int* skip = nullptr;
  // generic plans with a wide band: (sum_k B_k + F) u precomputed by the dense
  // operator passes; the kernel then adds only (V2 + beta u^2) u
  const double* Hu = nullptr;
};

// Device scalar block of a flow.  status: 0 running / converged, 2 non-finite, 3 iteration limit.
struct GpeScalars {
  double E, lam, c, nrm2, beta, tol;
  int done, iters, maxit, status;
};

enum class GpeStep : int { Energy = 0, Coef = 1, CoefInv = 2, Norm = 3 };

hipError_t launch_gpe_op(const GpeOpArgs& a, hipStream_t st);
hipError_t launch_wdot2(const GpeGrid& g, const double* x, const double* y, const double* z, double* partial,
                        double* partial2, const int* skip, hipStream_t st);
hipError_t launch_gpe_update(const GpeGrid& g, double* u, const double* gr, const double* gu, double tau,
                             const GpeScalars* sc, double* partial, const int* skip, hipStream_t st);
hipError_t launch_gpe_normalize(double* u, int64_t N, const GpeScalars* sc, const int* skip, hipStream_t st);
hipError_t launch_gpe_potential(const double* V2, const double* u, double beta, double* W, int64_t N,
                                hipStream_t st);
hipError_t launch_gpe_scalar(GpeStep what, GpeScalars* sc, const double* partial, const double* partial2,
                             double* hist, hipStream_t st);
hipError_t launch_gpe_init(GpeScalars* sc, double beta, double tol, int maxit, hipStream_t st);

}  // namespace ts
