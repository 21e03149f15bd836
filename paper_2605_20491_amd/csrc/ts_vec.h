// Launchers of the FP64 vector kernels (vec.hip): the stencil operator of
// eq. (general_system), deterministic reductions and the fused vector
// updates of PCG / iterative refinement.
#pragma once

#include "ts_internal.h"

namespace ts {

constexpr int kRedBlocks = 1024;  // fixed grid of every reduction: results are bitwise reproducible

// Output and reduction modes of the stencil kernel.
enum class StOut : int { Ax = 0, FminusAx = 1 };
enum class StDot : int { None = 0, UdotOut = 1, OutdotOut = 2 };

struct SolverScalars;

struct StencilArgs {
  int d = 0;
  int64_t N = 0;
  int64_t n[TS_MAX_D] = {};
  int64_t stride[TS_MAX_D] = {};
  double ih2[TS_MAX_D] = {};
  const double* f[TS_MAX_D] = {};  // device samples of f_k
  const double* V2 = nullptr;
  double s = 0.0;
  const double* u = nullptr;
  // Fused update of the PCG direction: with z set, the operator acts on
  // z + beta u (beta = bsc->beta), which is also written to unew (a buffer
  // other than u: neighbouring tiles still read the old u)
  const double* z = nullptr;
  const SolverScalars* bsc = nullptr;
  double* unew = nullptr;
  const double* rhs = nullptr;     // StOut::FminusAx: out = rhs - A u
  double* out = nullptr;
  StOut mode = StOut::Ax;
  StDot dot = StDot::None;
  double* partial = nullptr;       // [kRedBlocks] when dot != None
  const int* skip = nullptr;
  // Q^k SEM: per-axis operator bands [n_k][2 bw + 1] (entry (i, i - bw + t))
  // replace the h^-2 (-1, 2, -1) stencil when bw > 0
  int bw = 0;
  const double* band[TS_MAX_D] = {};
  // Generic plans with a wide band: the per-axis operators as FP64 pass
  // factors (the band is then not read), and two N-sized FP64 buffers for the
  // per-axis products
  const AxisFactor* dense[TS_MAX_D] = {};
  double* tmp0 = nullptr;
  double* tmp1 = nullptr;
};

hipError_t launch_stencil(const StencilArgs& a, hipStream_t st);

// Operator arguments of a plan: (H1 + V2 + s) on u into out, from the
// symmetric-form factors (sym: the solvers) or the public ones (defined in solvers.cpp).
StencilArgs stencil_args(const ts_plan* p, const double* V2, double s, const double* u, double* out, bool sym);

// y = x * prod_k w_k(i_k) pointwise (x may equal y); w_k device vectors of n_k.
hipError_t launch_axis_scale(const double* x, double* y, int d, const int64_t* n, const double* const* w,
                             hipStream_t st);

// Device scalar block used by the solvers (all FP64 except the int flags).
struct SolverScalars {
  double rz, rz_new, pq, zq, alpha, beta, rr, ff, tol2, rr_prev;
  double aux[6];
  int done, status, iters, pad;
};

// partial[b] = block b's share of sum x*y (and of sum x*w into partial2 if w).
hipError_t launch_dot(const double* x, const double* y, int64_t n, double* partial,
                      const double* w, double* partial2, const int* skip, hipStream_t st);

// x += alpha p; r -= alpha q; partial <- ||r||^2 shares.  alpha from sc.
// r16 (optional): r rounded to BF16 as the BF16 apply's input sweep rounds it.
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, int64_t n,
                            const SolverScalars* sc, double* partial, const int* skip, hipStream_t st,
                            uint16_t* r16 = nullptr);
// The same with r16 = the BF16 rounding of r folded along the axes of b (the
// input a BF16 apply with those folded axes reads, see bf16_fold_axes): the
// data walked by orbits of the reflections, four fastest-axis points per
// thread.  Needs n_{d-1} % 8 == 0, 16-byte aligned vectors and an 8-byte
// aligned r16 (cg_update_fold_ok).
bool cg_update_fold_ok(const ButterflyArgs& b, const double* x, const double* r, const double* p, const double* q,
                       const uint16_t* r16);
hipError_t launch_cg_update_fold(double* x, double* r, const double* p, const double* q, const ButterflyArgs& b,
                                 const SolverScalars* sc, double* partial, const int* skip, uint16_t* r16,
                                 hipStream_t st);

// p = z + beta p (beta from sc).
hipError_t launch_xpby(const double* z, double* p, int64_t n, const SolverScalars* sc, const int* skip,
                       hipStream_t st);

// x += y (iterative refinement correction).
hipError_t launch_axpy1(double* x, const double* y, int64_t n, const int* skip, hipStream_t st);

// y = x / sqrt(sc->aux[0]).
hipError_t launch_scale_invnorm(const double* x, double* y, int64_t n, const SolverScalars* sc, hipStream_t st);

// Zero the scalar block and set its tolerance, on the device.
hipError_t launch_init_scalars(SolverScalars* sc, double tol2, hipStream_t st);

// Scalar steps of PCG, one thread block each.  `what` selects the step.
enum class ScalarStep : int {
  InitRR = 0,      // rr <- sum(partial), ff <- sum(partial2) ; done if rr <= tol2 * ff
  InitRZ = 1,      // rz <- sum(partial)
  Alpha = 2,       // pq <- sum(partial); alpha = rz / pq (breakdown if pq <= 0)
  RR = 3,          // rr <- sum(partial); iters++; done if rr <= tol2 * ff or iters >= maxit
  Beta = 4,        // rz_new <- sum(partial), zq <- sum(partial2); beta (standard or flexible)
  SetRR = 5,       // rr <- sum(partial) (no decision)
  SetAux0 = 6,     // aux[0] <- sum(partial)
};
hipError_t launch_scalar(ScalarStep what, SolverScalars* sc, const double* partial, const double* partial2,
                         int flexible, int maxit, hipStream_t st);

}  // namespace ts
