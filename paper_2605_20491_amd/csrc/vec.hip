// HBM-bound FP64 kernels around the separable apply: the non-separable
// operator by its (2d+1)-point stencil (paper eq. (general_system)), and the
// deterministic reductions and fused vector updates of PCG (Sec. 3.2) and
// iterative refinement.
//
// Reductions are two-stage with a fixed grid (kRedBlocks blocks): each block
// writes one partial sum, and a one-block "scalar" kernel adds the partials in
// index order and takes the solver decision (alpha, beta, convergence) on the
// device.  Results are bitwise reproducible from run to run.
#include "bf16_round.h"
#include "modeprod_common.h"
#include "ts_internal.h"
#include "ts_reduce.h"
#include "ts_vec.h"

namespace ts {
namespace {

// Stencil tiles: the grid is viewed as [P][NY][NX] with NX = n_{d-1}, NY =
// n_{d-2} and P the flattened slower axes 0..d-3.  A block covers a TY x TX
// patch of one (y, x) plane and marches through `planes` consecutive planes p:
// the patch and its one-point halo are staged in LDS for the y and x
// neighbours, the neighbours along axis d-3 (p -+ 1) stay in registers, and
// the neighbours along axes 0..d-4 are read from memory.  Every value of u is
// read from HBM once (plus the halo).
constexpr int kTX = 64, kTYT = 4, kRows = 4, kTY = kTYT * kRows;
constexpr int kLX = kTX + 2;  // LDS row length

template <int MODE, int DOT>
__global__ __launch_bounds__(RT) void k_stencil(StencilArgs a, int64_t tx_tiles, int64_t ty_tiles,
                                                int64_t p_tiles, int64_t planes) {
  if (a.skip && *a.skip) {
    if (DOT && threadIdx.x == 0 && blockIdx.x < kRedBlocks) a.partial[blockIdx.x] = 0.0;
    return;
  }
  __shared__ double tile[kTY + 2][kLX];
  const int d = a.d;
  const int ax = d - 1, ay = d - 2, ap = d - 3;  // ay < 0 if d == 1, ap < 0 if d <= 2
  const int64_t NX = a.n[ax], NY = ay >= 0 ? a.n[ay] : 1, NXY = NX * NY;
  const int64_t P = a.N / NXY;
  const int64_t np = ap >= 0 ? a.n[ap] : 1;  // extent of the marching axis
  const double ihx = a.ih2[ax], ihy = ay >= 0 ? a.ih2[ay] : 0.0, ihp = ap >= 0 ? a.ih2[ap] : 0.0;
  const int tx = threadIdx.x & (kTX - 1), ty = threadIdx.x / kTX;
  const int64_t ntask = tx_tiles * ty_tiles * p_tiles;
  // operand: u, or z + beta u when the PCG direction update is fused in.  A
  // value is fetched raw (z and u) and combined only where it is used, so the
  // loads of later planes stay in flight across the LDS-only barriers.
  const double* __restrict__ zz = a.z;
  const double beta = zz ? a.bsc->beta : 0.0;
  struct Raw { double z, u; };
  auto fetch = [&](bool in, int64_t i) -> Raw {
    Raw r{0.0, 0.0};
    if (in) {
      r.u = a.u[i];
      if (zz) r.z = zz[i];
    }
    return r;
  };
  auto val = [&](const Raw& r) -> double { return zz ? r.z + beta * r.u : r.u; };
  auto ld = [&](int64_t i) -> double { return zz ? zz[i] + beta * a.u[i] : a.u[i]; };
  // the halo value this thread stages for plane q (one of rows y0 - 1, y0 + kTY,
  // columns x0 - 1, x0 + kTX), or none
  auto halo = [&](int64_t q, int64_t bx, int64_t by, int64_t x) -> Raw {
    const int64_t y0 = by * kTY, x0 = bx * kTX;
    const int64_t pb = q * NXY;
    if (ty < 2) {
      const int64_t yh = ty == 0 ? y0 - 1 : y0 + kTY;
      return fetch(x < NX && yh >= 0 && yh < NY, pb + yh * NX + x);
    } else if (tx < kTY) {
      const int64_t xh = ty == 2 ? x0 - 1 : x0 + kTX, yh = y0 + tx;
      return fetch(xh >= 0 && xh < NX && yh < NY, pb + yh * NX + xh);
    }
    return Raw{0.0, 0.0};
  };
  double dsum = 0.0;
  for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
    const int64_t bx = task % tx_tiles, rest = task / tx_tiles;
    const int64_t by = rest % ty_tiles, bp = rest / ty_tiles;
    const int64_t x = bx * kTX + tx;
    const int64_t p0 = bp * planes, p1 = p0 + planes < P ? p0 + planes : P;
    const bool xin = x < NX;
    // um, uc, nx: planes p - 1, p, p + 1 of this thread's rows; raw values of
    // plane p + 2 and the halo of plane p + 1 are requested one plane ahead
    double fxy[kRows], um[kRows], uc[kRows], nx[kRows];
    int64_t yy[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      yy[j] = by * kTY + ty + kTYT * j;
      const bool in = xin && yy[j] < NY;
      fxy[j] = in ? a.f[ax][x] + (ay >= 0 ? a.f[ay][yy[j]] : 0.0) : 0.0;
      const int64_t idx = (p0 * NY + yy[j]) * NX + x;
      uc[j] = in ? ld(idx) : 0.0;
      um[j] = (in && p0 > 0) ? ld(idx - NXY) : 0.0;
      nx[j] = (in && p0 + 1 < P) ? ld(idx + NXY) : 0.0;
    }
    double hcur = val(halo(p0, bx, by, x));
    for (int64_t p = p0; p < p1; ++p) {
      // requests for the next planes first
      Raw nn[kRows];
#pragma unroll
      for (int j = 0; j < kRows; ++j)
        nn[j] = fetch(xin && yy[j] < NY && p + 2 < P, ((p + 2) * NY + yy[j]) * NX + x);
      const Raw hnext = p + 1 < p1 ? halo(p + 1, bx, by, x) : Raw{0.0, 0.0};
      // position of plane p on the slower axes: diagonal part and neighbours
      const int64_t jp = ap >= 0 ? p % np : 0;
      double fp = a.s + (ap >= 0 ? a.f[ap][jp] : 0.0);
      unsigned lo_ok = 0, hi_ok = 0;
      {
        int64_t rem = ap >= 0 ? p / np : 0;
        for (int k = ap - 1; k >= 0; --k) {
          const int64_t j = rem % a.n[k];
          rem /= a.n[k];
          fp += a.f[k][j];
          if (j > 0) lo_ok |= 1u << k;
          if (j + 1 < a.n[k]) hi_ok |= 1u << k;
        }
      }
      const bool has_dn = jp > 0, has_up = jp + 1 < np;
#pragma unroll
      for (int j = 0; j < kRows; ++j) tile[ty + kTYT * j + 1][tx + 1] = uc[j];
      if (ty < 2) tile[ty == 0 ? 0 : kTY + 1][tx + 1] = hcur;
      else if (tx < kTY) tile[tx + 1][ty == 2 ? 0 : kLX - 1] = hcur;
      mp::lds_barrier();
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const int ly = ty + kTYT * j + 1;
        const bool in = xin && yy[j] < NY;
        if (in) {
          const int64_t idx = (p * NY + yy[j]) * NX + x;
          const double u0 = uc[j];
          double acc = 0.0;
          // axes 0 .. d-4 from memory, then the marching axis, then y and x (axis order)
          for (int k = 0; k < ap; ++k) {
            const int64_t st = a.stride[k];
            const double lo = ((lo_ok >> k) & 1u) ? ld(idx - st) : 0.0;
            const double hi = ((hi_ok >> k) & 1u) ? ld(idx + st) : 0.0;
            acc += a.ih2[k] * (2.0 * u0 - lo - hi);
          }
          if (ap >= 0) acc += ihp * (2.0 * u0 - (has_dn ? um[j] : 0.0) - (has_up ? nx[j] : 0.0));
          if (ay >= 0) acc += ihy * (2.0 * u0 - tile[ly - 1][tx + 1] - tile[ly + 1][tx + 1]);
          acc += ihx * (2.0 * u0 - tile[ly][tx] - tile[ly][tx + 2]);
          const double diag = fp + fxy[j] + (a.V2 ? a.V2[idx] : 0.0);
          double v = acc + diag * u0;
          if (MODE == (int)StOut::FminusAx) v = a.rhs[idx] - v;
          a.out[idx] = v;
          if (zz) a.unew[idx] = u0;
          if (DOT == (int)StDot::UdotOut) dsum += u0 * v;
          if (DOT == (int)StDot::OutdotOut) dsum += v * v;
        }
        um[j] = uc[j];
        uc[j] = nx[j];
        nx[j] = val(nn[j]);
      }
      hcur = val(hnext);
      mp::lds_barrier();
    }
  }
  if (DOT) {
    double sm = block_sum(dsum);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = sm;
  }
}

// Banded per-axis operator of Q^k SEM: sum_k (I x .. x B_k x .. x I) u plus
// the diagonal (sum_k f_k + V2 + s) u, one output point per thread.  The
// 2 bw + 1 neighbours of every axis are read in place (the fastest axis from
// the same cache lines, the others from L2 / the last-level cache).
template <int MODE, int DOT>
__global__ __launch_bounds__(RT) void k_band(StencilArgs a) {
  if (a.skip && *a.skip) {
    if (DOT && threadIdx.x == 0 && blockIdx.x < kRedBlocks) a.partial[blockIdx.x] = 0.0;
    return;
  }
  const int w = 2 * a.bw + 1;
  double dsum = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)RT + threadIdx.x; idx < a.N; idx += (int64_t)gridDim.x * RT) {
    double acc = 0.0;
    double diag = a.s + (a.V2 ? a.V2[idx] : 0.0);
    int64_t rem = idx;
    for (int k = a.d - 1; k >= 0; --k) {
      const int64_t nk = a.n[k];
      const int64_t i = rem % nk;
      rem /= nk;
      diag += a.f[k][i];
      const double* row = a.band[k] + i * w;
      const int64_t st = a.stride[k];
      const int64_t j0 = i - a.bw;
      for (int t = 0; t < w; ++t) {
        const int64_t j = j0 + t;
        if (j >= 0 && j < nk) acc += row[t] * a.u[idx + (j - i) * st];
      }
    }
    const double uc = a.u[idx];
    double v = acc + diag * uc;
    if (MODE == (int)StOut::FminusAx) v = a.rhs[idx] - v;
    a.out[idx] = v;
    if (DOT == (int)StDot::UdotOut) dsum += uc * v;
    if (DOT == (int)StDot::OutdotOut) dsum += v * v;
  }
  if (DOT) {
    double s = block_sum(dsum);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
  }
}

// Dense per-axis operators (generic plans with a wide band): the per-axis
// products sum_k (I x .. x B_k x .. x I) u come from MFMA passes, summed in
// tmp0 (+ tmp1); this kernel adds the diagonal (sum_k f_k + V2 + s) u and
// forms the output and its dot product exactly as k_band does.
__global__ __launch_bounds__(RT) void k_add_to(double* y, const double* x, int64_t N, const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < N; i += (int64_t)gridDim.x * RT) y[i] += x[i];
}

template <int MODE, int DOT>
__global__ __launch_bounds__(RT) void k_combine(StencilArgs a) {
  if (a.skip && *a.skip) {
    if (DOT && threadIdx.x == 0 && blockIdx.x < kRedBlocks) a.partial[blockIdx.x] = 0.0;
    return;
  }
  double dsum = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)RT + threadIdx.x; idx < a.N; idx += (int64_t)gridDim.x * RT) {
    double diag = a.s + (a.V2 ? a.V2[idx] : 0.0);
    int64_t rem = idx;
    for (int k = a.d - 1; k >= 0; --k) {
      diag += a.f[k][rem % a.n[k]];
      rem /= a.n[k];
    }
    const double acc = a.tmp0[idx] + (a.d > 1 ? a.tmp1[idx] : 0.0);
    const double uc = a.u[idx];
    double v = acc + diag * uc;
    if (MODE == (int)StOut::FminusAx) v = a.rhs[idx] - v;
    a.out[idx] = v;
    if (DOT == (int)StDot::UdotOut) dsum += uc * v;
    if (DOT == (int)StDot::OutdotOut) dsum += v * v;
  }
  if (DOT) {
    double s = block_sum(dsum);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
  }
}

struct ScaleArgs {
  int d;
  int64_t n[TS_MAX_D];
  const double* w[TS_MAX_D];
};

__global__ __launch_bounds__(RT) void k_axis_scale(const double* x, double* y, int64_t N, ScaleArgs a) {
  for (int64_t idx = blockIdx.x * (int64_t)RT + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * RT) {
    double s = 1.0;
    int64_t rem = idx;
    for (int k = a.d - 1; k >= 0; --k) {
      s *= a.w[k][rem % a.n[k]];
      rem /= a.n[k];
    }
    y[idx] = x[idx] * s;
  }
}

__global__ __launch_bounds__(RT) void k_dot(const double* x, const double* y, int64_t n, double* partial,
                                            const double* w, double* partial2, const int* skip) {
  if (skip && *skip) {
    if (threadIdx.x == 0) {
      partial[blockIdx.x] = 0.0;
      if (partial2) partial2[blockIdx.x] = 0.0;
    }
    return;
  }
  double s = 0.0, s2 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const double xi = x[i];
    s += xi * y[i];
    if (w) s2 += xi * w[i];
  }
  double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
  if (w) {
    double t2 = block_sum(s2);
    if (threadIdx.x == 0) partial2[blockIdx.x] = t2;
  }
}

// r16 (optional): also write r rounded to BF16 (FP64 -> FP32 -> BF16, as the
// BF16 apply's input sweep rounds it), so that sweep can be skipped.
__global__ __launch_bounds__(RT) void k_cg_update(double* x, double* r, const double* p, const double* q,
                                                  int64_t n, const SolverScalars* sc, double* partial,
                                                  const int* skip, uint16_t* r16) {
  if (skip && *skip) {
    if (threadIdx.x == 0) partial[blockIdx.x] = 0.0;
    return;
  }
  const double alpha = sc->alpha;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (r16) r16[i] = bf16_from_f32((float)ri);
    s += ri * ri;
  }
  double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// The same update walking the data by orbits of the reflections of the axes
// the next BF16 apply folds (b.ax: the slow ones in slots 0 .. NSLOW - 1, the
// fastest last when FAST; four consecutive fastest-axis points per thread, as
// the folding input sweep of the apply): after x and r of an orbit are
// updated, its r values are folded (s = r_i + r_{n-1-i} at i, d = r_i -
// r_{n-1-i} at n-1-i, in FP64, fastest axis first) and rounded FP64 -> FP32
// -> BF16 into r16, which is exactly what that sweep would write.  <r, r> is
// summed in orbit order.
template <int NSLOW, bool FAST>
__global__ __launch_bounds__(RT) void k_cg_update_fold(double* x, double* r, const double* p, const double* q,
                                                       ButterflyArgs b, int64_t units, const SolverScalars* sc,
                                                       double* partial, const int* skip, uint16_t* r16) {
  if (skip && *skip) {
    if (threadIdx.x == 0) partial[blockIdx.x] = 0.0;
    return;
  }
  constexpr int NB = NSLOW + (FAST ? 1 : 0);
  constexpr int NV = 1 << NB;
  const double alpha = sc->alpha;
  const int64_t nf = b.n[b.d - 1];
  const int64_t gq = (FAST ? nf / 2 : nf) / 4;
  double s = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)RT + threadIdx.x; e < units; e += (int64_t)gridDim.x * RT) {
    int64_t rest = e / gq;
    const int64_t qg = e - rest * gq;
    int64_t off = 4 * qg, stride = nf;
    int64_t delta[NB > 0 ? NB : 1];
    bool act[NB > 0 ? NB : 1];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      delta[j] = 0;
      act[j] = false;
    }
    if (FAST) {
      act[NB - 1] = true;
      delta[NB - 1] = nf - 4 - 8 * qg;
    }
    for (int k = b.d - 2; k >= 0; --k) {
      int jf = -1;
#pragma unroll
      for (int j = 0; j < NSLOW; ++j)
        if (b.ax[j] == k) jf = j;
      const int64_t ext = jf >= 0 ? b.n[k] - b.hh[jf] : b.n[k];
      const int64_t qq = rest / ext;
      const int64_t i = rest - qq * ext;
      rest = qq;
      off += i * stride;
#pragma unroll
      for (int j = 0; j < NSLOW; ++j)
        if (j == jf && i < b.hh[j]) {
          act[j] = true;
          delta[j] = (b.n[k] - 1 - 2 * i) * stride;
        }
      stride *= b.n[k];
    }
    double v[NV][4];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      bool ok = true;
      int64_t o = off;
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (m & (1 << j)) {
          ok = ok && act[j];
          o += delta[j];
        }
      if (ok) {
        const double2 x0 = *(const double2*)(x + o), x1 = *(const double2*)(x + o + 2);
        const double2 p0 = *(const double2*)(p + o), p1 = *(const double2*)(p + o + 2);
        const double2 r0 = *(const double2*)(r + o), r1 = *(const double2*)(r + o + 2);
        const double2 q0 = *(const double2*)(q + o), q1 = *(const double2*)(q + o + 2);
        *(double2*)(x + o) = make_double2(x0.x + alpha * p0.x, x0.y + alpha * p0.y);
        *(double2*)(x + o + 2) = make_double2(x1.x + alpha * p1.x, x1.y + alpha * p1.y);
        v[m][0] = r0.x - alpha * q0.x;
        v[m][1] = r0.y - alpha * q0.y;
        v[m][2] = r1.x - alpha * q1.x;
        v[m][3] = r1.y - alpha * q1.y;
        *(double2*)(r + o) = make_double2(v[m][0], v[m][1]);
        *(double2*)(r + o + 2) = make_double2(v[m][2], v[m][3]);
#pragma unroll
        for (int c = 0; c < 4; ++c) s += v[m][c] * v[m][c];
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[m][c] = 0.0;
      }
    }
    if (FAST) {
      constexpr int fb = FAST ? 1 << (NB - 1) : 0;
#pragma unroll
      for (int m = 0; m < NV; ++m)
        if (!(m & fb)) {
          double t0[4], t1[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            t0[c] = v[m][c] + v[m | fb][3 - c];
            t1[3 - c] = v[m][c] - v[m | fb][3 - c];
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            v[m][c] = t0[c];
            v[m | fb][c] = t1[c];
          }
        }
    }
#pragma unroll
    for (int j = 0; j < NSLOW; ++j) {
      if (!act[j]) continue;
#pragma unroll
      for (int m = 0; m < NV; ++m)
        if (!(m & (1 << j))) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double x0 = v[m][c], x1 = v[m | (1 << j)][c];
            v[m][c] = x0 + x1;
            v[m | (1 << j)][c] = x0 - x1;
          }
        }
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      bool ok = true;
      int64_t o = off;
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (m & (1 << j)) {
          ok = ok && act[j];
          o += delta[j];
        }
      if (ok)
        *(uint2*)(r16 + o) =
            make_uint2((uint32_t)bf16_from_f32((float)v[m][0]) | ((uint32_t)bf16_from_f32((float)v[m][1]) << 16),
                       (uint32_t)bf16_from_f32((float)v[m][2]) | ((uint32_t)bf16_from_f32((float)v[m][3]) << 16));
    }
  }
  double t = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(RT) void k_xpby(const double* z, double* p, int64_t n, const SolverScalars* sc,
                                             const int* skip) {
  if (skip && *skip) return;
  const double beta = sc->beta;
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT)
    p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(RT) void k_axpy1(double* x, const double* y, int64_t n, const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) x[i] += y[i];
}

// y = x / sqrt(sc->aux[0])  (normalisation by a norm^2 reduced on the device)
__global__ __launch_bounds__(RT) void k_scale_invnorm(const double* x, double* y, int64_t n,
                                                      const SolverScalars* sc) {
  const double inv = 1.0 / sqrt(sc->aux[0]);
  for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) y[i] = x[i] * inv;
}

// Reset the scalar block on the device (no host round trip).
__global__ void k_init_scalars(SolverScalars* sc, double tol2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    SolverScalars z{};
    z.tol2 = tol2;
    *sc = z;
  }
}

// Status codes written by the scalar kernel.
enum { ST_RUN = 0, ST_BREAKDOWN = 1, ST_NONFINITE = 2, ST_MAXIT = 3 };

__global__ __launch_bounds__(RT) void k_scalar(int what, SolverScalars* sc, const double* partial,
                                               const double* partial2, int flexible, int maxit) {
  // fixed-order sums of the partials: thread t adds t, t+RT, ...; then the block tree
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += RT) {
    a += partial[i];
    if (partial2) b += partial2[i];
  }
  a = block_sum(a);
  if (partial2) b = block_sum(b);
  if (threadIdx.x != 0) return;
  if (sc->done && what != (int)ScalarStep::SetRR && what != (int)ScalarStep::SetAux0) return;
  switch (what) {
    case (int)ScalarStep::InitRR:
      sc->rr = a;
      sc->ff = b;
      sc->iters = 0;
      sc->status = ST_RUN;
      if (!isfinite(a) || !isfinite(b)) { sc->status = ST_NONFINITE; sc->done = 1; }
      else if (a <= sc->tol2 * b) sc->done = 1;
      break;
    case (int)ScalarStep::InitRZ:
      sc->rz = a;
      if (!isfinite(a)) { sc->status = ST_NONFINITE; sc->done = 1; }
      break;
    case (int)ScalarStep::Alpha:
      sc->pq = a;
      if (!isfinite(a)) { sc->status = ST_NONFINITE; sc->done = 1; }
      else if (!(a > 0.0)) { sc->status = ST_BREAKDOWN; sc->done = 1; }
      else sc->alpha = sc->rz / a;
      break;
    case (int)ScalarStep::RR:
      sc->rr_prev = sc->rr;
      sc->rr = a;
      sc->iters += 1;
      if (!isfinite(a)) { sc->status = ST_NONFINITE; sc->done = 1; }
      else if (a <= sc->tol2 * sc->ff) sc->done = 1;
      else if (sc->iters >= maxit) { sc->status = ST_MAXIT; sc->done = 1; }
      break;
    case (int)ScalarStep::Beta: {
      // standard: beta = <z', r'> / <z, r>;  flexible (Polak-Ribiere):
      // beta = <z', r' - r> / <z, r> = (<z', r'> - <z', r>) / <z, r>, and
      // r' - r = -alpha q, so <z', r' - r> = -alpha <z', q>
      const double rz_new = a;
      double beta = flexible ? (-sc->alpha * b) / sc->rz : rz_new / sc->rz;
      if (!isfinite(beta)) { sc->status = ST_NONFINITE; sc->done = 1; }
      sc->rz_new = rz_new;
      sc->zq = b;
      sc->beta = beta;
      sc->rz = rz_new;
      break;
    }
    case (int)ScalarStep::SetRR:
      sc->rr = a;
      break;
    case (int)ScalarStep::SetAux0:
      sc->aux[0] = a;
      break;
  }
}

inline int red_grid(int64_t n) { (void)n; return kRedBlocks; }

}  // namespace

// Dense operators: d FP64 passes (axis k into tmp0 for k = 0, else tmp1, with
// tmp1 added into tmp0 before the next pass overwrites it), then k_combine.
static hipError_t launch_dense_operator(const StencilArgs& a, hipStream_t st) {
  if (!a.tmp0 || !a.tmp1) return hipErrorOutOfMemory;
  const unsigned g = (unsigned)std::min<int64_t>((a.N + RT - 1) / RT, 1 << 20);
  for (int k = 0; k < a.d; ++k) {
    PassArgs pa;
    pa.X = a.u;
    pa.Y = k == 0 ? a.tmp0 : a.tmp1;
    pa.tin = pa.tout = DT::F64;
    pa.prec = 0;
    pa.fac = a.dense[k];
    pa.forward = true;
    pa.n = a.n[k];
    pa.P = 1;
    pa.R = 1;
    for (int m = 0; m < k; ++m) pa.P *= a.n[m];
    for (int m = k + 1; m < a.d; ++m) pa.R *= a.n[m];
    pa.skip = a.skip;
    pa.kband = a.dense[k]->bw;  // SEM: band half-width k; generic dense operators: 0 (all of K)
    hipError_t e = launch_pass(pa, st);
    if (e != hipSuccess) return e;
    if (k >= 1 && k + 1 < a.d) {
      hipLaunchKernelGGL(k_add_to, dim3(g), dim3(RT), 0, st, a.tmp0, a.tmp1, a.N, a.skip);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  const unsigned gc = a.dot != StDot::None ? kRedBlocks : g;
  const int m = (int)a.mode, dt = (int)a.dot;
#define TS_CB(M, D) \
  if (m == M && dt == D) { hipLaunchKernelGGL((k_combine<M, D>), dim3(gc), dim3(RT), 0, st, a); return hipGetLastError(); }
  TS_CB(0, 0) TS_CB(0, 1) TS_CB(0, 2) TS_CB(1, 0) TS_CB(1, 1) TS_CB(1, 2)
#undef TS_CB
  return hipErrorInvalidValue;
}

hipError_t launch_stencil(const StencilArgs& a, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  if (a.z && (a.dense[0] || a.bw > 0 || !a.bsc || !a.unew || a.unew == a.u)) return hipErrorInvalidValue;
  if (a.dense[0]) return launch_dense_operator(a, st);
  if (a.bw > 0) {
    const unsigned g = a.dot != StDot::None ? kRedBlocks
                                            : (unsigned)std::min<int64_t>((a.N + RT - 1) / RT, 1 << 20);
    const int m = (int)a.mode, dt = (int)a.dot;
#define TS_BD(M, D) \
  if (m == M && dt == D) { hipLaunchKernelGGL((k_band<M, D>), dim3(g), dim3(RT), 0, st, a); return hipGetLastError(); }
    TS_BD(0, 0) TS_BD(0, 1) TS_BD(0, 2) TS_BD(1, 0) TS_BD(1, 1) TS_BD(1, 2)
#undef TS_BD
    return hipErrorInvalidValue;
  }
  const int64_t NX = a.n[a.d - 1], NY = a.d >= 2 ? a.n[a.d - 2] : 1;
  const int64_t P = a.N / (NX * NY);
  const int64_t txt = (NX + kTX - 1) / kTX, tyt = (NY + kTY - 1) / kTY;
  // planes per task: long marches (fewer halo and first-plane loads), but at
  // least ~2048 tasks when the grid allows
  const int64_t planes = std::max<int64_t>(1, std::min<int64_t>(32, P * txt * tyt / 2048));
  const int64_t pt = (P + planes - 1) / planes;
  const int64_t ntask = txt * tyt * pt;
  unsigned grid;
  if (a.dot != StDot::None) grid = kRedBlocks;  // one partial per block, every slot written
  else grid = (unsigned)std::min<int64_t>(ntask, 1 << 20);
  const int m = (int)a.mode, dt = (int)a.dot;
#define TS_ST(M, D) \
  if (m == M && dt == D) {                                                                            \
    hipLaunchKernelGGL((k_stencil<M, D>), dim3(grid), dim3(RT), 0, st, a, txt, tyt, pt, planes);       \
    return hipGetLastError();                                                                         \
  }
  TS_ST(0, 0) TS_ST(0, 1) TS_ST(0, 2) TS_ST(1, 0) TS_ST(1, 1) TS_ST(1, 2)
#undef TS_ST
  return hipErrorInvalidValue;
}

hipError_t launch_axis_scale(const double* x, double* y, int d, const int64_t* n, const double* const* w,
                             hipStream_t st) {
  ScaleArgs a;
  a.d = d;
  int64_t N = 1;
  for (int k = 0; k < d; ++k) {
    a.n[k] = n[k];
    a.w[k] = w[k];
    N *= n[k];
  }
  if (N <= 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>((N + RT - 1) / RT, 1 << 20);
  hipLaunchKernelGGL(k_axis_scale, dim3(g), dim3(RT), 0, st, x, y, N, a);
  return hipGetLastError();
}

hipError_t launch_dot(const double* x, const double* y, int64_t n, double* partial, const double* w,
                      double* partial2, const int* skip, hipStream_t st) {
  hipLaunchKernelGGL(k_dot, dim3(red_grid(n)), dim3(RT), 0, st, x, y, n, partial, w, partial2, skip);
  return hipGetLastError();
}

hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, int64_t n,
                            const SolverScalars* sc, double* partial, const int* skip, hipStream_t st,
                            uint16_t* r16) {
  hipLaunchKernelGGL(k_cg_update, dim3(red_grid(n)), dim3(RT), 0, st, x, r, p, q, n, sc, partial, skip, r16);
  return hipGetLastError();
}

bool cg_update_fold_ok(const ButterflyArgs& b, const double* x, const double* r, const double* p, const double* q,
                       const uint16_t* r16) {
  const uintptr_t al = ((uintptr_t)x | (uintptr_t)r | (uintptr_t)p | (uintptr_t)q) & 15;
  if (b.nax < 1 || b.nax > 4 || b.ncomp != 1 || b.n[b.d - 1] % 8 != 0 || al != 0 || (((uintptr_t)r16) & 7) != 0)
    return false;
  int nslow = 0;
  for (int j = 0; j < b.nax; ++j)
    if (b.ax[j] != b.d - 1) ++nslow;
  return nslow <= 3;
}

hipError_t launch_cg_update_fold(double* x, double* r, const double* p, const double* q, const ButterflyArgs& a,
                                 const SolverScalars* sc, double* partial, const int* skip, uint16_t* r16,
                                 hipStream_t st) {
  if (!cg_update_fold_ok(a, x, r, p, q, r16)) return hipErrorInvalidValue;
  ButterflyArgs b = a;  // the slow axes in slots 0 .. nslow - 1 (order kept)
  int nslow = 0;
  bool fast = false;
  for (int j = 0; j < a.nax; ++j) {
    if (a.ax[j] == a.d - 1) {
      fast = true;
      continue;
    }
    b.ax[nslow] = a.ax[j];
    b.hh[nslow] = a.hh[j];
    ++nslow;
  }
  int64_t units = 1;
  for (int k = 0; k < a.d - 1; ++k) {
    int64_t ext = a.n[k];
    for (int j = 0; j < nslow; ++j)
      if (b.ax[j] == k) ext = a.n[k] - b.hh[j];
    units *= ext;
  }
  units *= (fast ? a.n[a.d - 1] / 2 : a.n[a.d - 1]) / 4;
  const dim3 grid(red_grid(units)), block(RT);
#define TS_UPD_FOLD(NS)                                                                                        \
  if (fast)                                                                                                  \
    hipLaunchKernelGGL((k_cg_update_fold<NS, true>), grid, block, 0, st, x, r, p, q, b, units, sc, partial, skip, \
                       r16);                                                                                 \
  else                                                                                                       \
    hipLaunchKernelGGL((k_cg_update_fold<NS, false>), grid, block, 0, st, x, r, p, q, b, units, sc, partial,     \
                       skip, r16);
  switch (nslow) {
    case 0:
      hipLaunchKernelGGL((k_cg_update_fold<0, true>), grid, block, 0, st, x, r, p, q, b, units, sc, partial, skip,
                         r16);
      break;
    case 1: TS_UPD_FOLD(1) break;
    case 2: TS_UPD_FOLD(2) break;
    case 3: TS_UPD_FOLD(3) break;
    default: return hipErrorInvalidValue;
  }
#undef TS_UPD_FOLD
  return hipGetLastError();
}

hipError_t launch_xpby(const double* z, double* p, int64_t n, const SolverScalars* sc, const int* skip,
                       hipStream_t st) {
  unsigned grid = (unsigned)std::min<int64_t>((n + RT - 1) / RT, 4096);
  hipLaunchKernelGGL(k_xpby, dim3(grid), dim3(RT), 0, st, z, p, n, sc, skip);
  return hipGetLastError();
}

hipError_t launch_axpy1(double* x, const double* y, int64_t n, const int* skip, hipStream_t st) {
  unsigned grid = (unsigned)std::min<int64_t>((n + RT - 1) / RT, 4096);
  hipLaunchKernelGGL(k_axpy1, dim3(grid), dim3(RT), 0, st, x, y, n, skip);
  return hipGetLastError();
}

hipError_t launch_scale_invnorm(const double* x, double* y, int64_t n, const SolverScalars* sc, hipStream_t st) {
  unsigned grid = (unsigned)std::min<int64_t>((n + RT - 1) / RT, 4096);
  hipLaunchKernelGGL(k_scale_invnorm, dim3(grid), dim3(RT), 0, st, x, y, n, sc);
  return hipGetLastError();
}

hipError_t launch_init_scalars(SolverScalars* sc, double tol2, hipStream_t st) {
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, st, sc, tol2);
  return hipGetLastError();
}

hipError_t launch_scalar(ScalarStep what, SolverScalars* sc, const double* partial, const double* partial2,
                         int flexible, int maxit, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(RT), 0, st, (int)what, sc, partial, partial2, flexible, maxit);
  return hipGetLastError();
}

}  // namespace ts
