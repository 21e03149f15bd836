// Small-extent mode products (n_k <= 32 on every axis: the 6D / 9D grids of
// the splitting workloads and small serving requests), HBM-bound.
//
// Consecutive axes are grouped so that a tile [PB][G][RT] of the tensor
// viewed as [P][G][R] (G = product of the group's extents, R = faster
// extents x components) fits in LDS.  One pass loads a tile, applies the
// group's mode products one axis after the other inside LDS (one fibre per
// thread in registers, the n x n factor staged in LDS and read as a broadcast),
// and stores the tile back to the same place (passes run in place).  The
// slowest group's pass also carries the diagonal scaling between its forward
// and backward products (paper Sec. 2.1 steps 2-4, eq. (exact_prop)), so an
// apply with g groups makes 2g - 1 round trips through HBM instead of 2d.
// The pointwise potential factor e^{-i theta V2} of the splitting schemes
// (Sec. 5.1) can be fused into the first load and the last store.
#include "modeprod_common.h"
#include "ts_internal.h"
#include "ts_small.h"

namespace ts {
namespace {

using namespace mp;

constexpr int GT = 256;  // threads per block

template <typename T> __device__ __forceinline__ void sincos_t(T x, T* s, T* c);
template <> __device__ __forceinline__ void sincos_t<double>(double x, double* s, double* c) { sincos(x, s, c); }
template <> __device__ __forceinline__ void sincos_t<float>(float x, float* s, float* c) { sincosf(x, s, c); }

// VW consecutive values of one tile row move together: one 16-byte access
// when the rows allow it (VEC), else VW single accesses (VW = 2 keeps the two
// parts of a complex value together).  Row r of the tile [PB][G][RT] starts at
// global offset (p0 G + r) R + r0.
template <typename TIO> struct Vec16;
template <> struct Vec16<double> { using V = double2; };
template <> struct Vec16<float> { using V = float4; };

template <typename TIO, int VW, bool VEC>
__device__ __forceinline__ void vload(const TIO* p, TIO (&v)[VW]) {
  if constexpr (VEC) {
    static_assert(VW * sizeof(TIO) == 16, "16-byte chunks");
    const typename Vec16<TIO>::V w = *(const typename Vec16<TIO>::V*)p;
    const TIO* e = (const TIO*)&w;
#pragma unroll
    for (int m = 0; m < VW; ++m) v[m] = e[m];
  } else {
#pragma unroll
    for (int m = 0; m < VW; ++m) v[m] = p[m];
  }
}
template <typename TIO, int VW, bool VEC>
__device__ __forceinline__ void vstore(TIO* p, const TIO (&v)[VW]) {
  if constexpr (VEC) {
    typename Vec16<TIO>::V w;
    TIO* e = (TIO*)&w;
#pragma unroll
    for (int m = 0; m < VW; ++m) e[m] = v[m];
    *(typename Vec16<TIO>::V*)p = w;
  } else {
#pragma unroll
    for (int m = 0; m < VW; ++m) p[m] = v[m];
  }
}

template <typename TIO, typename TC, int MT, bool CPLX, int VW, bool VEC>
__global__ __launch_bounds__(GT) void k_group(GroupArgs a) {
  if (a.skip && *a.skip) return;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  TC* tile = (TC*)smem;

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t lb = xcd_logical_block(blockIdx.x, a.nblocks);
  const int64_t ptile = lb / a.rtiles, rtile = lb % a.rtiles;
  const int64_t p0 = ptile * a.PB, r0 = rtile * a.RT;
  const int pb = (int)(a.P - p0 < a.PB ? a.P - p0 : a.PB);
  const int rt = (int)(a.R - r0 < a.RT ? a.R - r0 : a.RT);
  const int G = a.G, RT = a.RT;
  const int elems = a.PB * G * RT;
  const int rows = a.PB * G, live_rows = pb * G;
  const int cpr = RT / VW, cpr_sh = a.cpr_shift;  // chunks of VW values per row (shift if a power of 2)
  const int nchunks = rows * cpr;
  const int64_t gbase = p0 * (int64_t)G * a.R + r0;
  const TIO* Xin = (const TIO*)a.Xin;
  TIO* Xout = (TIO*)a.Xout;
  const TIO* V2 = (const TIO*)a.V2;

  // ---- load (optionally multiplied by e^{-i th_pre V2}); padding rows/columns are zero ----
  for (int k = t; k < nchunks; k += GT) {
    const int row = cpr_sh >= 0 ? (k >> cpr_sh) : k / cpr;
    const int rl = (k - row * cpr) * VW;
    TIO v[VW];
    const bool ok = row < live_rows && rl < rt;
    const int64_t gi = gbase + (int64_t)row * a.R + rl;
    if (ok) vload<TIO, VW, VEC>(Xin + gi, v);
    TC c[VW];
#pragma unroll
    for (int m = 0; m < VW; ++m) c[m] = ok ? (TC)v[m] : (TC)0;
    if (CPLX && a.pre && ok) {
#pragma unroll
      for (int m = 0; m < VW; m += 2) {
        TC sn, cs;
        sincos_t<TC>((TC)(-a.th_pre) * (TC)V2[(gi + m) >> 1], &sn, &cs);
        const TC re = c[m], im = c[m + 1];
        c[m] = cs * re - sn * im;
        c[m + 1] = sn * re + cs * im;
      }
    }
#pragma unroll
    for (int m = 0; m < VW; ++m) tile[row * RT + rl + m] = c[m];
  }
  __syncthreads();

  for (int s = 0; s < a.nsteps; ++s) {
    const GroupStep S = a.step[s];
    const int n = S.n;
    // The tile is [B][n][W] along this axis (W = stride x RT contiguous values
    // per row); the step is the batched product Y_b = F^T X_b over the B x W
    // columns, 16 columns per MFMA chunk: A = F^T (M = output row, K = input
    // row, from the zero-padded factor in registers), B = 4 input rows x 16
    // columns read from LDS, accumulators written back in place (a chunk's
    // columns belong to one wave, which reads all their rows first).
    const int W = S.stride * RT;
    const int ncols = elems / n;
    const int kt = (n + 3) >> 2;
    const TC* F = (const TC*)S.Q;
    TC af[MT][8];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int k = 0; k < 8; ++k)
        af[m][k] = k < kt ? F[(int64_t)(k * 4 + lk) * S.ld + m * 16 + lr] : (TC)0;
    for (int c0 = wave * 16; c0 < ncols; c0 += (GT / 64) * 16) {
      const int c = c0 + lr;
      const bool cok = c < ncols;
      const int b = c / W;
      const int base = b * n * W + (c - b * W);
      typename AccT<TC>::V acc[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = {0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k < kt) {
          const int i = k * 4 + lk;
          const TC x = (cok && i < n) ? tile[base + i * W] : (TC)0;
#pragma unroll
          for (int m = 0; m < MT; ++m) acc[m] = mfma(af[m][k], x, acc[m]);
        }
      }
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = m * 16 + out_row<TC>(lane, r);
          if (cok && j < n) tile[base + j * W] = acc[m][r];
        }
    }
    __syncthreads();
    if (s == a.scale_after) {
      // diagonal of the slowest group's pass: element (g, q) with q = (r0 + rl) / ncomp
      for (int k = t; k < nchunks; k += GT) {
        const int row = cpr_sh >= 0 ? (k >> cpr_sh) : k / cpr;
        const int rl = (k - row * cpr) * VW;
        if (rl >= rt) continue;
        const int g = row % G;
        TC* e = tile + row * RT + rl;
        if (CPLX) {
          const double2 f1 = a.Eg[g];
#pragma unroll
          for (int m = 0; m < VW; m += 2) {
            const double2 f2 = a.Er[(r0 + rl + m) >> 1];
            const double fr = f1.x * f2.x - f1.y * f2.y, fi = f1.x * f2.y + f1.y * f2.x;
            const double re = e[m], im = e[m + 1];
            e[m] = (TC)(fr * re - fi * im);
            e[m + 1] = (TC)(fi * re + fr * im);
          }
        } else {
          const double lg = a.Lg[g];
#pragma unroll
          for (int m = 0; m < VW; ++m) e[m] = (TC)((double)e[m] / (lg + a.Lr[r0 + rl + m] + a.shift));
        }
      }
      __syncthreads();
    }
  }

  // ---- store (optionally multiplied by e^{-i th_post V2}) ----
  for (int k = t; k < nchunks; k += GT) {
    const int row = cpr_sh >= 0 ? (k >> cpr_sh) : k / cpr;
    const int rl = (k - row * cpr) * VW;
    if (row >= live_rows || rl >= rt) continue;
    const int64_t gi = gbase + (int64_t)row * a.R + rl;
    TC c[VW];
#pragma unroll
    for (int m = 0; m < VW; ++m) c[m] = tile[row * RT + rl + m];
    if (CPLX && a.post) {
#pragma unroll
      for (int m = 0; m < VW; m += 2) {
        TC sn, cs;
        sincos_t<TC>((TC)(-a.th_post) * (TC)V2[(gi + m) >> 1], &sn, &cs);
        const TC re = c[m], im = c[m + 1];
        c[m] = cs * re - sn * im;
        c[m + 1] = sn * re + cs * im;
      }
    }
    TIO v[VW];
#pragma unroll
    for (int m = 0; m < VW; ++m) v[m] = (TIO)c[m];
    vstore<TIO, VW, VEC>(Xout + gi, v);
  }
}

template <typename TIO, typename TC, bool CPLX, int VW, bool VEC>
hipError_t launch_vw(const GroupArgs& a, int nmax, hipStream_t st) {
  const size_t lds = sizeof(TC) * (size_t)a.tile_elems;
  dim3 grid((unsigned)a.nblocks), block(GT);
  if (nmax <= 16) hipLaunchKernelGGL((k_group<TIO, TC, 1, CPLX, VW, VEC>), grid, block, lds, st, a);
  else if (nmax <= 32) hipLaunchKernelGGL((k_group<TIO, TC, 2, CPLX, VW, VEC>), grid, block, lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// 16-byte chunks when every tile row starts 16-byte aligned and holds whole
// chunks (R, RT multiples of the vector width, aligned buffers), else single
// values (pairs for complex data).
template <typename TIO, typename TC, bool CPLX>
hipError_t launch_nmax(GroupArgs a, int nmax, hipStream_t st) {
  constexpr int V = 16 / (int)sizeof(TIO);
  constexpr int S = CPLX ? 2 : 1;
  const bool vec = a.R % V == 0 && a.RT % V == 0 && ((uintptr_t)a.Xin & 15) == 0 && ((uintptr_t)a.Xout & 15) == 0;
  const int cpr = a.RT / (vec ? V : S);
  a.cpr_shift = (cpr & (cpr - 1)) == 0 ? __builtin_ctz((unsigned)cpr) : -1;
  return vec ? launch_vw<TIO, TC, CPLX, V, true>(a, nmax, st) : launch_vw<TIO, TC, CPLX, S, false>(a, nmax, st);
}

}  // namespace

int small_nmax(int64_t n) {
  if (n <= 8) return 8;
  if (n <= 16) return 16;
  if (n <= 24) return 24;
  if (n <= 32) return 32;
  return 0;
}

hipError_t launch_group(const GroupArgs& a, DT tio, bool fp64_compute, bool cplx, int nmax, hipStream_t st) {
  if (a.nblocks <= 0) return hipSuccess;
  if (a.nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (tio == DT::F64 && fp64_compute)
    return cplx ? launch_nmax<double, double, true>(a, nmax, st) : launch_nmax<double, double, false>(a, nmax, st);
  if (tio == DT::F64 && !fp64_compute)
    return cplx ? launch_nmax<double, float, true>(a, nmax, st) : launch_nmax<double, float, false>(a, nmax, st);
  if (tio == DT::F32 && !fp64_compute)
    return cplx ? launch_nmax<float, float, true>(a, nmax, st) : launch_nmax<float, float, false>(a, nmax, st);
  if (tio == DT::F32 && fp64_compute)
    return cplx ? launch_nmax<float, double, true>(a, nmax, st) : launch_nmax<float, double, false>(a, nmax, st);
  return hipErrorInvalidValue;
}

// ---- pointwise e^{-i theta V2} on interleaved complex data (generic path) ----
template <typename T>
__global__ __launch_bounds__(256) void k_phase(T* psi, const T* V2, double theta, int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    T sn, cs;
    sincos_t<T>((T)(-theta) * V2[i], &sn, &cs);
    const T re = psi[2 * i], im = psi[2 * i + 1];
    psi[2 * i] = cs * re - sn * im;
    psi[2 * i + 1] = sn * re + cs * im;
  }
}

hipError_t launch_phase(void* psi, const void* V2, double theta, int64_t N, bool fp64, hipStream_t st) {
  const unsigned grid = (unsigned)std::min<int64_t>((N + 255) / 256, 8192);
  if (grid == 0) return hipSuccess;
  if (fp64) hipLaunchKernelGGL(k_phase<double>, dim3(grid), dim3(256), 0, st, (double*)psi, (const double*)V2, theta, N);
  else hipLaunchKernelGGL(k_phase<float>, dim3(grid), dim3(256), 0, st, (float*)psi, (const float*)V2, theta, N);
  return hipGetLastError();
}

// ---- FP64 tables over two axis ranges [0, split) and [split, d) ----
// mode 0: sums of eigenvalues (Lg, Lr); mode 1: products of e^{-i tau lam} (Eg, Er).
__global__ void k_range_tables(RangeTableArgs a) {
  const int64_t total = a.n_lo + a.n_hi;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const bool lo = e < a.n_lo;
    int64_t idx = lo ? e : e - a.n_lo;
    const int kb = lo ? 0 : a.split, ke = lo ? a.split : a.d;
    double sum = 0.0, re = 1.0, im = 0.0;
    for (int k = ke - 1; k >= kb; --k) {
      const int64_t j = idx % a.n[k];
      idx /= a.n[k];
      const double l = a.lam[k][j];
      if (a.mode == 0) {
        sum += l;
      } else {
        double sn, cs;
        sincos(a.tau * l, &sn, &cs);
        const double nr = re * cs + im * sn, ni = im * cs - re * sn;  // times (cs - i sn)
        re = nr;
        im = ni;
      }
    }
    if (a.mode == 0) (lo ? a.L_lo : a.L_hi)[lo ? e : e - a.n_lo] = sum;
    else (lo ? a.E_lo : a.E_hi)[lo ? e : e - a.n_lo] = make_double2(re, im);
  }
}

hipError_t launch_range_tables(const RangeTableArgs& a, hipStream_t st) {
  const int64_t total = a.n_lo + a.n_hi;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_range_tables, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace ts
