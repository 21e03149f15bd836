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
#include <algorithm>

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

// Visits the items k = t, t + GT, t + 2 GT, ... of a tile of rows x per_row
// items without dividing: row and column advance by fixed steps with a carry,
// and the global offset of the item follows them.
struct Walk {
  int row, col, dr, dc, per_row;
  int64_t goff, dgoff, carry;
  __device__ __forceinline__ Walk(int t, int per_row_, int64_t gbase, int64_t R, int width) {
    per_row = per_row_;
    row = t / per_row;
    col = t - row * per_row;
    dr = GT / per_row;
    dc = GT - dr * per_row;
    goff = gbase + (int64_t)row * R + (int64_t)col * width;
    dgoff = (int64_t)dr * R + (int64_t)dc * width;
    carry = R - (int64_t)per_row * width;
  }
  __device__ __forceinline__ void next() {
    col += dc;
    row += dr;
    goff += dgoff;
    if (col >= per_row) {
      col -= per_row;
      ++row;
      goff += carry;
    }
  }
};

// Multiplies the live complex values of this thread's chunks of the tile by
// e^{-i th V2} (the potential factor of the splitting schemes).
template <typename TIO, typename TC, int VW>
__device__ __forceinline__ void phase_chunks(TC* tile, const TIO* V2, double th, Walk w, int nchunks,
                                             int live_rows, int live) {
  for (int k = threadIdx.x; k < nchunks; k += GT) {
    if (w.row < live_rows && w.col * VW < live) {
#pragma unroll
      for (int m = 0; m < VW; m += 2) {
        TC sn, cs;
        sincos_t<TC>((TC)(-th) * (TC)V2[(w.goff + m) >> 1], &sn, &cs);
        TC* x = tile + k * VW + m;
        const TC re = x[0], im = x[1];
        x[0] = cs * re - sn * im;
        x[1] = sn * re + cs * im;
      }
    }
    w.next();
  }
}

// Output row carried by A row `row` of a 16-row MFMA block, chosen so that
// accumulator register r of lane group g holds output g + 4 r: the FP64
// MFMA already lays its output out that way; the FP32 one holds 4 g + r, so
// its A rows are permuted by (row / 4) + 4 (row % 4).
template <typename TC> __device__ __forceinline__ int rowperm(int row);
template <> __device__ __forceinline__ int rowperm<double>(int row) { return row; }
template <> __device__ __forceinline__ int rowperm<float>(int row) { return (row >> 2) + 4 * (row & 3); }

// Whether a pass stages each step's factor in LDS (FP32 compute) or reads the
// fragments from memory (FP64 compute).
template <typename TC> constexpr bool kFacLds = sizeof(TC) == 4;

// One axis step of a grouped pass over the tile seen as [B][n][W]: the batched
// product Y_b = F^T X_b over its B x W columns, 16 columns per MFMA chunk.
// A = F^T (M = output row, K = input row; fragments af from the zero-padded
// factor), B = 4 input rows x 16 columns read from LDS, KT steps of 4 rows;
// the accumulators go back in place (a chunk's columns belong to one wave,
// which reads all their rows first).  Column c lies in batch b = c / W, found
// as the high half of c times the host's ceil(2^32 / W) (wmul; 0 when W = 1).
template <int KT, int MT, typename TC>
__device__ __forceinline__ void group_step(TC* tile_generic, const TC (&af)[MT][8], int n, int W, uint32_t wmul,
                                           int ncols, int wave, int lane, int elems) {
  // LDS-typed pointer: 32-bit offsets, no flat-address arithmetic
  typedef __attribute__((address_space(3))) TC lds_t;
  lds_t* tile = (lds_t*)tile_generic;
  const int lr = lane & 15, lk = lane >> 4;
  const int skip_b = (n - 1) * W;
  const int discard = elems + lane;
  for (int c0 = wave * 16; c0 < ncols; c0 += (GT / 64) * 16) {
    const int c = c0 + lr;
    const bool cok = c < ncols;
    const int b = wmul ? (int)__umulhi((unsigned)c, wmul) : c;
    const int base = cok ? c + b * skip_b : 0;
    // every lane reads (element 0 when its row or column lies outside), then masks
    TC x[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int i = k * 4 + lk;
      const bool ok = cok && i < n;
      const TC v = tile[ok ? base + i * W : 0];
      x[k] = ok ? v : (TC)0;
    }
    typename AccT<TC>::V acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < KT; ++k)
#pragma unroll
      for (int m = 0; m < MT; ++m) acc[m] = mfma(af[m][k], x[k], acc[m]);
    // outputs outside the tile (rows j >= n, columns past the end) go to a
    // per-lane discard slot behind the tile, so every lane stores
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = m * 16 + lk + 4 * r;
        tile[(cok && j < n) ? base + j * W : discard] = acc[m][r];
      }
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
  const int live_rows = pb * G;
  const int nchunks = elems / VW;
  TC* fac = tile + elems + 64;  // the current step's factor, n x n, behind the discard slots
  const int64_t gbase = p0 * (int64_t)G * a.R + r0;
  const TIO* Xin = (const TIO*)a.Xin;
  TIO* Xout = (TIO*)a.Xout;
  const TIO* V2 = (const TIO*)a.V2;

  // Geometry of the load and the store: chunk k is values [k VW, k VW + VW)
  // of the tile in LDS.  A tile of the fastest group (RT = R) is one
  // contiguous run of global memory, seen as a single row; otherwise row r of
  // the tile [PB][G][RT] starts at global offset gbase + r R.
  const bool flat = a.flat;
  const int io_per_row = flat ? nchunks : RT / VW;
  const int io_live_rows = flat ? 1 : live_rows;
  const int io_live = flat ? live_rows * RT : rt;  // live values per io row

  // ---- load (then multiplied by e^{-i th_pre V2} if asked); padding rows/columns are zero ----
  // kLoadBatch chunks per thread are requested before any is used, so their
  // memory latencies overlap instead of adding up
  constexpr int kLoadBatch = 8;
  {
    const Walk w_first(t, io_per_row, gbase, a.R, VW);
    Walk w = w_first;
    for (int k0 = t; k0 < nchunks; k0 += GT * kLoadBatch) {
      TIO v[kLoadBatch][VW];
      bool ok[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        // chunks outside the live data read the first chunk instead (then zeroed): no branch
        ok[u] = k0 + u * GT < nchunks && w.row < io_live_rows && w.col * VW < io_live;
        vload<TIO, VW, VEC>(Xin + (ok[u] ? w.goff : 0), v[u]);
        w.next();
      }
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        const int k = k0 + u * GT;
        if (k >= nchunks) break;
#pragma unroll
        for (int m = 0; m < VW; ++m) tile[k * VW + m] = ok[u] ? (TC)v[u][m] : (TC)0;
      }
    }
    // each thread rotates the chunks it loaded itself: no barrier needed
    if (CPLX && a.pre) phase_chunks<TIO, TC, VW>(tile, V2, a.th_pre, w_first, nchunks, io_live_rows, io_live);
  }
  __syncthreads();

  for (int s = 0; s < a.nsteps; ++s) {
    const GroupStep S = a.step[s];
    const int n = S.n;
    // this axis's step: the tile seen as [B][n][W], W = stride x RT values per row
    const int W = S.stride * RT;
    const int ncols = elems / n;
    const int kt = (n + 3) >> 2;
    const TC* F = (const TC*)S.Q;
    // A row lr of output block m is output m 16 + rowperm<TC>(lr): then lane
    // group lk holds outputs m 16 + lk + 4 r in both precisions, and the
    // stores of one accumulator register hit 4 consecutive rows, as the reads do.
    // FP32: the n x n factor goes to LDS once per block (a few loads per block
    // instead of 8 MT scattered loads per lane, which kept the vector memory
    // return path busy); FP64 reads the fragments from memory, because the LDS
    // copy would cost a block per CU on the common tiles.
    TC af[MT][8];
    if constexpr (kFacLds<TC>) {
      for (int e = t; e < n * n; e += GT) {
        const int i = e / n;
        fac[e] = F[(int64_t)i * S.ld + (e - i * n)];
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = k * 4 + lk, j = m * 16 + rowperm<TC>(lr);
          const bool ok = k < kt && i < n && j < n;
          const TC v = fac[ok ? i * n + j : 0];
          af[m][k] = ok ? v : (TC)0;
        }
    } else {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int k = 0; k < 8; ++k)
          af[m][k] = k < kt ? F[(int64_t)(k * 4 + lk) * S.ld + m * 16 + rowperm<TC>(lr)] : (TC)0;
    }
    // the number of 4-row k-steps is uniform over the block: one branch-free
    // instance per count, so every LDS read of a chunk is issued before its MFMAs
    switch (kt) {
      case 1: group_step<1, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
      case 2: group_step<2, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
      case 3: group_step<3, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
      case 4: group_step<4, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
      case 5: if constexpr (MT == 2) group_step<5, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
      case 6: if constexpr (MT == 2) group_step<6, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
      case 7: if constexpr (MT == 2) group_step<7, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
      default: if constexpr (MT == 2) group_step<8, MT>(tile, af, n, W, S.wmul, ncols, wave, lane, elems); break;
    }
    __syncthreads();
    if (s == a.scale_after) {
      // diagonal of the slowest group's pass: value (g, q) of the tile, with
      // q the index of the value (or complex value) r0 + col in the faster axes
      constexpr int SC = CPLX ? 2 : 1;
      const int per_row = RT / SC;
      Walk w(t, per_row, 0, 0, 0);
      const int drg = w.dr % G;
      int g = w.row % G;
      // with a fixed column per thread (dc = 0) the faster axes' factor is read once
      double2 f2c = make_double2(0.0, 0.0);
      double lrc = 0.0;
      if (w.dc == 0 && w.col * SC < rt) {
        if (CPLX) f2c = a.Er[r0 / SC + w.col];
        else lrc = a.Lr[r0 + w.col];
      }
      for (int e = t; e < elems / SC; e += GT) {
        if (w.col * SC < rt) {
          TC* x = tile + e * SC;
          const int64_t q = r0 / SC + w.col;
          if (CPLX) {
            const double2 f1 = a.Eg[g], f2 = w.dc == 0 ? f2c : a.Er[q];
            const double fr = f1.x * f2.x - f1.y * f2.y, fi = f1.x * f2.y + f1.y * f2.x;
            const double re = x[0], im = x[1];
            x[0] = (TC)(fr * re - fi * im);
            x[1] = (TC)(fi * re + fr * im);
          } else {
            x[0] = (TC)((double)x[0] / (a.Lg[g] + (w.dc == 0 ? lrc : a.Lr[q]) + a.shift));
          }
        }
        const int row0 = w.row;
        w.next();
        g += drg + (w.row - row0 - w.dr);
        if (g >= G) g -= G;
      }
      __syncthreads();
    }
  }

  // ---- store (multiplied by e^{-i th_post V2} first if asked) ----
  {
    const Walk w_first(t, io_per_row, gbase, a.R, VW);
    // each thread rotates the chunks it stores itself: no barrier needed
    if (CPLX && a.post) phase_chunks<TIO, TC, VW>(tile, V2, a.th_post, w_first, nchunks, io_live_rows, io_live);
    Walk w = w_first;
    for (int k = t; k < nchunks; k += GT) {
      if (w.row < io_live_rows && w.col * VW < io_live) {
        TIO v[VW];
#pragma unroll
        for (int m = 0; m < VW; ++m) v[m] = (TIO)tile[k * VW + m];
        vstore<TIO, VW, VEC>(Xout + w.goff, v);
      }
      w.next();
    }
  }
}

template <typename TIO, typename TC, bool CPLX, int VW, bool VEC>
hipError_t launch_vw(const GroupArgs& a, int nmax, hipStream_t st) {
  // the tile, 64 discard slots and (FP32) the largest n x n factor of the pass
  int nf = 0;
  for (int s = 0; s < a.nsteps; ++s) nf = std::max(nf, a.step[s].n);
  const size_t lds = sizeof(TC) * ((size_t)a.tile_elems + 64 + (kFacLds<TC> ? (size_t)nf * nf : 0));
  dim3 grid((unsigned)a.nblocks), block(GT);
  if (nmax <= 16) hipLaunchKernelGGL((k_group<TIO, TC, 1, CPLX, VW, VEC>), grid, block, lds, st, a);
  else if (nmax <= 32) hipLaunchKernelGGL((k_group<TIO, TC, 2, CPLX, VW, VEC>), grid, block, lds, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// 16-byte chunks when every chunk starts 16-byte aligned and the live part of
// every tile holds whole chunks, else single values (pairs for complex data).
// A tile of the fastest group (RT = R) is moved as one contiguous run.
template <typename TIO, typename TC, bool CPLX>
hipError_t launch_nmax(GroupArgs a, int nmax, hipStream_t st) {
  constexpr int V = 16 / (int)sizeof(TIO);
  const bool aligned = ((uintptr_t)a.Xin & 15) == 0 && ((uintptr_t)a.Xout & 15) == 0;
  a.flat = a.RT == a.R;
  const bool vec = aligned && (a.flat ? ((int64_t)a.G * a.R) % V == 0 : a.R % V == 0 && a.RT % V == 0);
  if (a.nsteps > 8 || a.tile_elems <= 0) return hipErrorInvalidValue;
  for (int s = 0; s < a.nsteps; ++s) {
    // b = c / W as the high half of c * ceil(2^32 / W): exact while c (W - 1) < 2^32
    const int64_t W = (int64_t)a.step[s].stride * a.RT;
    if (W <= 0 || (int64_t)a.tile_elems * W >= (1LL << 32)) return hipErrorInvalidValue;
    a.step[s].wmul = W == 1 ? 0u : (uint32_t)(((1ULL << 32) + (uint64_t)W - 1) / (uint64_t)W);
  }
  return vec ? launch_vw<TIO, TC, CPLX, V, true>(a, nmax, st) : launch_vw<TIO, TC, CPLX, CPLX ? 2 : 1, false>(a, nmax, st);
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
