// Device helpers shared by the FP64/FP32 and BF16 mode-product kernels.
#pragma once

#include "bf16_round.h"
#include "ts_internal.h"

namespace ts {
namespace mp {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct AccT;
template <> struct AccT<double> { using V = d4; };
template <> struct AccT<float> { using V = f4; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row (within a 16x16 output block) of accumulator element r held by lane l.
// Measured on gfx950: the FP64 form interleaves rows across lane groups.
template <typename T> __device__ __forceinline__ int out_row(int l, int r);
template <> __device__ __forceinline__ int out_row<double>(int l, int r) { return (l >> 4) + 4 * r; }
template <> __device__ __forceinline__ int out_row<float>(int l, int r) { return 4 * (l >> 4) + r; }

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits for every outstanding global load, which would cut short a register
// prefetch of the next tile issued before it; with this barrier such loads
// stay in flight (the compiler still waits for them before their registers
// are used).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- element conversions ----
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return bf16_from_f32(f); }  // nearest even

template <typename TIn, typename TC> __device__ __forceinline__ TC cvt_in(TIn x);
template <> __device__ __forceinline__ double cvt_in<double, double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt_in<double, float>(double x) { return (float)x; }
template <> __device__ __forceinline__ float cvt_in<float, float>(float x) { return x; }
template <> __device__ __forceinline__ double cvt_in<float, double>(float x) { return (double)x; }
template <> __device__ __forceinline__ float cvt_in<uint16_t, float>(uint16_t x) { return bf16_to_f32(x); }

template <typename TOut> __device__ __forceinline__ TOut cvt_out(double x);
template <> __device__ __forceinline__ double cvt_out<double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt_out<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ uint16_t cvt_out<uint16_t>(double x) { return f32_to_bf16((float)x); }

struct KArgs {
  const void* X;
  void* Y;
  const void* S;      // resident factor, [kpad][ld], k-major
  int64_t ld;
  int64_t P, n, R;    // data view [P][n][R]
  int64_t M, N;       // GEMM extents (K = n)
  int64_t mt, nt;     // tiles along M and N
  int64_t nblocks;
  const double* lam;  // epilogue tables
  const double* Lp;
  const double* Lr;
  double shift;
  const double2* Ep;
  const double2* Er;
  const double2* es;
  const int* skip;
  bool rows;          // row pass (fastest axis) rather than column pass
  // half-extent passes of a reflection-symmetric axis (fold = 1 forward, 2 backward):
  // tiles [0, te) of the split dimension belong to the even part, the rest to the odd part
  int64_t ne, no, hh, cc, te;
  const void* Se;     // half factors, k-major [fld][fld]
  const void* So;
  int64_t fld;
  int64_t kband;      // > 0: the factor vanishes for |k - output| > kband
};

// Map the hardware block id to a logical tile id so that consecutive logical
// tiles (which share an operand panel) run on the same XCD: blocks are handed
// to the 8 XCDs round-robin.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t bid, int64_t nblocks) {
  int64_t q = nblocks / 8, rmd = nblocks % 8;
  int64_t x = bid % 8, loc = bid / 8;
  return x * q + (x < rmd ? x : rmd) + loc;
}


// Fill the kernel arguments of one pass for tiles of bm x bn outputs.
inline void fill_kargs(const PassArgs& pa, KArgs& a, const void* S, int bm, int bn) {
  a.X = pa.X;
  a.Y = pa.Y;
  a.S = S;
  a.ld = pa.fac->ld;
  a.P = pa.P;
  a.n = pa.n;
  a.R = pa.R;
  a.lam = pa.fac->lam;
  a.Lp = pa.Lp;
  a.Lr = pa.Lr;
  a.shift = pa.shift;
  a.Ep = pa.Ep;
  a.Er = pa.Er;
  a.es = pa.es;
  a.skip = pa.skip;
  a.kband = pa.kband;
  a.rows = (pa.R == 1 || (pa.cplx && pa.R == 2)) && pa.epi == Epi::None;
  if (a.rows) {
    a.M = pa.P * (pa.cplx ? 2 : 1);
    a.N = pa.n;
    a.mt = (a.M + bm - 1) / bm;
    a.nt = (a.N + bn - 1) / bn;
    a.nblocks = a.mt * a.nt;
  } else {
    a.M = pa.n;
    a.N = pa.R;
    a.mt = (a.M + bm - 1) / bm;
    a.nt = (a.N + bn - 1) / bn;
    a.nblocks = a.mt * a.nt * pa.P;
  }
}

// Store one output of a row pass: element (m, col) of the (M x n) result,
// rows m = 2p + c for interleaved complex data.
template <typename TOut, bool CPLX>
__device__ __forceinline__ void store_rows(const KArgs& a, TOut* Y, int64_t m, int64_t col, double v) {
  if (m < a.M && col < a.n) {
    if (!CPLX) Y[m * a.n + col] = cvt_out<TOut>(v);
    else Y[(((m >> 1) * a.n + col) << 1) + (m & 1)] = cvt_out<TOut>(v);
  }
}

// Scale (scaling axis only) and store one output (p, m, col) of a column pass.
// For Exp, `partner` is the other component of the same complex element
// (taken from the neighbouring lane by the caller).
template <typename TOut, bool CPLX, int EPI>
__device__ __forceinline__ void store_cols(const KArgs& a, TOut* Y, int64_t p, int64_t m, int64_t col,
                                           double v, double partner) {
  if (m >= a.n || col >= a.R) return;
  if (EPI == (int)Epi::Exp) {
    double2 f1 = a.es[m], f2 = a.Ep[p], f3 = a.Er[col >> 1];
    double fr = f1.x * f2.x - f1.y * f2.y, fi = f1.x * f2.y + f1.y * f2.x;
    double gr = fr * f3.x - fi * f3.y, gi = fr * f3.y + fi * f3.x;
    v = (col & 1) ? (gi * partner + gr * v) : (gr * v - gi * partner);
  } else if (EPI == (int)Epi::Inv) {
    const int64_t q = CPLX ? (col >> 1) : col;
    v = v / (a.lam[m] + a.Lp[p] + a.Lr[q] + a.shift);
  }
  Y[(p * a.n + m) * a.R + col] = cvt_out<TOut>(v);
}

}  // namespace mp
}  // namespace ts
