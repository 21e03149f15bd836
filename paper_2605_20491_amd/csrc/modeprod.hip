// Mode-k contraction passes of the separable apply on CDNA4 (gfx950) MFMA.
//
// One pass computes, for a grid function X viewed as [P][n][R] (axis k has
// extent n, P = product of the slower extents, R = product of the faster
// extents times 2 for interleaved complex data):
//     forward  (paper Sec. 2.1 step 2):  Y[p, j, r] = sum_i Q[i][j] X[p, i, r]
//     backward (paper Sec. 2.1 step 4):  Y[p, j, r] = sum_i Q[j][i] X[p, i, r]
// as a GEMM on the 16x16x4 FP64 / FP32 matrix cores:
//   "column" passes (any axis but the fastest): for each p, C = A B with
//       A = the n x n factor (resident, LDS-staged), B = X[p] (n x R, R contiguous)
//   "row" passes (fastest axis, R == 1 or 2): C = A B with
//       A = X viewed as (P or 2P) x n rows (streamed, transposed into LDS),
//       B = the n x n factor.
// The factor matrices are stored k-major and zero-padded by the plan, so their
// tiles load without predicates; data tiles are predicated and zero-filled.
// The last forward pass optionally scales each output in its epilogue:
//     Inv: y / (lam_k[j] + Lp[p] + Lr[q] + shift)       (FP64 denominator)
//     Exp: y * es[j] * Ep[p] * Er[q]                     (FP64 phase factors)
// where q indexes the faster axes (r, or r/2 for complex data).
//
// Reflection-symmetric axes (FOLD != 0) contract half the extent: every
// eigenvector is even or odd, the spectral index is ordered [even | odd], and
//   forward  (FOLD = 1): y_even = Fe^T s,  y_odd = Fo^T d,
//            s_i = x_i + x_{n-1-i} (s_h = x_h for odd n), d_i = x_i - x_{n-1-i}
//            (the fold is applied as the data tile is loaded);
//   backward (FOLD = 2): E = Be^T z_even, O = Bo^T z_odd, written with O's
//            rows reversed (row n-1-i), then x_i = E_i + O_i and
//            x_{n-1-i} = E_i - O_i by the in-place butterfly k_unfold;
//   forward on folded data (FOLD = 3): the input already holds s_i at row i
//            and d_i at row n-1-i (the same butterfly, applied beforehand to
//            every folded axis at once by k_butterfly), so the pass reads
//            rows [0, h + c) for the even half and [h + c, n) for the odd
//            half against Fr, Fo with its rows reversed: no mirror loads.
// The butterflies commute with the passes over the other axes, so an apply
// with several folded axes folds its input once and unfolds its output once
// (two data sweeps in place of one per folded axis).
// Tiles of the output dimension are split between the two halves, so each
// tile runs one half-size GEMM: half the MFMA work of the plain pass.
#include <type_traits>

#include "ts_internal.h"
#include "modeprod_common.h"

namespace ts {
namespace {

using namespace mp;

constexpr int BM = 128, BN = 128, BK = 16, NT = 256;
constexpr int LDS_LD = BM + 4;  // padded LDS row length (elements)


// 8 consecutive elements through 16-byte accesses (16-byte aligned addresses).
__device__ __forceinline__ void load8(const double* src, double* d) {
  const double2* s2 = (const double2*)src;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 v = s2[i];
    d[2 * i] = v.x;
    d[2 * i + 1] = v.y;
  }
}
__device__ __forceinline__ void load8(const float* src, float* d) {
  const float4* s4 = (const float4*)src;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float4 v = s4[i];
    d[4 * i] = v.x;
    d[4 * i + 1] = v.y;
    d[4 * i + 2] = v.z;
    d[4 * i + 3] = v.w;
  }
}
__device__ __forceinline__ void store8(double* dst, const double* v) {
  double2* d2 = (double2*)dst;
#pragma unroll
  for (int i = 0; i < 4; ++i) d2[i] = make_double2(v[2 * i], v[2 * i + 1]);
}
__device__ __forceinline__ void store8(float* dst, const float* v) {
  float4* d4 = (float4*)dst;
#pragma unroll
  for (int i = 0; i < 2; ++i) d4[i] = make_float4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
}

// COAL: the data of this pass allow no 16-byte access (odd extents); the data
// tiles then move element by element with consecutive lanes on consecutive
// elements of one row (cols: one k-row of the tile; rows: one data row), so
// every load instruction is coalesced.  A separate instance keeps the 16-byte
// paths free of its registers.
template <typename TC, typename TIn, typename TOut, bool ROWS, bool CPLX, int EPI, int FOLD, bool COAL>
__global__ __launch_bounds__(NT, 2) void k_mode_mfma(KArgs a) {
  if (a.skip && *a.skip) return;
  __shared__ TC As[2][BK][LDS_LD];
  __shared__ TC Bs[2][BK][LDS_LD];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;

  const int64_t lb = xcd_logical_block(blockIdx.x, a.nblocks);
  int64_t p = 0, mtile, ntile;
  if (ROWS) {
    mtile = lb / a.nt;
    ntile = lb % a.nt;
  } else {
    mtile = lb % a.mt;
    int64_t rest = lb / a.mt;
    ntile = rest % a.nt;
    p = rest / a.nt;
  }
  // half-extent passes: which half this tile belongs to, its GEMM K and factor
  bool odd = false;
  int64_t K = a.n;
  const TC* S = (const TC*)a.S;
  int64_t ldS = a.ld;
  if (FOLD) {
    int64_t& split = ROWS ? ntile : mtile;
    odd = split >= a.te;
    if (odd) split -= a.te;
    K = FOLD == 1 ? (odd ? a.hh : a.hh + a.cc) : (odd ? a.no : a.ne);  // FOLD 3: as 2
    S = (const TC*)(odd ? a.So : a.Se);
    ldS = a.fld;
  }
  const int64_t m0 = mtile * BM, n0 = ntile * BN;
  const TIn* X = (const TIn*)a.X;
  // input row (along the pass axis) feeding GEMM index k; FOLD = 1 adds the mirror
  const int64_t koff = (FOLD >= 2 && odd) ? a.ne : 0;

  TC rres0[8], rres1[8];
  TIn rdat0[8], rdat1[8];

  // ---- global -> registers for k-tile kt ----
  // Factor tiles and column-pass data tiles: thread t owns row t >> 4 of the
  // 16-row tile and 8 consecutive columns 8 (t & 15) .. +7, moved with 16-byte
  // loads and stores.  Data rows need R % (16 / sizeof) == 0 for that (always
  // true for the factor); otherwise those loads fall back to single elements.
  const int vr = t >> 4, vc = 8 * (t & 15);
  const bool vec_data = !ROWS && (a.R % (16 / (int)sizeof(TIn)) == 0) && ((((uintptr_t)a.X) & 15) == 0);
  // row passes: rows of n (real) or 2n (complex) elements, starting k offsets multiples of 4
  const int64_t VW = 16 / (int64_t)sizeof(TIn);
  const bool vec_rows = ROWS && ((((uintptr_t)a.X) & 15) == 0) &&
                        ((CPLX ? 2 * a.n : a.n) % VW == 0) && ((CPLX ? 2 * koff : koff) % VW == 0);
  // FOLD = 1: the mirror values of the 16-byte paths wait in rmir until the
  // tile is stored, so the loads stay in flight during the MFMA work
  TIn rmir[8];
  bool mpend = false;
  auto load_tile = [&](int64_t k0, TC (&rres)[8], TIn (&rdat)[8]) {
    const int64_t f0 = ROWS ? n0 : m0;
    if (FOLD == 1) mpend = false;
    load8(S + (k0 + vr) * ldS + f0 + vc, rres);  // resident factor tile, always in bounds
    if constexpr (COAL && !ROWS) {
      // element (k0 + 2e + (t >> 7), n0 + (t & 127)), e = 0..7
      const int64_t col = n0 + (t & 127);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + 2 * e + (t >> 7);
        TIn v = (TIn)0, w = (TIn)0;
        if (k < K && col < a.R) {
          v = X[(p * a.n + koff + k) * a.R + col];
          if (FOLD == 1 && k < a.hh) w = X[(p * a.n + (a.n - 1 - k)) * a.R + col];
        }
        rdat[e] = v;
        if (FOLD == 1) rmir[e] = w;
      }
      if (FOLD == 1) mpend = true;
    } else if constexpr (COAL && ROWS && !CPLX) {
      // element (m0 + 16e + (t >> 4), k0 + (t & 15)), e = 0..7
      const int64_t k = k0 + (t & 15);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t m = m0 + 16 * e + (t >> 4);
        TIn v = (TIn)0, w = (TIn)0;
        if (m < a.M && k < K) {
          v = X[m * a.n + koff + k];
          if (FOLD == 1 && k < a.hh) w = X[m * a.n + (a.n - 1 - k)];
        }
        rdat[e] = v;
        if (FOLD == 1) rmir[e] = w;
      }
      if (FOLD == 1) mpend = true;
    } else if (!ROWS) {
      // B = X[p] row k, columns n0 + vc .. +7
      const int64_t k = k0 + vr, col = n0 + vc;
      if (k < K && vec_data && col + 8 <= a.R) {
        load8(X + (p * a.n + koff + k) * a.R + col, rdat);
        if (FOLD == 1 && k < a.hh) {
          load8(X + (p * a.n + (a.n - 1 - k)) * a.R + col, rmir);
          mpend = true;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          TIn v = (TIn)0;
          if (k < K && col + e < a.R) {
            v = X[(p * a.n + koff + k) * a.R + col + e];
            if (FOLD == 1 && k < a.hh) {
              const TIn w = X[(p * a.n + (a.n - 1 - k)) * a.R + col + e];
              v = odd ? v - w : v + w;
            }
          }
          rdat[e] = v;
        }
      }
    } else if (!CPLX) {
      // A = X rows: thread t owns row m0 + (t >> 1) and k0 + 8 (t & 1) .. +7
      const int64_t m = m0 + (t >> 1), kb = k0 + 8 * (t & 1);
      const TIn* row = X + m * a.n;
      if (vec_rows && m < a.M && kb + 8 <= K) {
        load8(row + koff + kb, rdat);
        if (FOLD == 1 && kb + 8 <= a.hh) {
          TIn w[8];  // row[n-1-kb-7 .. n-1-kb], reversed
          load8(row + (a.n - 8 - kb), w);
#pragma unroll
          for (int e = 0; e < 8; ++e) rmir[e] = w[7 - e];
          mpend = true;
        } else if (FOLD == 1) {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (kb + e < a.hh) rdat[e] = odd ? rdat[e] - row[a.n - 1 - kb - e] : rdat[e] + row[a.n - 1 - kb - e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t k = kb + e;
          TIn v = (TIn)0;
          if (m < a.M && k < K) {
            v = row[koff + k];
            if (FOLD == 1 && k < a.hh) {
              const TIn w = row[a.n - 1 - k];
              v = odd ? v - w : v + w;
            }
          }
          rdat[e] = v;
        }
      }
    } else {
      // A rows 2 pp (re) and 2 pp + 1 (im): thread t owns pp = m0 / 2 + (t >> 2) and
      // k0 + 4 (t & 3) .. +3, i.e. 8 consecutive interleaved values
      const int64_t pp = (m0 >> 1) + (t >> 2), kb = k0 + 4 * (t & 3);
      const TIn* row = X + ((pp * a.n) << 1);
      if (vec_rows && pp < a.P && kb + 4 <= K) {
        load8(row + ((koff + kb) << 1), rdat);
        if (FOLD == 1 && kb + 4 <= a.hh) {
          TIn w[8];  // complex elements n-1-kb-3 .. n-1-kb, reversed
          load8(row + ((a.n - 4 - kb) << 1), w);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            rmir[2 * e] = w[6 - 2 * e];
            rmir[2 * e + 1] = w[7 - 2 * e];
          }
          mpend = true;
        } else if (FOLD == 1) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (kb + e < a.hh) {
              const int64_t mk = (a.n - 1 - kb - e) << 1;
              rdat[2 * e] = odd ? rdat[2 * e] - row[mk] : rdat[2 * e] + row[mk];
              rdat[2 * e + 1] = odd ? rdat[2 * e + 1] - row[mk + 1] : rdat[2 * e + 1] + row[mk + 1];
            }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t k = kb + e;
          TIn vr0 = (TIn)0, vi0 = (TIn)0;
          if (pp < a.P && k < K) {
            vr0 = row[(koff + k) << 1];
            vi0 = row[((koff + k) << 1) + 1];
            if (FOLD == 1 && k < a.hh) {
              const TIn wr = row[(a.n - 1 - k) << 1], wi = row[((a.n - 1 - k) << 1) + 1];
              vr0 = odd ? vr0 - wr : vr0 + wr;
              vi0 = odd ? vi0 - wi : vi0 + wi;
            }
          }
          rdat[2 * e] = vr0;
          rdat[2 * e + 1] = vi0;
        }
      }
    }
  };
  auto store_tile = [&](int buf, TC (&rres)[8], TIn (&rdat)[8]) {
    if (FOLD == 1 && mpend) {
#pragma unroll
      for (int e = 0; e < 8; ++e) rdat[e] = odd ? rdat[e] - rmir[e] : rdat[e] + rmir[e];
    }
    TC(*Res)[LDS_LD] = ROWS ? Bs[buf] : As[buf];
    store8(&Res[vr][vc], rres);
    if constexpr (COAL && !ROWS) {
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][2 * e + (t >> 7)][t & 127] = cvt_in<TIn, TC>(rdat[e]);
    } else if constexpr (COAL && ROWS && !CPLX) {
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][t & 15][16 * e + (t >> 4)] = cvt_in<TIn, TC>(rdat[e]);
    } else if (!ROWS) {
      TC cv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) cv[e] = cvt_in<TIn, TC>(rdat[e]);
      store8(&Bs[buf][vr][vc], cv);
    } else if (!CPLX) {
      const int ml = t >> 1, kl = 8 * (t & 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][kl + e][ml] = cvt_in<TIn, TC>(rdat[e]);
    } else {
      const int pl = t >> 2, kl = 4 * (t & 3);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        As[buf][kl + e][2 * pl] = cvt_in<TIn, TC>(rdat[2 * e]);
        As[buf][kl + e][2 * pl + 1] = cvt_in<TIn, TC>(rdat[2 * e + 1]);
      }
    }
  };

  using V = typename AccT<TC>::V;
  V acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = V{0, 0, 0, 0};

  // banded factor (a block-banded operator, |i - j| <= kband): only the k-tiles
  // that meet the band of this tile's outputs contribute (the others are zero)
  int64_t kbeg = 0, kend = K;
  if (a.kband > 0) {
    const int64_t o0 = ROWS ? n0 : m0, o1 = o0 + (ROWS ? BN : BM);
    kbeg = o0 > a.kband ? o0 - a.kband : 0;
    kbeg -= kbeg % BK;
    kend = o1 + a.kband < K ? o1 + a.kband : K;
  }
  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  auto compute = [&](int cur) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int krow = kk * 4 + lk;
      TC av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[cur][krow][wm * 64 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[cur][krow][wn * 64 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma(av[i], bv[j], acc[i][j]);
    }
  };
  load_tile(kbeg, rres0, rdat0);
  store_tile(0, rres0, rdat0);
  // Two k-tiles in flight in registers (the tile stored at the end of stage kt
  // was loaded at the start of stage kt - 1), except in the folding forward
  // pass, whose mirror loads leave no registers for a second set, and in the
  // element-wise instance, whose per-element addresses do not either.
  constexpr bool kDeep = FOLD != 1 && !COAL;
  if (kDeep) {
    if (nk > 1) load_tile(kbeg + BK, rres0, rdat0);
    lds_barrier();
    // LDS-only barriers: the loads of tile kt + 2 stay in flight across the
    // barrier that ends stage kt
    auto stage = [&](int64_t kt, TC (&ra)[8], TIn (&da)[8], TC (&rb)[8], TIn (&db)[8]) {
      const int cur = (int)(kt & 1);
      if (kt + 2 < nk) load_tile(kbeg + (kt + 2) * BK, rb, db);
      compute(cur);
      if (kt + 1 < nk) store_tile(cur ^ 1, ra, da);
      lds_barrier();
    };
    for (int64_t kt = 0; kt < nk; kt += 2) {
      stage(kt, rres0, rdat0, rres1, rdat1);
      if (kt + 1 < nk) stage(kt + 1, rres1, rdat1, rres0, rdat0);
    }
  } else {
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
      const int cur = (int)(kt & 1);
      if (kt + 1 < nk) load_tile(kbeg + (kt + 1) * BK, rres0, rdat0);
      compute(cur);
      if (kt + 1 < nk) store_tile(cur ^ 1, rres0, rdat0);
      __syncthreads();
    }
  }

  // ---- epilogue ----
  TOut* Y = (TOut*)a.Y;
  if constexpr (EPI != 0 && !ROWS) {
    // Scaling pass: the table entries of this thread's rows and columns are read
    // once (the stores below may alias the tables as far as the compiler can
    // tell, so it would reload them for every element); same arithmetic and
    // order as store_cols.
    double tr[4];
    double2 er[4], ep = make_double2(0.0, 0.0);
    if (EPI == (int)Epi::Exp) ep = a.Ep[p];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = n0 + wn * 64 + j * 16 + lr;
      const bool ok = col < a.R;
      if (EPI == (int)Epi::Inv) tr[j] = ok ? a.Lr[CPLX ? (col >> 1) : col] : 0.0;
      else er[j] = ok ? a.Er[col >> 1] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int64_t dm[4];
      double tm[4];
      double2 fm[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 64 + i * 16 + out_row<TC>(lane, r);
        int64_t dst = m;
        bool ok = m < a.n;
        if (FOLD) {
          const int64_t cnt = FOLD != 2 ? (odd ? a.no : a.ne) : (odd ? a.hh : a.hh + a.cc);
          ok = m < cnt;
          dst = FOLD != 2 ? (odd ? a.ne + m : m) : (odd ? a.n - 1 - m : m);
        }
        dm[r] = ok ? dst : -1;
        if (EPI == (int)Epi::Inv) {
          tm[r] = ok ? a.lam[dst] + a.Lp[p] : 0.0;
        } else {
          const double2 f1 = ok ? a.es[dst] : make_double2(0.0, 0.0);
          fm[r] = make_double2(f1.x * ep.x - f1.y * ep.y, f1.x * ep.y + f1.y * ep.x);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t col = n0 + wn * 64 + j * 16 + lr;
          double v = (double)acc[i][j][r];
          double partner = 0.0;
          // (re, im) of one element sit in lanes 2u, 2u+1 (columns col, col^1)
          if (EPI == (int)Epi::Exp) partner = __shfl_xor(v, 1);
          if (dm[r] < 0 || col >= a.R) continue;
          if (EPI == (int)Epi::Inv) {
            v = v / (tm[r] + tr[j] + a.shift);
          } else {
            const double gr = fm[r].x * er[j].x - fm[r].y * er[j].y, gi = fm[r].x * er[j].y + fm[r].y * er[j].x;
            v = (col & 1) ? (gi * partner + gr * v) : (gr * v - gi * partner);
          }
          Y[(p * a.n + dm[r]) * a.R + col] = cvt_out<TOut>(v);
        }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 64 + i * 16 + out_row<TC>(lane, r);
        const int64_t col = n0 + wn * 64 + j * 16 + lr;
        double v = (double)acc[i][j][r];
        double partner = 0.0;
        // (re, im) of one element sit in lanes 2u, 2u+1 (columns col, col^1)
        if (EPI == (int)Epi::Exp) partner = __shfl_xor(v, 1);
        if (FOLD) {
          // index along the pass axis within this half, and its place in the output
          const int64_t loc = ROWS ? col : m;
          const int64_t cnt = FOLD != 2 ? (odd ? a.no : a.ne) : (odd ? a.hh : a.hh + a.cc);
          if (loc >= cnt) continue;
          const int64_t dst = FOLD != 2 ? (odd ? a.ne + loc : loc) : (odd ? a.n - 1 - loc : loc);
          if (ROWS) store_rows<TOut, CPLX>(a, Y, m, dst, v);
          else store_cols<TOut, CPLX, EPI>(a, Y, p, dst, col, v, partner);
        } else if (ROWS) {
          store_rows<TOut, CPLX>(a, Y, m, col, v);
        } else {
          store_cols<TOut, CPLX, EPI>(a, Y, p, m, col, v, partner);
        }
      }
}

template <typename TC, typename TIn, typename TOut, int FOLD, bool COAL>
hipError_t launch_fold(const KArgs& a, const PassArgs& pa, hipStream_t st) {
  dim3 grid((unsigned)a.nblocks), block(NT);
  if (a.rows) {
    if (pa.cplx) hipLaunchKernelGGL((k_mode_mfma<TC, TIn, TOut, true, true, 0, FOLD, false>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_mode_mfma<TC, TIn, TOut, true, false, 0, FOLD, COAL>), grid, block, 0, st, a);
  } else if (pa.epi == Epi::Exp) {
    if (!pa.cplx) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_mode_mfma<TC, TIn, TOut, false, true, (int)Epi::Exp, FOLD, false>), grid, block, 0, st, a);
  } else if (pa.epi == Epi::Inv) {
    if (pa.cplx)
      hipLaunchKernelGGL((k_mode_mfma<TC, TIn, TOut, false, true, (int)Epi::Inv, FOLD, false>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_mode_mfma<TC, TIn, TOut, false, false, (int)Epi::Inv, FOLD, COAL>), grid, block, 0, st, a);
  } else {
    hipLaunchKernelGGL((k_mode_mfma<TC, TIn, TOut, false, false, 0, FOLD, COAL>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

// x_i, x_{n-1-i} <- x_i + x_{n-1-i}, x_i - x_{n-1-i} for i < hh, over [P][n][R].
template <typename T>
__global__ __launch_bounds__(256) void k_unfold(T* Y, int64_t P, int64_t n, int64_t R, int64_t hh) {
  const int64_t total = P * hh * R;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e % R;
    const int64_t q = e / R;
    const int64_t i = q % hh, p = q / hh;
    T* lo = Y + (p * n + i) * R + r;
    T* hi = Y + (p * n + (n - 1 - i)) * R + r;
    const T a = *lo, b = *hi;
    *lo = a + b;
    *hi = a - b;
  }
}

// The same with 16-byte accesses: V holds W consecutive r of one row (R % W == 0,
// rows 16-byte aligned).
template <typename V, int W>
__global__ __launch_bounds__(256) void k_unfold_vec(V* Y, int64_t P, int64_t n, int64_t Rv, int64_t hh) {
  const int64_t total = P * hh * Rv;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e % Rv;
    const int64_t q = e / Rv;
    const int64_t i = q % hh, p = q / hh;
    V* lo = Y + (p * n + i) * Rv + r;
    V* hi = Y + (p * n + (n - 1 - i)) * Rv + r;
    const V a = *lo, b = *hi;
    V s, d;
    if constexpr (W == 2) {
      s = V{a.x + b.x, a.y + b.y};
      d = V{a.x - b.x, a.y - b.y};
    } else {
      s = V{a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w};
      d = V{a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w};
    }
    *lo = s;
    *hi = d;
  }
}

template <typename T>
hipError_t launch_unfold(T* Y, int64_t P, int64_t n, int64_t R, int64_t hh, hipStream_t st) {
  constexpr int W = 16 / (int)sizeof(T);
  const bool vec = (R % W == 0) && ((((uintptr_t)Y) & 15) == 0);
  const int64_t Rv = vec ? R / W : R;
  const int64_t total = P * hh * Rv;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  if (vec) {
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    hipLaunchKernelGGL((k_unfold_vec<V, W>), dim3(blocks), dim3(256), 0, st, (V*)Y, P, n, Rv, hh);
  } else {
    hipLaunchKernelGGL((k_unfold<T>), dim3(blocks), dim3(256), 0, st, Y, P, n, R, hh);
  }
  return hipGetLastError();
}

// The butterfly along NAX axes at once: thread e owns one point with i_a <= n_a - 1 - i_a
// on every listed axis and the up to 2^NAX points of its orbit under the reflections.
// An axis on which the point is its own mirror (the middle of odd n) is left as it is.
template <typename T, int NAX>
__global__ __launch_bounds__(256) void k_butterfly(const T* X, T* Y, ButterflyArgs a, int64_t total) {
  if (a.skip && *a.skip) return;
  constexpr int NV = 1 << NAX;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    // coordinates of the representative point, fastest (the component) first
    int64_t rest = e / a.ncomp;
    int64_t off = e - rest * a.ncomp;
    int64_t stride = a.ncomp;
    int64_t delta[NAX];
    bool act[NAX];
#pragma unroll
    for (int j = 0; j < NAX; ++j) {
      delta[j] = 0;
      act[j] = false;
    }
    for (int k = a.d - 1; k >= 0; --k) {
      int jf = -1;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (a.ax[j] == k) jf = j;
      const int64_t ext = jf >= 0 ? a.n[k] - a.hh[jf] : a.n[k];  // h + c representatives
      const int64_t q = rest / ext;
      const int64_t i = rest - q * ext;
      rest = q;
      off += i * stride;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (j == jf && i < a.hh[j]) {
          act[j] = true;
          delta[j] = (a.n[k] - 1 - 2 * i) * stride;
        }
      stride *= a.n[k];
    }
    T v[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      bool ok = true;
      int64_t o = off;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (m & (1 << j)) {
          ok = ok && act[j];
          o += delta[j];
        }
      v[m] = ok ? X[o] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < NAX; ++j) {
      if (!act[j]) continue;
#pragma unroll
      for (int m = 0; m < NV; ++m)
        if (!(m & (1 << j))) {
          const T x0 = v[m], x1 = v[m | (1 << j)];
          v[m] = x0 + x1;
          v[m | (1 << j)] = x0 - x1;
        }
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      bool ok = true;
      int64_t o = off;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (m & (1 << j)) {
          ok = ok && act[j];
          o += delta[j];
        }
      if (ok) Y[o] = v[m];
    }
  }
}

// The same on 2-element units, moved with one 8- or 16-byte access each:
// complex data (a unit is one element, both components), or real data whose
// fastest axis is folded with n % 4 == 0 (SWAP: a unit is the pair i, i+1 of
// the lower half, its mirror the pair n-2-i, n-1-i, so the fastest-axis
// butterfly pairs a.x with b.y and a.y with b.x).
template <typename T, int NAX, bool SWAP>
__global__ __launch_bounds__(256) void k_butterfly_v2(const T* X, T* Y, ButterflyArgs a, int64_t total) {
  using V = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  if (a.skip && *a.skip) return;
  constexpr int NV = 1 << NAX;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int64_t rest = e, off = 0, stride = 2;  // offsets in elements of T
    int64_t delta[NAX];
    bool act[NAX];
    int jl = -1;  // the fastest axis's slot (SWAP)
#pragma unroll
    for (int j = 0; j < NAX; ++j) {
      delta[j] = 0;
      act[j] = false;
    }
    for (int k = a.d - 1; k >= 0; --k) {
      int jf = -1;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (a.ax[j] == k) jf = j;
      if (SWAP && k == a.d - 1) {
        const int64_t ext = a.hh[jf] / 2;  // pairs of the lower half
        const int64_t q = rest / ext;
        const int64_t i = rest - q * ext;
        rest = q;
        off = 2 * i;
        jl = jf;
#pragma unroll
        for (int j = 0; j < NAX; ++j)
          if (j == jf) {
            act[j] = true;
            delta[j] = a.n[k] - 2 - 4 * i;
          }
        stride = a.n[k];
        continue;
      }
      const int64_t ext = jf >= 0 ? a.n[k] - a.hh[jf] : a.n[k];
      const int64_t q = rest / ext;
      const int64_t i = rest - q * ext;
      rest = q;
      off += i * stride;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (j == jf && i < a.hh[j]) {
          act[j] = true;
          delta[j] = (a.n[k] - 1 - 2 * i) * stride;
        }
      stride *= a.n[k];
    }
    V v[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      bool ok = true;
      int64_t o = off;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (m & (1 << j)) {
          ok = ok && act[j];
          o += delta[j];
        }
      v[m] = ok ? *(const V*)(X + o) : V{};
    }
#pragma unroll
    for (int j = 0; j < NAX; ++j) {
      if (!act[j]) continue;
      const bool sw = SWAP && j == jl;
#pragma unroll
      for (int m = 0; m < NV; ++m)
        if (!(m & (1 << j))) {
          const V x0 = v[m], x1 = v[m | (1 << j)];
          if (sw) {
            v[m] = V{x0.x + x1.y, x0.y + x1.x};
            v[m | (1 << j)] = V{x0.y - x1.x, x0.x - x1.y};
          } else {
            v[m] = V{x0.x + x1.x, x0.y + x1.y};
            v[m | (1 << j)] = V{x0.x - x1.x, x0.y - x1.y};
          }
        }
    }
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      bool ok = true;
      int64_t o = off;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (m & (1 << j)) {
          ok = ok && act[j];
          o += delta[j];
        }
      if (ok) *(V*)(Y + o) = v[m];
    }
  }
}

template <typename T>
hipError_t launch_butterfly_t(const ButterflyArgs& a, hipStream_t st) {
  int64_t total = a.ncomp;
  for (int k = 0; k < a.d; ++k) {
    int64_t ext = a.n[k];
    for (int j = 0; j < a.nax; ++j)
      if (a.ax[j] == k) ext = a.n[k] - a.hh[j];
    total *= ext;
  }
  if (total <= 0) return hipSuccess;
  const T* X = (const T*)a.X;
  T* Y = (T*)a.Y;
  // 2-element units: complex data, or a folded fastest axis with n % 4 == 0
  const uintptr_t al = 2 * sizeof(T) - 1;
  const bool aligned = ((((uintptr_t)X) | ((uintptr_t)Y)) & al) == 0;
  int jlast = -1;
  for (int j = 0; j < a.nax; ++j)
    if (a.ax[j] == a.d - 1) jlast = j;
  const bool cplx_units = aligned && a.ncomp == 2;
  const bool pair_units = aligned && a.ncomp == 1 && jlast >= 0 && a.n[a.d - 1] % 4 == 0;
  if (cplx_units || pair_units) {
    const int64_t units = total / 2;  // pair_units: the fastest axis holds n / 2 representatives, i.e. n / 4 pairs
    const unsigned blocks = (unsigned)std::min<int64_t>((units + 255) / 256, 1 << 20);
#define TS_BFLY_V2(N)                                                                                  \
  if (pair_units)                                                                                      \
    hipLaunchKernelGGL((k_butterfly_v2<T, N, true>), dim3(blocks), dim3(256), 0, st, X, Y, a, units); \
  else                                                                                                 \
    hipLaunchKernelGGL((k_butterfly_v2<T, N, false>), dim3(blocks), dim3(256), 0, st, X, Y, a, units);
    switch (a.nax) {
      case 1: TS_BFLY_V2(1) break;
      case 2: TS_BFLY_V2(2) break;
      case 3: TS_BFLY_V2(3) break;
      case 4: TS_BFLY_V2(4) break;
      default: return hipErrorInvalidValue;
    }
#undef TS_BFLY_V2
    return hipGetLastError();
  }
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  switch (a.nax) {
    case 1: hipLaunchKernelGGL((k_butterfly<T, 1>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    case 2: hipLaunchKernelGGL((k_butterfly<T, 2>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    case 3: hipLaunchKernelGGL((k_butterfly<T, 3>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    case 4: hipLaunchKernelGGL((k_butterfly<T, 4>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TC, typename TIn, typename TOut>
hipError_t launch_typed(const PassArgs& pa, hipStream_t st) {
  KArgs a{};
  const AxisFactor* F = pa.fac;
  const bool dbl = std::is_same<TC, double>::value;
  const void* S;
  if (dbl) S = pa.forward ? (const void*)F->Q64 : (const void*)F->QT64;
  else S = pa.forward ? (const void*)F->Q32 : (const void*)F->QT32;
  fill_kargs(pa, a, S, BM, BN);
  const int fold = pa.fold ? (pa.forward ? (pa.deferred ? 3 : 1) : 2) : 0;
  if (fold) {
    a.ne = F->ne;
    a.no = F->no;
    a.hh = F->hh;
    a.cc = F->cc;
    a.fld = F->fkp;
    if (pa.forward) {
      a.Se = dbl ? (const void*)F->Fe64 : (const void*)F->Fe32;
      if (fold == 3) a.So = dbl ? (const void*)F->Fr64 : (const void*)F->Fr32;
      else a.So = dbl ? (const void*)F->Fo64 : (const void*)F->Fo32;
    } else {
      a.Se = dbl ? (const void*)F->Be64 : (const void*)F->Be32;
      a.So = dbl ? (const void*)F->Bo64 : (const void*)F->Bo32;
    }
    // outputs of each half along the pass axis
    const int64_t me = fold != 2 ? F->ne : F->hh + F->cc, mo = fold != 2 ? F->no : F->hh;
    const int64_t tb = a.rows ? BN : BM;
    a.te = (me + tb - 1) / tb;
    const int64_t tsplit = a.te + (mo + tb - 1) / tb;
    if (a.rows) {
      a.nt = tsplit;
      a.nblocks = a.mt * a.nt;
    } else {
      a.mt = tsplit;
      a.nblocks = a.mt * a.nt * pa.P;
    }
  }
  if (a.nblocks <= 0) return hipSuccess;
  if (a.nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  // real data that allow no 16-byte access at all: the element-wise instance
  constexpr int64_t VW = 16 / (int64_t)sizeof(TIn);
  const bool aligned = (((uintptr_t)pa.X) & 15) == 0;
  const bool coal = !pa.cplx && (a.rows ? !(aligned && pa.n % VW == 0 && (fold < 2 || F->ne % VW == 0))
                                        : !(aligned && pa.R % VW == 0));
  hipError_t e;
  if (coal) {
    if (fold == 1) e = launch_fold<TC, TIn, TOut, 1, true>(a, pa, st);
    else if (fold == 2) e = launch_fold<TC, TIn, TOut, 2, true>(a, pa, st);
    else if (fold == 3) e = launch_fold<TC, TIn, TOut, 3, true>(a, pa, st);
    else e = launch_fold<TC, TIn, TOut, 0, true>(a, pa, st);
  } else {
    if (fold == 1) e = launch_fold<TC, TIn, TOut, 1, false>(a, pa, st);
    else if (fold == 2) e = launch_fold<TC, TIn, TOut, 2, false>(a, pa, st);
    else if (fold == 3) e = launch_fold<TC, TIn, TOut, 3, false>(a, pa, st);
    else e = launch_fold<TC, TIn, TOut, 0, false>(a, pa, st);
  }
  if (e != hipSuccess || fold != 2 || pa.deferred || F->hh == 0) return e;
  // butterfly of the backward pass, in place on its output (R: real values per (p, i))
  return launch_unfold<TOut>((TOut*)pa.Y, pa.P, pa.n, pa.R, F->hh, st);
}

}  // namespace

hipError_t launch_butterfly(const ButterflyArgs& a, hipStream_t st) {
  if (a.nax < 1 || a.nax > 4 || a.d < 1 || a.d > TS_MAX_D || (a.ncomp != 1 && a.ncomp != 2))
    return hipErrorInvalidValue;
  if (!a.X || !a.Y) return hipErrorInvalidValue;
  for (int j = 0; j < a.nax; ++j) {
    if (a.ax[j] < 0 || a.ax[j] >= a.d || a.hh[j] != a.n[a.ax[j]] / 2) return hipErrorInvalidValue;
    for (int i = 0; i < j; ++i)
      if (a.ax[i] == a.ax[j]) return hipErrorInvalidValue;
  }
  if (a.t == DT::F64) return launch_butterfly_t<double>(a, st);
  if (a.t == DT::F32) return launch_butterfly_t<float>(a, st);
  return hipErrorInvalidValue;
}

hipError_t launch_pass(const PassArgs& pa, hipStream_t st) {
  if (pa.prec == 0) {
    if (pa.tin == DT::F64 && pa.tout == DT::F64) return launch_typed<double, double, double>(pa, st);
    if (pa.tin == DT::F32 && pa.tout == DT::F32) return launch_typed<double, float, float>(pa, st);
    return hipErrorInvalidValue;
  }
  if (pa.prec == 1) {
    if (pa.tin == DT::F64 && pa.tout == DT::F64) return launch_typed<float, double, double>(pa, st);
    if (pa.tin == DT::F64 && pa.tout == DT::F32) return launch_typed<float, double, float>(pa, st);
    if (pa.tin == DT::F32 && pa.tout == DT::F32) return launch_typed<float, float, float>(pa, st);
    if (pa.tin == DT::F32 && pa.tout == DT::F64) return launch_typed<float, float, double>(pa, st);
    return hipErrorInvalidValue;
  }
  if (pa.prec == 2) return launch_pass_bf16(pa, st);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Phase tables of the propagator (FP64): products of per-axis factors
// e^{-i tau lam}.  Entry ranges: [0, P) -> Ep, [P, P+R) -> Er, then es.
// ---------------------------------------------------------------------------
__global__ void k_phase_tables(PhaseTableArgs a) {
  const int64_t total = a.P + a.R + a.n[a.s];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double re = 1.0, im = 0.0;
    int lo, hi;
    int64_t idx;
    double2* dst;
    if (e < a.P) { lo = 0; hi = a.s; idx = e; dst = a.Ep + e; }
    else if (e < a.P + a.R) { lo = a.s + 1; hi = a.d; idx = e - a.P; dst = a.Er + (e - a.P); }
    else { lo = a.s; hi = a.s + 1; idx = e - a.P - a.R; dst = a.es + idx; }
    for (int k = hi - 1; k >= lo; --k) {
      int64_t j = idx % a.n[k];
      idx /= a.n[k];
      double sn, cs;
      sincos(a.tau * a.lam[k][j], &sn, &cs);
      // multiply by (cs - i sn)
      double nr = re * cs + im * sn, ni = im * cs - re * sn;
      re = nr;
      im = ni;
    }
    *dst = make_double2(re, im);
  }
}

hipError_t launch_phase_tables(const PhaseTableArgs& a, hipStream_t st) {
  int64_t total = a.P + a.R + a.n[a.s];
  int blocks = (int)std::min<int64_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_phase_tables, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

__global__ void k_cast_f32(const double* x, float* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
// A data array to BF16 for the BF16 passes, four elements per thread (x
// 16-byte, y 8-byte aligned, n % 4 == 0), stopping at once when *skip is set.
// Rounded as the pass kernels round FP64 data they load (FP64 -> FP32 -> BF16,
// each to nearest even), so an apply gives the same result either way.
__global__ __launch_bounds__(256) void k_cast_bf16_x4(const double2* x, uint2* y, int64_t n4, const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
    const double2 a = x[2 * i], b = x[2 * i + 1];
    y[i] = make_uint2((uint32_t)cvt_out<uint16_t>(a.x) | ((uint32_t)cvt_out<uint16_t>(a.y) << 16),
                      (uint32_t)cvt_out<uint16_t>(b.x) | ((uint32_t)cvt_out<uint16_t>(b.y) << 16));
  }
}

hipError_t launch_data_to_bf16(const double* x, uint16_t* y, int64_t n, const int* skip, hipStream_t st) {
  if (n % 4 != 0 || (((uintptr_t)x) & 15) != 0 || (((uintptr_t)y) & 7) != 0) return hipErrorInvalidValue;
  const int64_t n4 = n / 4;
  if (n4 == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n4 + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_cast_bf16_x4, dim3(blocks), dim3(256), 0, st, (const double2*)x, (uint2*)y, n4, skip);
  return hipGetLastError();
}

// y[j][i] = bf16(x[i][j]) for a square [ld][ld] matrix: the K-contiguous BF16
// copy of a k-major factor.
__global__ void k_cast_bf16_t(const double* x, uint16_t* y, int64_t ld) {
  const int64_t total = ld * ld;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / ld, i = e % ld;  // output row j, column i
    y[e] = bf16_from_f64(x[i * ld + j]);
  }
}

hipError_t launch_cast_f64_to_bf16_t(const double* x, uint16_t* y, int64_t ld, hipStream_t st) {
  int blocks = (int)std::min<int64_t>(4096, (ld * ld + 255) / 256);
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_cast_bf16_t, dim3(blocks), dim3(256), 0, st, x, y, ld);
  return hipGetLastError();
}

hipError_t launch_cast_f64_to_f32(const double* x, float* y, int64_t n, hipStream_t st) {
  int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f32, dim3(blocks), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

}  // namespace ts
