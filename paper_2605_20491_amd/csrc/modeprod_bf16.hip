// BF16 mode-product passes: BF16 operands on the 16x16x32 matrix cores of
// gfx950 with FP32 accumulation (the reduced-precision transforms used inside
// PCG and refinement; paper Sec. 2.2 runs the same apply in BF16).
//
// Same pass structure as modeprod.hip (column passes: factor x X[p]; row
// passes on the fastest axis: X rows x factor), but both LDS operands are
// stored "free index major, K contiguous" because one MFMA lane consumes 8
// consecutive K values of one row (A) or one column (B): each fragment is a
// single 128-bit LDS read.  The factor tiles therefore come from the
// transposed copy of the role the FP64 kernel uses (forward: Q^T, backward:
// Q), stored in HBM as BF16 with the same zero padding.  Data tiles are
// converted to BF16 on the way into LDS (FP64 -> FP32 -> BF16, each round to
// nearest even); the column operand is transposed there.
#include <algorithm>
#include <type_traits>

#include "modeprod_common.h"
#include "ts_internal.h"

namespace ts {
namespace {

using namespace mp;

typedef short s8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte register chunk

constexpr int BM = 128, BN = 128, BK = 64, NT = 256;
constexpr int LDK = BK + 8;  // padded row: 144 B, fragment reads are bank-conflict free

// Column passes store the data tile transposed (one k-run per column row), and
// rows 8 apart share a bank under any 16-byte-multiple row length; their 16-byte
// k-chunks are therefore XOR-swizzled by the row group.  Position of k-chunk
// `chunk` (8 elements) of row `row`, in elements:
__device__ __forceinline__ int swz8(int row, int chunk) { return 8 * (chunk ^ ((row >> 3) & 7)); }

__device__ __forceinline__ uint16_t to_bf16(double x) { return f32_to_bf16((float)x); }
__device__ __forceinline__ uint16_t to_bf16(float x) { return f32_to_bf16(x); }
__device__ __forceinline__ uint16_t to_bf16(uint16_t x) { return x; }

// 8 consecutive elements by 16-byte loads (the caller guarantees alignment).
__device__ __forceinline__ void load_vec8(const double* src, double* dst) {
  const double2* s2 = (const double2*)src;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double2 v = s2[i];
    dst[2 * i] = v.x;
    dst[2 * i + 1] = v.y;
  }
}
__device__ __forceinline__ void load_vec8(const float* src, float* dst) {
  const float4* s4 = (const float4*)src;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    float4 v = s4[i];
    dst[4 * i] = v.x;
    dst[4 * i + 1] = v.y;
    dst[4 * i + 2] = v.z;
    dst[4 * i + 3] = v.w;
  }
}
__device__ __forceinline__ void load_vec8(const uint16_t* src, uint16_t* dst) {
  uint4 v = *(const uint4*)src;
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    dst[2 * i] = (uint16_t)(w[i] & 0xffffu);
    dst[2 * i + 1] = (uint16_t)(w[i] >> 16);
  }
}

// One 16-byte chunk (16 / sizeof(T) consecutive elements; the caller guarantees alignment).
__device__ __forceinline__ void load_vec16(const double* src, double* dst) {
  const double2 v = *(const double2*)src;
  dst[0] = v.x;
  dst[1] = v.y;
}
__device__ __forceinline__ void load_vec16(const float* src, float* dst) {
  const float4 v = *(const float4*)src;
  dst[0] = v.x;
  dst[1] = v.y;
  dst[2] = v.z;
  dst[3] = v.w;
}
__device__ __forceinline__ void load_vec16(const uint16_t* src, uint16_t* dst) { load_vec8(src, dst); }

template <typename TIn> __device__ __forceinline__ TIn fold_add(TIn x, TIn y, bool sub) {
  return sub ? x - y : x + y;
}
template <> __device__ __forceinline__ uint16_t fold_add<uint16_t>(uint16_t x, uint16_t y, bool sub) {
  const float r = sub ? bf16_to_f32(x) - bf16_to_f32(y) : bf16_to_f32(x) + bf16_to_f32(y);
  return f32_to_bf16(r);
}

// FOLD as in modeprod.hip: 1 = forward half-extent pass (x_i +- x_{n-1-i} folded while
// loading), 2 = backward half-extent pass (halves written apart, butterfly afterwards).
// COAL: the data in this pass allow no 16-byte access (odd extents); every
// block then uses an element-wise mapping in which consecutive lanes read
// consecutive elements of one row (cols: one k-row of the tile; rows: one data
// row), so every load instruction is coalesced.  A separate instance keeps the
// 16-byte paths free of its registers.
// Two accumulators of a staged BF16 output (rows r and r + 1 of one column),
// rounded to nearest even by the packed conversion of gfx950 (the rounding
// of f32_to_bf16 for finite values, in one instruction).  Scaling pass: each
// is first multiplied by the reciprocal of its FP64 denominator rounded to
// FP32 (v_rcp_f32, within 1 ulp), i.e. within about 2^-22 of the FP64
// quotient, far below the BF16 step; a division, FP64 or FP32, would cost the
// epilogue more than the pass's products.  Entries outside the grid are
// staged and never written.
template <int EPI>
__device__ __forceinline__ uint32_t stage_pair(float v0, float v1, double den0, double den1) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  if (EPI == (int)Epi::Inv) {
    v0 *= __builtin_amdgcn_rcpf((float)den0);
    v1 *= __builtin_amdgcn_rcpf((float)den1);
  }
  const f32x2 v = {v0, v1};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

template <typename TIn, typename TOut, bool ROWS, bool CPLX, int EPI, int FOLD, bool COAL>
__global__ __launch_bounds__(NT, 2) void k_mode_bf16(KArgs a) {
  if (a.skip && *a.skip) return;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN][LDK];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;

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
  bool odd = false;
  int64_t K = a.n;
  const uint16_t* S = (const uint16_t*)a.S;
  int64_t ldS = a.ld;
  if (FOLD) {
    int64_t& split = ROWS ? ntile : mtile;
    odd = split >= a.te;
    if (odd) split -= a.te;
    K = FOLD == 1 ? (odd ? a.hh : a.hh + a.cc) : (odd ? a.no : a.ne);
    S = (const uint16_t*)(odd ? a.So : a.Se);
    ldS = a.fld;
  }
  const int64_t koff = (FOLD == 2 && odd) ? a.ne : 0;
  const int64_t m0 = mtile * BM, n0 = ntile * BN;
  const TIn* X = (const TIn*)a.X;

  // resident factor tile: 128 rows (free index) x 64 k; 4 x 16 bytes per thread
  uint4 rres0, rres1, rres2, rres3;
  // data: 32 elements per thread
  TIn rdat[32];

  const int64_t f0 = ROWS ? n0 : m0;
  const bool base_aligned = (((uintptr_t)a.X) & 15) == 0;
  constexpr bool coal_cols = COAL && !ROWS;
  constexpr bool coal_rows = COAL && ROWS && !CPLX;
  auto load_tile = [&](int64_t k0) {
    {
      const int row = t >> 1, half = t & 1;  // 32 k per thread
      const uint4* src = (const uint4*)(S + (f0 + row) * ldS + k0 + 32 * half);
      rres0 = src[0];
      rres1 = src[1];
      rres2 = src[2];
      rres3 = src[3];
    }
    if (!ROWS && coal_cols) {
      // element (k0 + 2c + (t >> 7), n0 + (t & 127)) for c = 0..31
      const int64_t col = n0 + (t & 127);
#pragma unroll
      for (int c = 0; c < 32; ++c) {
        const int64_t k = k0 + 2 * c + (t >> 7);
        TIn v = (TIn)0;
        if (k < K && col < a.R) {
          v = X[(p * a.n + koff + k) * a.R + col];
          if (FOLD == 1 && k < a.hh) v = fold_add(v, X[(p * a.n + (a.n - 1 - k)) * a.R + col], odd);
        }
        rdat[c] = v;
      }
    } else if (ROWS && coal_rows) {
      // element (m0 + 4c + (t >> 6), k0 + (t & 63)) for c = 0..31
      const int64_t k = k0 + (t & 63);
#pragma unroll
      for (int c = 0; c < 32; ++c) {
        const int64_t m = m0 + 4 * c + (t >> 6);
        TIn v = (TIn)0;
        if (m < a.M && k < K) {
          v = X[m * a.n + koff + k];
          if (FOLD == 1 && k < a.hh) v = fold_add(v, X[m * a.n + (a.n - 1 - k)], odd);
        }
        rdat[c] = v;
      }
    } else if (!ROWS) {
      // X[p] rows k0 + 4*kq .. +3, columns n0 + 8*oc .. +7
      const int oc = t & 15, kq = t >> 4;
      const int64_t col0 = n0 + 8 * oc;
      const bool vec = base_aligned && (a.R % (16 / (int)sizeof(TIn)) == 0) && (col0 + 8 <= a.R);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t k = k0 + 4 * kq + rr;
        const TIn* src = X + (p * a.n + koff + k) * a.R + col0;
        const TIn* mir = X + (p * a.n + (a.n - 1 - k)) * a.R + col0;
        const bool fold_k = FOLD == 1 && k < a.hh;
        if (k < K && vec) {
          load_vec8(src, &rdat[rr * 8]);
          if (fold_k) {
            TIn w[8];
            load_vec8(mir, w);
#pragma unroll
            for (int c = 0; c < 8; ++c) rdat[rr * 8 + c] = fold_add(rdat[rr * 8 + c], w[c], odd);
          }
        } else {
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            TIn v = (k < K && col0 + c < a.R) ? src[c] : (TIn)0;
            if (fold_k && col0 + c < a.R) v = fold_add(v, mir[c], odd);
            rdat[rr * 8 + c] = v;
          }
        }
      }
    } else if (!CPLX && FOLD != 1) {
      // data rows in 16-byte chunks: consecutive lanes take consecutive chunks of
      // one row (BK / VW lanes per row), so every load instruction is coalesced
      constexpr int VW = 16 / (int)sizeof(TIn), TPR = BK / VW, RPS = NT / TPR, NS = BM / RPS;
      const int c = t % TPR, rg = t / TPR;
      const int64_t kk = k0 + VW * c;
      const bool vec = base_aligned && (a.n % VW) == 0 && (koff % VW) == 0 && kk + VW <= K;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int64_t m = m0 + RPS * s + rg;
        const TIn* src = X + m * a.n + koff + kk;
        if (m < a.M && vec) {
          load_vec16(src, &rdat[VW * s]);
        } else {
#pragma unroll
          for (int e = 0; e < VW; ++e) rdat[VW * s + e] = (m < a.M && kk + e < K) ? src[e] : (TIn)0;
        }
      }
    } else if (!CPLX) {
      const int row = t >> 1, half = t & 1;
      const int64_t m = m0 + row;
      const int64_t kb = k0 + 32 * half;
      const TIn* rowp = X + m * a.n;
      const TIn* src = rowp + koff + kb;
      const int64_t VW = 16 / (int64_t)sizeof(TIn);
      if (base_aligned && m < a.M && kb + 32 <= K && (a.n % VW) == 0 && (koff % VW) == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) load_vec8(src + 8 * c, &rdat[8 * c]);
        if (FOLD == 1 && kb + 32 <= a.hh) {
          // mirror elements n-1-kb-31 .. n-1-kb, reversed
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            TIn w[8];
            load_vec8(rowp + (a.n - 32 - kb) + 8 * c, w);
#pragma unroll
            for (int e = 0; e < 8; ++e) rdat[31 - 8 * c - e] = fold_add(rdat[31 - 8 * c - e], w[e], odd);
          }
        } else if (FOLD == 1) {
#pragma unroll
          for (int c = 0; c < 32; ++c)
            if (kb + c < a.hh) rdat[c] = fold_add(rdat[c], rowp[a.n - 1 - kb - c], odd);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 32; ++c) {
          TIn v = (m < a.M && kb + c < K) ? src[c] : (TIn)0;
          if (FOLD == 1 && m < a.M && kb + c < a.hh) v = fold_add(v, rowp[a.n - 1 - kb - c], odd);
          rdat[c] = v;
        }
      }
    } else {
      // rows 2p (re) and 2p+1 (im): p = pl, 16 consecutive k, both components
      const int pl = t >> 2, quarter = t & 3;
      const int64_t pp = (m0 >> 1) + pl;
      const int64_t kb = k0 + 16 * quarter;
      const TIn* rowp = X + ((pp * a.n) << 1);
      const TIn* src = rowp + ((koff + kb) << 1);
      // 2n values per row: 16-byte alignment of every row start needs 2n % VW == 0
      const int64_t VW = 16 / (int64_t)sizeof(TIn);
      if (base_aligned && pp < a.P && kb + 16 <= K && ((2 * a.n) % VW) == 0 && ((2 * koff) % VW) == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) load_vec8(src + 8 * c, &rdat[8 * c]);
        if (FOLD == 1 && kb + 16 <= a.hh) {
          // complex elements n-1-kb-15 .. n-1-kb, reversed
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            TIn w[8];
            load_vec8(rowp + ((a.n - 16 - kb) << 1) + 8 * c, w);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int d = 15 - 4 * c - e;  // complex element within this thread's 16
              rdat[2 * d] = fold_add(rdat[2 * d], w[2 * e], odd);
              rdat[2 * d + 1] = fold_add(rdat[2 * d + 1], w[2 * e + 1], odd);
            }
          }
        } else if (FOLD == 1) {
#pragma unroll
          for (int d = 0; d < 16; ++d)
            if (kb + d < a.hh) {
              const int64_t mk = (a.n - 1 - kb - d) << 1;
              rdat[2 * d] = fold_add(rdat[2 * d], rowp[mk], odd);
              rdat[2 * d + 1] = fold_add(rdat[2 * d + 1], rowp[mk + 1], odd);
            }
        }
      } else {
#pragma unroll
        for (int c = 0; c < 32; ++c) {
          const int64_t k = kb + (c >> 1);
          TIn v = (pp < a.P && k < K) ? src[c] : (TIn)0;
          if (FOLD == 1 && pp < a.P && k < a.hh) v = fold_add(v, rowp[((a.n - 1 - k) << 1) + (c & 1)], odd);
          rdat[c] = v;
        }
      }
    }
  };
  auto store_tile = [&](int buf) {
    uint16_t(*Res)[LDK] = ROWS ? Bs[buf] : As[buf];
    {
      const int row = t >> 1, half = t & 1;
      uint4* dst = (uint4*)&Res[row][32 * half];
      dst[0] = rres0;
      dst[1] = rres1;
      dst[2] = rres2;
      dst[3] = rres3;
    }
    if (!ROWS && coal_cols) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {  // k = 2c + (t >> 7) with c = 4q + r lies in chunk q
        uint16_t* dst = &Bs[buf][t & 127][swz8(t & 127, q) + (t >> 7)];
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[2 * r] = to_bf16(rdat[4 * q + r]);
      }
    } else if (ROWS && coal_rows) {
#pragma unroll
      for (int c = 0; c < 32; ++c) As[buf][4 * c + (t >> 6)][t & 63] = to_bf16(rdat[c]);
    } else if (!ROWS) {
      // transpose: Bs[col][4 kq .. 4 kq + 3] for each of 8 columns
      const int oc = t & 15, kq = t >> 4;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        uint32_t lo = (uint32_t)to_bf16(rdat[0 * 8 + c]) | ((uint32_t)to_bf16(rdat[1 * 8 + c]) << 16);
        uint32_t hi = (uint32_t)to_bf16(rdat[2 * 8 + c]) | ((uint32_t)to_bf16(rdat[3 * 8 + c]) << 16);
        const int row = 8 * oc + c;
        *(uint2*)&Bs[buf][row][swz8(row, kq >> 1) + 4 * (kq & 1)] = make_uint2(lo, hi);
      }
    } else if (!CPLX && FOLD != 1) {
      constexpr int VW = 16 / (int)sizeof(TIn), TPR = BK / VW, RPS = NT / TPR, NS = BM / RPS;
      const int c = t % TPR, rg = t / TPR;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        uint16_t* dst = &As[buf][RPS * s + rg][VW * c];
        uint32_t w[VW / 2];
#pragma unroll
        for (int e = 0; e < VW / 2; ++e)
          w[e] = (uint32_t)to_bf16(rdat[VW * s + 2 * e]) | ((uint32_t)to_bf16(rdat[VW * s + 2 * e + 1]) << 16);
        if constexpr (VW == 2) *(uint32_t*)dst = w[0];
        else if constexpr (VW == 4) *(uint2*)dst = make_uint2(w[0], w[1]);
        else *(uint4*)dst = make_uint4(w[0], w[1], w[2], w[3]);
      }
    } else if (!CPLX) {
      const int row = t >> 1, half = t & 1;
      uint32_t w[16];
#pragma unroll
      for (int c = 0; c < 16; ++c)
        w[c] = (uint32_t)to_bf16(rdat[2 * c]) | ((uint32_t)to_bf16(rdat[2 * c + 1]) << 16);
      uint4* dst = (uint4*)&As[buf][row][32 * half];
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
    } else {
      const int pl = t >> 2, quarter = t & 3;
      uint32_t wr[8], wi[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        // rdat holds (re, im) pairs for k = 2c and 2c + 1
        wr[c] = (uint32_t)to_bf16(rdat[4 * c]) | ((uint32_t)to_bf16(rdat[4 * c + 2]) << 16);
        wi[c] = (uint32_t)to_bf16(rdat[4 * c + 1]) | ((uint32_t)to_bf16(rdat[4 * c + 3]) << 16);
      }
      uint4* dr = (uint4*)&As[buf][2 * pl][16 * quarter];
      uint4* di = (uint4*)&As[buf][2 * pl + 1][16 * quarter];
      dr[0] = make_uint4(wr[0], wr[1], wr[2], wr[3]);
      dr[1] = make_uint4(wr[4], wr[5], wr[6], wr[7]);
      di[0] = make_uint4(wi[0], wi[1], wi[2], wi[3]);
      di[1] = make_uint4(wi[4], wi[5], wi[6], wi[7]);
    }
  };

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0, 0, 0, 0};

  const int64_t nk = (K + BK - 1) / BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nk) load_tile((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
      s8 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = *(const s8*)&As[cur][wm * 64 + i * 16 + lr][ks * 32 + 8 * lg];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = wn * 64 + j * 16 + lr;
        bv[j] = *(const s8*)&Bs[cur][row][ROWS ? ks * 32 + 8 * lg : swz8(row, 4 * ks + lg)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile(cur ^ 1);
    __syncthreads();
  }

  TOut* Y = (TOut*)a.Y;
  // BF16 output of a plain (or scaling, real) pass with rows of a multiple of 8
  // outputs: the tile is staged in LDS as BF16 and written back with one 16-byte
  // store per 8 consecutive outputs (the MFMA layout alone gives 2-byte stores,
  // 16 per row segment; for other row lengths the direct stores are faster)
  constexpr bool kStage = !CPLX && FOLD == 0 && EPI != (int)Epi::Exp && std::is_same<TOut, uint16_t>::value;
  if (kStage && ((((uintptr_t)a.Y) & 15) == 0) && ((ROWS ? a.n : a.R) % 8) == 0) {
    constexpr int LT = BN + 8;  // staged row length (elements): 272 B, 16-byte aligned rows
    static_assert(BM * LT <= 2 * BM * LDK, "staged tile must fit in the A buffers");
    uint16_t* Ts = &As[0][0][0];
    double tr[4] = {0.0, 0.0, 0.0, 0.0};
    if (EPI == (int)Epi::Inv) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = n0 + wn * 64 + j * 16 + lr;
        tr[j] = col < a.R ? a.Lr[col] : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double tm[4] = {0.0, 0.0, 0.0, 0.0};
      if (EPI == (int)Epi::Inv) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = m0 + wm * 64 + i * 16 + out_row<float>(lane, r);
          tm[r] = m < a.n ? a.lam[m] + a.Lp[p] : 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
          const int ml = wm * 64 + i * 16 + out_row<float>(lane, r), cl = wn * 64 + j * 16 + lr;
          const uint32_t w = stage_pair<EPI>(acc[i][j][r], acc[i][j][r + 1], tm[r] + tr[j] + a.shift,
                                             tm[r + 1] + tr[j] + a.shift);
          Ts[ml * LT + cl] = (uint16_t)w;  // rows ml and ml + 1 (out_row of r and r + 1)
          Ts[(ml + 1) * LT + cl] = (uint16_t)(w >> 16);
        }
    }
    __syncthreads();
    const int64_t rowlen = ROWS ? a.n : a.R;
#pragma unroll
    for (int q = 0; q < (BM * BN / 8) / NT; ++q) {
      const int idx = q * NT + t, lrow = idx >> 4, ch = idx & 15;
      const int64_t mg = m0 + lrow, cg = n0 + 8 * ch;
      if (ROWS ? mg >= a.M : mg >= a.n) continue;
      const int64_t base = ROWS ? mg * a.n : (p * a.n + mg) * a.R;
      const uint16_t* src = &Ts[lrow * LT + 8 * ch];
      if (cg + 8 <= rowlen) {
        *(uint4*)(Y + base + cg) = *(const uint4*)src;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (cg + e < rowlen) Y[base + cg + e] = src[e];
      }
    }
    return;
  }
  if constexpr (EPI != 0 && !ROWS) {
    // Scaling pass: the table entries of this thread's rows and columns are read
    // once (the stores below may alias the tables as far as the compiler can
    // tell); same arithmetic and order as store_cols.
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
        const int64_t m = m0 + wm * 64 + i * 16 + out_row<float>(lane, r);
        int64_t dst = m;
        bool ok = m < a.n;
        if (FOLD) {
          const int64_t cnt = FOLD == 1 ? (odd ? a.no : a.ne) : (odd ? a.hh : a.hh + a.cc);
          ok = m < cnt;
          dst = FOLD == 1 ? (odd ? a.ne + m : m) : (odd ? a.n - 1 - m : m);
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
        const int64_t m = m0 + wm * 64 + i * 16 + out_row<float>(lane, r);
        const int64_t col = n0 + wn * 64 + j * 16 + lr;
        double v = (double)acc[i][j][r];
        double partner = 0.0;
        if (EPI == (int)Epi::Exp) partner = __shfl_xor(v, 1);
        if (FOLD) {
          const int64_t loc = ROWS ? col : m;
          const int64_t cnt = FOLD == 1 ? (odd ? a.no : a.ne) : (odd ? a.hh : a.hh + a.cc);
          if (loc >= cnt) continue;
          const int64_t dst = FOLD == 1 ? (odd ? a.ne + loc : loc) : (odd ? a.n - 1 - loc : loc);
          if (ROWS) store_rows<TOut, CPLX>(a, Y, m, dst, v);
          else store_cols<TOut, CPLX, EPI>(a, Y, p, dst, col, v, partner);
        } else if (ROWS) {
          store_rows<TOut, CPLX>(a, Y, m, col, v);
        } else {
          store_cols<TOut, CPLX, EPI>(a, Y, p, m, col, v, partner);
        }
      }
}

// ---- 256 x 256 output tiles (real BF16 data, no fold, 16-byte aligned rows) ----
// With 128 x 128 tiles every operand element is fetched from L2 once per
// tile it feeds: 2 M N K (1/BM + 1/BN) bytes per pass, 32 GB at 1000^3, which
// the L2-to-CU path cannot deliver at the rate the matrix cores consume it.
// Doubling both tile sides halves that traffic.  A block of 512 threads (8
// waves as 2 x 4, each a 128 x 64 sub-tile of 8 x 4 MFMA blocks, 128 FP32
// accumulators per lane) owns one CU's LDS (two stages of 256 x 64 BF16 for
// each operand, 144 KB).  K is consumed in the same order as by k_mode_bf16
// (64-wide k-tiles, two 32-wide MFMA steps each), so both kernels give
// bitwise equal results.
constexpr int BB = 256, NTB = 512;

// F3: forward half-extent pass on data folded beforehand (s_i at row or
// column i < h + c, d_i at n - 1 - i; see modeprod.hip): tiles [0, te) of the
// output dimension take the even modes from the first h + c entries against
// Fe, the others the odd modes from the last h entries against Fr (Fo with its
// rows reversed), so each tile runs one half-size product.  Row passes then
// move data and outputs in 8-byte pieces (the odd half starts at h, a multiple
// of 4 but not always of 8).
// ACC (FP64 output): the pass adds its result to Y instead of storing it.
// NU (row pass with FP64 output, the last pass of a BF16 apply whose other
// passes all ran over half extents): the data are folded along the NU slower
// axes (u_i at i, w_i at n - 1 - i on each), and the tile's rows are gathered
// by reflection orbits, the 2^NU rows of an orbit consecutive, so that one
// lane holds a whole orbit of outputs (its four accumulator rows) and unfolds
// them, x_i = u_i + w_i and x_{n-1-i} = u_i - w_i along each axis, before
// the FP64 stores.
struct UGeom {
  int64_t na = 0;  // extent of the slowest axis
  int64_t nb = 1;  // NU = 2: extent of the next axis
  int64_t hb = 1;  // NU = 2: nb / 2
  int64_t no = 0;  // orbits: (na / 2) (nb / 2)
};
template <int NU>
__device__ __forceinline__ int64_t unf_row(const UGeom& u, int64_t o, int b) {
  if constexpr (NU == 1) {
    return b ? u.na - 1 - o : o;
  } else {
    const int64_t i0 = o / u.hb, i1 = o - i0 * u.hb;
    return ((b & 2) ? u.na - 1 - i0 : i0) * u.nb + ((b & 1) ? u.nb - 1 - i1 : i1);
  }
}

template <bool ROWS, int EPI, typename TOut, bool F3, bool ACC = false, int NU = 0>
__global__ __launch_bounds__(NTB, 1) void k_mode_bf16_big(KArgs a, UGeom u) {
  static_assert(NU == 0 || (ROWS && !F3 && EPI == 0 && std::is_same<TOut, double>::value),
                "orbit-gathered rows: row passes with FP64 output only");
  if (a.skip && *a.skip) return;
  __shared__ __attribute__((aligned(16))) uint16_t smem_big[4 * BB * LDK];
  typedef uint16_t Row[LDK];
  Row* As = (Row*)smem_big;                  // [2][BB] rows
  Row* Bs = As + 2 * BB;                     // [2][BB] rows

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;   // 128-row x 64-column wave tile
  const int lr = lane & 15, lg = lane >> 4;

  const int64_t lb = xcd_logical_block(blockIdx.x, a.nblocks);
  int64_t p = 0, mtile, ntile;
  if (ROWS) {
    mtile = lb / a.nt;
    ntile = lb % a.nt;
  } else {
    mtile = lb % a.mt;
    const int64_t rest = lb / a.mt;
    ntile = rest % a.nt;
    p = rest / a.nt;
  }
  bool odd = false;
  int64_t K = a.n, koff = 0, ldS = a.ld;
  const uint16_t* S = (const uint16_t*)a.S;
  if (F3) {
    int64_t& split = ROWS ? ntile : mtile;
    odd = split >= a.te;
    if (odd) split -= a.te;
    const int64_t sh = (a.hh + a.cc) & 7;  // the odd half read from n - h - sh (a multiple of 8)
    K = odd ? a.hh + sh : a.hh + a.cc;
    koff = odd ? a.hh + a.cc - sh : 0;
    S = (const uint16_t*)(odd ? a.So : a.Se);
    ldS = a.fld;
  }
  const int64_t m0 = mtile * BB, n0 = ntile * BB;
  const uint16_t* X = (const uint16_t*)a.X;
  const int64_t f0 = ROWS ? n0 : m0;  // first factor row of this tile
  // NU: the data rows this thread loads (tile row 64 s2 + t / 8 is member
  // (row & (2^NU - 1)) of orbit mtile 256 / 2^NU + row / 2^NU; orbits past the
  // last are clamped to it, and their outputs are not stored)
  int64_t urow[4] = {0, 0, 0, 0};
  if constexpr (NU > 0) {
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int rho = 64 * s2 + (t >> 3);
      int64_t o = mtile * (BB >> NU) + (rho >> NU);
      o = o < u.no ? o : u.no - 1;
      urow[s2] = unf_row<NU>(u, o, rho & ((1 << NU) - 1));
    }
  }

  // One k-tile on its way to LDS: 64 bytes of the factor tile and 64 bytes of
  // the data tile per thread, as raw 16-byte chunks.
  // Every load is unconditional (no branches, so the compiler can wait for
  // exactly the loads each step needs): out-of-range indices are clamped to
  // the last row or column.  The duplicates they fetch are finite values that
  // meet only zero factor entries (k past n: the factor's zero padding) or feed
  // outputs that are never stored (factor rows past the stored padding, data
  // rows or columns past the grid).
  auto load_factor = [&](int64_t k0, u32x4 (&rf)[4]) __attribute__((always_inline)) {
    const int row = t >> 1, half = t & 1;
    const int64_t fr = f0 + row < ldS ? f0 + row : ldS - 1;
    const u32x4* src = (const u32x4*)(S + fr * ldS + k0 + 32 * half);
#pragma unroll
    for (int i = 0; i < 4; ++i) rf[i] = src[i];
  };
  auto load_data = [&](int64_t k0, u32x4 (&rx)[4]) __attribute__((always_inline)) {
    if (!ROWS) {
      // rows k0 + 4 kq .. + 3 of X[p], columns n0 + 8 oc .. + 7 (32 lanes per row: coalesced)
      const int oc = t & 31, kq = t >> 5;
      const int64_t col0 = n0 + 8 * oc < a.R ? n0 + 8 * oc : 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t k = k0 + 4 * kq + r < K ? k0 + 4 * kq + r : K - 1;
        rx[r] = *(const u32x4*)(X + (p * a.n + koff + k) * a.R + col0);
      }
    } else {
      // rows m0 + 64 s + rg, k-chunk c of 8 (8 lanes per row: coalesced); with
      // F3 the chunks of a half start at koff, a multiple of 8, and a chunk
      // may reach past K into entries that meet zero factor columns
      const int c = t & 7, rg = t >> 3;
      const int64_t kk = koff + (k0 + 8 * c < K ? k0 + 8 * c : (K - 1) / 8 * 8);
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int64_t m = NU ? urow[s2] : (m0 + 64 * s2 + rg < a.M ? m0 + 64 * s2 + rg : a.M - 1);
        rx[s2] = *(const u32x4*)(X + m * a.n + kk);
      }
    }
  };
  auto store_factor = [&](int buf, const u32x4 (&rf)[4]) __attribute__((always_inline)) {
    Row* Fs = (ROWS ? Bs : As) + buf * BB;
    const int row = t >> 1, half = t & 1;
    u32x4* dst = (u32x4*)&Fs[row][32 * half];
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = rf[i];
  };
  auto store_data = [&](int buf, const u32x4 (&rx)[4]) __attribute__((always_inline)) {
    if (!ROWS) {
      // transpose 4 k x 8 columns into Bs[col][k], k-chunks swizzled by row group
      const int oc = t & 31, kq = t >> 5;
      Row* D = Bs + buf * BB;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int sh = 16 * (c & 1);
        const uint32_t v0 = (rx[0][c >> 1] >> sh) & 0xffffu, v1 = (rx[1][c >> 1] >> sh) & 0xffffu;
        const uint32_t v2 = (rx[2][c >> 1] >> sh) & 0xffffu, v3 = (rx[3][c >> 1] >> sh) & 0xffffu;
        const int row = 8 * oc + c;
        *(uint2*)&D[row][swz8(row, kq >> 1) + 4 * (kq & 1)] = make_uint2(v0 | (v1 << 16), v2 | (v3 << 16));
      }
    } else {
      const int c = t & 7, rg = t >> 3;
      Row* D = As + buf * BB;
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) *(u32x4*)&D[64 * s2 + rg][8 * c] = rx[s2];
    }
  };

  f4 acc[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0, 0, 0, 0};

  const int64_t nk = (K + BK - 1) / BK;
  auto compute = [&](int cur) __attribute__((always_inline)) {
    const Row* Ac = As + cur * BB;
    const Row* Bc = Bs + cur * BB;
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
      s8 bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = wn * 64 + j * 16 + lr;
        bv[j] = *(const s8*)&Bc[row][ROWS ? ks * 32 + 8 * lg : swz8(row, 4 * ks + lg)];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const s8 av = *(const s8*)&Ac[wm * 128 + i * 16 + lr][ks * 32 + 8 * lg];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  // The data tile (from HBM) is requested two stages ahead: the one stored to
  // LDS at the end of stage kt was requested at the start of stage kt - 1, so
  // it has two compute phases (about 2 x 2048 MFMA cycles per SIMD) to arrive;
  // the factor tile (resident in L2) one stage ahead.
  u32x4 rf[4], rx0[4];
  load_factor(0, rf);
  load_data(0, rx0);
  store_factor(0, rf);
  store_data(0, rx0);
  if constexpr (ROWS) {
    // Row passes keep the data tile two stages ahead in registers (the one
    // stored at the end of stage kt was requested at the start of stage kt - 1)
    // and the factor tile, resident in L2, one stage ahead; the barriers order
    // LDS only, so those loads stay in flight across them.  The number of
    // k-tiles is made even: with nk odd the extra tile [64 nk, 64 nk + 64)
    // still lies inside the stored factor (whose extent ld is a multiple of
    // 128) and is all zero padding there, so it adds only zero products; the
    // loop body then runs without branches (past the last k-tile the stages
    // re-request the last tile and fill the idle LDS buffer, which nothing
    // reads afterwards), and the compiler waits for exactly the loads each
    // step needs.  (The column passes' transposing stores need the registers
    // of the second stage.)
    const int64_t nke = (nk + 1) & ~(int64_t)1;
    u32x4 rx1[4];
    load_data(BK, rx0);
    lds_barrier();
    auto stage = [&](int64_t kt, u32x4 (&xa)[4], u32x4 (&xb)[4]) __attribute__((always_inline)) {
      const int cur = (int)(kt & 1);
      // the factor first: the loads complete in order, so waiting for it at the
      // end of the stage does not wait for the data requested for stage kt + 2
      load_factor((kt + 1 < nke ? kt + 1 : nke - 1) * BK, rf);
      load_data((kt + 2 < nke ? kt + 2 : nke - 1) * BK, xb);
      compute(cur);
      store_factor(cur ^ 1, rf);
      store_data(cur ^ 1, xa);
      lds_barrier();
    };
    for (int64_t kt = 0; kt < nke; kt += 2) {
      stage(kt, rx0, rx1);
      stage(kt + 1, rx1, rx0);
    }
  } else {
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
      const int cur = (int)(kt & 1);
      if (kt + 1 < nk) {
        load_factor((kt + 1) * BK, rf);
        load_data((kt + 1) * BK, rx0);
      }
      compute(cur);
      if (kt + 1 < nk) {
        store_factor(cur ^ 1, rf);
        store_data(cur ^ 1, rx0);
      }
      __syncthreads();
    }
  }

  TOut* Y = (TOut*)a.Y;
  static_assert(!F3 || std::is_same<TOut, uint16_t>::value, "folded passes write BF16");
  // outputs of this tile's half: the first `cnt` of the split dimension are
  // valid and land at `base` on (F3 odd tiles: after the ne even modes)
  const int64_t cnt = F3 ? (odd ? a.no : a.ne) : a.n;
  const int64_t base = F3 && odd ? a.ne : 0;
  const int64_t rowlen = ROWS ? cnt : a.R;   // outputs per output row (within the half)
  const int64_t nrows = ROWS ? a.M : cnt;    // output rows (within the half)
  if constexpr (std::is_same<TOut, uint16_t>::value) {
    // stage the BF16 tile in LDS (rows of 264 elements: 528 B) and write 16 bytes per 8 outputs
    constexpr int LT = BB + 8;
    static_assert(BB * LT <= 4 * BB * LDK, "staged tile must fit in the operand buffers");
    uint16_t* Ts = smem_big;
    double tr[4] = {0.0, 0.0, 0.0, 0.0};
    const double* tmS = nullptr;
    if constexpr (EPI == (int)Epi::Inv) {
      // the row parts lam + Lp of the denominators of the tile's 256 rows: one
      // load per thread into LDS behind the staged tile (the main loop's last
      // barrier left LDS idle), instead of each lane loading its 32 just
      // before their use, one dependent round trip per 16-row block
      static_assert(BB * LT * sizeof(uint16_t) + BB * sizeof(double) <= 4 * BB * LDK * sizeof(uint16_t),
                    "denominator table must fit behind the staged tile");
      double* tmw = (double*)(smem_big + BB * LT);
      if (t < BB) {
        const int64_t m = m0 + t;
        tmw[t] = m < cnt ? a.lam[base + m] + a.Lp[p] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = n0 + wn * 64 + j * 16 + lr;
        tr[j] = col < a.R ? a.Lr[col] : 0.0;
      }
      __syncthreads();
      tmS = tmw;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      double tm[4] = {0.0, 0.0, 0.0, 0.0};
      if constexpr (EPI == (int)Epi::Inv) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tm[r] = tmS[wm * 128 + i * 16 + out_row<float>(lane, r)];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
          const int ml = wm * 128 + i * 16 + out_row<float>(lane, r), cl = wn * 64 + j * 16 + lr;
          const uint32_t w = stage_pair<EPI>(acc[i][j][r], acc[i][j][r + 1], tm[r] + tr[j] + a.shift,
                                             tm[r + 1] + tr[j] + a.shift);
          Ts[ml * LT + cl] = (uint16_t)w;  // rows ml and ml + 1 (out_row of r and r + 1)
          Ts[(ml + 1) * LT + cl] = (uint16_t)(w >> 16);
        }
    }
    __syncthreads();
    if (ROWS && F3) {
      // 8 bytes per 4 outputs: the odd half starts at column ne (a multiple of 4)
#pragma unroll
      for (int q = 0; q < (BB * BB / 4) / NTB; ++q) {
        const int idx = q * NTB + t, lrow = idx >> 6, ch = idx & 63;
        const int64_t mg = m0 + lrow, cg = n0 + 4 * ch;
        if (mg >= nrows || cg >= rowlen) continue;
        *(uint2*)(Y + mg * a.n + base + cg) = *(const uint2*)&Ts[lrow * LT + 4 * ch];
      }
    } else {
#pragma unroll
      for (int q = 0; q < (BB * BB / 8) / NTB; ++q) {
        const int idx = q * NTB + t, lrow = idx >> 5, ch = idx & 31;
        const int64_t mg = m0 + lrow, cg = n0 + 8 * ch;
        if (mg >= nrows || cg >= rowlen) continue;
        const int64_t off = ROWS ? mg * a.n : (p * a.n + base + mg) * a.R;
        *(uint4*)(Y + off + cg) = *(const uint4*)&Ts[lrow * LT + 8 * ch];
      }
    }
  } else if constexpr (NU > 0) {
    // rows 4 lg .. 4 lg + 3 of each 16-row block are the lane's accumulator
    // rows r = 0..3: one orbit (NU = 2) or two (NU = 1)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int rho = wm * 128 + i * 16 + 4 * lg;
      // ACC: the block's 16 old values are loaded together before its stores (a
      // load after a store waits for it: one load and add per store would make
      // every element a round trip)
      double yo[4][4];
      if constexpr (ACC) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t col = n0 + wn * 64 + j * 16 + lr;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t o = mtile * (BB >> NU) + ((rho + r) >> NU);
            yo[j][r] = col < a.n && o < u.no ? Y[unf_row<NU>(u, o, (rho + r) & ((1 << NU) - 1)) * a.n + col] : 0.0;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t col = n0 + wn * 64 + j * 16 + lr;
        if (col >= a.n) continue;
        double x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = (double)acc[i][j][r];
#pragma unroll
        for (int q = 0; q < 4; q += 2) {  // along the faster unfolded axis
          const double s0 = x[q] + x[q + 1], d0 = x[q] - x[q + 1];
          x[q] = s0;
          x[q + 1] = d0;
        }
        if constexpr (NU == 2) {
#pragma unroll
          for (int q = 0; q < 2; ++q) {  // along the slowest axis
            const double s0 = x[q] + x[q + 2], d0 = x[q] - x[q + 2];
            x[q] = s0;
            x[q + 2] = d0;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t o = mtile * (BB >> NU) + ((rho + r) >> NU);
          if (o >= u.no) continue;
          double* y = Y + unf_row<NU>(u, o, (rho + r) & ((1 << NU) - 1)) * a.n + col;
          if constexpr (ACC) *y = yo[j][r] + x[r];
          else *y = x[r];
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + wm * 128 + i * 16 + out_row<float>(lane, r);
        if (m >= nrows) continue;
        const double tm = EPI == (int)Epi::Inv ? a.lam[m] + a.Lp[p] : 0.0;
        // ACC: the row's four old values are loaded before its stores
        double yo[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (ACC) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wn * 64 + j * 16 + lr;
            if (col < rowlen) yo[j] = Y[(ROWS ? m * a.n : (p * a.n + m) * a.R) + col];
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t col = n0 + wn * 64 + j * 16 + lr;
          if (col >= rowlen) continue;
          double v = (double)acc[i][j][r];
          if (EPI == (int)Epi::Inv) v = v / (tm + a.Lr[col] + a.shift);
          TOut* y = Y + (ROWS ? m * a.n : (p * a.n + m) * a.R) + col;
          if constexpr (ACC) *y = yo[j] + v;
          else *y = cvt_out<TOut>(v);
        }
      }
    }
  }
}

// Whether a pass runs on the 256 x 256 tiles: real BF16 input, no fold, rows
// whose length is a multiple of 8 (every 16-byte chunk aligned) and n >= 192.
// Chosen by default when it pads the factor's extent by at most 10 % more than
// 128-wide tiles do and still gives every compute unit a tile.
template <typename TIn>
bool bf16_big_ok(const KArgs& a, const PassArgs& pa, int fold) {
  if (!std::is_same<TIn, uint16_t>::value || pa.cplx || fold || pa.epi == Epi::Exp) return false;
  if (a.rows && pa.epi != Epi::None) return false;  // the row instance has no scaling epilogue
  if (pa.bf16_tile == 128) return false;
  if ((((uintptr_t)a.X) & 15) != 0 || (((uintptr_t)a.Y) & 15) != 0) return false;
  if ((a.rows ? a.n : a.R) % 8 != 0 || a.n < 192) return false;
  if (pa.bf16_tile == 256) return true;
  const int64_t pad256 = (a.n + BB - 1) / BB * BB, pad128 = (a.n + BM - 1) / BM * BM;
  if (pad256 * 10 > pad128 * 11) return false;
  const int64_t mt = (a.M + BB - 1) / BB, nt = (a.N + BB - 1) / BB;
  return mt * nt * (a.rows ? 1 : pa.P) >= 256;
}

// Whether a forward pass on data folded beforehand runs on the 256 x 256 tiles
// (the only BF16 kernel with that input layout): real BF16 data in and out,
// 16-byte aligned buffers, a reflection-symmetric axis of n >= 192, no
// scaling epilogue on a row pass, and rows of a multiple of 8 values; a row
// pass also needs n % 8 == 0, so that both halves start on 4-value boundaries.
// A backward pass runs the same kernel on the spectral [even | odd] order with
// the backward half factors (Be, and Bo with its physical index reversed): it
// leaves u_i at i and w_i at n - 1 - i, the folded layout, for the unfolding
// last pass.
bool fold3_ok(const KArgs& a, const PassArgs& pa) {
  const AxisFactor* F = pa.fac;
  if (pa.tin != DT::BF16 || pa.tout != DT::BF16 || pa.cplx || pa.epi == Epi::Exp) return false;
  if (!pa.forward && pa.epi != Epi::None) return false;
  if (!F->fold || pa.bf16_tile == 128 || a.n < 192) return false;
  if (pa.forward ? (!F->Fe16w || !F->Fr16w) : (!F->Be16w || !F->Br16w)) return false;
  if ((((uintptr_t)a.X) & 15) != 0 || (((uintptr_t)a.Y) & 15) != 0) return false;
  if (a.rows) return pa.epi == Epi::None && a.n % 8 == 0;
  return a.R % 8 == 0;
}

template <typename TOut>
hipError_t launch_bf16_big(KArgs a, const PassArgs& pa, hipStream_t st) {
  a.mt = (a.M + BB - 1) / BB;
  a.nt = (a.N + BB - 1) / BB;
  a.nblocks = a.mt * a.nt * (a.rows ? 1 : pa.P);
  if (a.nblocks <= 0) return hipSuccess;
  if (a.nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)a.nblocks), block(NTB);
  if (pa.accumulate) {
    if (!std::is_same<TOut, double>::value || pa.epi != Epi::None) return hipErrorInvalidValue;
    if (a.rows) hipLaunchKernelGGL((k_mode_bf16_big<true, 0, TOut, false, true>), grid, block, 0, st, a, UGeom{});
    else hipLaunchKernelGGL((k_mode_bf16_big<false, 0, TOut, false, true>), grid, block, 0, st, a, UGeom{});
    return hipGetLastError();
  }
  if (a.rows) {
    hipLaunchKernelGGL((k_mode_bf16_big<true, 0, TOut, false>), grid, block, 0, st, a, UGeom{});
  } else if (pa.epi == Epi::Inv) {
    hipLaunchKernelGGL((k_mode_bf16_big<false, (int)Epi::Inv, TOut, false>), grid, block, 0, st, a, UGeom{});
  } else {
    hipLaunchKernelGGL((k_mode_bf16_big<false, 0, TOut, false>), grid, block, 0, st, a, UGeom{});
  }
  return hipGetLastError();
}

// Forward pass on folded data: the split dimension holds ceil(ne / 256) even
// tiles followed by ceil(no / 256) odd ones.
hipError_t launch_bf16_big_fold3(KArgs a, const PassArgs& pa, hipStream_t st) {
  const AxisFactor* F = pa.fac;
  a.ne = F->ne;
  a.no = F->no;
  a.hh = F->hh;
  a.cc = F->cc;
  a.fld = F->fldw;
  a.Se = pa.forward ? F->Fe16w : F->Be16w;
  a.So = pa.forward ? F->Fr16w : F->Br16w;
  a.te = (F->ne + BB - 1) / BB;
  const int64_t split = a.te + (F->no + BB - 1) / BB;
  if (a.rows) {
    a.mt = (a.M + BB - 1) / BB;
    a.nt = split;
  } else {
    a.mt = split;
    a.nt = (a.N + BB - 1) / BB;
  }
  a.nblocks = a.mt * a.nt * (a.rows ? 1 : pa.P);
  if (a.nblocks <= 0) return hipSuccess;
  if (a.nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)a.nblocks), block(NTB);
  if (a.rows) {
    hipLaunchKernelGGL((k_mode_bf16_big<true, 0, uint16_t, true>), grid, block, 0, st, a, UGeom{});
  } else if (pa.epi == Epi::Inv) {
    hipLaunchKernelGGL((k_mode_bf16_big<false, (int)Epi::Inv, uint16_t, true>), grid, block, 0, st, a, UGeom{});
  } else {
    hipLaunchKernelGGL((k_mode_bf16_big<false, 0, uint16_t, true>), grid, block, 0, st, a, UGeom{});
  }
  return hipGetLastError();
}

// The last pass of a BF16 apply whose other passes all ran over half extents:
// a row pass with FP64 output on data folded along the pa.unf slower axes
// (extents pa.un[0..unf-1], all even), unfolded in registers (k_mode_bf16_big, NU).
bool unfold_ok(const KArgs& a, const PassArgs& pa) {
  if (pa.unf < 1 || pa.unf > 2 || !a.rows || pa.cplx || pa.epi != Epi::None || pa.forward) return false;
  if (pa.tin != DT::BF16 || pa.tout != DT::F64 || pa.bf16_tile == 128 || a.n < 192 || a.n % 8 != 0) return false;
  if ((((uintptr_t)a.X) & 15) != 0 || (((uintptr_t)a.Y) & 15) != 0) return false;
  int64_t M = 1;
  for (int j = 0; j < pa.unf; ++j) {
    if (pa.un[j] < 2 || pa.un[j] % 2 != 0) return false;
    M *= pa.un[j];
  }
  if (M != a.M) return false;
  if (pa.bf16_tile == 256) return true;
  // by default only where the tiles pad the extent as little as 128-wide ones
  // would and every compute unit gets one (as bf16_big_ok)
  const int64_t pad256 = (a.n + BB - 1) / BB * BB, pad128 = (a.n + BM - 1) / BM * BM;
  return pad256 * 10 <= pad128 * 11 && ((a.M + BB - 1) / BB) * ((a.N + BB - 1) / BB) >= 256;
}

hipError_t launch_bf16_big_unfold(KArgs a, const PassArgs& pa, hipStream_t st) {
  UGeom u;
  u.na = pa.un[0];
  u.nb = pa.unf == 2 ? pa.un[1] : 1;
  u.hb = u.nb / 2 > 0 ? u.nb / 2 : 1;
  u.no = (u.na / 2) * (pa.unf == 2 ? u.nb / 2 : 1);
  a.mt = (a.M + BB - 1) / BB;  // 256 / 2^NU orbits of 2^NU rows per tile
  a.nt = (a.N + BB - 1) / BB;
  a.nblocks = a.mt * a.nt;
  if (a.nblocks <= 0) return hipSuccess;
  if (a.nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)a.nblocks), block(NTB);
  if (pa.unf == 2) {
    if (pa.accumulate) hipLaunchKernelGGL((k_mode_bf16_big<true, 0, double, false, true, 2>), grid, block, 0, st, a, u);
    else hipLaunchKernelGGL((k_mode_bf16_big<true, 0, double, false, false, 2>), grid, block, 0, st, a, u);
  } else {
    if (pa.accumulate) hipLaunchKernelGGL((k_mode_bf16_big<true, 0, double, false, true, 1>), grid, block, 0, st, a, u);
    else hipLaunchKernelGGL((k_mode_bf16_big<true, 0, double, false, false, 1>), grid, block, 0, st, a, u);
  }
  return hipGetLastError();
}

// Whether a pass's data allow no 16-byte access at all (then the element-wise,
// coalesced instance runs; such passes do not fold).
template <typename TIn>
bool bf16_coalesced(const KArgs& a, const PassArgs& pa) {
  constexpr int64_t VW = 16 / (int64_t)sizeof(TIn);
  const bool aligned = (((uintptr_t)a.X) & 15) == 0;
  return !pa.cplx && (a.rows ? !(aligned && a.n % VW == 0) : !(aligned && a.R % VW == 0));
}

template <typename TIn, typename TOut, int FOLD>
hipError_t launch_bf16_fold(const KArgs& a, const PassArgs& pa, hipStream_t st) {
  dim3 grid((unsigned)a.nblocks), block(NT);
  constexpr bool kCoal = FOLD == 0;  // element-wise instances exist only without the fold
  const bool coal = kCoal && bf16_coalesced<TIn>(a, pa);
  if (a.rows) {
    if (pa.cplx) hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, true, true, 0, FOLD, false>), grid, block, 0, st, a);
    else if (coal) hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, true, false, 0, FOLD, kCoal>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, true, false, 0, FOLD, false>), grid, block, 0, st, a);
  } else if (pa.epi == Epi::Exp) {
    if (!pa.cplx) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, false, true, (int)Epi::Exp, FOLD, false>), grid, block, 0, st, a);
  } else if (pa.epi == Epi::Inv) {
    if (pa.cplx)
      hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, false, true, (int)Epi::Inv, FOLD, false>), grid, block, 0, st, a);
    else if (coal)
      hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, false, false, (int)Epi::Inv, FOLD, kCoal>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, false, false, (int)Epi::Inv, FOLD, false>), grid, block, 0, st, a);
  } else if (coal) {
    hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, false, false, 0, FOLD, kCoal>), grid, block, 0, st, a);
  } else {
    hipLaunchKernelGGL((k_mode_bf16<TIn, TOut, false, false, 0, FOLD, false>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

// Butterfly of a backward half-extent pass, x_i, x_{n-1-i} <- x_i + x_{n-1-i}, x_i - x_{n-1-i}
// for i < hh over [P][n][R]; BF16 values are combined in FP32 and rounded once.
__device__ __forceinline__ void butterfly(double& x, double& y) {
  const double s = x + y, d = x - y;
  x = s;
  y = d;
}
__device__ __forceinline__ void butterfly(float& x, float& y) {
  const float s = x + y, d = x - y;
  x = s;
  y = d;
}
__device__ __forceinline__ void butterfly(uint16_t& x, uint16_t& y) {
  const float a = bf16_to_f32(x), b = bf16_to_f32(y);
  x = f32_to_bf16(a + b);
  y = f32_to_bf16(a - b);
}
template <typename T>
__global__ __launch_bounds__(256) void k_unfold_any(T* Y, int64_t P, int64_t n, int64_t R, int64_t hh) {
  const int64_t total = P * hh * R;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e % R;
    const int64_t q = e / R;
    const int64_t i = q % hh, p = q / hh;
    T* lo = Y + (p * n + i) * R + r;
    T* hi = Y + (p * n + (n - 1 - i)) * R + r;
    T x = *lo, y = *hi;
    butterfly(x, y);
    *lo = x;
    *hi = y;
  }
}

template <typename TIn, typename TOut>
hipError_t launch_bf16_typed(const PassArgs& pa, hipStream_t st) {
  KArgs a{};
  const AxisFactor* F = pa.fac;
  fill_kargs(pa, a, pa.forward ? (const void*)F->QT16 : (const void*)F->Q16, BM, BN);
  if (pa.fold && pa.deferred) {
    // data folded beforehand: only the 256 x 256 tiles read that layout
    if (!fold3_ok(a, pa)) return hipErrorInvalidValue;
    return launch_bf16_big_fold3(a, pa, st);
  }
  if (pa.unf > 0) {
    if constexpr (std::is_same<TIn, uint16_t>::value && std::is_same<TOut, double>::value) {
      if (!unfold_ok(a, pa)) return hipErrorInvalidValue;
      return launch_bf16_big_unfold(a, pa, st);
    }
    return hipErrorInvalidValue;
  }
  const int fold = (pa.fold && !bf16_coalesced<TIn>(a, pa)) ? (pa.forward ? 1 : 2) : 0;
  if (bf16_big_ok<TIn>(a, pa, fold)) return launch_bf16_big<TOut>(a, pa, st);
  if (pa.accumulate) return hipErrorInvalidValue;  // only the large tiles add into their output
  if (fold) {
    a.ne = F->ne;
    a.no = F->no;
    a.hh = F->hh;
    a.cc = F->cc;
    a.fld = F->fkp;
    a.Se = pa.forward ? (const void*)F->Fe16 : (const void*)F->Be16;
    a.So = pa.forward ? (const void*)F->Fo16 : (const void*)F->Bo16;
    const int64_t me = fold == 1 ? F->ne : F->hh + F->cc, mo = fold == 1 ? F->no : F->hh;
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
  hipError_t e;
  if (fold == 1) e = launch_bf16_fold<TIn, TOut, 1>(a, pa, st);
  else if (fold == 2) e = launch_bf16_fold<TIn, TOut, 2>(a, pa, st);
  else e = launch_bf16_fold<TIn, TOut, 0>(a, pa, st);
  if (e != hipSuccess || fold != 2 || F->hh == 0) return e;
  const int64_t total = pa.P * F->hh * pa.R;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL((k_unfold_any<TOut>), dim3(blocks), dim3(256), 0, st, (TOut*)pa.Y, pa.P, pa.n, pa.R, F->hh);
  return hipGetLastError();
}

// Input of a BF16 apply whose forward passes read folded data: the
// butterfly s_i = x_i + x_{n-1-i} (at i), d_i = x_i - x_{n-1-i} (at n-1-i)
// along every listed axis, taken in FP64 on the FP64 input, each result then
// rounded FP64 -> FP32 -> BF16 as the unfolded input sweep rounds its values.
// One thread per orbit of the reflections (a point with i_a <= n_a - 1 - i_a
// on every listed axis, fastest axis first); an axis on which the point is its
// own mirror (the middle of odd n) leaves it as it is.
template <int NAX>
__global__ __launch_bounds__(256) void k_fold_to_bf16(const double* X, uint16_t* Y, ButterflyArgs a, int64_t total) {
  if (a.skip && *a.skip) return;
  constexpr int NV = 1 << NAX;
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int64_t rest = e, off = 0, stride = 1;
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
    double v[NV];
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
      v[m] = ok ? X[o] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NAX; ++j) {
      if (!act[j]) continue;
#pragma unroll
      for (int m = 0; m < NV; ++m)
        if (!(m & (1 << j))) {
          const double x0 = v[m], x1 = v[m | (1 << j)];
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
      if (ok) Y[o] = cvt_out<uint16_t>(v[m]);
    }
  }
}

// The same with four consecutive points of the fastest axis per thread
// (n_{d-1} % 8 == 0): 16-byte loads, 8-byte stores.  With the fastest axis
// folded (FAST), the group 4q .. 4q + 3 of its lower half pairs with the
// mirror group n - 4 - 4q .. n - 1 - 4q in reverse order; the other listed
// axes (slots 0 .. NAX - 1 of a.ax, the fastest one excluded) as above.
template <int NAX, bool FAST>
__global__ __launch_bounds__(256) void k_fold_to_bf16_x4(const double* X, uint16_t* Y, ButterflyArgs a, int64_t total) {
  if (a.skip && *a.skip) return;
  constexpr int NB = NAX + (FAST ? 1 : 0);  // orbit bits: the slow axes, then the fastest
  constexpr int NV = 1 << NB;
  const int64_t nf = a.n[a.d - 1];
  const int64_t gq = (FAST ? nf / 2 : nf) / 4;  // groups of 4 along the fastest axis
  for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int64_t rest = e / gq;
    const int64_t q = e - rest * gq;
    int64_t off = 4 * q, stride = nf;
    int64_t delta[NB > 0 ? NB : 1];
    bool act[NB > 0 ? NB : 1];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      delta[j] = 0;
      act[j] = false;
    }
    if (FAST) {
      act[NB - 1] = true;
      delta[NB - 1] = nf - 4 - 8 * q;  // start of the mirror group
    }
    for (int k = a.d - 2; k >= 0; --k) {
      int jf = -1;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (a.ax[j] == k) jf = j;
      const int64_t ext = jf >= 0 ? a.n[k] - a.hh[jf] : a.n[k];
      const int64_t qq = rest / ext;
      const int64_t i = rest - qq * ext;
      rest = qq;
      off += i * stride;
#pragma unroll
      for (int j = 0; j < NAX; ++j)
        if (j == jf && i < a.hh[j]) {
          act[j] = true;
          delta[j] = (a.n[k] - 1 - 2 * i) * stride;
        }
      stride *= a.n[k];
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
      double2 lo = make_double2(0.0, 0.0), hi = make_double2(0.0, 0.0);
      if (ok) {
        lo = *(const double2*)(X + o);
        hi = *(const double2*)(X + o + 2);
      }
      v[m][0] = lo.x;
      v[m][1] = lo.y;
      v[m][2] = hi.x;
      v[m][3] = hi.y;
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
    for (int j = 0; j < NAX; ++j) {
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
        *(uint2*)(Y + o) = make_uint2((uint32_t)cvt_out<uint16_t>(v[m][0]) | ((uint32_t)cvt_out<uint16_t>(v[m][1]) << 16),
                                      (uint32_t)cvt_out<uint16_t>(v[m][2]) | ((uint32_t)cvt_out<uint16_t>(v[m][3]) << 16));
    }
  }
}

}  // namespace

hipError_t launch_fold_to_bf16(const ButterflyArgs& a, hipStream_t st) {
  if (a.ncomp != 1) return hipErrorInvalidValue;
  int64_t total = 1;
  for (int k = 0; k < a.d; ++k) {
    int64_t ext = a.n[k];
    for (int j = 0; j < a.nax; ++j)
      if (a.ax[j] == k) ext = a.n[k] - a.hh[j];
    total *= ext;
  }
  if (total <= 0) return hipSuccess;
  const double* X = (const double*)a.X;
  uint16_t* Y = (uint16_t*)a.Y;
  // four points of the fastest axis per thread: 16-byte aligned input rows and
  // groups that never straddle the middle of a folded fastest axis
  const int64_t nf = a.n[a.d - 1];
  int jl = -1;
  for (int j = 0; j < a.nax; ++j)
    if (a.ax[j] == a.d - 1) jl = j;
  if (nf % 8 == 0 && ((((uintptr_t)X) & 15) == 0) && ((((uintptr_t)Y) & 7) == 0)) {
    ButterflyArgs b = a;  // the slow axes in slots 0 .. nslow - 1
    int nslow = 0;
    for (int j = 0; j < a.nax; ++j)
      if (j != jl) {
        b.ax[nslow] = a.ax[j];
        b.hh[nslow] = a.hh[j];
        ++nslow;
      }
    const int64_t units = total / 4;
    const unsigned blocks = (unsigned)std::min<int64_t>((units + 255) / 256, 1 << 20);
#define TS_FOLD_X4(N)                                                                                       \
  if (jl >= 0)                                                                                            \
    hipLaunchKernelGGL((k_fold_to_bf16_x4<N, true>), dim3(blocks), dim3(256), 0, st, X, Y, b, units);    \
  else                                                                                                    \
    hipLaunchKernelGGL((k_fold_to_bf16_x4<N, false>), dim3(blocks), dim3(256), 0, st, X, Y, b, units);
    switch (nslow) {
      case 0:  // only the fastest axis is listed
        hipLaunchKernelGGL((k_fold_to_bf16_x4<0, true>), dim3(blocks), dim3(256), 0, st, X, Y, b, units);
        break;
      case 1: TS_FOLD_X4(1) break;
      case 2: TS_FOLD_X4(2) break;
      case 3: TS_FOLD_X4(3) break;
      default: return hipErrorInvalidValue;
    }
#undef TS_FOLD_X4
    return hipGetLastError();
  }
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  switch (a.nax) {
    case 1: hipLaunchKernelGGL((k_fold_to_bf16<1>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    case 2: hipLaunchKernelGGL((k_fold_to_bf16<2>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    case 3: hipLaunchKernelGGL((k_fold_to_bf16<3>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    case 4: hipLaunchKernelGGL((k_fold_to_bf16<4>), dim3(blocks), dim3(256), 0, st, X, Y, a, total); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool bf16_big_pass_ok(const PassArgs& pa) {
  KArgs a{};
  fill_kargs(pa, a, pa.forward ? (const void*)pa.fac->QT16 : (const void*)pa.fac->Q16, BM, BN);
  return pa.tin == DT::BF16 && bf16_big_ok<uint16_t>(a, pa, 0);
}

bool bf16_fold_pass_ok(const PassArgs& pa) {
  KArgs a{};
  fill_kargs(pa, a, pa.fac->QT16, BM, BN);
  return fold3_ok(a, pa);
}

bool bf16_unfold_pass_ok(const PassArgs& pa) {
  KArgs a{};
  fill_kargs(pa, a, pa.fac->Q16, BM, BN);
  return unfold_ok(a, pa);
}

hipError_t launch_pass_bf16(const PassArgs& pa, hipStream_t st) {
  // intermediates are BF16; the first pass may read FP64/FP32 and the last write FP64/FP32
  const DT i = pa.tin, o = pa.tout;
  if (i == DT::F64 && o == DT::BF16) return launch_bf16_typed<double, uint16_t>(pa, st);
  if (i == DT::F32 && o == DT::BF16) return launch_bf16_typed<float, uint16_t>(pa, st);
  if (i == DT::BF16 && o == DT::BF16) return launch_bf16_typed<uint16_t, uint16_t>(pa, st);
  if (i == DT::BF16 && o == DT::F64) return launch_bf16_typed<uint16_t, double>(pa, st);
  if (i == DT::BF16 && o == DT::F32) return launch_bf16_typed<uint16_t, float>(pa, st);
  if (i == DT::F64 && o == DT::F64) return launch_bf16_typed<double, double>(pa, st);
  if (i == DT::F32 && o == DT::F32) return launch_bf16_typed<float, float>(pa, st);
  return hipErrorInvalidValue;
}

}  // namespace ts
