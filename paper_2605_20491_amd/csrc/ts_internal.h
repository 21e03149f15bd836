// Internal declarations of the MI355X separable tensor-product solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#define TS_MAX_D 12

namespace ts {

// ---- host eigensolver (eig_tridiag.cpp) ----
bool tridiag_eig(int64_t n, const double* diag, const double* off, double* lam, double* Q);

// ---- error plumbing (ts_api.cpp) ----
void set_error(const std::string& msg);

// Tile geometry shared by launchers and the plan's padded matrix storage.
constexpr int kTileF = 128;   // free-index tile width of the MFMA kernels
constexpr int kBandMax = 32;  // widest operator band read by the band loop; wider: MFMA passes
constexpr int64_t kOpPassMinN = 128;  // SEM plans with an axis this long apply the operator as banded MFMA passes
constexpr int kTileK = 32;    // K padding granularity (covers BK of every kernel)

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Per-axis eigen-factors of one distinct axis operator on the device.  A pass
// computes y_j = sum_i W[i][j] x_i with W stored k-major and zero-padded to
// [kpad][ld], so an MFMA tile of either operand role reads whole padded rows:
//   Q  : forward  W = (T^{-1})^T   (FD: W[i][j] = Q[i][j])
//   QT : backward W = T^T          (FD: W[i][j] = Q[j][i])
// For Q^k SEM T = M^{-1/2} Q; a plan holds these mass-scaled factors for its
// public applies and a second, orthogonal set (T = Q) for the solvers, which
// work with the symmetric operator M^{-1/2} S M^{-1/2} + F.
struct AxisFactor {
  int64_t n = 0, ld = 0, kpad = 0;
  double L = 0;
  std::vector<double> lam_h;  // ascending
  std::vector<double> Q_h;    // row-major n x n, orthonormal eigenvectors of the symmetric form
  double ih2 = 0;             // FD: h^-2, h = 2L/(n+1)
  double* lam = nullptr;      // device [n]
  double* f = nullptr;        // device [n]: the samples f_k(x_j)
  double* Q64 = nullptr;      // device [kpad][ld]
  double* QT64 = nullptr;
  float* Q32 = nullptr;
  float* QT32 = nullptr;
  // BF16 copies for the BF16 passes, whose operands are K-contiguous: QT16 is
  // the transpose of Q (forward), Q16 the transpose of QT (backward)
  uint16_t* Q16 = nullptr;
  uint16_t* QT16 = nullptr;
  double* mass = nullptr;     // device [n]: L^2 quadrature weights (FD: h; SEM: lumped mass)
  // SEM and generic plans: operator band [n][2 bw + 1] (entry (i, i - bw + t); null when
  // bw > kBandMax, the operator then runs as op_pass), M^{1/2} and M^{-1/2}
  int bw = 0;
  double* band = nullptr;
  double* msq = nullptr;
  double* imsq = nullptr;
  std::vector<double> m_h;    // lumped mass
  std::vector<double> x_h;    // grid nodes (interior), ascending
  // Reflection symmetry (f_k(x) = f_k(-x) on a symmetric grid): every
  // eigenvector is even or odd, and the passes on this axis contract half the
  // extent.  The internal spectral order is then [even modes | odd modes]
  // (each ascending), used by lam, lam_int_h and the full factors alike.
  // Half factors, k-major [fkp][fkp]:
  //   Fe / Fo: forward, rows = physical i < h + c (resp. h), columns = even (odd) modes
  //   Be / Bo: backward, rows = even (odd) modes, columns = physical i < h + c (resp. h)
  bool fold = false;
  int64_t ne = 0, no = 0, hh = 0, cc = 0, fkp = 0;
  double *Fe64 = nullptr, *Fo64 = nullptr, *Be64 = nullptr, *Bo64 = nullptr;
  float *Fe32 = nullptr, *Fo32 = nullptr, *Be32 = nullptr, *Bo32 = nullptr;
  // Fr: Fo with its rows reversed (row r is physical i = h - 1 - r), for a
  // forward pass on data folded beforehand, where d_i sits at row n - 1 - i
  double* Fr64 = nullptr;
  float* Fr32 = nullptr;
  // BF16, K-contiguous (transposed) copies of Fe, Fo, Be, Bo for the BF16 passes
  uint16_t *Fe16 = nullptr, *Fo16 = nullptr, *Be16 = nullptr, *Bo16 = nullptr;
  // BF16 forward pass on folded data, [fldw][fldw], K-contiguous: Fe (K from
  // 0), and Fr with its K index shifted by sh = (h + c) % 8 (column k holds
  // Fr row k - sh; the pass reads the odd half from n - h - sh, a multiple of
  // 8, and the sh even entries it takes along meet zero columns)
  uint16_t *Fe16w = nullptr, *Fr16w = nullptr;
  // and of the backward pass that leaves its output folded: Be (K from 0), and
  // Br = Bo with its physical index reversed (row r is i = h - 1 - r, written
  // at n - h + r) and its K index shifted by sh, both [fldw][fldw]
  uint16_t *Be16w = nullptr, *Br16w = nullptr;
  int64_t fldw = 0;
  std::vector<double> lam_int_h;  // eigenvalues in the internal spectral order
  // Generic plans whose operator band is wide: the axis operator itself as an
  // FP64 pass factor (Q64 holds W with y_j = sum_i W[i][j] x_i, i.e. y = B x),
  // so that the operator apply runs on the matrix cores instead of the band loop
  std::shared_ptr<AxisFactor> op_pass;
  ~AxisFactor();
};

// Element types of the per-pass data.
enum class DT : int { F64 = 0, F32 = 1, BF16 = 2 };

enum class Epi : int { None = 0, Inv = 1, Exp = 2 };

// Arguments of one mode-k pass over X viewed as [P][n][R] (R real values per
// (p, i), including the factor 2 of interleaved complex data).
struct PassArgs {
  const void* X = nullptr;
  void* Y = nullptr;
  DT tin = DT::F64, tout = DT::F64;
  int prec = 0;                // 0 fp64, 1 fp32, 2 bf16 (MFMA arithmetic)
  const AxisFactor* fac = nullptr;
  bool forward = true;         // forward uses Q (y = Q^T x), backward uses Q^T
  int64_t P = 1, n = 1, R = 1;
  bool cplx = false;           // data are interleaved complex
  Epi epi = Epi::None;
  // epilogue tables (device, FP64), indexed by p, by r / (cplx ? 2 : 1), by j
  const double* Lp = nullptr;  // Inv: sum of eigenvalues of the axes before
  const double* Lr = nullptr;  //      and after the pass axis
  double shift = 0.0;          // Inv: denominator = lam[j] + Lp[p] + Lr[q] + shift
  const double2* Ep = nullptr; // Exp: factor = es[j] * Ep[p] * Er[q]
  const double2* Er = nullptr;
  const double2* es = nullptr;
  const int* skip = nullptr;   // if non-null and *skip != 0 the kernel returns
  bool fold = false;           // half-extent pass of a symmetric axis
  // with fold: a forward pass reads data already folded along this axis
  // (launch_butterfly), a backward pass leaves its butterfly to the caller
  bool deferred = false;
  // FP64 output of a BF16 pass on 256 x 256 tiles: Y += the result instead of
  // Y = the result (bf16_big_pass_ok tells whether the pass runs there)
  bool accumulate = false;
  // BF16 row pass with FP64 output, the last of an apply whose other passes
  // left the data folded along the unf (1 or 2) slower axes of extents un[]
  // (slowest first): the pass unfolds them (bf16_unfold_pass_ok)
  int unf = 0;
  int64_t un[2] = {0, 0};
  int64_t kband = 0;           // > 0: the factor is banded, |k - output| <= kband (FP64 passes)
  int bf16_tile = 0;           // BF16 passes: 0 picks the tile size, 128 or 256 forces it where allowed
};

hipError_t launch_pass(const PassArgs& a, hipStream_t st);
hipError_t launch_pass_bf16(const PassArgs& a, hipStream_t st);
// Whether a BF16 pass can read data folded beforehand (pa.fold and pa.deferred
// set; a backward pass also leaves its output folded): the 256 x 256-tile
// kernel is the only one with that layout.
bool bf16_fold_pass_ok(const PassArgs& pa);
// Whether a BF16 pass of BF16 input runs on the 256 x 256 tiles.
bool bf16_big_pass_ok(const PassArgs& pa);
// Whether the last pass of a BF16 apply can unfold its input (pa.unf, pa.un).
bool bf16_unfold_pass_ok(const PassArgs& pa);

// Butterfly y_i, y_{n-1-i} = x_i + x_{n-1-i}, x_i - x_{n-1-i} (i < hh), in
// place or not, along up to four axes of a [n_0]...[n_{d-1}][ncomp] array at once
// (the axes' reflections commute, so their order does not matter).  The same
// map folds the input of an apply and unfolds its output.
struct ButterflyArgs {
  const void* X = nullptr;      // input (may equal Y)
  void* Y = nullptr;
  DT t = DT::F64;
  int d = 0, ncomp = 1;
  int64_t n[TS_MAX_D] = {};
  int nax = 0;                  // 1..4
  int ax[4] = {};               // the axes, as indices into n
  int64_t hh[4] = {};           // floor(n / 2) of each
  const int* skip = nullptr;    // if non-null and *skip != 0 the kernel returns
};
hipError_t launch_butterfly(const ButterflyArgs& a, hipStream_t st);
// The same butterflies on FP64 data a.X written as BF16 to a.Y (a BF16 apply's
// input sweep when its forward passes read folded data); real data only.
hipError_t launch_fold_to_bf16(const ButterflyArgs& a, hipStream_t st);

// Phase tables for the propagator: es[j] = e^{-i tau lam_s[j]},
// Ep[p] = prod_{m<s} e^{-i tau lam_m[j_m(p)]}, Er[q] = prod_{m>s} (...).
struct PhaseTableArgs {
  int d = 0, s = 0;
  int64_t n[TS_MAX_D] = {};
  const double* lam[TS_MAX_D] = {};
  double tau = 0;
  double2* Ep = nullptr;
  double2* Er = nullptr;
  double2* es = nullptr;
  int64_t P = 1, R = 1;
};
hipError_t launch_phase_tables(const PhaseTableArgs& a, hipStream_t st);

// Device-side casts for the plan's reduced-precision copies of Q.
hipError_t launch_cast_f64_to_f32(const double* x, float* y, int64_t n, hipStream_t st);
// FP64 data -> BF16 as the BF16 pass kernels round what they load (through
// FP32, each step to nearest even), four per thread: n % 4 == 0, x 16-byte and
// y 8-byte aligned (else hipErrorInvalidValue); honours *skip.
hipError_t launch_data_to_bf16(const double* x, uint16_t* y, int64_t n, const int* skip, hipStream_t st);
// Transposing cast of a square [ld][ld] factor: y[j][i] = bf16(x[i][j]).
hipError_t launch_cast_f64_to_bf16_t(const double* x, uint16_t* y, int64_t ld, hipStream_t st);

// Scratch of one stream of work on a plan: the apply's ping-pong workspace,
// the propagator's phase tables, the small path's diagonal tables and the
// solvers' vectors, plus a pinned host mirror of the solver scalars.  A plan
// owns a growable context for the plain entry points; the serving loop hands
// each admitted request a fixed context carved from its memory arena.
enum CtxSlot : int { kSlotWork = 0, kSlotPhase = 1, kSlotTab = 2, kSlotSolver = 3, kSlotOp = 4, kSlots = 5 };
struct ExecCtx {
  bool growable = true;
  void* buf[kSlots] = {};
  size_t bytes[kSlots] = {};
  void* host = nullptr;  // pinned, >= 256 bytes
  std::mutex mu;
  ExecCtx() = default;
  ExecCtx(const ExecCtx&) = delete;
  ExecCtx& operator=(const ExecCtx&) = delete;
  ~ExecCtx();
};
// Pointer to at least `bytes` of the slot (grown with hipMalloc if growable).
int ctx_get(ExecCtx& c, int slot, size_t bytes, void** out);
int ctx_host(ExecCtx& c, void** out);

}  // namespace ts

// The opaque plan of the C ABI.
struct ts_plan {
  int d = 0;
  int64_t n[TS_MAX_D] = {};
  int64_t N = 0;
  double L = 0, sigma = 0;
  int device = 0;
  std::vector<std::shared_ptr<ts::AxisFactor>> ax;      // factors of the public applies
  std::vector<std::shared_ptr<ts::AxisFactor>> ax_sym;  // orthogonal factors of the solvers (FD: = ax)
  int sem_k = 0;               // 0: FD or generic; k >= 1: Q^k SEM
  bool massed = false;         // SEM or generic: mass inner product, banded operator
  bool fold_enabled = true;    // use the half-extent passes on symmetric axes
  bool bf16_bwd_fold = true;   // BF16 applies: backward passes over half extents too (ts_set_fold)
  int bf16_tile = 0;           // BF16 pass tile: 0 automatic, 128 or 256 forced
  int s = 0;                   // axis whose forward pass carries the scaling
  int64_t Ps = 1, Rs = 1;      // products of the extents before / after axis s
  double* Lp = nullptr;        // device FP64 [Ps]
  double* Lr = nullptr;        // device FP64 [Rs]
  double lam_min = 0;          // lowest eigenvalue of H1
  ts::ExecCtx ctx;             // scratch of the plain (non-serving) entry points
  ~ts_plan();
};
