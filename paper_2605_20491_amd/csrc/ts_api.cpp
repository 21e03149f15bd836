// C ABI of the separable tensor-product solver: plan setup (paper Sec. 2.1,
// step 1), the inverse and propagator applies (steps 2-4, eq. (exact_prop)),
// accessors and error plumbing.  Solvers built on the applies live in
// solvers.cpp.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/ts.h"
#include "bf16_round.h"
#include "ts_internal.h"
#include "ts_apply.h"
#include "ts_sem.h"
#include "ts_small.h"

namespace ts {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

AxisFactor::~AxisFactor() {
  hipFree(lam);
  hipFree(f);
  hipFree(Q64);
  hipFree(QT64);
  hipFree(Q32);
  hipFree(QT32);
  hipFree(Q16);
  hipFree(QT16);
  hipFree(band);
  hipFree(Fe64);
  hipFree(Fo64);
  hipFree(Be64);
  hipFree(Bo64);
  hipFree(Fe32);
  hipFree(Fo32);
  hipFree(Be32);
  hipFree(Bo32);
  hipFree(Fr64);
  hipFree(Fr32);
  hipFree(Fe16);
  hipFree(Fo16);
  hipFree(Be16);
  hipFree(Bo16);
  if (Fe16w != Fe16) hipFree(Fe16w);  // the same array when the widths agree
  hipFree(Fr16w);
  if (Be16w != Be16) hipFree(Be16w);
  hipFree(Br16w);
  hipFree(mass);
  hipFree(msq);
  hipFree(imsq);
}

namespace {

// Even/odd structure of a reflection-symmetric axis.  The operator A
// (A[n-1-i][n-1-j] = A[i][j]) leaves the even and odd subspaces invariant.
// In the orthonormal bases (e_i +- e_{n-1-i}) / sqrt(2), i < h (plus e_h for
// odd n), its blocks are
//   even: A[i][j] + A[i][n-1-j]   (i, j < h),  sqrt(2) A[i][h],  A[h][h]
//   odd:  A[i][j] - A[i][n-1-j]   (i, j < h),
// each diagonalised on its own, so every eigenvector has exact parity even
// where the two subspaces hold nearly equal eigenvalues (for instance the top
// modes of a confining potential, localised at the two walls).  The spectral
// order inside the plan is then [even modes | odd modes], each ascending.
struct FoldPlan {
  bool on = false;            // the passes may fold (n >= 64)
  std::vector<int64_t> perm;  // internal spectral index -> ascending index
  int64_t ne = 0, no = 0, hh = 0, cc = 0;
};

// f reflection-symmetric up to the rounding of its samples: |f_i - f_{n-1-i}|
// within 8 ulps of max(1, max|f|).  The split eigensolvers then use the
// average of each mirrored pair, which moves the operator by at most half that.
bool symmetric_samples(int64_t n, const double* f) {
  double fmax = 0.0, fasym = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    fmax = std::max(fmax, std::fabs(f[i]));
    fasym = std::max(fasym, std::fabs(f[i] - f[n - 1 - i]));
  }
  return fasym <= 8.0 * DBL_EPSILON * std::max(1.0, fmax);
}

// Assemble the full eigenvectors from the two blocks (Ue: ne x ne, Uo: no x no,
// row-major, column = eigenvector), sort ascending, sign: largest entry
// positive (lowest index on ties).  Fills lam, Q (n x n) and the fold plan.
void assemble_split(int64_t n, const std::vector<double>& le, const std::vector<double>& Ue,
                    const std::vector<double>& lo, const std::vector<double>& Uo, double* lam, double* Q,
                    FoldPlan& fp) {
  const int64_t hh = n / 2, cc = n % 2, ne = hh + cc, no = hh;
  const double r2 = 1.0 / std::sqrt(2.0);
  std::vector<double> V((size_t)(n * n), 0.0);  // column c: even modes first, then odd
  std::vector<double> lv(n);
  for (int64_t j = 0; j < ne; ++j) {
    lv[j] = le[j];
    for (int64_t i = 0; i < hh; ++i) {
      const double v = Ue[(size_t)(i * ne + j)] * r2;
      V[(size_t)(i * n + j)] = v;
      V[(size_t)((n - 1 - i) * n + j)] = v;
    }
    if (cc) V[(size_t)(hh * n + j)] = Ue[(size_t)(hh * ne + j)];
  }
  for (int64_t j = 0; j < no; ++j) {
    lv[ne + j] = lo[j];
    for (int64_t i = 0; i < hh; ++i) {
      const double v = Uo[(size_t)(i * no + j)] * r2;
      V[(size_t)(i * n + ne + j)] = v;
      V[(size_t)((n - 1 - i) * n + ne + j)] = -v;
    }
  }
  // public order: ascending eigenvalue (ties: even first)
  std::vector<int64_t> order(n);
  for (int64_t c = 0; c < n; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return lv[a] < lv[b]; });
  std::vector<int64_t> pos(n);  // internal column -> ascending index
  for (int64_t j = 0; j < n; ++j) pos[order[j]] = j;
  for (int64_t j = 0; j < n; ++j) {
    const int64_t c = order[j];
    int64_t arg = 0;
    for (int64_t i = 1; i < n; ++i)
      if (std::fabs(V[(size_t)(i * n + c)]) > std::fabs(V[(size_t)(arg * n + c)])) arg = i;
    const double sg = V[(size_t)(arg * n + c)] < 0.0 ? -1.0 : 1.0;
    lam[j] = lv[c];
    for (int64_t i = 0; i < n; ++i) Q[(size_t)(i * n + j)] = sg * V[(size_t)(i * n + c)];
  }
  fp.hh = hh;
  fp.cc = cc;
  fp.ne = ne;
  fp.no = no;
  fp.perm.resize(n);
  for (int64_t c = 0; c < n; ++c) fp.perm[c] = pos[c];
  fp.on = n >= 64;
}

// Tridiagonal symmetric operator (diag, off constant-free): the two blocks are tridiagonal too.
bool split_eig_tridiag(int64_t n, const double* dg, const double* off, double* lam, double* Q, FoldPlan& fp) {
  const int64_t hh = n / 2, cc = n % 2, ne = hh + cc, no = hh;
  if (hh == 0) return false;
  std::vector<double> de(ne), oe(ne > 1 ? ne - 1 : 1, 0.0), dd(no), od(no > 1 ? no - 1 : 1, 0.0);
  for (int64_t i = 0; i < hh; ++i) {  // mirrored pairs averaged (equal up to rounding)
    de[i] = 0.5 * (dg[i] + dg[n - 1 - i]);
    dd[i] = de[i];
  }
  for (int64_t i = 0; i + 1 < hh; ++i) oe[i] = od[i] = 0.5 * (off[i] + off[n - 2 - i]);
  if (cc) {
    de[hh] = dg[hh];
    oe[hh - 1] = std::sqrt(2.0) * 0.5 * (off[hh - 1] + off[hh]);  // e_{h-1} pair coupled to the centre
  } else {
    de[hh - 1] += off[hh - 1];  // the pair h-1, h = n-1-(h-1) couples to itself
    dd[hh - 1] -= off[hh - 1];
  }
  std::vector<double> le(ne), Ue((size_t)(ne * ne)), lo(no), Uo((size_t)(no * no));
  if (!tridiag_eig(ne, de.data(), oe.data(), le.data(), Ue.data())) return false;
  if (!tridiag_eig(no, dd.data(), od.data(), lo.data(), Uo.data())) return false;
  assemble_split(n, le, Ue, lo, Uo, lam, Q, fp);
  return true;
}

// Even and odd blocks of a reflection-symmetric operator (row-major n x n),
// mirrored entries averaged, each block made exactly symmetric.
template <class T>
void reflection_blocks(int64_t n, const T* A, std::vector<T>& He, std::vector<T>& Ho) {
  const int64_t hh = n / 2, cc = n % 2, ne = hh + cc, no = hh;
  auto a = [&](int64_t i, int64_t j) {  // reflection average
    return (T)0.5 * (A[(size_t)(i * n + j)] + A[(size_t)((n - 1 - i) * n + (n - 1 - j))]);
  };
  He.assign((size_t)(ne * ne), (T)0);
  Ho.assign((size_t)(no * no), (T)0);
  for (int64_t i = 0; i < hh; ++i)
    for (int64_t j = 0; j < hh; ++j) {
      He[(size_t)(i * ne + j)] = a(i, j) + a(i, n - 1 - j);
      Ho[(size_t)(i * no + j)] = a(i, j) - a(i, n - 1 - j);
    }
  if (cc) {
    const T r2 = std::sqrt((T)2);
    for (int64_t i = 0; i < hh; ++i) He[(size_t)(i * ne + hh)] = He[(size_t)(hh * ne + i)] = r2 * a(i, hh);
    He[(size_t)(hh * ne + hh)] = a(hh, hh);
  }
  for (int64_t i = 0; i < ne; ++i)  // exact symmetry of the blocks
    for (int64_t j = 0; j < i; ++j)
      He[(size_t)(i * ne + j)] = He[(size_t)(j * ne + i)] = (T)0.5 * (He[(size_t)(i * ne + j)] + He[(size_t)(j * ne + i)]);
  for (int64_t i = 0; i < no; ++i)
    for (int64_t j = 0; j < i; ++j)
      Ho[(size_t)(i * no + j)] = Ho[(size_t)(j * no + i)] = (T)0.5 * (Ho[(size_t)(i * no + j)] + Ho[(size_t)(j * no + i)]);
}

// Dense reflection-symmetric operator (row-major n x n); Aex: the same
// operator in long double, against which each block's eigenvectors are
// refined (null: refined against the double blocks).
bool split_eig_dense(int64_t n, const std::vector<double>& A, double* lam, double* Q, FoldPlan& fp,
                     const std::vector<long double>* Aex = nullptr) {
  const int64_t hh = n / 2, cc = n % 2, ne = hh + cc, no = hh;
  if (hh == 0) return false;
  std::vector<double> He, Ho;
  reflection_blocks(n, A.data(), He, Ho);
  std::vector<long double> HeL, HoL;
  if (Aex) reflection_blocks(n, Aex->data(), HeL, HoL);
  std::vector<double> le(ne), Ue((size_t)(ne * ne)), lo(no), Uo((size_t)(no * no));
  if (!dense_sym_eig(ne, He, le.data(), Ue.data(), Aex ? HeL.data() : nullptr)) return false;
  if (!dense_sym_eig(no, Ho, lo.data(), Uo.data(), Aex ? HoL.data() : nullptr)) return false;
  assemble_split(n, le, Ue, lo, Uo, lam, Q, fp);
  return true;
}

// Upload one factor set.  Fwd and Bwd are row-major n x n with the pass
// convention y_j = sum_i W[i][j] x_i; they are zero-padded to [kpad][ld].
// m: the axis's L^2 weights; band (n * (2 bw + 1) entries) and the mass
// roots (roots = true) are for SEM.
int upload_factor(AxisFactor& F, const double* f, const std::vector<double>& Fwd0, const std::vector<double>& Bwd0,
                  const std::vector<double>* band, const std::vector<double>& m, bool roots, const FoldPlan& fp) {
  const int64_t n = F.n;
  // internal spectral order: columns of Fwd and rows of Bwd, and lam
  std::vector<double> Fwd = Fwd0, Bwd = Bwd0;
  F.lam_int_h = F.lam_h;
  if (fp.on) {
    for (int64_t jj = 0; jj < n; ++jj) {
      const int64_t j = fp.perm[jj];
      F.lam_int_h[jj] = F.lam_h[j];
      for (int64_t i = 0; i < n; ++i) {
        Fwd[(size_t)(i * n + jj)] = Fwd0[(size_t)(i * n + j)];
        Bwd[(size_t)(jj * n + i)] = Bwd0[(size_t)(j * n + i)];
      }
    }
  }
  F.ld = round_up(n, kTileF);
  F.kpad = F.ld;  // square padding: every kernel's tiles stay inside
  const size_t padded = (size_t)(F.kpad * F.ld);
  std::vector<double> Qp(padded, 0.0), QTp(padded, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      Qp[(size_t)(i * F.ld + j)] = Fwd[(size_t)(i * n + j)];
      QTp[(size_t)(i * F.ld + j)] = Bwd[(size_t)(i * n + j)];
    }
  std::vector<double> ms, ims;
  if (roots) {
    ms.resize(n);
    ims.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      ms[i] = std::sqrt(m[i]);
      ims[i] = 1.0 / ms[i];
    }
  }
  hipError_t e = hipSuccess;
  e = hipMalloc(&F.lam, sizeof(double) * n);
  if (e == hipSuccess) e = hipMalloc(&F.f, sizeof(double) * n);
  if (e == hipSuccess) e = hipMalloc(&F.Q64, sizeof(double) * padded);
  if (e == hipSuccess) e = hipMalloc(&F.QT64, sizeof(double) * padded);
  if (e == hipSuccess) e = hipMalloc(&F.Q32, sizeof(float) * padded);
  if (e == hipSuccess) e = hipMalloc(&F.QT32, sizeof(float) * padded);
  if (e == hipSuccess) e = hipMalloc(&F.Q16, sizeof(uint16_t) * padded);
  if (e == hipSuccess) e = hipMalloc(&F.QT16, sizeof(uint16_t) * padded);
  if (e == hipSuccess && band) e = hipMalloc(&F.band, sizeof(double) * band->size());
  if (e == hipSuccess) e = hipMalloc(&F.mass, sizeof(double) * n);
  if (e == hipSuccess && roots) e = hipMalloc(&F.msq, sizeof(double) * n);
  if (e == hipSuccess && roots) e = hipMalloc(&F.imsq, sizeof(double) * n);
  if (e != hipSuccess) {
    set_error(std::string("device allocation of factors failed: ") + hipGetErrorString(e));
    return TS_ERR_NOMEM;
  }
  // upload on a private non-blocking stream: setup never waits for other work
  hipStream_t st = nullptr;
  e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMemcpyAsync(F.lam, F.lam_int_h.data(), sizeof(double) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(F.f, f, sizeof(double) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(F.Q64, Qp.data(), sizeof(double) * padded, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(F.QT64, QTp.data(), sizeof(double) * padded, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && band)
    e = hipMemcpyAsync(F.band, band->data(), sizeof(double) * band->size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(F.mass, m.data(), sizeof(double) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && roots) e = hipMemcpyAsync(F.msq, ms.data(), sizeof(double) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && roots) e = hipMemcpyAsync(F.imsq, ims.data(), sizeof(double) * n, hipMemcpyHostToDevice, st);
  // reduced-precision copies are cast on the device from the FP64 copy
  if (e == hipSuccess) e = launch_cast_f64_to_f32(F.Q64, F.Q32, (int64_t)padded, st);
  if (e == hipSuccess) e = launch_cast_f64_to_f32(F.QT64, F.QT32, (int64_t)padded, st);
  if (e == hipSuccess) e = launch_cast_f64_to_bf16_t(F.Q64, F.QT16, F.ld, st);
  if (e == hipSuccess) e = launch_cast_f64_to_bf16_t(F.QT64, F.Q16, F.ld, st);
  // half factors of a symmetric axis
  std::vector<double> H[5];
  std::vector<uint16_t> Hw[4];
  if (e == hipSuccess && fp.on) {
    F.fold = true;
    F.ne = fp.ne;
    F.no = fp.no;
    F.hh = fp.hh;
    F.cc = fp.cc;
    F.fkp = round_up(fp.hh + fp.cc, kTileF);
    const int64_t kp = F.fkp;
    for (auto& h : H) h.assign((size_t)(kp * kp), 0.0);
    for (int64_t i = 0; i < fp.hh + fp.cc; ++i)
      for (int64_t j = 0; j < fp.ne; ++j) {
        H[0][(size_t)(i * kp + j)] = Fwd[(size_t)(i * n + j)];  // Fe[i][j']
        H[2][(size_t)(j * kp + i)] = Bwd[(size_t)(j * n + i)];  // Be[j'][i]
      }
    for (int64_t i = 0; i < fp.hh; ++i)
      for (int64_t j = 0; j < fp.no; ++j) {
        H[1][(size_t)(i * kp + j)] = Fwd[(size_t)(i * n + fp.ne + j)];  // Fo[i][j'']
        H[4][(size_t)((fp.hh - 1 - i) * kp + j)] = H[1][(size_t)(i * kp + j)];  // Fr
        H[3][(size_t)(j * kp + i)] = Bwd[(size_t)((fp.ne + j) * n + i)];  // Bo[j''][i]
      }
    double** d64[4] = {&F.Fe64, &F.Fo64, &F.Be64, &F.Bo64};
    float** d32[4] = {&F.Fe32, &F.Fo32, &F.Be32, &F.Bo32};
    uint16_t** d16[4] = {&F.Fe16, &F.Fo16, &F.Be16, &F.Bo16};
    const size_t cnt = (size_t)(kp * kp);
    for (int q = 0; q < 4 && e == hipSuccess; ++q) {
      e = hipMalloc(d64[q], sizeof(double) * cnt);
      if (e == hipSuccess) e = hipMalloc(d32[q], sizeof(float) * cnt);
      if (e == hipSuccess) e = hipMalloc(d16[q], sizeof(uint16_t) * cnt);
      if (e == hipSuccess) e = hipMemcpyAsync(*d64[q], H[q].data(), sizeof(double) * cnt, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = launch_cast_f64_to_f32(*d64[q], *d32[q], (int64_t)cnt, st);
      if (e == hipSuccess) e = launch_cast_f64_to_bf16_t(*d64[q], *d16[q], kp, st);
    }
    // BF16 factors of the 256 x 256-tile forward pass on folded data: Fe, and
    // Fr with its K index shifted by sh, both K-contiguous with a common width
    // covering h + c and h + sh in 128-wide k-tiles (Fe16 itself when that is
    // its own width)
    const int64_t sh = (fp.hh + fp.cc) % 8, lw = round_up(std::max(fp.hh + fp.cc, fp.hh + sh), kTileF);
    F.fldw = lw;
    if (lw != kp) {
      Hw[0].assign((size_t)(lw * lw), 0);
      for (int64_t j = 0; j < fp.ne; ++j)
        for (int64_t i = 0; i < fp.hh + fp.cc; ++i) Hw[0][(size_t)(j * lw + i)] = bf16_from_f64(H[0][(size_t)(i * kp + j)]);
    }
    Hw[1].assign((size_t)(lw * lw), 0);
    for (int64_t j = 0; j < fp.no; ++j)
      for (int64_t r = 0; r < fp.hh; ++r) Hw[1][(size_t)(j * lw + r + sh)] = bf16_from_f64(H[4][(size_t)(r * kp + j)]);
    // the backward pass that leaves its output folded: Be (rows = physical
    // i < h + c, K = even modes), and Bo with its rows reversed (row r is
    // i = h - 1 - r) and its K index (odd modes) shifted by sh
    if (lw != kp) {
      Hw[2].assign((size_t)(lw * lw), 0);
      for (int64_t i = 0; i < fp.hh + fp.cc; ++i)
        for (int64_t j = 0; j < fp.ne; ++j) Hw[2][(size_t)(i * lw + j)] = bf16_from_f64(H[2][(size_t)(j * kp + i)]);
    }
    Hw[3].assign((size_t)(lw * lw), 0);
    for (int64_t r = 0; r < fp.hh; ++r)
      for (int64_t j = 0; j < fp.no; ++j)
        Hw[3][(size_t)(r * lw + j + sh)] = bf16_from_f64(H[3][(size_t)(j * kp + (fp.hh - 1 - r))]);
    if (lw != kp) {
      if (e == hipSuccess) e = hipMalloc(&F.Fe16w, sizeof(uint16_t) * (size_t)(lw * lw));
      if (e == hipSuccess)
        e = hipMemcpyAsync(F.Fe16w, Hw[0].data(), sizeof(uint16_t) * Hw[0].size(), hipMemcpyHostToDevice, st);
    } else {
      F.Fe16w = F.Fe16;
    }
    if (e == hipSuccess) e = hipMalloc(&F.Fr16w, sizeof(uint16_t) * (size_t)(lw * lw));
    if (e == hipSuccess)
      e = hipMemcpyAsync(F.Fr16w, Hw[1].data(), sizeof(uint16_t) * Hw[1].size(), hipMemcpyHostToDevice, st);
    if (lw != kp) {
      if (e == hipSuccess) e = hipMalloc(&F.Be16w, sizeof(uint16_t) * (size_t)(lw * lw));
      if (e == hipSuccess)
        e = hipMemcpyAsync(F.Be16w, Hw[2].data(), sizeof(uint16_t) * Hw[2].size(), hipMemcpyHostToDevice, st);
    } else {
      F.Be16w = F.Be16;  // K-contiguous Be at width kp is the same matrix
    }
    if (e == hipSuccess) e = hipMalloc(&F.Br16w, sizeof(uint16_t) * (size_t)(lw * lw));
    if (e == hipSuccess)
      e = hipMemcpyAsync(F.Br16w, Hw[3].data(), sizeof(uint16_t) * Hw[3].size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMalloc(&F.Fr64, sizeof(double) * cnt);
    if (e == hipSuccess) e = hipMalloc(&F.Fr32, sizeof(float) * cnt);
    if (e == hipSuccess) e = hipMemcpyAsync(F.Fr64, H[4].data(), sizeof(double) * cnt, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_cast_f64_to_f32(F.Fr64, F.Fr32, (int64_t)cnt, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (st) hipStreamDestroy(st);
  if (e != hipSuccess) {
    set_error(std::string("factor upload failed: ") + hipGetErrorString(e));
    return TS_ERR_DEVICE;
  }
  return TS_OK;
}

std::vector<double> transpose(const std::vector<double>& A, int64_t n) {
  std::vector<double> T(A.size());
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) T[(size_t)(j * n + i)] = A[(size_t)(i * n + j)];
  return T;
}

}  // namespace

// Build and upload the factors of H = h^-2 tridiag(-1,2,-1) + diag(f).
static int build_axis(int64_t n, double L, const double* f, std::shared_ptr<AxisFactor>& out) {
  auto F = std::make_shared<AxisFactor>();
  F->n = n;
  F->L = L;
  const double h = 2.0 * L / (double)(n + 1);
  const double ih2 = 1.0 / (h * h);
  F->ih2 = ih2;
  std::vector<double> dg(n), off(n > 1 ? n - 1 : 1, 0.0);
  for (int64_t i = 0; i < n; ++i) dg[i] = 2.0 * ih2 + f[i];
  for (int64_t i = 0; i + 1 < n; ++i) off[i] = -ih2;
  F->lam_h.resize(n);
  F->Q_h.resize((size_t)(n * n));
  FoldPlan fp;
  const bool split = n >= 2 && symmetric_samples(n, f);
  const bool ok = split ? split_eig_tridiag(n, dg.data(), off.data(), F->lam_h.data(), F->Q_h.data(), fp)
                        : tridiag_eig(n, dg.data(), off.data(), F->lam_h.data(), F->Q_h.data());
  if (!ok) {
    set_error("tridiagonal eigensolver did not converge");
    return TS_ERR_INVALID;
  }
  int rc = upload_factor(*F, f, F->Q_h, transpose(F->Q_h, n), nullptr, std::vector<double>(n, h), false, fp);
  if (rc) return rc;
  F->x_h.resize(n);
  for (int64_t j = 0; j < n; ++j) F->x_h[j] = -L + h * (double)(j + 1);
  out = F;
  return TS_OK;
}

// Eigenpairs of the symmetric form A + diag(f) (row-major n x n, A is
// overwritten): exact symmetry imposed, the even and odd blocks solved apart
// when the operator is reflection-symmetric, and the eigenvectors refined
// against Aex + diag(f) (the operator before rounding, long double) when given.
static bool massed_eig(int64_t n, std::vector<double>& A, std::vector<long double>* Aex, const double* f, bool reflect,
                       double* lam, double* Q, FoldPlan& fp) {
  for (int64_t i = 0; i < n; ++i) A[(size_t)(i * n + i)] += f[i];
  for (int64_t i = 0; i < n; ++i)  // exact symmetry (the input is symmetric up to rounding)
    for (int64_t j = 0; j < i; ++j) {
      const double a = 0.5 * (A[(size_t)(i * n + j)] + A[(size_t)(j * n + i)]);
      A[(size_t)(i * n + j)] = A[(size_t)(j * n + i)] = a;
    }
  if (Aex) {
    auto& E = *Aex;
    for (int64_t i = 0; i < n; ++i) E[(size_t)(i * n + i)] += f[i];
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < i; ++j)
        E[(size_t)(i * n + j)] = E[(size_t)(j * n + i)] = 0.5L * (E[(size_t)(i * n + j)] + E[(size_t)(j * n + i)]);
  }
  return n >= 2 && reflect ? split_eig_dense(n, A, lam, Q, fp, Aex)
                           : dense_sym_eig(n, A, lam, Q, Aex ? Aex->data() : nullptr);
}

// SEM axis operator M^{-1/2} S M^{-1/2}, formed in long double (Al) and
// rounded once (A, and its band bsym); bphys = the band of M^{-1} S.
static void sem_operator(const SemAxis& ax, std::vector<long double>& Al, std::vector<double>& A,
                         std::vector<double>* bsym, std::vector<double>* bphys) {
  const int64_t n = ax.n;
  const int k = ax.k, w = 2 * k + 1;
  std::vector<long double> msl(n);
  Al.assign((size_t)(n * n), 0.0L);
  A.assign((size_t)(n * n), 0.0);
  if (bsym) bsym->assign((size_t)(n * w), 0.0);
  if (bphys) bphys->assign((size_t)(n * w), 0.0);
  for (int64_t i = 0; i < n; ++i) msl[i] = std::sqrt(ax.ml[i]);
  for (int64_t i = 0; i < n; ++i)
    for (int t = 0; t < w; ++t) {
      const int64_t j = i - k + t;
      if (j < 0 || j >= n) continue;
      const long double sij = ax.Sl[(size_t)(i * w + t)];
      const long double aij = sij / (msl[i] * msl[j]);
      Al[(size_t)(i * n + j)] = aij;
      A[(size_t)(i * n + j)] = (double)aij;
      if (bsym) (*bsym)[(size_t)(i * w + t)] = (double)aij;
      if (bphys) (*bphys)[(size_t)(i * w + t)] = (double)(sij / ax.ml[i]);
    }
}

// Axis of a mass-weighted operator H = K + diag(f) with K self-adjoint in the
// weights m (diag(m) K symmetric; Q^k SEM: K = M^{-1} S).  Q diagonalises the
// symmetric A = M^{1/2} K M^{-1/2} + F (eq. (eigen_decomp)).
//   A: dense M^{1/2} K M^{-1/2} (row-major; f is added here)
//   bsym, bphys: bands [n][2 bw + 1] of M^{1/2} K M^{-1/2} and of K
//   reflect: K, m and f are reflection-symmetric (even/odd eigensolve, fold)
// sym: factors (Q, Q^T), band bsym, mass roots; the solvers use it.
// phys: T^{-1} = Q^T M^{1/2}, T = M^{-1/2} Q, band bphys; the public applies use it.
static int build_axis_massed(int64_t n, double L, std::vector<double>& A, const std::vector<double>* bsym,
                             const std::vector<double>* bphys, int bw, const std::vector<double>& m,
                             const std::vector<double>& x, const double* f, bool reflect,
                             std::shared_ptr<AxisFactor>& phys, std::shared_ptr<AxisFactor>& sym,
                             std::vector<long double>* Aex = nullptr) {
  std::vector<double> ms(n);
  for (int64_t i = 0; i < n; ++i) ms[i] = std::sqrt(m[i]);
  auto S = std::make_shared<AxisFactor>();
  S->n = n;
  S->L = L;
  S->lam_h.resize(n);
  S->Q_h.resize((size_t)(n * n));
  FoldPlan fp;
  if (!massed_eig(n, A, Aex, f, reflect, S->lam_h.data(), S->Q_h.data(), fp)) {
    set_error("symmetric eigensolver did not converge");
    return TS_ERR_INVALID;
  }
  S->bw = bw;
  S->m_h = m;
  S->x_h = x;
  int rc = upload_factor(*S, f, S->Q_h, transpose(S->Q_h, n), bsym, m, true, fp);
  if (rc) return rc;
  auto P = std::make_shared<AxisFactor>();
  P->n = n;
  P->L = L;
  P->lam_h = S->lam_h;
  P->Q_h = S->Q_h;
  P->bw = bw;
  P->m_h = m;
  P->x_h = x;
  std::vector<double> Fwd((size_t)(n * n)), Bwd((size_t)(n * n));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const double q = S->Q_h[(size_t)(i * n + j)];
      Fwd[(size_t)(i * n + j)] = ms[i] * q;   // (T^{-1})^T = M^{1/2} Q
      Bwd[(size_t)(j * n + i)] = q / ms[i];   // T^T = Q^T M^{-1/2}
    }
  rc = upload_factor(*P, f, Fwd, Bwd, bphys, m, true, fp);
  if (rc) return rc;
  phys = P;
  sym = S;
  return TS_OK;
}

static int upload_op_pass(int64_t n, const std::vector<double>& B, std::shared_ptr<AxisFactor>& out);

// Dense row-major n x n matrix of a band [n][2 bw + 1] (entry (i, i - bw + t)).
static std::vector<double> band_to_dense(int64_t n, int bw, const std::vector<double>& band) {
  const int64_t w = 2 * (int64_t)bw + 1;
  std::vector<double> B((size_t)(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t t = 0; t < w; ++t) {
      const int64_t j = i - bw + t;
      if (j >= 0 && j < n) B[(size_t)(i * n + j)] = band[(size_t)(i * w + t)];
    }
  return B;
}

// Q^k SEM axis: K = M^{-1} S from the Gauss-Lobatto mass and stiffness band.
// op: also keep the operator as banded FP64 pass factors (the plan applies its
// operator as matrix-core passes restricted to the band).
static int build_axis_sem(int k, int64_t cells, double L, const double* f, bool op, std::shared_ptr<AxisFactor>& phys,
                          std::shared_ptr<AxisFactor>& sym) {
  SemAxis ax;
  if (!sem_axis(k, cells, L, ax)) { set_error("bad SEM axis"); return TS_ERR_INVALID; }
  const int64_t n = ax.n;
  std::vector<long double> Al;
  std::vector<double> A, bsym, bphys;
  sem_operator(ax, Al, A, &bsym, &bphys);
  // the mesh is symmetric; with symmetric f the operator is reflection-symmetric
  int rc = build_axis_massed(n, L, A, &bsym, &bphys, k, ax.m, ax.x, f, symmetric_samples(n, f), phys, sym, &Al);
  if (rc || !op) return rc;
  rc = upload_op_pass(n, band_to_dense(n, k, bsym), sym->op_pass);
  if (rc) return rc;
  rc = upload_op_pass(n, band_to_dense(n, k, bphys), phys->op_pass);
  if (rc) return rc;
  sym->op_pass->bw = k;
  phys->op_pass->bw = k;
  return TS_OK;
}

// FP64 pass factor of a dense operator B (row-major n x n): the pass computes
// y = B x along its axis (W[i][j] = B[j][i], zero-padded to [ld][ld]).
static int upload_op_pass(int64_t n, const std::vector<double>& B, std::shared_ptr<AxisFactor>& out) {
  auto F = std::make_shared<AxisFactor>();
  F->n = n;
  F->ld = round_up(n, kTileF);
  F->kpad = F->ld;
  std::vector<double> W((size_t)(F->kpad * F->ld), 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) W[(size_t)(i * F->ld + j)] = B[(size_t)(j * n + i)];
  if (hipMalloc(&F->Q64, sizeof(double) * W.size()) != hipSuccess) {
    set_error("operator factor allocation failed");
    return TS_ERR_NOMEM;
  }
  if (hipMemcpy(F->Q64, W.data(), sizeof(double) * W.size(), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("operator factor upload failed");
    return TS_ERR_DEVICE;
  }
  out = F;
  return TS_OK;
}

// Generic axis from a dense K and weights m (NULL: unit weights); bw is the
// band half-width of every axis of the plan (the largest over the axes).
static int build_axis_general(int64_t n, const double* K, const double* m_in, const double* x_in, const double* f,
                              int bw, std::shared_ptr<AxisFactor>& phys, std::shared_ptr<AxisFactor>& sym) {
  std::vector<double> m(n, 1.0), x(n), ms(n);
  if (m_in) std::memcpy(m.data(), m_in, sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    if (!(m[i] > 0.0) || !std::isfinite(m[i])) { set_error("weights must be positive and finite"); return TS_ERR_INVALID; }
    ms[i] = std::sqrt(m[i]);
    x[i] = x_in ? x_in[i] : (double)i;
  }
  // bands only for the band loop; wider operators run as dense passes and keep none
  const bool banded = bw <= kBandMax;
  const int64_t w = banded ? 2 * (int64_t)bw + 1 : 0;
  std::vector<double> A((size_t)(n * n)), bsym((size_t)(n * w), 0.0), bphys((size_t)(n * w), 0.0);
  double amax = 0.0, asym = 0.0, arefl = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const double kij = K[(size_t)(i * n + j)];
      if (!std::isfinite(kij)) { set_error("K has a non-finite entry"); return TS_ERR_NONFINITE; }
      A[(size_t)(i * n + j)] = ms[i] * kij / ms[j];
      amax = std::max(amax, std::fabs(A[(size_t)(i * n + j)]));
    }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      asym = std::max(asym, std::fabs(A[(size_t)(i * n + j)] - A[(size_t)(j * n + i)]));
      arefl = std::max(arefl, std::fabs(A[(size_t)(i * n + j)] - A[(size_t)((n - 1 - i) * n + (n - 1 - j))]));
    }
  if (asym > 1e-10 * amax) {
    set_error("K is not self-adjoint in the weights m (diag(m) K not symmetric to 1e-10)");
    return TS_ERR_INVALID;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t t = 0; t < w; ++t) {
      const int64_t j = i - bw + t;
      if (j < 0 || j >= n) continue;
      bsym[(size_t)(i * w + t)] = 0.5 * (A[(size_t)(i * n + j)] + A[(size_t)(j * n + i)]);
      bphys[(size_t)(i * w + t)] = K[(size_t)(i * n + j)];
    }
  const bool reflect = arefl <= 1e-11 * amax && symmetric_samples(n, m.data()) && symmetric_samples(n, f);
  std::vector<double> A0;
  if (bw > kBandMax) {  // the operator apply runs as MFMA passes: keep M^{1/2} K M^{-1/2} before f is added
    A0 = A;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < i; ++j)
        A0[(size_t)(i * n + j)] = A0[(size_t)(j * n + i)] = 0.5 * (A[(size_t)(i * n + j)] + A[(size_t)(j * n + i)]);
  }
  int rc = build_axis_massed(n, 0.0, A, banded ? &bsym : nullptr, banded ? &bphys : nullptr, bw, m, x, f, reflect,
                             phys, sym);
  if (rc || bw <= kBandMax) return rc;
  rc = upload_op_pass(n, A0, sym->op_pass);
  if (rc) return rc;
  return upload_op_pass(n, std::vector<double>(K, K + n * n), phys->op_pass);
}

// Device bytes held by a plan: factors of every distinct axis (all
// precisions, half factors of folded axes), per-axis vectors and the scaling
// tables.  Scratch contexts are not counted.
size_t plan_device_bytes(const ts_plan* p) {
  std::vector<const AxisFactor*> seen;
  size_t b = sizeof(double) * (size_t)(p->Ps + p->Rs);
  std::function<void(const AxisFactor*)> add = [&](const AxisFactor* F) {
    if (!F || std::find(seen.begin(), seen.end(), F) != seen.end()) return;
    seen.push_back(F);
    b += (size_t)(F->kpad * F->ld) * (8 + 8 + 4 + 4 + 2 + 2);
    b += sizeof(double) * (size_t)F->n * (F->msq ? 5 : 3);
    if (F->band) b += sizeof(double) * (size_t)F->n * (2 * F->bw + 1);
    if (F->fold)
      b += (size_t)(F->fkp * F->fkp) * (5 * 8 + 5 * 4 + 4 * 2) + (size_t)(F->fldw * F->fldw) * 2 * (F->fldw == F->fkp ? 2 : 4);
    add(F->op_pass.get());
  };
  for (const auto& F : p->ax) add(F.get());
  for (const auto& F : p->ax_sym) add(F.get());
  return b;
}

ExecCtx::~ExecCtx() {
  if (!growable) return;
  for (int i = 0; i < kSlots; ++i) hipFree(buf[i]);
  if (host) hipHostFree(host);
}

// Growing a slot synchronises the device so that no queued kernel still uses
// the old buffer.
int ctx_get(ExecCtx& c, int slot, size_t bytes, void** out) {
  std::lock_guard<std::mutex> g(c.mu);
  if (bytes == 0) bytes = 256;
  if (c.bytes[slot] < bytes) {
    if (!c.growable) {
      set_error("request scratch too small (" + std::to_string(c.bytes[slot]) + " < " + std::to_string(bytes) + " bytes)");
      return TS_ERR_NOMEM;
    }
    if (c.buf[slot]) {
      hipDeviceSynchronize();
      hipFree(c.buf[slot]);
      c.buf[slot] = nullptr;
      c.bytes[slot] = 0;
    }
    if (hipMalloc(&c.buf[slot], bytes) != hipSuccess) {
      c.buf[slot] = nullptr;
      set_error("scratch allocation of " + std::to_string(bytes) + " bytes failed");
      return TS_ERR_NOMEM;
    }
    c.bytes[slot] = bytes;
  }
  *out = c.buf[slot];
  return TS_OK;
}

int ctx_host(ExecCtx& c, void** out) {
  std::lock_guard<std::mutex> g(c.mu);
  if (!c.host) {
    if (!c.growable || hipHostMalloc(&c.host, 256, hipHostMallocDefault) != hipSuccess) {
      c.host = nullptr;
      set_error("pinned host allocation failed");
      return TS_ERR_NOMEM;
    }
  }
  *out = c.host;
  return TS_OK;
}

size_t need_inverse(const ts_plan* p, int slot) {
  if (plan_is_small(p)) return slot == kSlotTab ? small_table_bytes(p, false, true, false) : 0;
  return slot == kSlotWork ? (size_t)p->N * 8 : 0;
}

size_t need_exp(const ts_plan* p, int slot) {
  if (plan_is_small(p)) return slot == kSlotTab ? small_table_bytes(p, true, false, true) : 0;
  if (slot == kSlotWork) return (size_t)p->N * 16;
  if (slot == kSlotPhase) return sizeof(double2) * (size_t)(p->Ps + p->Rs + p->n[p->s]);
  return 0;
}

static DT dt_of(int dtype) { return (dtype == TS_F64 || dtype == TS_C128) ? DT::F64 : DT::F32; }

bool bf16_fold_axes(const ts_plan* p, const void* in, void* out, bool sym, ButterflyArgs& b) {
  b = ButterflyArgs{};
  if (!p->fold_enabled || in == out || p->N % 4 != 0 || (((uintptr_t)in) & 15) != 0 || (((uintptr_t)out) & 15) != 0)
    return false;
  const int d = p->d;
  b.X = in;
  b.Y = out;
  b.t = DT::F64;
  b.d = d;
  b.ncomp = 1;
  for (int k = 0; k < d; ++k) b.n[k] = p->n[k];
  for (int k = d - 1; k >= 0 && b.nax < 4; --k) {  // fastest first, as the sweep applies them
    const AxisFactor* F = (sym ? p->ax_sym : p->ax)[k].get();
    if (!F->fold) continue;
    PassArgs q;
    q.X = out;
    q.Y = out;  // the work buffers are library allocations, 256-byte aligned like out's check
    q.tin = DT::BF16;
    q.tout = DT::BF16;
    q.prec = TS_PREC_BF16;
    q.fac = F;
    q.forward = true;
    q.n = p->n[k];
    q.P = 1;
    for (int m = 0; m < k; ++m) q.P *= p->n[m];
    q.R = 1;
    for (int m = k + 1; m < d; ++m) q.R *= p->n[m];
    q.epi = k == p->s ? Epi::Inv : Epi::None;
    q.bf16_tile = p->bf16_tile;
    if (!bf16_fold_pass_ok(q)) continue;
    b.ax[b.nax] = k;
    b.hh[b.nax] = p->n[k] / 2;
    ++b.nax;
  }
  return b.nax > 0;
}

// Whether a BF16 apply whose input sweep folds along fb's axes also runs its
// backward passes over the slower axes on half extents: d = 2 or 3 with every
// slower axis folded and of even extent; those passes leave their output
// folded, and the last pass, backward over the fastest axis, unfolds it
// before its FP64 stores.  `buf` stands for the buffers the passes use (the
// caller's output and the library's 256-byte aligned workspace).
static bool bf16_unfold_route(const ts_plan* p, const ButterflyArgs& fb, bool sym, const void* buf, bool accumulate) {
  const int d = p->d;
  if (!p->bf16_bwd_fold || (d != 2 && d != 3)) return false;
  for (int k = 0; k < d - 1; ++k) {
    bool in = false;
    for (int j = 0; j < fb.nax; ++j) in = in || fb.ax[j] == k;
    if (!in || p->n[k] % 2 != 0) return false;
  }
  PassArgs q;
  q.X = buf;
  q.Y = (void*)buf;
  q.tin = DT::BF16;
  q.prec = TS_PREC_BF16;
  q.forward = false;
  q.bf16_tile = p->bf16_tile;
  for (int k = 0; k < d; ++k) {
    q.fac = (sym ? p->ax_sym : p->ax)[k].get();
    q.n = p->n[k];
    q.P = 1;
    for (int m = 0; m < k; ++m) q.P *= p->n[m];
    q.R = 1;
    for (int m = k + 1; m < d; ++m) q.R *= p->n[m];
    if (k < d - 1) {
      q.tout = DT::BF16;
      q.fold = q.deferred = true;
      if (!bf16_fold_pass_ok(q)) return false;
    } else {
      q.tout = DT::F64;
      q.fold = q.deferred = false;
      q.accumulate = accumulate;
      q.unf = d - 1;
      for (int m = 0; m < d - 1; ++m) q.un[m] = p->n[m];
      if (!bf16_unfold_pass_ok(q)) return false;
    }
  }
  return true;
}

// Run the 2d passes of one apply.  Intermediates have the precision's type.
int run_apply(ts_plan* p, const ApplyParams& ap, hipStream_t st) {
  const int d = p->d;
  const bool cplx = ap.cplx;
  const int ncomp = cplx ? 2 : 1;
  // (FP64 transforms of FP32-stored data keep FP32 intermediates: the output
  // buffer, which holds every other intermediate, has room for no more)
  DT inter = ap.prec == TS_PREC_FP64 ? (ap.tin == DT::F32 && ap.tout == DT::F32 ? DT::F32 : DT::F64)
                                     : (ap.prec == TS_PREC_FP32 ? DT::F32 : DT::BF16);
  // pass order: forward over every axis but s (fastest first), then s with the
  // scaling epilogue; backward over s first, then the others.
  std::vector<int> order;
  for (int k = d - 1; k >= 0; --k)
    if (k != p->s) order.push_back(k);
  order.push_back(p->s);
  const int T = 2 * d;
  const void* src = ap.in;
  DT src_t = ap.tin;
  // Several folded axes: fold the input along all of them in one sweep (into
  // the output buffer, which the last pass overwrites), run the forward passes
  // on folded data and the backward passes without their butterflies, then
  // unfold the output in one sweep.  The butterflies act on one axis each and
  // so commute with the passes over the other axes.
  int fax[TS_MAX_D];
  int nf = 0;
  if (p->fold_enabled && ap.prec != TS_PREC_BF16 && ap.tin == ap.tout)
    for (int k = 0; k < d; ++k)
      if ((ap.sym ? p->ax_sym : p->ax)[k]->fold) fax[nf++] = k;
  const bool deferred = nf >= 2;
  auto butterfly = [&](const void* X, void* Y, DT t) -> int {
    for (int j0 = 0; j0 < nf; j0 += 4) {
      ButterflyArgs b;
      b.X = j0 == 0 ? X : Y;
      b.Y = Y;
      b.t = t;
      b.d = d;
      b.ncomp = ncomp;
      for (int k = 0; k < d; ++k) b.n[k] = p->n[k];
      b.nax = std::min(4, nf - j0);
      for (int j = 0; j < b.nax; ++j) {
        b.ax[j] = fax[j0 + j];
        b.hh[j] = p->n[b.ax[j]] / 2;
      }
      b.skip = ap.skip;
      hipError_t e = launch_butterfly(b, st);
      if (e != hipSuccess) {
        set_error(std::string("butterfly launch failed: ") + hipGetErrorString(e));
        return TS_ERR_DEVICE;
      }
    }
    return TS_OK;
  };
  if (deferred) {
    int rc = butterfly(ap.in, ap.out, ap.tin);
    if (rc) return rc;
    src = ap.out;
  }
  // BF16 transforms of FP64 data: the input sweep also folds the data along
  // the symmetric axes whose forward pass can read folded data (256 x 256
  // tiles), and those forward passes contract half the extent; the backward
  // passes run over the full extent on the spectral [even | odd] order, which
  // needs no unfolding afterwards.  (A caller that wrote the input itself,
  // in_rounded, folded it along the same axes when in_folded is set.)
  // With accumulate (out += the result), the intermediates that would go to
  // out go to the upper half of the workspace instead (BF16: 2 bytes a value,
  // the workspace holds 8).
  if (ap.accumulate && (ap.prec != TS_PREC_BF16 || ap.tout != DT::F64 || cplx || ap.in_rounded || ap.in == ap.out)) {
    set_error("accumulating applies are BF16 applies of FP64 data");
    return TS_ERR_INVALID;
  }
  void* const ob = ap.accumulate ? (void*)((char*)ap.work + 2 * (size_t)p->N) : ap.out;
  ButterflyArgs fb;
  int nb = 0;
  const int* bax = fb.ax;
  if (!cplx && ap.tin == DT::F64 && ap.tout == DT::F64 && (!ap.in_rounded || ap.in_folded) &&
      ap.epi != Epi::Exp && ap.prec == TS_PREC_BF16 && bf16_fold_axes(p, ap.in, ob, ap.sym, fb))
    nb = fb.nax;
  if (nb > 0 && (((uintptr_t)ap.work) & 15) != 0) {  // the folded passes read 16-byte chunks of it
    if (ap.in_folded) {
      set_error("BF16 apply on folded input needs a 16-byte aligned workspace");
      return TS_ERR_INVALID;
    }
    nb = 0;
  }
  auto bf16_folded = [&](int k) {
    for (int j = 0; j < nb; ++j)
      if (bax[j] == k) return true;
    return false;
  };
  // with every slower axis folded, the backward passes over them run on half
  // extents too, and the fastest axis goes last to unfold the output
  const bool unfold = nb > 0 && ap.tout == DT::F64 && bf16_unfold_route(p, fb, ap.sym, ap.out, ap.accumulate);
  std::vector<int> border{p->s};
  if (unfold) {
    for (int k = 0; k < d - 1; ++k)
      if (k != p->s) border.push_back(k);
    border.push_back(d - 1);
  } else {
    for (int j = 0; j + 1 < d; ++j) border.push_back(order[j]);
  }
  // BF16 transforms of FP64 data: round the input to BF16 in one streaming
  // sweep (into the output buffer, which the last pass overwrites), so that
  // the first pass reads 2 instead of 8 bytes per value (rounded as the pass
  // kernels would round it while loading)
  const int64_t Ntot = p->N * ncomp;
  if (ap.in_rounded) {
    // the caller's producer of the input already wrote its BF16 rounding to out
    src = ap.out;
    src_t = DT::BF16;
  } else if (nb > 0) {
    fb.skip = ap.skip;
    hipError_t e = launch_fold_to_bf16(fb, st);
    if (e != hipSuccess) {
      set_error(std::string("BF16 folding launch failed: ") + hipGetErrorString(e));
      return TS_ERR_DEVICE;
    }
    src = ob;
    src_t = DT::BF16;
  } else if (ap.prec == TS_PREC_BF16 && ap.tin == DT::F64 && ap.in != ap.out && Ntot % 4 == 0 &&
      ((((uintptr_t)ap.in) & 15) == 0) && ((((uintptr_t)ob) & 7) == 0)) {
    hipError_t e = launch_data_to_bf16((const double*)ap.in, (uint16_t*)ob, Ntot, ap.skip, st);
    if (e != hipSuccess) {
      set_error(std::string("BF16 rounding launch failed: ") + hipGetErrorString(e));
      return TS_ERR_DEVICE;
    }
    src = ob;
    src_t = DT::BF16;
  }
  for (int t = 1; t <= T; ++t) {
    const bool fwd = t <= d;
    const int k = fwd ? order[t - 1] : border[t - d - 1];
    void* dst = ((T - t) % 2 == 0) ? (t == T ? ap.out : ob) : ap.work;
    DT dst_t = (t == T) ? ap.tout : inter;
    PassArgs pa;
    pa.X = src;
    pa.Y = dst;
    pa.tin = src_t;
    pa.tout = dst_t;
    pa.prec = ap.prec;
    pa.fac = (ap.sym ? p->ax_sym : p->ax)[k].get();
    pa.forward = fwd;
    pa.n = p->n[k];
    pa.P = 1;
    for (int m = 0; m < k; ++m) pa.P *= p->n[m];
    pa.R = (int64_t)ncomp;
    for (int m = k + 1; m < d; ++m) pa.R *= p->n[m];
    pa.cplx = cplx;
    pa.skip = ap.skip;
    // BF16 passes fold only as forward passes on data the input sweep folded
    // (above): folding while loading (mirror loads) and a butterfly after each
    // backward pass cost the 128 x 128 BF16 tiles more than the halved products
    pa.fold = pa.fac->fold && p->fold_enabled && ap.prec != TS_PREC_BF16;
    pa.deferred = deferred && pa.fold;
    if (ap.prec == TS_PREC_BF16 && fwd && bf16_folded(k)) pa.fold = pa.deferred = true;
    if (unfold && !fwd) {
      if (t < T) {
        pa.fold = pa.deferred = true;
      } else {
        pa.unf = d - 1;
        for (int m = 0; m < d - 1; ++m) pa.un[m] = p->n[m];
      }
    }
    pa.accumulate = ap.accumulate && t == T;
    pa.bf16_tile = p->bf16_tile;
    if (fwd && t == d) {
      pa.epi = ap.epi;
      pa.Lp = p->Lp;
      pa.Lr = p->Lr;
      pa.shift = ap.shift;
      pa.Ep = ap.phase;
      pa.Er = ap.phase ? ap.phase + p->Ps : nullptr;
      pa.es = ap.phase ? ap.phase + p->Ps + p->Rs : nullptr;
    }
    hipError_t e = launch_pass(pa, st);
    if (e != hipSuccess) {
      set_error(std::string("mode pass launch failed: ") + hipGetErrorString(e));
      return TS_ERR_DEVICE;
    }
    src = dst;
    src_t = dst_t;
  }
  return deferred ? butterfly(ap.out, ap.out, ap.tout) : TS_OK;
}

bool bf16_sweep_applies(const ts_plan* p, const void* in, const void* out) {
  return !plan_is_small(p) && in != out && p->N % 4 == 0 && (((uintptr_t)in) & 15) == 0 &&
         (((uintptr_t)out) & 7) == 0;
}

bool bf16_accumulate_ok(const ts_plan* p, const void* in, const void* out, bool sym) {
  if (plan_is_small(p) || in == out || p->N % 8 != 0 || (((uintptr_t)out) & 15) != 0) return false;
  ButterflyArgs fb;
  if (bf16_fold_axes(p, in, (void*)out, sym, fb) && bf16_unfold_route(p, fb, sym, out, true)) return true;
  // the last pass (run_apply's order): backward along the lowest axis other
  // than the scaling axis s, or along s itself in 1D
  const int d = p->d;
  int k = p->s;
  for (int m = d - 1; m >= 0; --m)
    if (m != p->s) k = m;
  PassArgs q;
  q.X = out;  // stands for the workspace (library allocation, 256-byte aligned)
  q.Y = (void*)out;
  q.tin = DT::BF16;
  q.tout = DT::F64;
  q.prec = TS_PREC_BF16;
  q.fac = (sym ? p->ax_sym : p->ax)[k].get();
  q.forward = false;
  q.n = p->n[k];
  q.P = 1;
  for (int m = 0; m < k; ++m) q.P *= p->n[m];
  q.R = 1;
  for (int m = k + 1; m < d; ++m) q.R *= p->n[m];
  q.bf16_tile = p->bf16_tile;
  q.accumulate = true;
  return bf16_big_pass_ok(q);
}

int apply_inverse_impl(ts_plan* p, double shift, const void* b, void* u, int dtype, int prec,
                       hipStream_t st, ExecCtx& c, const int* skip, bool sym, bool in_rounded, bool in_folded,
                       bool accumulate) {
  if (!p || !b || !u) { set_error("null argument"); return TS_ERR_INVALID; }
  if (dtype != TS_F64 && dtype != TS_F32) { set_error("inverse apply needs TS_F64 or TS_F32 data"); return TS_ERR_INVALID; }
  if (prec < TS_PREC_FP64 || prec > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  if (!(p->lam_min + shift > 0.0)) {
    set_error("H1 + sigma is not positive definite: lambda_min(H1) + sigma = " + std::to_string(p->lam_min + shift));
    return TS_ERR_NOT_SPD;
  }
  if (plan_is_small(p)) {
    SmallApply sa;
    sa.in = b;
    sa.out = u;
    sa.tio = dt_of(dtype);
    sa.fp64 = prec == TS_PREC_FP64;
    sa.cplx = false;
    sa.epi = Epi::Inv;
    sa.shift = shift;
    sa.skip = skip;
    sa.sym = sym;
    return run_small_apply(p, sa, st, c);
  }
  void* work = nullptr;
  int rc = ctx_get(c, kSlotWork, need_inverse(p, kSlotWork), &work);
  if (rc) return rc;
  ApplyParams ap;
  ap.in = b;
  ap.out = u;
  ap.work = work;
  ap.tin = ap.tout = dt_of(dtype);
  ap.prec = prec;
  ap.cplx = false;
  ap.epi = Epi::Inv;
  ap.shift = shift;
  ap.skip = skip;
  ap.sym = sym;
  ap.in_rounded = in_rounded && prec == TS_PREC_BF16 && dtype == TS_F64 && bf16_sweep_applies(p, b, u);
  ap.in_folded = ap.in_rounded && in_folded;
  ap.accumulate = accumulate;
  return run_apply(p, ap, st);
}

static int check_exp_args(ts_plan* p, double tau, const void* in, const void* out, int dtype, int prec) {
  if (!p || !in || !out) { set_error("null argument"); return TS_ERR_INVALID; }
  if (dtype != TS_C128 && dtype != TS_C64) { set_error("propagator needs TS_C128 or TS_C64 data"); return TS_ERR_INVALID; }
  if (prec < TS_PREC_FP64 || prec > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  if (!std::isfinite(tau)) { set_error("tau is not finite"); return TS_ERR_INVALID; }
  return TS_OK;
}

// The MFMA-path propagator: phase tables for the scaling axis, then 2d passes.
static int exp_mfma(ts_plan* p, double tau, const void* in, void* out, int dtype, int prec, hipStream_t st,
                    ExecCtx& c) {
  void *work = nullptr, *tabs = nullptr;
  int rc = ctx_get(c, kSlotWork, need_exp(p, kSlotWork), &work);
  if (rc) return rc;
  rc = ctx_get(c, kSlotPhase, need_exp(p, kSlotPhase), &tabs);
  if (rc) return rc;
  double2* phase = (double2*)tabs;
  PhaseTableArgs pt;
  pt.d = p->d;
  pt.s = p->s;
  for (int k = 0; k < p->d; ++k) {
    pt.n[k] = p->n[k];
    pt.lam[k] = p->ax[k]->lam;
  }
  pt.tau = tau;
  pt.Ep = phase;
  pt.Er = phase + p->Ps;
  pt.es = phase + p->Ps + p->Rs;
  pt.P = p->Ps;
  pt.R = p->Rs;
  hipError_t e = launch_phase_tables(pt, st);
  if (e != hipSuccess) { set_error("phase table launch failed"); return TS_ERR_DEVICE; }
  ApplyParams ap;
  ap.in = in;
  ap.out = out;
  ap.work = work;
  ap.tin = ap.tout = dt_of(dtype);
  ap.prec = prec;
  ap.cplx = true;
  ap.epi = Epi::Exp;
  ap.phase = phase;
  return run_apply(p, ap, st);
}

int apply_exp_impl(ts_plan* p, double tau, const void* in, void* out, int dtype, int prec,
                   hipStream_t st, ExecCtx& c) {
  int rc = check_exp_args(p, tau, in, out, dtype, prec);
  if (rc) return rc;
  if (plan_is_small(p)) {
    SmallApply sa;
    sa.in = in;
    sa.out = out;
    sa.tio = dt_of(dtype);
    sa.fp64 = prec == TS_PREC_FP64;
    sa.cplx = true;
    sa.epi = Epi::Exp;
    sa.tau = tau;
    return run_small_apply(p, sa, st, c);
  }
  return exp_mfma(p, tau, in, out, dtype, prec, st, c);
}

int apply_exp_phased(ts_plan* p, double tau, void* psi, int dtype, int prec, const Phases& ph,
                     hipStream_t st, ExecCtx& c) {
  int rc = check_exp_args(p, tau, psi, psi, dtype, prec);
  if (rc) return rc;
  const bool fp64_data = dtype == TS_C128;
  if (plan_is_small(p)) {
    SmallApply sa;
    sa.in = psi;
    sa.out = psi;
    sa.tio = dt_of(dtype);
    sa.fp64 = prec == TS_PREC_FP64;
    sa.cplx = true;
    sa.epi = Epi::Exp;
    sa.tau = tau;
    sa.V2 = ph.V2;
    sa.pre = ph.pre;
    sa.post = ph.post;
    sa.th_pre = ph.th_pre;
    sa.th_post = ph.th_post;
    return run_small_apply(p, sa, st, c);
  }
  hipError_t e;
  if (ph.pre) {
    e = launch_phase(psi, ph.V2, ph.th_pre, p->N, fp64_data, st);
    if (e != hipSuccess) { set_error("phase launch failed"); return TS_ERR_DEVICE; }
  }
  rc = exp_mfma(p, tau, psi, psi, dtype, prec, st, c);
  if (rc) return rc;
  if (ph.post) {
    e = launch_phase(psi, ph.V2, ph.th_post, p->N, fp64_data, st);
    if (e != hipSuccess) { set_error("phase launch failed"); return TS_ERR_DEVICE; }
  }
  return TS_OK;
}

}  // namespace ts

ts_plan::~ts_plan() {
  hipFree(Lp);
  hipFree(Lr);
}

namespace ts {
// Eigenvalue bound, scaling axis and its eigenvalue-sum tables (shared by FD
// and SEM setup).
static int finish_plan(ts_plan* p) {
  const int d = p->d;
  if (p->ax_sym.empty()) p->ax_sym = p->ax;
  p->lam_min = 0.0;
  for (int k = 0; k < d; ++k) p->lam_min += p->ax[k]->lam_h[0];
  // scaling axis: a non-fastest axis balancing the two table lengths
  p->s = 0;
  if (d >= 2) {
    int64_t best = -1;
    for (int s = 0; s <= d - 2; ++s) {
      int64_t P = 1, R = 1;
      for (int m = 0; m < s; ++m) P *= p->n[m];
      for (int m = s + 1; m < d; ++m) R *= p->n[m];
      int64_t c = std::max(P, R);
      if (best < 0 || c < best) { best = c; p->s = s; }
    }
  }
  p->Ps = 1;
  p->Rs = 1;
  for (int m = 0; m < p->s; ++m) p->Ps *= p->n[m];
  for (int m = p->s + 1; m < d; ++m) p->Rs *= p->n[m];
  // eigenvalue-sum tables of the axes before / after s (FP64, host-built)
  std::vector<double> Lp(p->Ps), Lr(p->Rs);
  for (int64_t i = 0; i < p->Ps; ++i) {
    int64_t idx = i;
    double s = 0.0;
    for (int m = p->s - 1; m >= 0; --m) { s += p->ax[m]->lam_int_h[idx % p->n[m]]; idx /= p->n[m]; }
    Lp[i] = s;
  }
  for (int64_t i = 0; i < p->Rs; ++i) {
    int64_t idx = i;
    double s = 0.0;
    for (int m = d - 1; m > p->s; --m) { s += p->ax[m]->lam_int_h[idx % p->n[m]]; idx /= p->n[m]; }
    Lr[i] = s;
  }
  hipError_t e = hipMalloc(&p->Lp, sizeof(double) * p->Ps);
  if (e == hipSuccess) e = hipMalloc(&p->Lr, sizeof(double) * p->Rs);
  if (e != hipSuccess) { set_error("table allocation failed"); return TS_ERR_NOMEM; }
  e = hipMemcpy(p->Lp, Lp.data(), sizeof(double) * p->Ps, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->Lr, Lr.data(), sizeof(double) * p->Rs, hipMemcpyHostToDevice);
  if (e != hipSuccess) { set_error("table upload failed"); return TS_ERR_DEVICE; }
  return TS_OK;
}

}  // namespace ts

using namespace ts;

extern "C" {

const char* ts_last_error(void) { return g_err.c_str(); }

int ts_setup(int d, const int64_t* n, double L, const double* const* f, double sigma, ts_plan** out) {
  set_error("");
  if (!out || !n || !f) { set_error("null argument"); return TS_ERR_INVALID; }
  *out = nullptr;
  if (d < 1 || d > TS_MAX_D) { set_error("d must be in [1, 12]"); return TS_ERR_INVALID; }
  if (!(L > 0.0) || !std::isfinite(L)) { set_error("L must be positive"); return TS_ERR_INVALID; }
  if (!std::isfinite(sigma)) { set_error("sigma must be finite"); return TS_ERR_INVALID; }
  int64_t N = 1;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1 || n[k] > 16384) { set_error("n[k] must be in [1, 16384]"); return TS_ERR_INVALID; }
    if (!f[k]) { set_error("f[k] is null"); return TS_ERR_INVALID; }
    for (int64_t j = 0; j < n[k]; ++j)
      if (!std::isfinite(f[k][j])) { set_error("f[k] has a non-finite sample"); return TS_ERR_NONFINITE; }
    N *= n[k];
    if (N >= (int64_t(1) << 40)) { set_error("grid too large"); return TS_ERR_INVALID; }
  }
  auto p = std::unique_ptr<ts_plan>(new ts_plan());
  p->d = d;
  p->N = N;
  p->L = L;
  p->sigma = sigma;
  hipGetDevice(&p->device);
  std::map<std::pair<int64_t, std::string>, std::shared_ptr<AxisFactor>> cache;
  for (int k = 0; k < d; ++k) {
    p->n[k] = n[k];
    std::string key((const char*)f[k], sizeof(double) * (size_t)n[k]);
    auto it = cache.find({n[k], key});
    if (it != cache.end()) {
      p->ax.push_back(it->second);
      continue;
    }
    std::shared_ptr<AxisFactor> F;
    int rc = build_axis(n[k], L, f[k], F);
    if (rc) return rc;
    cache[{n[k], key}] = F;
    p->ax.push_back(F);
  }
  int rc = finish_plan(p.get());
  if (rc) return rc;
  *out = p.release();
  return TS_OK;
}

int ts_setup_sem(int d, const int64_t* cells, int k, double L, const double* const* f, double sigma,
                 ts_plan** out) {
  set_error("");
  if (!out || !cells || !f) { set_error("null argument"); return TS_ERR_INVALID; }
  *out = nullptr;
  if (d < 1 || d > TS_MAX_D) { set_error("d must be in [1, 12]"); return TS_ERR_INVALID; }
  if (k < 1 || k > kMaxSemOrder) { set_error("k must be in [1, 32]"); return TS_ERR_INVALID; }
  if (!(L > 0.0) || !std::isfinite(L)) { set_error("L must be positive"); return TS_ERR_INVALID; }
  if (!std::isfinite(sigma)) { set_error("sigma must be finite"); return TS_ERR_INVALID; }
  int64_t N = 1;
  for (int a = 0; a < d; ++a) {
    const int64_t n = (int64_t)k * cells[a] - 1;
    if (cells[a] < 1 || n < 1 || n > 8192) { set_error("k * cells[a] - 1 must be in [1, 8192]"); return TS_ERR_INVALID; }
    if (!f[a]) { set_error("f[a] is null"); return TS_ERR_INVALID; }
    for (int64_t j = 0; j < n; ++j)
      if (!std::isfinite(f[a][j])) { set_error("f[a] has a non-finite sample"); return TS_ERR_NONFINITE; }
    N *= n;
    if (N >= (int64_t(1) << 40)) { set_error("grid too large"); return TS_ERR_INVALID; }
  }
  auto p = std::unique_ptr<ts_plan>(new ts_plan());
  p->d = d;
  p->N = N;
  p->L = L;
  p->sigma = sigma;
  p->sem_k = k;
  p->massed = true;
  hipGetDevice(&p->device);
  std::map<std::pair<int64_t, std::string>, std::pair<std::shared_ptr<AxisFactor>, std::shared_ptr<AxisFactor>>> cache;
  bool op = false;  // one decision for the whole plan: every axis or none has operator pass factors
  for (int a = 0; a < d; ++a) op = op || (int64_t)k * cells[a] - 1 >= kOpPassMinN;
  for (int a = 0; a < d; ++a) {
    const int64_t n = (int64_t)k * cells[a] - 1;
    p->n[a] = n;
    std::string key((const char*)f[a], sizeof(double) * (size_t)n);
    auto it = cache.find({cells[a], key});
    if (it == cache.end()) {
      std::shared_ptr<AxisFactor> P, S;
      int rc = build_axis_sem(k, cells[a], L, f[a], op, P, S);
      if (rc) return rc;
      it = cache.insert({{cells[a], key}, {P, S}}).first;
    }
    p->ax.push_back(it->second.first);
    p->ax_sym.push_back(it->second.second);
  }
  int rc = finish_plan(p.get());
  if (rc) return rc;
  *out = p.release();
  return TS_OK;
}

int ts_setup_general(int d, const int64_t* n, const double* const* K, const double* const* m,
                     const double* const* x, const double* const* f, double sigma, ts_plan** out) {
  set_error("");
  if (!out || !n || !K || !f) { set_error("null argument"); return TS_ERR_INVALID; }
  *out = nullptr;
  if (d < 1 || d > TS_MAX_D) { set_error("d must be in [1, 12]"); return TS_ERR_INVALID; }
  if (!std::isfinite(sigma)) { set_error("sigma must be finite"); return TS_ERR_INVALID; }
  int64_t N = 1;
  int bw = 1;  // at least 1: the band path serves every generic plan
  for (int a = 0; a < d; ++a) {
    if (n[a] < 1 || n[a] > 8192) { set_error("n[a] must be in [1, 8192]"); return TS_ERR_INVALID; }
    if (!K[a] || !f[a]) { set_error("K[a] or f[a] is null"); return TS_ERR_INVALID; }
    for (int64_t j = 0; j < n[a]; ++j)
      if (!std::isfinite(f[a][j])) { set_error("f[a] has a non-finite sample"); return TS_ERR_NONFINITE; }
    for (int64_t i = 0; i < n[a]; ++i)
      for (int64_t j = 0; j < n[a]; ++j)
        if (K[a][(size_t)(i * n[a] + j)] != 0.0) bw = std::max<int>(bw, (int)std::llabs(i - j));
    N *= n[a];
    if (N >= (int64_t(1) << 40)) { set_error("grid too large"); return TS_ERR_INVALID; }
  }
  auto p = std::unique_ptr<ts_plan>(new ts_plan());
  p->d = d;
  p->N = N;
  p->L = 0.0;
  p->sigma = sigma;
  p->massed = true;
  hipGetDevice(&p->device);
  for (int a = 0; a < d; ++a) {
    p->n[a] = n[a];
    int b;  // reuse the factors of an earlier identical axis
    for (b = 0; b < a; ++b) {
      if (n[b] != n[a] || K[b] != K[a] || (m ? m[b] : nullptr) != (m ? m[a] : nullptr)) continue;
      if (std::memcmp(f[b], f[a], sizeof(double) * (size_t)n[a]) == 0) break;
    }
    if (b < a) {
      p->ax.push_back(p->ax[b]);
      p->ax_sym.push_back(p->ax_sym[b]);
      continue;
    }
    std::shared_ptr<AxisFactor> P, S;
    int rc = build_axis_general(n[a], K[a], m ? m[a] : nullptr, x ? x[a] : nullptr, f[a], bw, P, S);
    if (rc) return rc;
    p->ax.push_back(P);
    p->ax_sym.push_back(S);
  }
  int rc = finish_plan(p.get());
  if (rc) return rc;
  *out = p.release();
  return TS_OK;
}

int ts_sem_nodes(int k, int64_t cells, double L, double* x) {
  if (!x) { set_error("null argument"); return TS_ERR_INVALID; }
  SemAxis ax;
  if (!sem_axis(k, cells, L, ax)) { set_error("bad SEM axis (k in [1, 32], cells >= 1, L > 0)"); return TS_ERR_INVALID; }
  std::memcpy(x, ax.x.data(), sizeof(double) * (size_t)ax.n);
  return TS_OK;
}

int ts_sem_axis_eig(int k, int64_t cells, double L, const double* f, double* lam, double* Q, double* m) {
  if (!f || !lam || !Q) { set_error("null argument"); return TS_ERR_INVALID; }
  SemAxis ax;
  if (!sem_axis(k, cells, L, ax)) { set_error("bad SEM axis (k in [1, 32], cells >= 1, L > 0)"); return TS_ERR_INVALID; }
  const int64_t n = ax.n;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(f[i])) { set_error("f has a non-finite entry"); return TS_ERR_NONFINITE; }
  std::vector<long double> Al;
  std::vector<double> A;
  sem_operator(ax, Al, A, nullptr, nullptr);
  FoldPlan fp;
  if (!massed_eig(n, A, &Al, f, symmetric_samples(n, f), lam, Q, fp)) {
    set_error("symmetric eigensolver did not converge");
    return TS_ERR_NOCONV;
  }
  if (m) std::memcpy(m, ax.m.data(), sizeof(double) * (size_t)n);
  return TS_OK;
}

int ts_mass(const ts_plan* plan, int axis, double* out) {
  if (!plan || !out || axis < 0 || axis >= plan->d) { set_error("bad argument"); return TS_ERR_INVALID; }
  const auto& F = *plan->ax[axis];
  if (plan->massed) {
    std::memcpy(out, F.m_h.data(), sizeof(double) * (size_t)F.n);
  } else {
    const double h = 2.0 * plan->L / (double)(F.n + 1);
    for (int64_t i = 0; i < F.n; ++i) out[i] = h;
  }
  return TS_OK;
}

int ts_mode_pass(ts_plan* plan, int axis, int forward, const void* in, void* out, int dtype, int prec,
                 void* hip_stream) {
  if (!plan || !in || !out || axis < 0 || axis >= plan->d) { set_error("bad argument"); return TS_ERR_INVALID; }
  if (in == out) { set_error("in and out must not alias"); return TS_ERR_INVALID; }
  if (dtype != TS_F64 && dtype != TS_F32 && dtype != TS_C128 && dtype != TS_C64) { set_error("bad dtype"); return TS_ERR_INVALID; }
  if (prec != TS_PREC_FP64 && prec != TS_PREC_FP32 && prec != TS_PREC_BF16) { set_error("bad prec"); return TS_ERR_INVALID; }
  const bool f64 = dtype == TS_F64 || dtype == TS_C128;
  if (prec == TS_PREC_FP64 && !f64) { set_error("FP64 transforms need FP64 data"); return TS_ERR_INVALID; }
  if (forward < 0 || forward > 3) { set_error("forward must be 0, 1, 2 or 3"); return TS_ERR_INVALID; }
  if (forward >= 2 && prec == TS_PREC_BF16) {
    set_error("BF16 passes have no folded-data form (modes 2 and 3)");
    return TS_ERR_INVALID;
  }
  const bool cplx = dtype == TS_C128 || dtype == TS_C64;
  PassArgs pa;
  pa.X = in;
  pa.Y = out;
  pa.tin = pa.tout = f64 ? DT::F64 : DT::F32;
  pa.prec = prec;
  pa.fac = plan->ax[axis].get();
  pa.forward = forward == 1 || forward == 2;
  pa.n = plan->n[axis];
  pa.P = 1;
  for (int m = 0; m < axis; ++m) pa.P *= plan->n[m];
  pa.R = cplx ? 2 : 1;
  for (int m = axis + 1; m < plan->d; ++m) pa.R *= plan->n[m];
  pa.cplx = cplx;
  pa.fold = pa.fac->fold && plan->fold_enabled;
  pa.deferred = pa.fold && forward >= 2;
  pa.bf16_tile = plan->bf16_tile;
  hipError_t e = launch_pass(pa, (hipStream_t)hip_stream);
  if (e != hipSuccess) { set_error(std::string("mode pass launch failed: ") + hipGetErrorString(e)); return TS_ERR_DEVICE; }
  return TS_OK;
}

int ts_fold_butterfly(ts_plan* plan, int axes, const void* in, void* out, int dtype, void* hip_stream) {
  if (!plan || !in || !out) { set_error("null argument"); return TS_ERR_INVALID; }
  if (dtype != TS_F64 && dtype != TS_F32 && dtype != TS_C128 && dtype != TS_C64) { set_error("bad dtype"); return TS_ERR_INVALID; }
  if (axes <= 0 || axes >= (1 << plan->d)) { set_error("axes must be a non-empty mask of the plan's axes"); return TS_ERR_INVALID; }
  int ax[TS_MAX_D];
  int na = 0;
  for (int k = 0; k < plan->d; ++k)
    if (axes & (1 << k)) ax[na++] = k;
  const void* src = in;
  for (int j0 = 0; j0 < na; j0 += 4) {
    ButterflyArgs b;
    b.X = src;
    b.Y = out;
    b.t = (dtype == TS_F64 || dtype == TS_C128) ? DT::F64 : DT::F32;
    b.d = plan->d;
    b.ncomp = (dtype == TS_C128 || dtype == TS_C64) ? 2 : 1;
    for (int k = 0; k < plan->d; ++k) b.n[k] = plan->n[k];
    b.nax = std::min(4, na - j0);
    for (int j = 0; j < b.nax; ++j) {
      b.ax[j] = ax[j0 + j];
      b.hh[j] = plan->n[b.ax[j]] / 2;
    }
    hipError_t e = launch_butterfly(b, (hipStream_t)hip_stream);
    if (e != hipSuccess) { set_error(std::string("butterfly launch failed: ") + hipGetErrorString(e)); return TS_ERR_DEVICE; }
    src = out;
  }
  return TS_OK;
}

int ts_set_fold(ts_plan* plan, int enable) {
  if (!plan) { set_error("null plan"); return TS_ERR_INVALID; }
  if (enable < 0 || enable > 2) { set_error("fold mode must be 0, 1 or 2"); return TS_ERR_INVALID; }
  plan->fold_enabled = enable != 0;
  plan->bf16_bwd_fold = enable == 1;
  return TS_OK;
}

int ts_set_bf16_tile(ts_plan* plan, int tile) {
  if (!plan) { set_error("null plan"); return TS_ERR_INVALID; }
  if (tile != 0 && tile != 128 && tile != 256) { set_error("BF16 tile must be 0, 128 or 256"); return TS_ERR_INVALID; }
  plan->bf16_tile = tile;
  return TS_OK;
}

int ts_fold_axes(const ts_plan* plan, int* folded) {
  if (!plan || !folded) { set_error("null argument"); return TS_ERR_INVALID; }
  int mask = 0;
  for (int k = 0; k < plan->d; ++k)
    if (plan->ax[k]->fold) mask |= 1 << k;
  *folded = mask;
  return TS_OK;
}

int ts_destroy(ts_plan* plan) {
  if (!plan) return TS_OK;
  hipDeviceSynchronize();
  delete plan;
  return TS_OK;
}

int ts_apply_inverse(ts_plan* plan, const void* b, void* u, int dtype, int prec, void* hip_stream) {
  if (!plan) { set_error("null plan"); return TS_ERR_INVALID; }
  return apply_inverse_impl(plan, plan->sigma, b, u, dtype, prec, (hipStream_t)hip_stream, plan->ctx, nullptr);
}

int ts_apply_inverse_shift(ts_plan* plan, double s, const void* b, void* u, int dtype, int prec,
                           void* hip_stream) {
  if (!plan) { set_error("null plan"); return TS_ERR_INVALID; }
  if (!std::isfinite(s)) { set_error("shift is not finite"); return TS_ERR_INVALID; }
  return apply_inverse_impl(plan, s, b, u, dtype, prec, (hipStream_t)hip_stream, plan->ctx, nullptr);
}

int ts_apply_exp(ts_plan* plan, double tau, const void* psi_in, void* psi_out, int dtype, int prec,
                 void* hip_stream) {
  if (!plan) { set_error("null plan"); return TS_ERR_INVALID; }
  return apply_exp_impl(plan, tau, psi_in, psi_out, dtype, prec, (hipStream_t)hip_stream, plan->ctx);
}

int ts_eigvals(const ts_plan* plan, int axis, double* out) {
  if (!plan || !out || axis < 0 || axis >= plan->d) { set_error("bad argument"); return TS_ERR_INVALID; }
  const auto& F = *plan->ax[axis];
  std::memcpy(out, F.lam_h.data(), sizeof(double) * F.n);
  return TS_OK;
}

int ts_eigvecs(const ts_plan* plan, int axis, double* out) {
  if (!plan || !out || axis < 0 || axis >= plan->d) { set_error("bad argument"); return TS_ERR_INVALID; }
  const auto& F = *plan->ax[axis];
  std::memcpy(out, F.Q_h.data(), sizeof(double) * F.n * F.n);
  return TS_OK;
}

int ts_tridiag_eig(int64_t n, const double* diag, const double* off, double* lam, double* Q) {
  if (n < 1 || !diag || !lam || !Q || (n > 1 && !off)) { set_error("bad argument"); return TS_ERR_INVALID; }
  if (!tridiag_eig(n, diag, off, lam, Q)) { set_error("QL iteration limit reached"); return TS_ERR_NOCONV; }
  return TS_OK;
}

int ts_tridiag_eig_even_odd(int64_t n, const double* diag, const double* off, double* lam, double* Q) {
  if (n < 2 || !diag || !off || !lam || !Q) { set_error("bad argument"); return TS_ERR_INVALID; }
  for (int64_t i = 0; i < n; ++i)
    if (diag[i] != diag[n - 1 - i]) { set_error("diagonal is not reflection-symmetric"); return TS_ERR_INVALID; }
  for (int64_t i = 0; i + 1 < n; ++i)
    if (off[i] != off[n - 2 - i]) { set_error("off-diagonal is not reflection-symmetric"); return TS_ERR_INVALID; }
  FoldPlan fp;
  if (!split_eig_tridiag(n, diag, off, lam, Q, fp)) { set_error("QL iteration limit reached"); return TS_ERR_NOCONV; }
  return TS_OK;
}

int ts_bf16_round(int64_t n, const double* x, int route, uint16_t* y) {
  if (n < 0 || (n > 0 && (!x || !y)) || (route != 0 && route != 1)) { set_error("bad argument"); return TS_ERR_INVALID; }
  for (int64_t i = 0; i < n; ++i) y[i] = route == 0 ? bf16_from_f64(x[i]) : bf16_from_f32((float)x[i]);
  return TS_OK;
}

int ts_sym_eig(int64_t n, const double* A, double* lam, double* Q) {
  if (n < 1 || !A || !lam || !Q) { set_error("bad argument"); return TS_ERR_INVALID; }
  std::vector<double> W(A, A + n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) W[(size_t)(i * n + j)] = W[(size_t)(j * n + i)] = 0.5 * (A[i * n + j] + A[j * n + i]);
  if (!dense_sym_eig(n, W, lam, Q)) { set_error("QL iteration limit reached"); return TS_ERR_NOCONV; }
  return TS_OK;
}

int ts_workspace_bytes(const ts_plan* plan, int dtype, size_t* bytes) {
  if (!plan || !bytes) { set_error("bad argument"); return TS_ERR_INVALID; }
  size_t per = (dtype == TS_C128 || dtype == TS_C64) ? 16 : 8;
  *bytes = per * (size_t)plan->N;
  return TS_OK;
}

}  // extern "C"
