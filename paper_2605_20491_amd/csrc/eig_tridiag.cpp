// Host FP64 eigendecomposition of a symmetric tridiagonal matrix by the
// implicit QL method with Wilkinson-type shifts (Bowdler, Martin, Reinsch &
// Wilkinson, "The QR and QL algorithms for symmetric matrices", Numer. Math.
// 11 (1968); the "tql2" procedure of the Handbook for Automatic Computation).
//
// Used by plan setup for the per-axis matrices H_k = h^-2 tridiag(-1,2,-1) +
// diag(f_k) (paper Sec. 2.1, eq. (eigen_decomp)); the "one-time" O(n^3) step.
//
// Structure chosen for a many-core host: the QL sweeps on (diag, offdiag)
// are O(n^2) in total and run first, recording every Givens rotation in the
// order it is generated.  The O(n^3) eigenvector accumulation then applies
// that rotation sequence to independent column slices of Z^T in parallel,
// with no synchronisation between threads.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <thread>
#include <vector>

#include "ts_internal.h"

namespace ts {

namespace {

struct Rot {
  int32_t i;  // rotates rows i and i+1 of Z^T
  double c, s;
};

}  // namespace

// diag[n], off[n-1] (off[i] couples i and i+1).  On success returns true and
// fills lam (ascending) and Q (row-major n x n, column j = eigenvector j).
//
// QL chases from the bottom and keeps small eigenvalues to high relative
// accuracy when the matrix is graded with its large entries at the bottom;
// a matrix graded the other way (as Householder reduction leaves the Q^k SEM
// operators) is reversed first and its eigenvectors reversed back.
bool tridiag_eig(int64_t n, const double* diag, const double* off, double* lam, double* Q) {
  const bool flip = n > 1 && std::fabs(diag[0]) + std::fabs(off[0]) > std::fabs(diag[n - 1]) + std::fabs(off[n - 2]);
  std::vector<double> d(n);
  std::vector<double> e(n, 0.0);
  for (int64_t i = 0; i < n; ++i) d[i] = flip ? diag[n - 1 - i] : diag[i];
  for (int64_t i = 0; i + 1 < n; ++i) e[i] = flip ? off[n - 2 - i] : off[i];
  std::vector<Rot> rots;
  rots.reserve((size_t)std::max<int64_t>(16, 2 * n * n));
  const double eps = std::numeric_limits<double>::epsilon();

  for (int64_t l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      // find a negligible off-diagonal element at or after l
      int64_t m = l;
      for (; m + 1 < n; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;  // d[l] is an eigenvalue
      if (++iter > 60) return false;
      // shift: eigenvalue of the leading 2x2 block closer to d[l]
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool early = false;
      for (int64_t i = m - 1; i >= l; --i) {
        double f = s * e[i];
        double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // underflow: split the problem here
          d[i + 1] -= p;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        rots.push_back(Rot{(int32_t)i, c, s});
      }
      if (early) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }

  // Z^T starts as the identity; apply the recorded rotations to column slices.
  std::vector<double> Zt((size_t)(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i) Zt[(size_t)(i * n + i)] = 1.0;
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  int64_t nthreads = std::min<int64_t>(std::min<int64_t>(hw, 32), std::max<int64_t>(1, n / 32));
  auto work = [&](int64_t k0, int64_t k1) {
    for (const Rot& R : rots) {
      double* a = &Zt[(size_t)(R.i * n)];
      double* b = a + n;
      for (int64_t k = k0; k < k1; ++k) {
        double zb = b[k];
        b[k] = R.s * a[k] + R.c * zb;
        a[k] = R.c * a[k] - R.s * zb;
      }
    }
  };
  if (nthreads <= 1) {
    work(0, n);
  } else {
    std::vector<std::thread> th;
    int64_t chunk = (n + nthreads - 1) / nthreads;
    for (int64_t t = 0; t < nthreads; ++t) {
      int64_t k0 = t * chunk, k1 = std::min(n, k0 + chunk);
      if (k0 < k1) th.emplace_back(work, k0, k1);
    }
    for (auto& t : th) t.join();
  }

  // sort ascending; Q[:, j] = row perm[j] of Z^T; sign: largest entry positive
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
  for (int64_t j = 0; j < n; ++j) {
    const double* zr = &Zt[(size_t)(perm[j] * n)];
    auto z = [&](int64_t k) { return flip ? zr[n - 1 - k] : zr[k]; };
    int64_t arg = 0;
    for (int64_t k = 1; k < n; ++k)
      if (std::fabs(z(k)) > std::fabs(z(arg))) arg = k;
    double sg = z(arg) < 0.0 ? -1.0 : 1.0;
    lam[j] = d[perm[j]];
    for (int64_t k = 0; k < n; ++k) Q[k * n + j] = sg * z(k);
  }
  return true;
}

}  // namespace ts
