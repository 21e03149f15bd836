// Host setup of the Q^k spectral-element per-axis operators (paper Sec. 2,
// eq. (eigen_decomp)): Gauss-Lobatto nodes and weights, the Lagrange
// derivative matrix, the assembled stiffness S and lumped mass M of one axis,
// and a dense symmetric eigensolver for M^{-1/2} S M^{-1/2} + F.
//
// Element e of [-L, L] (he = 2L / cells) maps the reference nodes xi_j to
// -L + e he + (xi_j + 1) he / 2.  The element mass is diag(w) he / 2 and the
// element stiffness (2 / he) D^T diag(w) D.  After assembly the two end
// nodes are dropped (homogeneous Dirichlet), leaving n = k cells - 1 unknowns.
//
// The rule, the element matrices and the assembly run in long double (x87,
// 64-bit significand) and are rounded to double once: the operator's
// condition number grows like k^4 cells^2, and an assembly in double already
// moves the discrete solution of a Q^10 problem on 110 cells by 1e-11.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <limits>
#include <thread>
#include <vector>

#include "ts_internal.h"
#include "ts_sem.h"

namespace ts {

namespace {

// P_k(x) and P_k'(x) by the three-term recurrence
// (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}, and P_k' from
// (1 - x^2) P_k' = k (P_{k-1} - x P_k).
void legendre(int k, long double x, long double* P, long double* dP) {
  long double p0 = 1.0L, p1 = x;
  if (k == 0) {
    *P = 1.0;
    *dP = 0.0;
    return;
  }
  for (int m = 1; m < k; ++m) {
    long double p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  *dP = k * (p0 - x * p1) / (1.0L - x * x);
}

unsigned host_threads(int64_t work_rows) {
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(std::min<unsigned>(hw, 32), work_rows / 16));
}

template <class F>
void parallel_rows(int64_t lo, int64_t hi, F&& fn) {
  const int64_t rows = hi - lo;
  if (rows <= 0) return;
  const unsigned nt = host_threads(rows);
  if (nt <= 1) {
    fn(lo, hi);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (rows + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t a = lo + t * chunk, b = std::min(hi, a + chunk);
    if (a < b) th.emplace_back([&, a, b] { fn(a, b); });
  }
  for (auto& t : th) t.join();
}

}  // namespace

// Interior roots of P_k' by Newton's method, P_k'' taken from Legendre's
// equation (1 - x^2) P'' = 2 x P' - k (k+1) P; starting points are the
// Chebyshev-Lobatto points -cos(pi j / k), which interlace with the roots.
bool gll_rule(int k, long double* xi, long double* w) {
  if (k < 1 || k > kMaxSemOrder) return false;
  xi[0] = -1.0L;
  xi[k] = 1.0L;
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double tol = 4.0L * std::numeric_limits<long double>::epsilon();
  for (int j = 1; j < k; ++j) {
    long double x = -std::cos(pi * j / k);
    for (int it = 0; it < 100; ++it) {
      long double P, dP;
      legendre(k, x, &P, &dP);
      const long double d2P = (2.0L * x * dP - k * (k + 1.0L) * P) / (1.0L - x * x);
      const long double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < tol) break;
    }
    xi[j] = x;
  }
  for (int j = 0; j <= k; ++j) {
    long double P, dP;
    legendre(k, xi[j], &P, &dP);
    w[j] = 2.0L / (k * (k + 1.0L) * P * P);
  }
  return true;
}

// Derivative matrix of the Lagrange basis at the Gauss-Lobatto nodes, in its
// closed form: D[i][j] = P_k(xi_i) / (P_k(xi_j) (xi_i - xi_j)) for i != j,
// D[0][0] = -k(k+1)/4, D[k][k] = k(k+1)/4, other diagonal entries 0.
void gll_derivative(int k, const long double* xi, long double* D) {
  const int m = k + 1;
  std::vector<long double> P(m);
  for (int j = 0; j < m; ++j) {
    long double dP;
    legendre(k, xi[j], &P[j], &dP);
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) D[i * m + j] = i == j ? 0.0L : P[i] / (P[j] * (xi[i] - xi[j]));
  D[0] = -k * (k + 1.0L) / 4.0L;
  D[m * m - 1] = k * (k + 1.0L) / 4.0L;
}

bool sem_axis(int k, int64_t cells, double L, SemAxis& out) {
  if (k < 1 || k > kMaxSemOrder || cells < 1 || !(L > 0.0)) return false;
  using LD = long double;
  const int m = k + 1;
  std::vector<LD> xi(m), w(m), D(m * m), Se(m * m);
  if (!gll_rule(k, xi.data(), w.data())) return false;
  gll_derivative(k, xi.data(), D.data());
  const LD he = 2.0L * (LD)L / (LD)cells;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      LD s = 0.0L;
      for (int q = 0; q < m; ++q) s += w[q] * D[q * m + a] * D[q * m + b];
      Se[a * m + b] = (2.0L / he) * s;
    }
  const int64_t G = k * cells + 1, n = G - 2, wd = 2 * k + 1;
  out.k = k;
  out.n = n;
  std::vector<LD> xl(n, 0.0L);
  out.ml.assign(n, 0.0L);
  out.Sl.assign((size_t)(n * wd), 0.0L);  // band: row i, column i - k + t
  for (int64_t e = 0; e < cells; ++e)
    for (int a = 0; a < m; ++a) {
      const int64_t g = e * k + a - 1;  // interior index of global node e k + a
      if (g < 0 || g >= n) continue;
      xl[g] = -(LD)L + e * he + (xi[a] + 1.0L) * he / 2.0L;
      out.ml[g] += w[a] * he / 2.0L;
      for (int b = 0; b < m; ++b) {
        const int64_t h = e * k + b - 1;
        if (h < 0 || h >= n) continue;
        out.Sl[(size_t)(g * wd + (h - g + k))] += Se[a * m + b];
      }
    }
  out.x.resize(n);
  out.m.resize(n);
  out.S.resize(out.Sl.size());
  for (int64_t i = 0; i < n; ++i) {
    out.x[i] = (double)xl[i];
    out.m[i] = (double)out.ml[i];
  }
  for (size_t i = 0; i < out.Sl.size(); ++i) out.S[i] = (double)out.Sl[i];
  return true;
}

namespace {

// Rows of a symmetric matrix in long double, exact zeros dropped (the SEM
// operators are banded).
struct RowsLD {
  std::vector<int64_t> ptr, col;
  std::vector<long double> val;
};

template <class T>
RowsLD rows_of(int64_t n, const T* A) {
  RowsLD R;
  R.ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      const T a = A[(size_t)(i * n + j)];
      if (a != (T)0) {
        R.col.push_back(j);
        R.val.push_back((long double)a);
      }
    }
    R.ptr[i + 1] = (int64_t)R.col.size();
  }
  return R;
}

// C = A B^T for row-major n x n A, B: each entry a dot product of two
// contiguous rows, summed in index order (4 x 4 output blocks per pass).
void gemm_abt(int64_t n, const double* A, const double* B, double* C) {
  parallel_rows(0, (n + 3) / 4, [&](int64_t b0, int64_t b1) {
    for (int64_t ib = b0; ib < b1; ++ib) {
      const int64_t i0 = ib * 4, ni = std::min<int64_t>(4, n - i0);
      for (int64_t j0 = 0; j0 < n; j0 += 4) {
        const int64_t nj = std::min<int64_t>(4, n - j0);
        double acc[4][4] = {};
        const double* a[4];
        const double* b[4];
        for (int u = 0; u < 4; ++u) {
          a[u] = A + (size_t)((i0 + std::min<int64_t>(u, ni - 1)) * n);
          b[u] = B + (size_t)((j0 + std::min<int64_t>(u, nj - 1)) * n);
        }
        for (int64_t r = 0; r < n; ++r)
          for (int u = 0; u < 4; ++u)
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u][r] * b[v][r];
        for (int u = 0; u < ni; ++u)
          for (int v = 0; v < nj; ++v) C[(size_t)((i0 + u) * n + j0 + v)] = acc[u][v];
      }
    }
  });
}

// One step of the iterative refinement of Ogita and Aishima (Japan J. Indust.
// Appl. Math. 35 (2018), Algorithm 1) for A X = X diag(lam), with X row-major
// and the eigenvectors in its columns.  With the Rayleigh quotients lt_j and
// the residuals W = A X - X diag(lt), the off-diagonal correction is
// E_ij = (X^T W)_ij / (lt_j - lt_i) and the diagonal one (1 - |x_j|^2) / 2;
// X <- X + X E, lam <- lt.  The residuals are formed in long double and
// rounded once, so that the step reaches the accuracy of the long double A;
// X^T W and X E are small and formed in double.  Pairs closer than the step
// can separate (gap below twice the Frobenius norm of X^T W plus n eps |A|)
// only get their non-orthogonality removed, E_ij = -x_i.x_j / 2.
void refine_sym_eig(int64_t n, const RowsLD& A, double* lam, double* X) {
  std::vector<double> XT((size_t)(n * n)), WT((size_t)(n * n)), lt(n), rd(n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) XT[(size_t)(j * n + i)] = X[(size_t)(i * n + j)];
  parallel_rows(0, n, [&](int64_t j0, int64_t j1) {
    std::vector<long double> x(n), y(n);
    for (int64_t j = j0; j < j1; ++j) {
      const double* xj = &XT[(size_t)(j * n)];
      for (int64_t i = 0; i < n; ++i) x[i] = xj[i];
      long double nrm = 0.0L, xay = 0.0L;
      for (int64_t i = 0; i < n; ++i) {
        long double s = 0.0L;
        for (int64_t t = A.ptr[i]; t < A.ptr[i + 1]; ++t) s += A.val[t] * x[A.col[t]];
        y[i] = s;
        nrm += x[i] * x[i];
        xay += x[i] * s;
      }
      const long double rq = xay / nrm;
      for (int64_t i = 0; i < n; ++i) WT[(size_t)(j * n + i)] = (double)(y[i] - rq * x[i]);
      lt[j] = (double)rq;
      rd[j] = (double)(1.0L - nrm);
    }
  });
  std::vector<double> T((size_t)(n * n));
  gemm_abt(n, XT.data(), WT.data(), T.data());  // T = X^T W
  double tf = 0.0, amax = 0.0;
  for (size_t i = 0; i < T.size(); ++i) tf += T[i] * T[i];
  for (int64_t j = 0; j < n; ++j) amax = std::max(amax, std::fabs(lt[j]));
  const double delta = 2.0 * (std::sqrt(tf) + (double)n * DBL_EPSILON * amax);
  std::vector<double>& ET = WT;  // E^T, reusing the residual storage
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double e;
      if (i == j) {
        e = 0.5 * rd[j];
      } else if (std::fabs(lt[j] - lt[i]) > delta) {
        e = T[(size_t)(i * n + j)] / (lt[j] - lt[i]);
      } else {
        long double g = 0.0L;
        for (int64_t r = 0; r < n; ++r) g += (long double)XT[(size_t)(i * n + r)] * XT[(size_t)(j * n + r)];
        e = -0.5 * (double)g;
      }
      ET[(size_t)(j * n + i)] = e;
    }
  gemm_abt(n, X, ET.data(), T.data());  // T = X E
  for (size_t i = 0; i < T.size(); ++i) X[i] += T[i];
  for (int64_t j = 0; j < n; ++j) lam[j] = lt[j];
}

}  // namespace

// Householder reduction of the dense symmetric A (row-major, overwritten) to
// tridiagonal form A = P T P^T (Golub & Van Loan, Algorithm 8.3.1), the
// tridiagonal eigensolver on T, Q = P Z, and one refinement step against Aex
// (the same operator in long double) or, without it, against A itself.
bool dense_sym_eig(int64_t n, std::vector<double>& A, double* lam, double* Q, const long double* Aex) {
  const RowsLD R = Aex ? rows_of(n, Aex) : rows_of(n, A.data());
  std::vector<double> diag(n), off(n > 1 ? n - 1 : 1, 0.0);
  std::vector<double> V((size_t)(n * n), 0.0);  // Householder vectors, v_j in row j (entries j+1..n-1)
  std::vector<double> beta(n, 0.0), p(n), wv(n);
  for (int64_t j = 0; j + 2 < n; ++j) {
    double* v = &V[(size_t)(j * n)];
    double sigma = 0.0;
    for (int64_t i = j + 2; i < n; ++i) sigma += A[i * n + j] * A[i * n + j];
    const double x0 = A[(j + 1) * n + j];
    for (int64_t i = j + 1; i < n; ++i) v[i] = A[i * n + j];
    if (sigma == 0.0) {
      beta[j] = 0.0;
      continue;
    }
    const double mu = std::sqrt(x0 * x0 + sigma);
    // v_0 = x0 - mu, written without cancellation when x0 > 0; the reflector maps x to mu e_1
    const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
    beta[j] = 2.0 * v0 * v0 / (sigma + v0 * v0);
    for (int64_t i = j + 2; i < n; ++i) v[i] /= v0;
    v[j + 1] = 1.0;
    // p = beta A v over the trailing block, w = p - (beta p^T v / 2) v, then
    // A <- A - v w^T - w v^T (one thread: each step is a short O(n^2) sweep)
    for (int64_t r = j + 1; r < n; ++r) {
      const double* Ar = &A[(size_t)(r * n)];
      double s = 0.0;
      for (int64_t c = j + 1; c < n; ++c) s += Ar[c] * v[c];
      p[r] = beta[j] * s;
    }
    double pv = 0.0;
    for (int64_t i = j + 1; i < n; ++i) pv += p[i] * v[i];
    const double kf = beta[j] * pv / 2.0;
    for (int64_t i = j + 1; i < n; ++i) wv[i] = p[i] - kf * v[i];
    for (int64_t r = j + 1; r < n; ++r) {
      double* Ar = &A[(size_t)(r * n)];
      const double vr = v[r], wr = wv[r];
      for (int64_t c = j + 1; c < n; ++c) Ar[c] -= vr * wv[c] + wr * v[c];
    }
    // the reflector maps the column below the diagonal to mu e_1
    A[(j + 1) * n + j] = mu;
    A[j * n + j + 1] = mu;
  }
  for (int64_t i = 0; i < n; ++i) diag[i] = A[i * n + i];
  for (int64_t i = 0; i + 1 < n; ++i) off[i] = A[(i + 1) * n + i];
  std::vector<double> Z((size_t)(n * n));
  if (!tridiag_eig(n, diag.data(), off.data(), lam, Z.data())) return false;
  // Q = H_0 H_1 ... H_{n-3} Z, applied from the last reflector to the first,
  // each column of Z independently
  for (size_t i = 0; i < Z.size(); ++i) Q[i] = Z[i];
  parallel_rows(0, n, [&](int64_t c0, int64_t c1) {
    std::vector<double> col(n);
    for (int64_t c = c0; c < c1; ++c) {
      for (int64_t i = 0; i < n; ++i) col[i] = Q[i * n + c];
      for (int64_t j = n - 3; j >= 0; --j) {
        if (beta[j] == 0.0) continue;
        const double* v = &V[(size_t)(j * n)];
        double s = 0.0;
        for (int64_t i = j + 1; i < n; ++i) s += v[i] * col[i];
        s *= beta[j];
        for (int64_t i = j + 1; i < n; ++i) col[i] -= s * v[i];
      }
      for (int64_t i = 0; i < n; ++i) Q[i * n + c] = col[i];
    }
  });
  // sign: largest-magnitude entry of each column positive
  for (int64_t c = 0; c < n; ++c) {
    int64_t arg = 0;
    for (int64_t i = 1; i < n; ++i)
      if (std::fabs(Q[i * n + c]) > std::fabs(Q[arg * n + c])) arg = i;
    if (Q[arg * n + c] < 0.0)
      for (int64_t i = 0; i < n; ++i) Q[i * n + c] = -Q[i * n + c];
  }
  refine_sym_eig(n, R, lam, Q);
  // keep the ascending order (a refined pair can only swap inside a cluster)
  std::vector<int64_t> order(n);
  for (int64_t c = 0; c < n; ++c) order[c] = c;
  if (!std::is_sorted(lam, lam + n)) {
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return lam[a] < lam[b]; });
    std::vector<double> l2(lam, lam + n), Q2(Q, Q + n * n);
    for (int64_t j = 0; j < n; ++j) {
      lam[j] = l2[order[j]];
      for (int64_t i = 0; i < n; ++i) Q[i * n + j] = Q2[(size_t)(i * n + order[j])];
    }
  }
  return true;
}

}  // namespace ts
