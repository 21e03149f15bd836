// Host setup of the Q^k spectral-element per-axis operators (paper Sec. 2,
// eq. (eigen_decomp)): Gauss-Lobatto nodes and weights, the Lagrange
// derivative matrix, the assembled stiffness S and lumped mass M of one axis,
// and a dense symmetric eigensolver for M^{-1/2} S M^{-1/2} + F.
//
// Element e of [-L, L] (he = 2L / cells) maps the reference nodes xi_j to
// -L + e he + (xi_j + 1) he / 2.  The element mass is diag(w) he / 2 and the
// element stiffness (2 / he) D^T diag(w) D.  After assembly the two end
// nodes are dropped (homogeneous Dirichlet), leaving n = k cells - 1 unknowns.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "ts_internal.h"
#include "ts_sem.h"

namespace ts {

namespace {

// P_k(x) and P_k'(x) by the three-term recurrence
// (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}, and P_k' from
// (1 - x^2) P_k' = k (P_{k-1} - x P_k).
void legendre(int k, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x;
  if (k == 0) {
    *P = 1.0;
    *dP = 0.0;
    return;
  }
  for (int m = 1; m < k; ++m) {
    double p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  *dP = k * (p0 - x * p1) / (1.0 - x * x);
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
bool gll_rule(int k, double* xi, double* w) {
  if (k < 1 || k > kMaxSemOrder) return false;
  xi[0] = -1.0;
  xi[k] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int j = 1; j < k; ++j) {
    double x = -std::cos(pi * j / k);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(k, x, &P, &dP);
      const double d2P = (2.0 * x * dP - k * (k + 1.0) * P) / (1.0 - x * x);
      const double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    xi[j] = x;
  }
  for (int j = 0; j <= k; ++j) {
    double P, dP;
    legendre(k, xi[j], &P, &dP);
    w[j] = 2.0 / (k * (k + 1.0) * P * P);
  }
  return true;
}

// Derivative matrix of the Lagrange basis at the Gauss-Lobatto nodes, in its
// closed form: D[i][j] = P_k(xi_i) / (P_k(xi_j) (xi_i - xi_j)) for i != j,
// D[0][0] = -k(k+1)/4, D[k][k] = k(k+1)/4, other diagonal entries 0.
void gll_derivative(int k, const double* xi, double* D) {
  const int m = k + 1;
  std::vector<double> P(m);
  for (int j = 0; j < m; ++j) {
    double dP;
    legendre(k, xi[j], &P[j], &dP);
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) D[i * m + j] = i == j ? 0.0 : P[i] / (P[j] * (xi[i] - xi[j]));
  D[0] = -k * (k + 1.0) / 4.0;
  D[m * m - 1] = k * (k + 1.0) / 4.0;
}

bool sem_axis(int k, int64_t cells, double L, SemAxis& out) {
  if (k < 1 || k > kMaxSemOrder || cells < 1 || !(L > 0.0)) return false;
  const int m = k + 1;
  std::vector<double> xi(m), w(m), D(m * m), Se(m * m);
  if (!gll_rule(k, xi.data(), w.data())) return false;
  gll_derivative(k, xi.data(), D.data());
  const double he = 2.0 * L / (double)cells;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      double s = 0.0;
      for (int q = 0; q < m; ++q) s += w[q] * D[q * m + a] * D[q * m + b];
      Se[a * m + b] = (2.0 / he) * s;
    }
  const int64_t G = k * cells + 1, n = G - 2;
  out.k = k;
  out.n = n;
  out.x.assign(n, 0.0);
  out.m.assign(n, 0.0);
  out.S.assign((size_t)(n * (2 * k + 1)), 0.0);  // band: row i, column i - k + t
  for (int64_t e = 0; e < cells; ++e)
    for (int a = 0; a < m; ++a) {
      const int64_t g = e * k + a - 1;  // interior index of global node e k + a
      if (g < 0 || g >= n) continue;
      out.x[g] = -L + e * he + (xi[a] + 1.0) * he / 2.0;
      out.m[g] += w[a] * he / 2.0;
      for (int b = 0; b < m; ++b) {
        const int64_t h = e * k + b - 1;
        if (h < 0 || h >= n) continue;
        out.S[(size_t)(g * (2 * k + 1) + (h - g + k))] += Se[a * m + b];
      }
    }
  return true;
}

// Householder reduction of the dense symmetric A (row-major, overwritten) to
// tridiagonal form A = P T P^T (Golub & Van Loan, Algorithm 8.3.1), the
// tridiagonal eigensolver on T, and Q = P Z.
bool dense_sym_eig(int64_t n, std::vector<double>& A, double* lam, double* Q) {
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
  return true;
}

}  // namespace ts
