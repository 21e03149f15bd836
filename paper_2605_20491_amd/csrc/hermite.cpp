// Host setup of Hermite spectral collocation on the real line (paper,
// Appendix "Hermite spectral method on unbounded domains"): one axis's nodes,
// quadrature weights and second-derivative operator, as input for the generic
// per-axis plan.
//
// Nodes: the zeros of the degree-n Hermite polynomial, i.e. the eigenvalues of
// the Jacobi matrix J (zero diagonal, J[k-1][k] = sqrt(k/2)); found by Sturm
// bisection on J and one Newton step on psi_n.  The normalised Hermite
// functions follow psi_{k+1} = sqrt(2/(k+1)) x psi_k - sqrt(k/(k+1)) psi_{k-1}
// from psi_0 = pi^{-1/4} e^{-x^2/2}; the recurrence runs on psi e^{x^2/2} with
// a separate exponent, so nothing underflows at the outer nodes.
//
// With m_j = 1 / (n psi_{n-1}(x_j)^2) (the Gauss weights of the Hermite
// functions) the differentiation matrix D_ij = psi_{n-1}(x_i) /
// (psi_{n-1}(x_j) (x_i - x_j)) is M^{-1/2} E M^{1/2} with the skew-symmetric
// E_ij = s_i s_j / (x_i - x_j), s = sign psi_{n-1}.  So K = -D^2 =
// M^{-1/2} (E E^T) M^{1/2}: the Gram matrix E E^T is formed directly, which
// keeps M^{1/2} K M^{-1/2} symmetric to the last bit.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <thread>
#include <vector>

#include "../../include/ts.h"
#include "ts_internal.h"

namespace ts {

namespace {

// Number of eigenvalues of J below t (LDL^T Sturm count); b2[k] = J[k][k+1]^2.
int64_t sturm_below(int64_t n, const std::vector<double>& b2, double t) {
  int64_t cnt = 0;
  double q = -t;
  if (q < 0.0) ++cnt;
  for (int64_t k = 1; k < n; ++k) {
    const double prev = q != 0.0 ? q : 1e-300;
    q = -t - b2[(size_t)(k - 1)] / prev;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// psi_{n-1}(x) and psi_n(x) as mantissas with a common scale:
// psi_k(x) = mant_k * exp(lg - x^2/2).
void hermite_pair(int64_t n, double x, double& pnm1, double& pn, double& lg) {
  double prev = 0.0, cur = std::pow(M_PI, -0.25);  // psi_{-1}, psi_0 without e^{-x^2/2}
  lg = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const double next = std::sqrt(2.0 / (double)(k + 1)) * x * cur - std::sqrt((double)k / (double)(k + 1)) * prev;
    prev = cur;
    cur = next;
    if (std::fabs(cur) > 1e200) {
      cur *= 1e-200;
      prev *= 1e-200;
      lg += 200.0 * std::log(10.0);
    }
  }
  pnm1 = prev;
  pn = cur;
}

}  // namespace

int hermite_axis(int64_t n, double* x, double* m, double* K) {
  std::vector<double> b2((size_t)std::max<int64_t>(n - 1, 1));
  for (int64_t k = 1; k < n; ++k) b2[(size_t)(k - 1)] = 0.5 * (double)k;
  const double bound = std::sqrt(2.0 * (double)n) + 1.0;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int64_t nth = std::min<int64_t>(std::min<int64_t>(hw, 32), std::max<int64_t>(1, n / 64));
  auto run = [&](int64_t lo_j, int64_t hi_j, const std::function<void(int64_t, int64_t)>& body, bool tri) {
    if (nth <= 1) {
      body(lo_j, hi_j);
      return;
    }
    // equal work per thread: rows of cost ~ j (tri) or constant
    std::vector<int64_t> cut(nth + 1, hi_j);
    cut[0] = lo_j;
    for (int64_t t = 1; t < nth; ++t) {
      const double f = tri ? std::sqrt((double)t / (double)nth) : (double)t / (double)nth;
      cut[t] = lo_j + (int64_t)((double)(hi_j - lo_j) * f);
    }
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nth; ++t)
      if (cut[t] < cut[t + 1]) th.emplace_back(body, cut[t], cut[t + 1]);
    for (auto& t : th) t.join();
  };
  // the upper half by bisection (x_{n-1-j} = -x_j; the middle node of odd n is 0)
  run(n / 2, n, [&](int64_t j0, int64_t j1) {
    for (int64_t j = j0; j < j1; ++j) {
      if (n % 2 == 1 && j == n / 2) {
        x[j] = 0.0;
        continue;
      }
      double lo = 0.0, hi = bound;
      for (int it = 0; it < 200 && hi - lo > 2.0 * 2.3e-16 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_below(n, b2, mid) > j) hi = mid;
        else lo = mid;
      }
      double t = 0.5 * (lo + hi);
      double pnm1, pn, lg;
      hermite_pair(n, t, pnm1, pn, lg);
      const double dpn = std::sqrt(2.0 * (double)n) * pnm1 - t * pn;  // psi_n' in the same scale
      if (dpn != 0.0) {
        const double step = pn / dpn;
        if (std::fabs(step) <= 1e-10 * (1.0 + t)) t -= step;
      }
      x[j] = t;
      x[n - 1 - j] = -t;
    }
  }, false);
  std::vector<double> s((size_t)n), ms((size_t)n);
  for (int64_t j = 0; j < n; ++j) {
    double pnm1, pn, lg;
    hermite_pair(n, x[j], pnm1, pn, lg);
    const double logpsi = std::log(std::fabs(pnm1)) + lg - 0.5 * x[j] * x[j];
    m[j] = std::exp(-2.0 * logpsi) / (double)n;
    if (!(m[j] > 0.0) || !std::isfinite(m[j])) return TS_ERR_INVALID;
    ms[(size_t)j] = std::sqrt(m[j]);
    s[(size_t)j] = pnm1 < 0.0 ? -1.0 : 1.0;
  }
  // E = [s_i s_k / (x_i - x_k)] (n^2 doubles, the size of K itself), then its Gram matrix
  std::vector<double> Em((size_t)(n * n));
  run(0, n, [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i)
      for (int64_t k = 0; k < n; ++k)
        Em[(size_t)(i * n + k)] = i == k ? 0.0 : s[(size_t)i] * s[(size_t)k] / (x[i] - x[k]);
  }, false);
  auto rows = [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i) {
      const double* ei = &Em[(size_t)(i * n)];
      for (int64_t j = 0; j <= i; ++j) {
        const double* ej = &Em[(size_t)(j * n)];
        double g = 0.0;
        for (int64_t k = 0; k < n; ++k) g += ei[k] * ej[k];
        K[(size_t)(i * n + j)] = g * ms[(size_t)j] / ms[(size_t)i];
        K[(size_t)(j * n + i)] = g * ms[(size_t)i] / ms[(size_t)j];
      }
    }
  };
  run(0, n, rows, true);
  return TS_OK;
}

}  // namespace ts

extern "C" int ts_hermite_axis(int64_t n, double* x, double* m, double* K) {
  if (!x || !m || !K) {
    ts::set_error("null argument");
    return TS_ERR_INVALID;
  }
  if (n < 1 || n > 8192) {
    ts::set_error("n must be in [1, 8192]");
    return TS_ERR_INVALID;
  }
  const int rc = ts::hermite_axis(n, x, m, K);
  if (rc) ts::set_error("Hermite weights overflowed");
  return rc;
}
