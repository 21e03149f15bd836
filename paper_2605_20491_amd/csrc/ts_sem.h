// Q^k spectral-element per-axis operators (sem_setup.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace ts {

constexpr int kMaxSemOrder = 32;

// One axis of Q^k SEM on [-L, L] with `cells` elements, Dirichlet ends.
struct SemAxis {
  int k = 0;
  int64_t n = 0;               // k * cells - 1 interior nodes
  std::vector<double> x;       // interior nodes, ascending
  std::vector<double> m;       // lumped (Gauss-Lobatto) mass
  std::vector<double> S;       // stiffness band [n][2k+1]: S[i][i-k+t]
  std::vector<long double> ml, Sl;  // the mass and the band before rounding
};

bool gll_rule(int k, long double* xi, long double* w);              // k+1 nodes on [-1, 1]
void gll_derivative(int k, const long double* xi, long double* D);  // (k+1)^2, D[i][j] = l_j'(xi_i)
bool sem_axis(int k, int64_t cells, double L, SemAxis& out);
// Eigen-decomposition of a dense symmetric matrix (A is overwritten), refined
// once against Aex (row-major n x n, the same operator in long double) or,
// when Aex is null, against A as given.
bool dense_sym_eig(int64_t n, std::vector<double>& A, double* lam, double* Q, const long double* Aex = nullptr);

}  // namespace ts
