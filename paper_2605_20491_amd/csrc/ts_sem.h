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
};

bool gll_rule(int k, double* xi, double* w);                 // k+1 nodes on [-1, 1]
void gll_derivative(int k, const double* xi, double* D);     // (k+1)^2, D[i][j] = l_j'(xi_i)
bool sem_axis(int k, int64_t cells, double L, SemAxis& out);
// Eigen-decomposition of a dense symmetric matrix (A is overwritten).
bool dense_sym_eig(int64_t n, std::vector<double>& A, double* lam, double* Q);

}  // namespace ts
