/*
 * Plain CPU FP64 oracle for the separable tensor-product solver of -Delta + V1.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Everything here is written for a reader who holds the paper next to it:
 *   - Section 2.1, eq. (general_system)/(tensor_system): the discrete operator is
 *     the Kronecker sum of per-axis matrices H_k = K_k + F_k, where for Q^1
 *     elements (classical second-order finite differences) K_k is h^-2
 *     tridiag(-1, 2, -1) on the n interior nodes of [-L, L] and F_k = diag(f_k).
 *   - eq. (eigen_decomp): H_k = Q_k Lambda_k Q_k^T (mass matrix is a multiple of
 *     the identity for Q^1, so T_k = Q_k, T_k^{-1} = Q_k^T).
 *   - the four-step solve of Section 2.1 and eq. (exact_prop): forward transform
 *     with T^{-1} on every axis, pointwise divide by (sum of eigenvalues + sigma)
 *     or multiply by exp(-i tau * sum of eigenvalues), backward transform with T.
 * Accumulation is always FP64 in plain index order.  OpenMP parallelises only
 * over independent fibres / grid points, which does not change any result.
 *
 * Parity status of each function is stated in its comment; pins live in tests/.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Per-axis operator (Section 2.1, Q^1 = second-order FD; grid of n interior  */
/* nodes x_j = -L + j h, h = 2L/(n+1), homogeneous Dirichlet).                */
/* ------------------------------------------------------------------------- */

double or_grid_spacing(int64_t n, double L) { return 2.0 * L / (double)(n + 1); }

/* Dense row-major n x n matrix H = h^-2 tridiag(-1, 2, -1) + diag(f). */
void or_fd_axis_matrix(int64_t n, double L, const double* f, double* H) {
  double h = or_grid_spacing(n, L);
  double ih2 = 1.0 / (h * h);
  memset(H, 0, sizeof(double) * (size_t)(n * n));
  for (int64_t i = 0; i < n; ++i) {
    H[i * n + i] = 2.0 * ih2 + f[i];
    if (i > 0) H[i * n + i - 1] = -ih2;
    if (i + 1 < n) H[i * n + i + 1] = -ih2;
  }
}

/* ------------------------------------------------------------------------- */
/* Cyclic-by-row Jacobi eigensolver with Rutishauser's rotation and update   */
/* formulas (Golub & Van Loan, "Matrix Computations", Sec. 8.5; Rutishauser,  */
/* Handbook for Automatic Computation II/1, 1971).  Plain and slow on         */
/* purpose.  A is symmetric row-major n x n (not modified).  Output: w        */
/* ascending, V row-major with column j the unit eigenvector of w[j], sign    */
/* fixed so that its largest-magnitude entry (lowest index on ties) is > 0.   */
/* Returns the number of sweeps, or -1 if max_sweeps was reached.             */
/* ------------------------------------------------------------------------- */
static double offdiag_norm2(int64_t n, const double* A) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j)
      if (i != j) s += A[i * n + j] * A[i * n + j];
  return s;
}

int or_jacobi_eigh(int64_t n, const double* A_in, double* w, double* V, int max_sweeps) {
  double* A = (double*)malloc(sizeof(double) * (size_t)(n * n));
  memcpy(A, A_in, sizeof(double) * (size_t)(n * n));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  double fro2 = 0.0;
  for (int64_t i = 0; i < n * n; ++i) fro2 += A[i] * A[i];
  const double tol2 = 1e-30 * fro2; /* off(A) <= 1e-15 ||A||_F */
  int sweep = 0;
  int converged = 0;
  for (sweep = 0; sweep < max_sweeps; ++sweep) {
    if (offdiag_norm2(n, A) <= tol2) { converged = 1; break; }
    for (int64_t p = 0; p < n - 1; ++p) {
      for (int64_t q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        /* zero A[p][q] with J = [[c, s], [-s, c]] acting on rows/cols p, q */
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0);
        double s = t * c;
        double tau = s / (1.0 + c);
        /* A <- J^T A J with Rutishauser's update: the diagonal moves by
           -/+ t a_pq, every other entry of rows/columns p and q rotates as
           x_p <- x_p - s (x_q + tau x_p), x_q <- x_q + s (x_p - tau x_q). */
        A[p * n + p] = app - t * apq;
        A[q * n + q] = aqq + t * apq;
        A[p * n + q] = 0.0;
        A[q * n + p] = 0.0;
        for (int64_t k = 0; k < n; ++k) {
          if (k == p || k == q) continue;
          double akp = A[k * n + p], akq = A[k * n + q];
          double nkp = akp - s * (akq + tau * akp);
          double nkq = akq + s * (akp - tau * akq);
          A[k * n + p] = nkp;
          A[p * n + k] = nkp;
          A[k * n + q] = nkq;
          A[q * n + k] = nkq;
        }
        /* accumulate eigenvectors: V <- V J */
        for (int64_t k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = vkp - s * (vkq + tau * vkp);
          V[k * n + q] = vkq + s * (vkp - tau * vkq);
        }
      }
    }
  }
  if (!converged && offdiag_norm2(n, A) <= tol2) converged = 1;
  for (int64_t i = 0; i < n; ++i) w[i] = A[i * n + i];
  free(A);
  /* selection sort ascending (stable enough for a checker), columns follow */
  for (int64_t i = 0; i < n; ++i) {
    int64_t m = i;
    for (int64_t j = i + 1; j < n; ++j)
      if (w[j] < w[m]) m = j;
    if (m != i) {
      double tw = w[i]; w[i] = w[m]; w[m] = tw;
      for (int64_t k = 0; k < n; ++k) {
        double tv = V[k * n + i]; V[k * n + i] = V[k * n + m]; V[k * n + m] = tv;
      }
    }
  }
  /* sign: largest-magnitude component positive */
  for (int64_t j = 0; j < n; ++j) {
    int64_t arg = 0;
    for (int64_t k = 1; k < n; ++k)
      if (fabs(V[k * n + j]) > fabs(V[arg * n + j])) arg = k;
    if (V[arg * n + j] < 0.0)
      for (int64_t k = 0; k < n; ++k) V[k * n + j] = -V[k * n + j];
  }
  return converged ? sweep : -1;
}

/* ------------------------------------------------------------------------- */
/* Mode-k product on a d-way tensor stored C-contiguously (last axis fastest) */
/* with ncomp interleaved real components (1 = real, 2 = complex).  For every */
/* fibre x along `axis`:                                                       */
/*   transpose = 1:  y[j] = sum_i Q[i][j] x[i]   (y = Q^T x, the forward step) */
/*   transpose = 0:  y[j] = sum_i Q[j][i] x[i]   (y = Q x,   the backward step)*/
/* Sums run over i = 0..n-1 in order.  X and Y must not overlap.              */
/* ------------------------------------------------------------------------- */
void or_mode_product(int d, const int64_t* shape, int axis, const double* Q, int transpose,
                     int ncomp, const double* X, double* Y) {
  int64_t n = shape[axis];
  int64_t P = 1, R = 1;
  for (int k = 0; k < axis; ++k) P *= shape[k];
  for (int k = axis + 1; k < d; ++k) R *= shape[k];
  R *= ncomp; /* components behave like one more fastest axis */
  int64_t nfib = P * R;
#pragma omp parallel
  {
    double* x = (double*)malloc(sizeof(double) * (size_t)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
    for (int64_t f = 0; f < nfib; ++f) {
      int64_t p = f / R, r = f % R;
      const double* xs = X + p * n * R + r;
      double* ys = Y + p * n * R + r;
      for (int64_t i = 0; i < n; ++i) x[i] = xs[i * R];
      for (int64_t j = 0; j < n; ++j) y[j] = 0.0;
      if (transpose) {
        for (int64_t i = 0; i < n; ++i) {
          double xi = x[i];
          const double* qrow = Q + i * n;
          for (int64_t j = 0; j < n; ++j) y[j] += qrow[j] * xi;
        }
      } else {
        for (int64_t j = 0; j < n; ++j) {
          const double* qrow = Q + j * n;
          double acc = 0.0;
          for (int64_t i = 0; i < n; ++i) acc += qrow[i] * x[i];
          y[j] = acc;
        }
      }
      for (int64_t j = 0; j < n; ++j) ys[j * R] = y[j];
    }
    free(x);
    free(y);
  }
}

/* Multi-index of linear grid index `lin` (C order). */
static void unravel(int d, const int64_t* shape, int64_t lin, int64_t* idx) {
  for (int k = d - 1; k >= 0; --k) {
    idx[k] = lin % shape[k];
    lin /= shape[k];
  }
}

/* ------------------------------------------------------------------------- */
/* Four-step direct solve (Section 2.1): u = (H1 + sigma I)^{-1} b.           */
/* Q[k], lam[k]: eigenvectors (row-major, columns = vectors) and eigenvalues  */
/* of H_k.  Forward T^{-1} = Q^T on every axis, divide each entry by the      */
/* eigenvalue sum plus sigma (summed directly, per point, in FP64), backward  */
/* T = Q on every axis.  work has N doubles.  Real data.                      */
/* ------------------------------------------------------------------------- */
void or_apply_inverse(int d, const int64_t* shape, const double* const* Q, const double* const* lam,
                      double sigma, const double* b, double* u, double* work) {
  int64_t N = 1;
  for (int k = 0; k < d; ++k) N *= shape[k];
  /* forward: ping-pong so that after d products the result sits in `cur` */
  const double* src = b;
  double* bufs[2] = {work, u};
  int which = 0;
  for (int k = d - 1; k >= 0; --k) {
    or_mode_product(d, shape, k, Q[k], 1, 1, src, bufs[which]);
    src = bufs[which];
    which ^= 1;
  }
  double* cur = (double*)src;
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < N; ++lin) {
    int64_t idx[16];
    unravel(d, shape, lin, idx);
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += lam[k][idx[k]];
    cur[lin] = cur[lin] / (s + sigma);
  }
  for (int k = 0; k < d; ++k) {
    double* dst = (cur == u) ? work : u;
    or_mode_product(d, shape, k, Q[k], 0, 1, cur, dst);
    cur = dst;
  }
  if (cur != u) memcpy(u, cur, sizeof(double) * (size_t)N);
}

/* eq. (exact_prop): psi_out = T (exp(-i tau Lambda) .* (T^{-1} psi_in)).
 * Complex data interleaved (re, im).  The phase of each entry is formed from
 * the directly summed eigenvalue, exp(-i tau * sum_k lam_k), per point.       */
void or_apply_exp(int d, const int64_t* shape, const double* const* Q, const double* const* lam,
                  double tau, const double* psi_in, double* psi_out, double* work) {
  int64_t N = 1;
  for (int k = 0; k < d; ++k) N *= shape[k];
  const double* src = psi_in;
  double* bufs[2] = {work, psi_out};
  int which = 0;
  for (int k = d - 1; k >= 0; --k) {
    or_mode_product(d, shape, k, Q[k], 1, 2, src, bufs[which]);
    src = bufs[which];
    which ^= 1;
  }
  double* cur = (double*)src;
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < N; ++lin) {
    int64_t idx[16];
    unravel(d, shape, lin, idx);
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += lam[k][idx[k]];
    double ph = -tau * s;
    double c = cos(ph), sn = sin(ph);
    double re = cur[2 * lin], im = cur[2 * lin + 1];
    cur[2 * lin] = c * re - sn * im;
    cur[2 * lin + 1] = sn * re + c * im;
  }
  for (int k = 0; k < d; ++k) {
    double* dst = (cur == psi_out) ? work : psi_out;
    or_mode_product(d, shape, k, Q[k], 0, 2, cur, dst);
    cur = dst;
  }
  if (cur != psi_out) memcpy(psi_out, cur, sizeof(double) * (size_t)(2 * N));
}

/* ------------------------------------------------------------------------- */
/* The full (non-separable) operator of eq. (general_system), applied by its  */
/* stencil: (A u)_j = sum_k h_k^-2 (2 u_j - u_{j - e_k} - u_{j + e_k})        */
/*                    + (sum_k f_k[j_k] + V2_j + sigma) u_j,                  */
/* with zero values outside the grid (homogeneous Dirichlet).  V2 may be NULL.*/
/* ncomp = 2 applies the same real operator to interleaved complex data.      */
/* ------------------------------------------------------------------------- */
void or_stencil_apply(int d, const int64_t* shape, const double* hs, const double* const* f,
                      const double* V2, double sigma, int ncomp, const double* u, double* out) {
  int64_t N = 1;
  for (int k = 0; k < d; ++k) N *= shape[k];
  int64_t stride[16];
  stride[d - 1] = 1;
  for (int k = d - 2; k >= 0; --k) stride[k] = stride[k + 1] * shape[k + 1];
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < N; ++lin) {
    int64_t idx[16];
    unravel(d, shape, lin, idx);
    double diag = sigma + (V2 ? V2[lin] : 0.0);
    for (int k = 0; k < d; ++k) diag += f[k][idx[k]];
    for (int c = 0; c < ncomp; ++c) {
      double uc = u[lin * ncomp + c];
      double acc = diag * uc;
      for (int k = 0; k < d; ++k) {
        double ih2 = 1.0 / (hs[k] * hs[k]);
        double lo = (idx[k] > 0) ? u[(lin - stride[k]) * ncomp + c] : 0.0;
        double hi = (idx[k] + 1 < shape[k]) ? u[(lin + stride[k]) * ncomp + c] : 0.0;
        acc += ih2 * (2.0 * uc - lo - hi);
      }
      out[lin * ncomp + c] = acc;
    }
  }
}

/* Dense N x N matrix of the same operator, built entry by entry from the     */
/* stencil rule above (not from Kronecker products).  For brute force on tiny */
/* grids only.                                                                 */
void or_dense_operator(int d, const int64_t* shape, const double* hs, const double* const* f,
                       const double* V2, double sigma, double* H) {
  int64_t N = 1;
  for (int k = 0; k < d; ++k) N *= shape[k];
  int64_t stride[16];
  stride[d - 1] = 1;
  for (int k = d - 2; k >= 0; --k) stride[k] = stride[k + 1] * shape[k + 1];
  memset(H, 0, sizeof(double) * (size_t)(N * N));
  for (int64_t lin = 0; lin < N; ++lin) {
    int64_t idx[16];
    unravel(d, shape, lin, idx);
    double diag = sigma + (V2 ? V2[lin] : 0.0);
    for (int k = 0; k < d; ++k) {
      double ih2 = 1.0 / (hs[k] * hs[k]);
      diag += f[k][idx[k]] + 2.0 * ih2;
      if (idx[k] > 0) H[lin * N + lin - stride[k]] -= ih2;
      if (idx[k] + 1 < shape[k]) H[lin * N + lin + stride[k]] -= ih2;
    }
    H[lin * N + lin] += diag;
  }
}

/* ------------------------------------------------------------------------- */
/* Dense LU with partial pivoting, solve A x = b (A row-major N x N, kept).   */
/* Returns 0, or -1 on an exactly singular pivot.                              */
/* ------------------------------------------------------------------------- */
int or_lu_solve(int64_t N, const double* A_in, const double* b, double* x) {
  double* A = (double*)malloc(sizeof(double) * (size_t)(N * N));
  memcpy(A, A_in, sizeof(double) * (size_t)(N * N));
  memcpy(x, b, sizeof(double) * (size_t)N);
  int rc = 0;
  for (int64_t k = 0; k < N; ++k) {
    int64_t piv = k;
    for (int64_t i = k + 1; i < N; ++i)
      if (fabs(A[i * N + k]) > fabs(A[piv * N + k])) piv = i;
    if (A[piv * N + k] == 0.0) { rc = -1; break; }
    if (piv != k) {
      for (int64_t j = 0; j < N; ++j) {
        double t = A[k * N + j]; A[k * N + j] = A[piv * N + j]; A[piv * N + j] = t;
      }
      double t = x[k]; x[k] = x[piv]; x[piv] = t;
    }
    for (int64_t i = k + 1; i < N; ++i) {
      double l = A[i * N + k] / A[k * N + k];
      A[i * N + k] = l;
      for (int64_t j = k + 1; j < N; ++j) A[i * N + j] -= l * A[k * N + j];
      x[i] -= l * x[k];
    }
  }
  if (rc == 0)
    for (int64_t i = N - 1; i >= 0; --i) {
      double s = x[i];
      for (int64_t j = i + 1; j < N; ++j) s -= A[i * N + j] * x[j];
      x[i] = s / A[i * N + i];
    }
  free(A);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* exp(-i tau H) psi for a real symmetric dense H (N x N row-major), complex  */
/* psi interleaved.  Truncated Taylor series with scaling (Moler & Van Loan,  */
/* "Nineteen dubious ways ...", method 3): with B = -i tau H / 2^s and        */
/* ||B||_1 <= 1/2, psi is multiplied 2^s times by sum_{m=0}^{nterms} B^m/m!.  */
/* Used only for brute force on tiny grids.  Returns 2^s.                     */
/* ------------------------------------------------------------------------- */
int64_t or_expm_apply(int64_t N, const double* H, double tau, int nterms, const double* psi_in,
                      double* psi_out) {
  double norm1 = 0.0;
  for (int64_t j = 0; j < N; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += fabs(H[i * N + j]);
    if (s > norm1) norm1 = s;
  }
  double a = fabs(tau) * norm1;
  int64_t reps = 1;
  while (a / (double)reps > 0.5) reps *= 2;
  double t = tau / (double)reps; /* B = -i t H */
  double* v = (double*)malloc(sizeof(double) * (size_t)(2 * N));
  double* term = (double*)malloc(sizeof(double) * (size_t)(2 * N));
  double* nxt = (double*)malloc(sizeof(double) * (size_t)(2 * N));
  memcpy(v, psi_in, sizeof(double) * (size_t)(2 * N));
  for (int64_t r = 0; r < reps; ++r) {
    memcpy(term, v, sizeof(double) * (size_t)(2 * N));
    /* v accumulates sum of terms; term_m = B term_{m-1} / m */
    for (int m = 1; m <= nterms; ++m) {
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < N; ++i) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < N; ++j) {
          sr += H[i * N + j] * term[2 * j];
          si += H[i * N + j] * term[2 * j + 1];
        }
        /* (-i t)(sr + i si) / m = (t si - i t sr) / m */
        nxt[2 * i] = t * si / (double)m;
        nxt[2 * i + 1] = -t * sr / (double)m;
      }
      for (int64_t i = 0; i < 2 * N; ++i) {
        term[i] = nxt[i];
        v[i] += term[i];
      }
    }
  }
  memcpy(psi_out, v, sizeof(double) * (size_t)(2 * N));
  free(v);
  free(term);
  free(nxt);
  return reps;
}

/* exp(-i theta V) pointwise on interleaved complex psi (the potential factor */
/* of the splitting schemes, Section 5.1).  In place.                          */
void or_phase_apply(int64_t N, const double* V, double theta, double* psi) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double ph = -theta * V[i];
    double c = cos(ph), s = sin(ph);
    double re = psi[2 * i], im = psi[2 * i + 1];
    psi[2 * i] = c * re - s * im;
    psi[2 * i + 1] = s * re + c * im;
  }
}

/* Number of OpenMP threads the loops above use (reported by timing code). */
#ifdef _OPENMP
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
#else
int or_num_threads(void) { return 1; }
#endif
