/*
 * ts.h -- C ABI of the MI355X separable tensor-product solver for the
 * Schroedinger operator H = -Delta + V1 (+ V2), V1(x) = sum_k f_k(x_k).
 *
 * Discretisations (paper Sec. 2, Sec. 2.1, eq. (general_system), eq. (tensor_system)),
 * each giving per-axis operators H_k and H1 = sum_k I (x) ... (x) H_k (x) ... (x) I
 * (the Kronecker sum):
 *  - ts_setup: second-order finite differences (the Q^1 case) on n_k interior
 *    nodes of [-L, L], x_{k,j} = -L + j h_k, h_k = 2L/(n_k+1), homogeneous
 *    Dirichlet; H_k = h_k^-2 tridiag(-1, 2, -1) + diag(f_k(x_{k,j}));
 *  - ts_setup_sem: Q^k spectral elements with Gauss-Lobatto nodes and lumped
 *    mass, H_k = M_k^-1 S_k + diag(f_k);
 *  - ts_setup_general: any per-axis operator K_k self-adjoint in weights m_k
 *    (Hermite collocation on R from ts_hermite_axis is one such input).
 * The applies, solvers and splitting schemes below work on any of them.
 *
 * Data layout: a grid function is a C-contiguous array of shape
 * (n_0, ..., n_{d-1}); axis d-1 is the fastest index (the paper's x).
 * Complex data is interleaved (re, im).  Per-axis arrays f[k] follow the same
 * axis order.  All grid-function pointers are DEVICE pointers owned by the
 * caller; the library never frees them.  f[k] in ts_setup are HOST pointers.
 *
 * Streams: work is enqueued on the caller's HIP stream (hipStream_t passed as
 * void*, NULL = the legacy default stream) and the call returns without
 * synchronising, except where a scalar result is returned to the host
 * (iteration counts, residuals, eigenvalue histories): those calls
 * synchronise the stream before returning.
 *
 * Errors: every call returns a ts_status; no exception crosses the ABI.  A
 * human-readable message for the last failure on the calling thread is
 * available from ts_last_error().  On error, caller-owned outputs are left in
 * an unspecified state, and the plan stays valid.
 *
 * Concurrency: a plan is immutable after ts_setup except for its lazily
 * allocated scratch buffers; calls that use the same plan must be issued on
 * one stream (or otherwise ordered).  Distinct plans are independent.
 */
#ifndef TS_H
#define TS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ts_plan ts_plan;

typedef enum {
  TS_OK = 0,
  TS_ERR_INVALID = 1,   /* bad argument: null pointer, shape, dtype, precision   */
  TS_ERR_NOT_SPD = 2,   /* lambda_min(H1) + sigma <= 0: the inverse is undefined  */
  TS_ERR_NOMEM = 3,     /* device or host allocation failed                       */
  TS_ERR_DEVICE = 4,    /* a HIP runtime call failed                              */
  TS_ERR_NOCONV = 5,    /* iteration limit reached before the tolerance           */
  TS_ERR_NONFINITE = 6, /* NaN or Inf met in a residual or inner product          */
  TS_ERR_BUSY = 7,      /* serving: request not admitted yet (memory or slots)    */
  TS_ERR_BREAKDOWN = 8  /* PCG: <p, A p> <= 0 (operator not positive definite)    */
} ts_status;

/* Element type of the grid functions passed to an apply. */
typedef enum { TS_F64 = 0, TS_F32 = 1, TS_C128 = 2, TS_C64 = 3 } ts_dtype;

/* Arithmetic of the per-axis transforms inside an apply.
 * FP64: FP64 MFMA with FP64 factors; FP64 intermediates for FP64 data, and
 * for FP32 data (TS_F32, TS_C64) FP32 intermediates between HBM passes with
 * every pass computed in FP64 (the paper's complex64 runs with FP64
 * transforms, Sec. 6).  FP32: FP32 MFMA, FP32 intermediates.  BF16: BF16 MFMA
 * operands with FP32 accumulation, BF16 intermediates.  Denominators and phase
 * factors are always formed in FP64 and then cast. */
typedef enum { TS_PREC_FP64 = 0, TS_PREC_FP32 = 1, TS_PREC_BF16 = 2 } ts_prec;

/* Splitting schemes for ts_split_step (paper Sec. 5.1).  A = H1 (exact
 * propagator), B = V2 (pointwise).
 *   STRANG_BAB : e^{-iB dt/2} e^{-iA dt} e^{-iB dt/2}   (potential outside)
 *   STRANG_ABA : e^{-iA dt/2} e^{-iB dt} e^{-iA dt/2}   (= qHOP with M = 1)
 *   YOSHIDA_*  : eq. (yoshida) -- S(g1 dt) S(g2 dt) S(g1 dt) with the Strang
 *                step S of the same form, g1 = 1/(2 - 2^{1/3}),
 *                g2 = -2^{1/3}/(2 - 2^{1/3}).
 * Adjacent factors of the same operator are merged across sub-steps and steps
 * (Remark rem:cost_naive_merged), which changes rounding only. */
typedef enum {
  TS_STRANG_BAB = 0,
  TS_STRANG_ABA = 1,
  TS_YOSHIDA_BAB = 2,
  TS_YOSHIDA_ABA = 3
} ts_scheme;

/* ---------------------------------------------------------------- setup -- */

/* Build a plan for H1 + sigma I (Sec. 2.1, step 1 "off-line setup").
 *   d      : number of axes, 1 <= d <= 12
 *   n[k]   : interior nodes on axis k, 1 <= n[k] <= 16384, prod(n) < 2^40
 *   L      : half-width of the box [-L, L]^d, L > 0
 *   f[k]   : HOST array of n[k] samples f_k(x_{k,j}), j = 1..n[k]
 *   sigma  : shift; the inverse apply computes (H1 + sigma I)^{-1}
 *   out    : receives the plan (owned by the caller, release with ts_destroy)
 * Computes, on the host in FP64, the eigendecomposition H_k = Q_k diag(lam_k)
 * Q_k^T of every distinct axis (eq. (eigen_decomp); for FD the mass matrix is
 * a multiple of I, so T_k = Q_k and T_k^{-1} = Q_k^T), uploads Q_k, Q_k^T and
 * lam_k to the current HIP device, and derives FP32 and BF16 copies of Q_k on
 * the device from the FP64 copy (round to nearest even).  Synchronous.
 * Errors: TS_ERR_INVALID, TS_ERR_NOMEM, TS_ERR_DEVICE.  A negative definite
 * shift is not an error here (the propagator does not need it); the inverse
 * apply reports TS_ERR_NOT_SPD. */
int ts_setup(int d, const int64_t* n, double L, const double* const* f, double sigma,
             ts_plan** out);

/* Release a plan and every device buffer it owns.  NULL is a no-op.
 * Synchronises the device first, so pending work that uses the plan ends. */
int ts_destroy(ts_plan* plan);

/* Half-extent passes on reflection-symmetric axes.  When f_k is symmetric
 * (|f_k(x_j) - f_k(x_{n-1-j})| within 8 ulps of max(1, max|f_k|); the
 * eigensolver then uses the mean of each mirrored pair) every eigenvector of H_k is
 * even or odd; the passes on that axis (n_k >= 64, every transform precision)
 * then fold x into x_i +- x_{n-1-i} and contract half the extent against the
 * even and odd halves of the factor (half the MFMA work), with a butterfly
 * after each backward pass; with two or more such axes an apply folds its
 * input and unfolds its output once for all of them (ts_fold_butterfly) and
 * its passes run on folded data.  The result is the same up to rounding.  Applies
 * with BF16 transforms of FP64 data fold in the sweep that rounds the input to
 * BF16 (s_i and d_i are formed in FP64, then rounded) and run their forward
 * passes over half extents on 256 x 256 tiles; in 2D and 3D, with every axis
 * but the fastest folded and of even extent, the backward passes over those
 * axes also run over half extents and leave their output folded, and the last
 * pass (backward over the fastest axis, FP64 output) unfolds it in registers.
 * BF16 results differ from the unfolded BF16 apply by the different rounding
 * (both at the BF16 level); ts_mode_pass folds in every precision.
 * ts_set_fold(plan, 0) turns folding off for the plan, 1 turns it back on (the
 * default), 2 keeps it but runs the BF16 backward passes over full extents;
 * ts_fold_axes reports the axes that qualify as a bit mask (bit k = axis k).
 * Errors: TS_ERR_INVALID for a null plan or another mode. */
int ts_set_fold(ts_plan* plan, int enable);

/* Output tile of the BF16 passes (Sec. 2.2 runs the apply in BF16): 0 (the
 * default) lets the library choose, 128 forces 128 x 128 tiles, 256 asks for
 * 256 x 256 tiles wherever they apply (real BF16 input on a non-folded axis
 * of n >= 192 whose rows hold a multiple of 8 values, 16-byte aligned
 * buffers).  The larger tile fetches each operand element half as often from
 * L2; by default it is used when it still gives every compute unit a tile.
 * Both tiles consume K in the same order, so results are bitwise equal.
 * Returns TS_ERR_INVALID for a null plan or another value. */
int ts_set_bf16_tile(ts_plan* plan, int tile);

/* One pass of the apply (Sec. 2.1 step 2 or 4) on one axis, without the
 * scaling: forward out = in x_axis T_axis^{-1}, backward out = in x_axis
 * T_axis (spectral index in the plan's internal order, see ts_set_fold).
 * For measuring and checking the pass kernels on their own.  in, out: device
 * arrays of the grid (must not alias); dtype any of ts_dtype; prec FP64 (FP64
 * data), FP32, or BF16 (operands rounded to BF16, FP32 accumulation, result
 * stored in the data type).
 *   forward = 1: forward pass; 0: backward pass (with its butterfly on a
 *   folding axis);
 *   2: forward pass whose input is already folded along this axis
 *      (ts_fold_butterfly), as inside an apply with several folded axes;
 *   3: backward pass that leaves the butterfly out: E_i at row i (i < n - h)
 *      and O_i at row n - 1 - i (i < h, h = floor(n / 2)).
 * On an axis that does not fold, 2 and 3 are 1 and 0.  Modes 2 and 3 take
 * FP64 or FP32 transforms.  Errors: TS_ERR_INVALID, TS_ERR_DEVICE. */
int ts_mode_pass(ts_plan* plan, int axis, int forward, const void* in, void* out, int dtype, int prec,
                 void* hip_stream);
int ts_fold_axes(const ts_plan* plan, int* folded);

/* The butterfly of the half-extent passes along every axis k in the bit mask
 * `axes` (bit k = axis k): out_i = in_i + in_{n-1-i} and out_{n-1-i} = in_i -
 * in_{n-1-i} for i < floor(n_k / 2), the middle row of odd n_k copied (a
 * linear map on one axis each, so the order of the axes does not matter; two
 * applications give 2x the input per axis, except on the middle row).  It folds the input of the
 * forward passes and unfolds the output of the backward passes; an apply with
 * several folded axes runs it once before and once after its passes (up to
 * four axes per sweep over the data).  in, out: device arrays of the grid,
 * dtype any of ts_dtype (complex: on both components); out may equal in.
 * Enqueued on hip_stream.  Errors: TS_ERR_INVALID, TS_ERR_DEVICE. */
int ts_fold_butterfly(ts_plan* plan, int axes, const void* in, void* out, int dtype, void* hip_stream);

/* Plan of the Q^k spectral-element discretisation (Sec. 2, eq. (eigen_decomp)):
 * each axis of [-L, L] is split into cells[a] equal elements carrying the
 * k+1 Gauss-Lobatto nodes of degree k; n[a] = k cells[a] - 1 interior nodes
 * (ts_sem_nodes), homogeneous Dirichlet ends, lumped Gauss-Lobatto mass M
 * and assembled stiffness S.  H_a = M^{-1} S + diag(f_a); it is diagonalised
 * through the symmetric M^{-1/2} S M^{-1/2} + F = Q Lambda Q^T, so that
 * T = M^{-1/2} Q and T^{-1} = Q^T M^{1/2} (host FP64 Householder reduction
 * and QL).  k = 1 is the FD grid of ts_setup with N_cell = n + 1.
 *   cells : host int64[d], k * cells[a] - 1 in [1, 8192]
 *   k     : polynomial degree, 1..32
 *   f     : host FP64 arrays, f[a] holds f_a at the nodes of ts_sem_nodes
 * Every entry point then works on the nodal values of the SEM grid: the
 * applies compute (H1 + sigma)^{-1} and e^{-i tau H1} with the T factors;
 * ts_operator_apply applies M^{-1} S per axis (band of 2k+1 entries); the
 * solvers (PCG, refinement, inverse iteration) run in the mass inner product
 * sum_p (prod_a m_a) x_p y_p, in which H1 + V2 is self-adjoint, so their
 * residual norms and eigenvector normalisation are mass-weighted.  When an
 * axis has n[a] >= 128 the operator apply runs as one FP64 matrix-core pass
 * per axis restricted to the band |i - j| <= k, in two N-sized FP64 buffers
 * the plan allocates on first use and keeps until ts_destroy.
 * Errors: TS_ERR_INVALID, TS_ERR_NONFINITE, TS_ERR_NOMEM, TS_ERR_DEVICE. */
int ts_setup_sem(int d, const int64_t* cells, int k, double L, const double* const* f, double sigma,
                 ts_plan** out);

/* Plan of arbitrary per-axis operators (Appendix app:hermite: the solver needs
 * only a diagonalisable 1D operator K_a per axis).  Per axis a:
 *   K[a]: host FP64 n[a] x n[a], row-major: the 1D operator without the
 *         potential (for instance -D^2 of ts_hermite_axis)
 *   m[a]: host FP64 n[a] positive weights in which K[a] is self-adjoint
 *         (diag(m) K symmetric to 1e-10 relative); m == NULL or m[a] == NULL
 *         means unit weights (K symmetric)
 *   x[a]: host FP64 n[a] nodes, kept for reporting; x may be NULL
 *   f[a]: host FP64 n[a], the separable potential at the nodes
 * H_a = K_a + diag(f_a) is diagonalised through the symmetric
 * M^{1/2} H_a M^{-1/2} = Q Lambda Q^T (host FP64 Householder and QL), so
 * T = M^{-1/2} Q and T^{-1} = Q^T M^{1/2}, exactly as for ts_setup_sem; every
 * entry point then works on the nodal values, the solvers in the inner
 * product sum_p (prod_a m_a) x_p y_p.  The operator apply (ts_operator_apply,
 * PCG, GPE flows) reads each K_a as a band whose half-width b is the largest
 * |i - j| with K_a[i][j] != 0 over all axes; for b > 32 (for instance a dense
 * K, b = n - 1) it runs instead as one FP64 matrix-core pass per axis with
 * K_a as the factor, in two N-sized FP64 buffers the plan allocates on first
 * use and keeps until ts_destroy.
 * An axis whose K, m and f are reflection-symmetric (to 1e-11 / 1e-13
 * relative) gets the half-extent passes (ts_set_fold).  The plan has no
 * interval [-L, L]: ts_interpolate and the multi-level iteration reject it.
 * n[a] in [1, 8192].  The caller's arrays are copied; nothing is kept.
 * Errors: TS_ERR_INVALID (also for K not self-adjoint in m),
 * TS_ERR_NONFINITE, TS_ERR_NOMEM, TS_ERR_DEVICE. */
int ts_setup_general(int d, const int64_t* n, const double* const* K, const double* const* m,
                     const double* const* x, const double* const* f, double sigma, ts_plan** out);

/* Host: n-point Hermite spectral collocation on the real line (Appendix
 * app:hermite), the input of ts_setup_general for unbounded domains.
 *   x (n): the Gauss-Hermite nodes, the zeros of the degree-n Hermite
 *          polynomial (ascending, x[n-1-j] = -x[j] exactly)
 *   m (n): the Gauss weights of the Hermite functions, 1 / (n psi_{n-1}(x_j)^2)
 *   K (n x n, row-major): -D^2, with the differentiation matrix of the
 *          Hermite functions D_ij = psi_{n-1}(x_i) / (psi_{n-1}(x_j) (x_i - x_j)),
 *          D_ii = 0; diag(m) K is symmetric
 * psi_{n-1} comes from a rescaled three-term recurrence, so the outer nodes
 * do not underflow.  n in [1, 8192].  Errors: TS_ERR_INVALID. */
int ts_hermite_axis(int64_t n, double* x, double* m, double* K);

/* Host: the k cells - 1 interior nodes of Q^k SEM on [-L, L] (ascending),
 * the points at which f_a and V2 are sampled.  x: host array of k cells - 1
 * doubles.  Errors: TS_ERR_INVALID. */
int ts_sem_nodes(int k, int64_t cells, double L, double* x);

/* Host eigen-decomposition of one Q^k SEM axis in its symmetric form
 * M^{-1/2} S M^{-1/2} + diag(f) (Sec. 2, eq. (eigen_decomp)), computed exactly
 * as ts_setup_sem computes it for each axis: the Gauss-Lobatto rule, the
 * element matrices and the assembly in long double, rounded once; Householder
 * reduction and implicit QL in double (on the even and odd blocks when f is
 * reflection-symmetric); one refinement step of the eigenvectors against the
 * operator before rounding.  Needs no GPU.  f: n = k cells - 1 host doubles
 * at the nodes of ts_sem_nodes.  lam: n ascending eigenvalues; Q: row-major
 * n x n, column j = unit eigenvector of lam[j] (the physical eigenvectors are
 * M^{-1/2} Q); m: the n lumped masses, or NULL.  Host pointers.  Errors:
 * TS_ERR_INVALID (bad k, cells or L, null pointer), TS_ERR_NONFINITE,
 * TS_ERR_NOCONV. */
int ts_sem_axis_eig(int k, int64_t cells, double L, const double* f, double* lam, double* Q, double* m);

/* Host copy of the lumped mass of an axis (n[axis] doubles): the
 * Gauss-Lobatto weights times the element half-length, summed at element
 * interfaces; h for FD plans. */
int ts_mass(const ts_plan* plan, int axis, double* out);

/* --------------------------------------------------------------- applies -- */

/* u = (H1 + sigma I)^{-1} b by the four steps of Sec. 2.1: forward transform
 * with Q_k^T on every axis, divide by (sum_k lam_k[j_k] + sigma) formed in
 * FP64, backward transform with Q_k.
 *   b, u  : device arrays of prod(n) elements of dtype TS_F64 or TS_F32; u may
 *           alias b (in place)
 *   prec  : transform arithmetic (see ts_prec), any with either dtype
 * Errors: TS_ERR_INVALID (dtype/prec), TS_ERR_NOT_SPD, TS_ERR_NOMEM. */
int ts_apply_inverse(ts_plan* plan, const void* b, void* u, int dtype, int prec,
                     void* hip_stream);

/* Bytes of the device array that serves ts_apply_inverse_noalloc. */
#define TS_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* ts_apply_inverse for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and result as ts_apply_inverse (bitwise), but the
 * apply's scratch (the pass workspace, N x 8 bytes for grids with an axis of
 * n > 32; the diagonal tables of the grouped passes otherwise) is taken from
 * one static device array of TS_NOALLOC_SCRATCH_BYTES (256 MiB) that every
 * device holds from library load to process exit; the call makes no hipMalloc,
 * hipFree or other allocating call.  The plan's device must be current.  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (two streams, two threads) race and must be ordered by the caller.
 * Errors: as ts_apply_inverse; TS_ERR_INVALID also when the apply needs more
 * than TS_NOALLOC_SCRATCH_BYTES (FP64 grids of more than 2^25 points with an
 * axis of n > 32) or another device is current; TS_ERR_DEVICE if the array's
 * address cannot be obtained. */
int ts_apply_inverse_noalloc(ts_plan* plan, const void* b, void* u, int dtype, int prec,
                             void* hip_stream);

/* Same, with an explicit shift s replacing the plan's sigma: u = (H1 + s)^{-1} b.
 * Used for shifted inverse iteration, where s = -(shift) sits close to
 * -lambda_1 and the denominators must be formed in FP64. */
int ts_apply_inverse_shift(ts_plan* plan, double s, const void* b, void* u, int dtype, int prec,
                           void* hip_stream);

/* psi_out = exp(-i tau H1) psi_in (eq. (exact_prop)): forward transform,
 * multiply by exp(-i tau sum_k lam_k[j_k]) (per-axis FP64 phase factors,
 * multiplied together), backward transform.
 *   psi_in, psi_out : device arrays of prod(n) complex elements (TS_C128 or
 *                     TS_C64, interleaved); psi_out may alias psi_in
 *   tau             : any real time step, including 0 and negative values
 * Errors: TS_ERR_INVALID, TS_ERR_NOMEM. */
int ts_apply_exp(ts_plan* plan, double tau, const void* psi_in, void* psi_out, int dtype, int prec,
                 void* hip_stream);

/* --------------------------------------------------------------- solvers -- */

/* Solve (H1 + sigma I) u = f with the transforms in `inner` precision and
 * FP64 iterative refinement: u <- u + M^{-1}(f - (H1 + sigma) u), the
 * residual formed in FP64 with the (2d+1)-point stencil, until
 * ||r||_2 / ||f||_2 <= rtol or maxit sweeps.  f, u: device FP64.
 * u is an output (its input value is ignored).  If a sweep contracts the
 * residual by less than a factor 0.9 twice, the remaining work switches to
 * flexible CG with the same inner apply.  Synchronises.
 *   iters  : (out, may be NULL) sweeps + CG iterations used
 *   relres : (out, may be NULL) final true relative residual
 * Errors: TS_ERR_NOCONV (u holds the last iterate), TS_ERR_NONFINITE. */
int ts_solve_refined(ts_plan* plan, const double* f, double* u, int inner, double rtol, int maxit,
                     int* iters, double* relres, void* hip_stream);

/* PCG for (H1 + diag(V2) + sigma I) u = f (Sec. 3.2), preconditioner
 * (H1 + sigma I)^{-1} applied in `precond` precision with FP64 input and
 * output.  All vectors, inner products, alpha and beta are FP64 on the
 * device; with a reduced-precision preconditioner beta takes the flexible
 * (Polak-Ribiere) form <z_{k+1}, r_{k+1} - r_k> / <z_k, r_k>.
 *   V2     : device FP64 array of prod(n) values, or NULL for V2 = 0
 *   f      : device FP64 right-hand side
 *   u      : device FP64; in: initial guess, out: solution
 *   rtol   : stop when the recurrence residual ||r||/||f|| <= rtol; the true
 *            residual is then recomputed with the stencil and reported
 *   maxit  : iteration limit
 * Synchronises.  Errors: TS_ERR_NOCONV, TS_ERR_BREAKDOWN, TS_ERR_NONFINITE,
 * TS_ERR_NOT_SPD (H1 + sigma not positive definite). */
int ts_pcg_solve(ts_plan* plan, const double* V2, const double* f, double* u, double rtol, int maxit,
                 int precond, int* iters, double* relres, void* hip_stream);

/* Shifted inverse iteration for the lowest eigenpair of H = H1 + diag(V2)
 * (Sec. 4.1, Sec. 5.3.1).  Each step solves (H - shift) w = u by PCG
 * (preconditioner (H1 - shift)^{-1} in `precond` precision, denominators in
 * FP64), warm-started from the previous step's w, to pcg_rtol; then
 * u <- w / ||w||_2 and lambda <- u^T H u.  The plan's sigma is not used.
 *   V2        : device FP64 or NULL
 *   u         : device FP64; in: start vector (need not be normalised),
 *               out: final normalised eigenvector estimate
 *   steps     : number of steps
 *   lam_hist  : HOST array of steps + 1 doubles (lambda before the first
 *               step, then after each step), may be NULL
 *   pcg_iters : HOST array of `steps` ints, may be NULL
 * Requires H - shift positive definite (shift below lambda_1(H)).
 * Synchronises.  Errors: as ts_pcg_solve. */
int ts_inverse_iteration(ts_plan* plan, const double* V2, double shift, double* u, int steps,
                         double pcg_rtol, int maxit, int precond, double* lam_hist, int* pcg_iters,
                         void* hip_stream);

/* nsteps steps of a splitting scheme for i psi_t = (H1 + V2) psi (Sec. 5.1).
 *   V2    : device array of prod(n) real values, FP64 for TS_C128 data and
 *           FP32 for TS_C64 data
 *   psi   : device complex array (TS_C128 or TS_C64), updated in place
 *   dt    : time step; nsteps >= 0
 *   prec  : transform arithmetic of the exact propagator of H1
 * Errors: TS_ERR_INVALID, TS_ERR_NOMEM. */
int ts_split_step(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int scheme,
                  int dtype, int prec, void* hip_stream);

/* nsteps steps of the approximated qHOP (Sec. 5.1, eq. (qhop_product)) or,
 * with magnus2 != 0, of the approximated Magnus-2 (eq. (yoshida): three qHOP
 * steps of sizes g1 dt, g2 dt, g1 dt) for i psi_t = (A + B) psi, A = H1 of
 * the plan (exact propagator), B = V2 (pointwise).  One qHOP step of size h:
 *   e^{-iA h} prod_{k=1..M} e^{iA s_k} e^{-i w_k h B} e^{-iA s_k},
 * the k = 1 factor acting first, s_k = h x_k and w_k the M-point
 * Gauss-Legendre nodes and normalised weights on [0, 1] (ts_gauss_legendre).
 * It runs in the merged form of Remark rem:cost_naive_merged (M + 1
 * propagations for one step, M per step across steps, 3M per Magnus-2 step),
 * which changes rounding only.  M = 1 is STRANG_ABA and, with magnus2,
 * YOSHIDA_ABA.  For A = -Delta (the quantum-algorithm setting) pass a plan
 * with f = 0 and the whole potential in V2.
 *   V2, psi, dtype, prec : as ts_split_step
 *   dt, nsteps           : step size (may be negative) and count >= 0
 *   M                    : quadrature nodes, 1..64
 * Errors: TS_ERR_INVALID, TS_ERR_NOMEM, TS_ERR_DEVICE. */
int ts_qhop_step(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int M, int magnus2,
                 int dtype, int prec, void* hip_stream);

/* M-point Gauss-Legendre rule on [0, 1] (the s_k / dt and w_k of Sec. 5.1):
 * nodes ascending in (0, 1), weights positive and summing to 1.  Host
 * arrays of M doubles; no GPU needed.  Errors: TS_ERR_INVALID (M outside
 * 1..64 or a null pointer). */
int ts_gauss_legendre(int M, double* nodes, double* weights);

/* Tensor-product linear interpolation from the grid of `coarse` to the grid
 * of `fine` (Sec. 5.3.1): one axis at a time, each fine node taking the two
 * bracketing coarse nodes, with the Dirichlet zeros at -L and L.  The plans
 * must share d and L (FD or SEM grids, any extents).  uc, uf: device FP64
 * arrays of the two grids.  Synchronises the stream.  Errors: TS_ERR_INVALID,
 * TS_ERR_NOMEM, TS_ERR_DEVICE. */
int ts_interpolate(const ts_plan* coarse, const ts_plan* fine, const double* uc, double* uf, void* hip_stream);

/* u = the separable ground state of H1: the outer product of each axis's
 * lowest eigenvector (for SEM the column of T = M^{-1/2} Q), not normalised.
 * Device FP64.  Synchronises. */
int ts_separable_ground_state(const ts_plan* plan, double* u, void* hip_stream);

/* Multi-level shifted inverse iteration (Sec. 5.3.1, Table tab:multilevel)
 * for the lowest eigenpair of H = H1 + diag(V2) on a sequence of grids from
 * coarse to fine.  Level 0 starts from its separable ground state; every
 * later level starts from the previous level's eigenvector interpolated by
 * ts_interpolate.  On each level: the steps of ts_inverse_iteration until
 * |lambda_k - lambda_{k-1}| <= lam_tol |lambda_k| or max_steps.
 *   plans[l], V2[l] (device, may be NULL; V2 itself may be NULL), shifts[l]
 *   (host; below lambda_min(H1) of level l)
 *   u          : device FP64 of the finest grid, out: its eigenvector (unit
 *                norm in the plan's inner product, see ts_setup_sem)
 *   lam_levels, steps, pcg_iters : host arrays of nlevels (may be NULL):
 *                final lambda, steps and total PCG iterations per level
 * Errors: as ts_inverse_iteration. */
int ts_multilevel_inverse_iteration(int nlevels, ts_plan* const* plans, const double* const* V2,
                                    const double* shifts, double* u, int max_steps, double lam_tol,
                                    double pcg_rtol, int pcg_maxit, int precond, double* lam_levels,
                                    int* steps, int* pcg_iters, void* hip_stream);

/* ------------------------------------------------------- GPE flows -- */

/* Ground state of the GPE eq. (gpe), -Delta u + V u + beta u^3 = lambda u
 * with ||u||_{L^2} = 1, by the modified H^1 Riemannian gradient flow
 * (Sec. 4.3, eq. (riemannian_update), metric eq. (h1_metric)):
 *   R(u) = G^{-1} E'(u) - [(u, G^{-1} E'(u)) / (u, G^{-1} u)] G^{-1} u,
 *   u <- (u - tau R(u)) / ||u - tau R(u)||,   G = -Delta + alpha,
 * E'(u) = (-Delta + V + beta u^2) u; two applies of (-Delta + alpha)^{-1} per
 * step.  Inner products are the grid's L^2 sums (weights prod_k m_k, see
 * ts_mass).  Stops when |E_k - E_{k-1}| <= tol |E_k|, E of eq. (gpe_energy);
 * tol <= 0 runs exactly maxit steps (the eigenvalue, first order in the state
 * error, keeps converging after the energy has reached its rounding level).
 *   plan        : plan of -Delta alone (f = 0), FD or SEM; its sigma is unused
 *   V           : device FP64, the whole potential on the grid (may be NULL)
 *   u           : device FP64; in: start (normalised first), out: ground state
 *   maxit       : step limit; energy_hist: HOST array of maxit + 1 doubles or NULL
 *   iters       : steps taken; eigenvalue: lambda = (u, E'(u)); energy: E (host, may be NULL)
 * All vectors, sums and decisions stay on the device; the host polls every
 * few steps.  Errors: TS_ERR_INVALID, TS_ERR_NOT_SPD, TS_ERR_NOCONV (limit
 * reached; u holds the last iterate), TS_ERR_NONFINITE, TS_ERR_NOMEM. */
int ts_gpe_h1_flow(ts_plan* plan, const double* V, double beta, double alpha, double tau, double* u, int maxit,
                   double tol, double* energy_hist, int* iters, double* eigenvalue, double* energy,
                   void* hip_stream);

/* The a_u Riemannian flow (Sec. 4.3, metric eq. (au_metric)): G = G_u =
 * -Delta + V + beta u^2, so G^{-1} E'(u) = u and each step solves G_u z = u
 * by PCG with the preconditioner (-Delta + V1)^{-1} (ts_pcg_solve's solver,
 * warm-started from the previous z, in `precond` precision).
 *   plan          : plan of -Delta + V1 (sigma unused)
 *   V2            : device FP64, V - V1 on the grid, or NULL
 *   pcg_rtol/maxit: inner PCG tolerance and limit
 *   linear_iters  : total PCG iterations (host, may be NULL)
 * Other arguments as ts_gpe_h1_flow.  Errors: as ts_gpe_h1_flow and PCG's. */
int ts_gpe_au_flow(ts_plan* plan, const double* V2, double beta, double tau, double* u, int maxit, double tol,
                   double pcg_rtol, int pcg_maxit, int precond, double* energy_hist, int* iters,
                   int* linear_iters, double* eigenvalue, double* energy, void* hip_stream);

/* ---------------------------------------------------------- operators -- */

/* out = (H1 + diag(V2) + s I) u by the (2d+1)-point stencil, FP64, zero ghost
 * values (the operator of eq. (general_system)).  V2 may be NULL.  u and out
 * must not alias.  Device FP64 arrays. */
int ts_operator_apply(ts_plan* plan, const double* V2, double s, const double* u, double* out,
                      void* hip_stream);

/* ---------------------------------------------------------- accessors -- */

/* Host copy of the ascending eigenvalues of H_axis (n[axis] doubles). */
int ts_eigvals(const ts_plan* plan, int axis, double* out);

/* Host copy of Q_axis, row-major, column j = unit eigenvector of lam[j]
 * (n[axis]^2 doubles).  Eigenvectors are unique up to sign only.  For SEM
 * plans these are the eigenvectors of M^{-1/2} S M^{-1/2} + F; the nodal
 * eigenfunctions are the columns of T = M^{-1/2} Q (ts_mass). */
int ts_eigvecs(const ts_plan* plan, int axis, double* out);

/* Device bytes a single apply of the given dtype may allocate as scratch. */
int ts_workspace_bytes(const ts_plan* plan, int dtype, size_t* bytes);

/* Host FP64 eigendecomposition of the symmetric tridiagonal matrix with
 * diagonal diag[0..n-1] and off-diagonal off[0..n-2] by implicit QL
 * (the per-axis step of eq. (eigen_decomp) that ts_setup runs).  Needs no
 * GPU.  lam: n ascending eigenvalues; Q: row-major n x n, column j = unit
 * eigenvector of lam[j], sign chosen so its largest-magnitude entry is
 * positive.  Host pointers.  Errors: TS_ERR_INVALID, TS_ERR_NOCONV. */
int ts_tridiag_eig(int64_t n, const double* diag, const double* off, double* lam, double* Q);

/* Host: ts_tridiag_eig for a reflection-symmetric tridiagonal (diag[i] =
 * diag[n-1-i], off[i] = off[n-2-i], exactly), solved as the two blocks of its
 * even and odd subspaces (the way ts_setup treats a symmetric f): every
 * eigenvector has exact parity.  Same outputs and conventions as
 * ts_tridiag_eig; n >= 2.  Errors: TS_ERR_INVALID, TS_ERR_NOCONV. */
int ts_tridiag_eig_even_odd(int64_t n, const double* diag, const double* off, double* lam, double* Q);

/* Host FP64 eigendecomposition of a dense symmetric matrix (row-major n x n;
 * the symmetric part (A + A^T)/2 is used) by Householder reduction to
 * tridiagonal form and implicit QL, followed by one refinement step of the
 * eigenvectors against A (Ogita and Aishima, 2018), with the residuals formed
 * in long double (the per-axis step of eq. (eigen_decomp) that ts_setup_sem
 * runs).  Needs no GPU.  lam: n ascending eigenvalues; Q:
 * row-major, column j = unit eigenvector of lam[j], largest-magnitude entry
 * positive.  Host pointers.  Errors: TS_ERR_INVALID, TS_ERR_NOCONV. */
int ts_sym_eig(int64_t n, const double* A, double* lam, double* Q);

/* BF16 rounding exactly as the library applies it, run on the host (needs no
 * GPU); BF16 = 1 sign, 8 exponent, 7 fraction bits.  route 0: the factor
 * copies of the BF16 passes, FP64 rounded once to nearest, ties to even.
 * route 1: data entering a BF16 pass, FP64 rounded to FP32 and then to BF16,
 * each to nearest even (reading of the paper's BF16 runs: data are held in
 * FP32 and rounded to BF16 for the matrix cores).  x: n host doubles; y: n
 * host uint16 bit patterns.  Errors: TS_ERR_INVALID (null pointer, n < 0,
 * route not 0 or 1). */
int ts_bf16_round(int64_t n, const double* x, int route, uint16_t* y);

/* Message describing the last failure on the calling thread ("" if none). */
const char* ts_last_error(void);

/* ------------------------------------------------------------- serving -- */
/* A request loop over the applies and solvers above (not part of the paper):
 * requests of different d, n and kind are admitted as device memory frees
 * up, run concurrently on a pool of HIP streams, and keep their operator
 * factors resident in a plan cache.  Each admitted request advances in small
 * units (one apply, one refinement sweep, a few PCG iterations, a few split
 * steps), so requests that arrive while others run join between units.
 * Results do not depend on what else runs: every kernel is deterministic and
 * a request's arithmetic does not depend on the schedule. */
typedef struct ts_server ts_server;

typedef enum {
  TS_REQ_INVERSE = 0, /* solve: V2 == NULL and prec FP64 -> one direct apply;
                         V2 == NULL, prec FP32/BF16 -> refinement to rtol;
                         V2 != NULL -> PCG to rtol with a prec preconditioner */
  TS_REQ_EXP = 1      /* propagate: V2 == NULL -> exact e^{-i tau H1};
                         V2 != NULL -> Strang (BAB) steps of dt covering tau */
} ts_req_kind;

typedef struct {
  int kind;               /* ts_req_kind */
  int d;                  /* grid: as ts_setup (f[k] are HOST pointers, read at submit) */
  int64_t n[12];
  double L;
  const double* f[12];
  double sigma;
  int dtype;              /* TS_F64 for INVERSE; TS_C128 / TS_C64 for EXP */
  int prec;               /* ts_prec of the transforms */
  const void* in;         /* DEVICE, caller-owned, valid and unchanged until done */
  void* out;              /* DEVICE, caller-owned (may equal in) */
  const void* V2;         /* DEVICE or NULL: FP64 (INVERSE, C128) or FP32 (C64) */
  double tau;             /* EXP: total time */
  double dt;              /* EXP with V2: step (nsteps = ceil(|tau| / dt)) */
  double rtol;            /* INVERSE iterative forms */
  int maxit;
  uint64_t tag;           /* echoed in the result */
} ts_request;

typedef struct {
  int status;             /* ts_status of the request */
  int iters;              /* sweeps / PCG iterations / split steps */
  double relres;          /* true relative residual of iterative solves, else 0 */
  double t_submit, t_admit, t_done;  /* seconds on the server's clock */
  uint64_t tag;
} ts_result;

/* Create a server on the current device.  hbm_budget_bytes bounds the device
 * memory of the server: plan_reserve_bytes of it (0 = a quarter) hold the
 * resident factors of the plan cache (plans are keyed by grid and potential
 * samples; plans no queued or running request uses are evicted least recently
 * used first), the rest is the arena from which every admitted request's
 * scratch is carved (allocated once, here).  n_streams >= 1 non-blocking HIP streams of
 * default priority: each runs the next unit of the most urgent admitted
 * request (urgency = submit time + estimated GPU time), so at most n_streams
 * requests are in flight at once.  max_active caps the admitted requests (0 =
 * no cap); max_active = 1 makes the server a plain FIFO queue (arrival
 * order, one request at a time). */
int ts_serve_create(size_t hbm_budget_bytes, size_t plan_reserve_bytes, int n_streams, int max_active,
                    ts_server** out);

/* Queue a request; it is admitted when its scratch fits.  Returns a ticket.
 * Builds the request's plan here (host eigendecomposition) unless it is cached.
 * TS_ERR_NOMEM if the request could never fit the budget (scratch above the
 * arena or factors above the plan reserve), TS_ERR_BUSY if its plan does not
 * fit the plan reserve while queued or running requests hold the other plans
 * (resubmit later), TS_ERR_INVALID for a malformed request. */
int ts_serve_submit(ts_server* s, const ts_request* req, uint64_t* ticket);

/* Non-blocking: *done = 1 and *res filled once the request has finished. */
int ts_serve_poll(ts_server* s, uint64_t ticket, int* done, ts_result* res);

/* Block until every submitted request has finished. */
int ts_serve_drain(ts_server* s);

/* Seconds on the server's clock (for arrival timestamps). */
double ts_serve_clock(ts_server* s);

/* Stop the scheduler (after draining), release the arena, plans and streams. */
int ts_serve_destroy(ts_server* s);

#ifdef __cplusplus
}
#endif

#endif /* TS_H */
