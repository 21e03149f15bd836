"""Plain CPU FP64 oracle for the separable tensor-product Schroedinger solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the GPU library (``paper_2605_20491_amd``) and never imports it.

The heavy loops live in ``oracle.c`` (plain C, OpenMP over independent fibres
only); the solver drivers below are plain numpy, written in the paper's order:

* operator and per-axis eigendecomposition: Sec. 2.1, eq. (tensor_system),
  eq. (eigen_decomp); Q^1 elements = second-order finite differences.
* direct solve: the four steps of Sec. 2.1.  Propagator: eq. (exact_prop).
* PCG with preconditioner (-Delta + V1)^{-1}: Sec. 3.2 (textbook PCG,
  Saad, "Iterative Methods for Sparse Linear Systems", Alg. 9.1).
* shifted inverse iteration: Sec. 4.1 and Sec. 5.3.1 (each step solves
  (H - s) w = u by PCG, warm-started from the previous solution).
* splitting: Strang (Sec. 5.1), Yoshida composition eq. (yoshida), the
  approximated qHOP product eq. (qhop_product).

Parity status: every public function is pinned by a CPU test in
``tests/test_oracle_*.py`` (closed forms, brute force, printed values of the
paper, invariants) except where its docstring says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

# OpenMP threads of the C core must not spin between calls: numpy's own BLAS
# threads run in the gaps and spinning workers starve them.
os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIBRARY selects another build of the C part (a sanitizer build)
_LIB = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build_sanitized(out: str) -> str:
    """oracle.c with the address and undefined-behaviour sanitizers (ROCm's
    clang, serial, -O1), for the host sanitizer test."""
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    subprocess.check_call([clang, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-std=c11", "-o", out, _SRC,
                           "-lm"])
    return out


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no fast-math)."""
    if "ORACLE_LIBRARY" in os.environ:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.or_grid_spacing.restype = ctypes.c_double
        L.or_grid_spacing.argtypes = [ctypes.c_int64, ctypes.c_double]
        L.or_fd_axis_matrix.argtypes = [ctypes.c_int64, ctypes.c_double, _dp, _dp]
        L.or_jacobi_eigh.restype = ctypes.c_int
        L.or_jacobi_eigh.argtypes = [ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int]
        L.or_mode_product.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, _dp, ctypes.c_int,
                                      ctypes.c_int, _dp, _dp]
        L.or_apply_inverse.argtypes = [ctypes.c_int, _i64p, ctypes.POINTER(_dp),
                                       ctypes.POINTER(_dp), ctypes.c_double, _dp, _dp, _dp]
        L.or_apply_exp.argtypes = [ctypes.c_int, _i64p, ctypes.POINTER(_dp), ctypes.POINTER(_dp),
                                   ctypes.c_double, _dp, _dp, _dp]
        L.or_stencil_apply.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.POINTER(_dp), _dp,
                                       ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.or_dense_operator.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.POINTER(_dp), _dp,
                                        ctypes.c_double, _dp]
        L.or_lu_solve.restype = ctypes.c_int
        L.or_lu_solve.argtypes = [ctypes.c_int64, _dp, _dp, _dp]
        L.or_expm_apply.restype = ctypes.c_int64
        L.or_expm_apply.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.or_phase_apply.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, _dp]
        L.or_num_threads.restype = ctypes.c_int
        L.or_num_threads.argtypes = []
        _lib = L
    return _lib


def num_threads() -> int:
    """OpenMP threads used by the C loops."""
    return int(lib().or_num_threads())


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _shape(shape):
    arr = (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])
    return arr


def _real_view(x: np.ndarray) -> np.ndarray:
    """complex128 array -> float64 view with interleaved (re, im)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    return x.view(np.float64)


# --------------------------------------------------------------------------
# Per-axis operator and eigendecomposition (Sec. 2.1, eq. (eigen_decomp))
# --------------------------------------------------------------------------

def grid_spacing(n: int, L: float) -> float:
    """h = 2L/(n+1): n interior nodes of [-L, L]."""
    return lib().or_grid_spacing(int(n), float(L))


def fd_axis_matrix(n: int, L: float, f: np.ndarray) -> np.ndarray:
    """Dense H_k = h^-2 tridiag(-1, 2, -1) + diag(f_k) (Q^1 = second-order FD)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.shape == (n,)
    H = np.empty((n, n))
    lib().or_fd_axis_matrix(int(n), float(L), _ptr(f), _ptr(H))
    return H


def jacobi_eigh(A: np.ndarray, max_sweeps: int = 60):
    """Cyclic Jacobi: returns (w ascending, V with eigenvectors in columns)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n))
    sweeps = lib().or_jacobi_eigh(n, _ptr(A), _ptr(w), _ptr(V), int(max_sweeps))
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge in %d sweeps" % max_sweeps)
    return w, V


@dataclass
class Plan:
    """Per-axis data of the separable operator H1 = sum_k I x .. x H_k x .. x I.

    ``shape[k]`` and ``f[k]`` follow C order: axis d-1 is the fastest index
    (the paper's x).  ``Q[k]`` columns are eigenvectors, ``lam[k]`` ascending.
    For a Q^k SEM plan (``sem_k`` >= 1) ``m[k]`` is the lumped mass and
    ``K[k]`` the dense M^{-1} S of each axis, and ``Q[k]`` diagonalises the
    symmetric M^{-1/2} S M^{-1/2} + F of eq. (eigen_decomp).  A generic plan
    (``make_plan_general``) carries any K[k] with its weights m[k] the same way.
    """
    shape: tuple
    L: float
    f: list
    h: list = field(default_factory=list)
    Q: list = field(default_factory=list)
    lam: list = field(default_factory=list)
    sem_k: int = 0
    m: list = field(default_factory=list)
    K: list = field(default_factory=list)
    x: list = field(default_factory=list)   # grid nodes of each axis

    @property
    def d(self):
        return len(self.shape)

    @property
    def massed(self):
        """SEM and generic plans: H_k = K_k + F_k is self-adjoint in the mass
        inner product (m non-empty); FD plans use the Euclidean one."""
        return len(self.m) > 0

    @property
    def N(self):
        return int(np.prod(self.shape))


def make_plan(shape, L, f_list) -> Plan:
    shape = tuple(int(s) for s in shape)
    f_list = [np.ascontiguousarray(f, dtype=np.float64) for f in f_list]
    p = Plan(shape=shape, L=float(L), f=f_list)
    cache = {}
    for n, f in zip(shape, f_list):
        key = (n, f.tobytes())
        if key not in cache:
            w, V = jacobi_eigh(fd_axis_matrix(n, L, f))
            cache[key] = (w, V)
        w, V = cache[key]
        p.h.append(grid_spacing(n, L))
        p.Q.append(V)
        p.lam.append(w)
        p.x.append(-L + grid_spacing(n, L) * np.arange(1, n + 1))
    return p


# --------------------------------------------------------------------------
# Q^k spectral elements with Gauss-Lobatto quadrature (Sec. 2, eq. (eigen_decomp))
# --------------------------------------------------------------------------

def gll_rule(k: int):
    """(k+1)-point Gauss-Lobatto rule on [-1, 1]: the end points and the roots
    of P_k' (numpy's Legendre series), weights 2 / (k (k+1) P_k(x)^2)."""
    Pk = np.polynomial.legendre.Legendre.basis(int(k))
    inner = np.sort(Pk.deriv().roots().real) if k > 1 else np.zeros(0)
    x = np.concatenate([[-1.0], inner, [1.0]])
    return x, 2.0 / (k * (k + 1) * Pk(x) ** 2)


def lagrange_derivative_matrix(xi: np.ndarray) -> np.ndarray:
    """D[q, j] = l_j'(xi_q) for the Lagrange basis on the nodes xi, from the
    product rule applied to l_j(x) = prod_{a != j} (x - xi_a) / (xi_j - xi_a)."""
    m = len(xi)
    D = np.zeros((m, m))
    for q in range(m):
        for j in range(m):
            acc = 0.0
            for a in range(m):
                if a == j:
                    continue
                term = 1.0 / (xi[j] - xi[a])
                for l in range(m):
                    if l != j and l != a:
                        term *= (xi[q] - xi[l]) / (xi[j] - xi[l])
                acc += term
            D[q, j] = acc
    return D


def sem_axis(k: int, n_cells: int, L: float):
    """Interior nodes, lumped mass and dense stiffness of Q^k SEM on [-L, L]
    with n_cells equal elements and homogeneous Dirichlet ends.

    Element e maps the reference nodes xi to -L + e he + (xi + 1) he / 2,
    he = 2L / n_cells; mass m = sum over elements of (he/2) w; stiffness
    S = sum over elements of (2/he) D^T diag(w) D.  The k n_cells - 1 interior
    nodes are returned (the two end nodes carry the Dirichlet values)."""
    xi, w = gll_rule(k)
    D = lagrange_derivative_matrix(xi)
    he = 2.0 * L / n_cells
    G = k * n_cells + 1
    x = np.empty(G)
    m = np.zeros(G)
    S = np.zeros((G, G))
    Se = (2.0 / he) * (D.T * w) @ D
    for e in range(n_cells):
        idx = e * k + np.arange(k + 1)
        x[idx] = -L + e * he + (xi + 1.0) * he / 2.0
        m[idx] += w * he / 2.0
        S[np.ix_(idx, idx)] += Se
    return x[1:-1].copy(), m[1:-1].copy(), np.ascontiguousarray(S[1:-1, 1:-1])


def sem_nodes(k: int, n_cells: int, L: float) -> np.ndarray:
    return sem_axis(k, n_cells, L)[0]


# --------------------------------------------------------------------------
# Generic per-axis operators (Appendix app:hermite: the solver needs only a
# diagonalisable 1D operator per axis); Hermite spectral collocation
# --------------------------------------------------------------------------

def hermite_functions(kmax: int, x: np.ndarray) -> np.ndarray:
    """Rows 0..kmax: the normalised Hermite functions psi_k(x) by the three-term
    recurrence psi_{k+1} = sqrt(2/(k+1)) x psi_k - sqrt(k/(k+1)) psi_{k-1},
    psi_0 = pi^{-1/4} exp(-x^2/2) (which underflows for |x| beyond about 37)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((kmax + 1,) + x.shape)
    out[0] = np.pi ** -0.25 * np.exp(-0.5 * x * x)
    if kmax >= 1:
        out[1] = np.sqrt(2.0) * x * out[0]
    for k in range(1, kmax):
        out[k + 1] = np.sqrt(2.0 / (k + 1)) * x * out[k] - np.sqrt(k / (k + 1.0)) * out[k - 1]
    return out


def hermite_axis(n: int):
    """(x, m, K) of n-point Hermite spectral collocation on the real line
    (Appendix app:hermite).  Nodes: eigenvalues of the symmetric tridiagonal
    J with zero diagonal and J[k-1, k] = sqrt(k/2) (numpy's eigvalsh).
    D[i, j] = psi_{n-1}(x_i) / (psi_{n-1}(x_j) (x_i - x_j)), D[i, i] = 0, and
    K = -D^2.  m[j] = 1 / (n psi_{n-1}(x_j)^2), the Gauss weights of the
    Hermite functions, in which K is self-adjoint (diag(m) K symmetric)."""
    n = int(n)
    J = np.diag(np.sqrt(np.arange(1, n) / 2.0), 1)
    x = np.linalg.eigvalsh(J + J.T)
    psi = hermite_functions(n - 1, x)[n - 1]
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = psi[i] / (psi[j] * (x[i] - x[j]))
    K = -(D @ D)
    m = 1.0 / (n * psi * psi)
    return x, m, K


def make_plan_general(K_list, m_list, f_list, x_list=None) -> Plan:
    """Plan of arbitrary per-axis operators H_k = K_k + diag(f_k), with K_k
    self-adjoint in the weights m_k (diag(m_k) K_k symmetric; None = unit
    weights).  As for SEM, the symmetric M^{1/2} H_k M^{-1/2} is diagonalised
    (Jacobi) and T = M^{-1/2} Q, T^{-1} = Q^T M^{1/2}."""
    K_list = [np.ascontiguousarray(K, dtype=np.float64) for K in K_list]
    shape = tuple(K.shape[0] for K in K_list)
    f_list = [np.ascontiguousarray(f, dtype=np.float64) for f in f_list]
    m_list = [np.ones(K.shape[0]) if m is None else np.ascontiguousarray(m, dtype=np.float64)
              for K, m in zip(K_list, m_list)]
    p = Plan(shape=shape, L=float("nan"), f=f_list)
    for a, (K, m, f) in enumerate(zip(K_list, m_list, f_list)):
        sq = np.sqrt(m)
        A = sq[:, None] * K / sq[None, :] + np.diag(f)
        w, V = jacobi_eigh(0.5 * (A + A.T))
        p.h.append(float("nan"))
        p.Q.append(V)
        p.lam.append(w)
        p.m.append(m)
        p.K.append(K)
        p.x.append(np.arange(K.shape[0], dtype=np.float64) if x_list is None
                   else np.ascontiguousarray(x_list[a], dtype=np.float64))
    return p


def make_plan_sem(k: int, cells, L, f_list) -> Plan:
    """Q^k SEM plan: H_k = M^{-1} S + F = M^{-1/2} (M^{-1/2} S M^{-1/2} + F) M^{1/2}
    (eq. (eigen_decomp)); the symmetric middle factor is diagonalised by Jacobi."""
    cells = tuple(int(c) for c in cells)
    shape = tuple(k * c - 1 for c in cells)
    f_list = [np.ascontiguousarray(f, dtype=np.float64) for f in f_list]
    p = Plan(shape=shape, L=float(L), f=f_list, sem_k=int(k))
    for c, f in zip(cells, f_list):
        x, m, S = sem_axis(k, c, L)
        sq = np.sqrt(m)
        A = S / np.outer(sq, sq) + np.diag(f)
        w, V = jacobi_eigh(0.5 * (A + A.T))
        p.h.append(2.0 * L / c)
        p.Q.append(V)
        p.lam.append(w)
        p.m.append(m)
        p.K.append(np.ascontiguousarray(S / m[:, None]))
        p.x.append(x)
    return p


def _mass_root(plan: Plan, power: float) -> np.ndarray:
    """prod_k m_k(x_k)^power on the grid."""
    out = np.ones(())
    for m in plan.m:
        out = np.multiply.outer(out, m ** power)
    return out


def _arrays_ptrs(arrs):
    return (_dp * len(arrs))(*[_ptr(a) for a in arrs])


# --------------------------------------------------------------------------
# Separable apply (Sec. 2.1 four-step solve; eq. (exact_prop))
# --------------------------------------------------------------------------

def mode_product(shape, axis, Q, X, transpose: bool):
    """Mode-`axis` product with Q^T (transpose=True) or Q.  X real or complex."""
    cplx = np.iscomplexobj(X)
    Xr = _real_view(X) if cplx else np.ascontiguousarray(X, dtype=np.float64)
    Y = np.empty_like(Xr)
    lib().or_mode_product(len(shape), _shape(shape), int(axis), _ptr(np.ascontiguousarray(Q)),
                          1 if transpose else 0, 2 if cplx else 1, _ptr(Xr), _ptr(Y))
    return Y.view(np.complex128).reshape(shape) if cplx else Y.reshape(shape)


def apply_inverse(plan: Plan, b: np.ndarray, sigma: float) -> np.ndarray:
    """u = (H1 + sigma I)^{-1} b by the four-step solve (real FP64).  For SEM,
    T^{-1} = Q^T M^{1/2} and T = M^{-1/2} Q: the orthogonal solve between the
    two diagonal mass scalings."""
    if plan.massed:
        b = np.asarray(b, dtype=np.float64).reshape(plan.shape) * _mass_root(plan, 0.5)
        return _apply_inverse_q(plan, b, sigma) * _mass_root(plan, -0.5)
    return _apply_inverse_q(plan, b, sigma)


def _apply_inverse_q(plan: Plan, b: np.ndarray, sigma: float) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(plan.shape)
    u = np.empty_like(b)
    work = np.empty_like(b)
    lib().or_apply_inverse(plan.d, _shape(plan.shape), _arrays_ptrs(plan.Q), _arrays_ptrs(plan.lam),
                           float(sigma), _ptr(b), _ptr(u), _ptr(work))
    return u


def apply_exp(plan: Plan, psi: np.ndarray, tau: float) -> np.ndarray:
    """psi' = exp(-i tau H1) psi (eq. (exact_prop)), complex128; SEM as apply_inverse."""
    if plan.massed:
        x = np.asarray(psi, dtype=np.complex128).reshape(plan.shape) * _mass_root(plan, 0.5)
        return _apply_exp_q(plan, x, tau) * _mass_root(plan, -0.5)
    return _apply_exp_q(plan, psi, tau)


def _apply_exp_q(plan: Plan, psi: np.ndarray, tau: float) -> np.ndarray:
    x = _real_view(np.asarray(psi).reshape(plan.shape))
    out = np.empty_like(x)
    work = np.empty_like(x)
    lib().or_apply_exp(plan.d, _shape(plan.shape), _arrays_ptrs(plan.Q), _arrays_ptrs(plan.lam),
                       float(tau), _ptr(x), _ptr(out), _ptr(work))
    return out.view(np.complex128).reshape(plan.shape)


# --------------------------------------------------------------------------
# Non-separable operator by its stencil (eq. (general_system)) and brute force
# --------------------------------------------------------------------------

def stencil_apply(plan: Plan, u: np.ndarray, V2=None, sigma: float = 0.0) -> np.ndarray:
    """(H1 + diag V2 + sigma I) u, by the (2d+1)-point stencil with zero ghosts."""
    cplx = np.iscomplexobj(u)
    ur = _real_view(u.reshape(plan.shape)) if cplx else np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(ur)
    V2p = None if V2 is None else _ptr(np.ascontiguousarray(V2, dtype=np.float64).reshape(-1))
    hs = np.array(plan.h, dtype=np.float64)
    lib().or_stencil_apply(plan.d, _shape(plan.shape), _ptr(hs), _arrays_ptrs(plan.f), V2p,
                           float(sigma), 2 if cplx else 1, _ptr(ur), _ptr(out))
    return out.view(np.complex128).reshape(plan.shape) if cplx else out.reshape(plan.shape)


def operator_apply(plan: Plan, u: np.ndarray, V2=None, sigma: float = 0.0) -> np.ndarray:
    """(H1 + diag V2 + sigma I) u of eq. (general_system): the stencil for FD
    plans; for SEM plans sum_k (I x .. x K_k x .. x I) u by mode products with
    the dense K_k = M_k^{-1} S_k, plus (sum_k f_k + V2 + sigma) u."""
    if not plan.massed:
        return stencil_apply(plan, u, V2, sigma)
    u = np.asarray(u).reshape(plan.shape)
    out = np.zeros_like(u)
    diag = np.full(plan.shape, float(sigma))
    for k in range(plan.d):
        out = out + mode_product(plan.shape, k, plan.K[k], u, transpose=False)
        idx = [None] * plan.d
        idx[k] = slice(None)
        diag = diag + plan.f[k][tuple(idx)]
    if V2 is not None:
        diag = diag + np.asarray(V2, dtype=np.float64).reshape(plan.shape)
    return out + diag * u


def dense_operator(plan: Plan, V2=None, sigma: float = 0.0) -> np.ndarray:
    """Dense N x N matrix of H1 + diag V2 + sigma I: from the stencil rule for FD
    plans; for SEM plans the Kronecker sum of eq. (general_system) assembled
    with np.kron from the per-axis K_k + F_k."""
    if plan.massed:
        N = plan.N
        H = np.zeros((N, N))
        for k in range(plan.d):
            left = int(np.prod(plan.shape[:k]))
            right = int(np.prod(plan.shape[k + 1:]))
            Hk = plan.K[k] + np.diag(plan.f[k])
            H += np.kron(np.kron(np.eye(left), Hk), np.eye(right))
        diag = np.full(N, float(sigma))
        if V2 is not None:
            diag += np.asarray(V2, dtype=np.float64).reshape(-1)
        return H + np.diag(diag)
    N = plan.N
    H = np.empty((N, N))
    V2p = None if V2 is None else _ptr(np.ascontiguousarray(V2, dtype=np.float64).reshape(-1))
    hs = np.array(plan.h, dtype=np.float64)
    lib().or_dense_operator(plan.d, _shape(plan.shape), _ptr(hs), _arrays_ptrs(plan.f), V2p,
                            float(sigma), _ptr(H))
    return H


def lu_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Dense LU with partial pivoting."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    x = np.empty_like(b)
    if lib().or_lu_solve(A.shape[0], _ptr(A), _ptr(b), _ptr(x)) != 0:
        raise np.linalg.LinAlgError("singular")
    return x


def expm_apply(H: np.ndarray, tau: float, psi: np.ndarray, nterms: int = 30) -> np.ndarray:
    """exp(-i tau H) psi by truncated Taylor series with scaling (dense H)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    x = _real_view(np.asarray(psi).reshape(-1))
    out = np.empty_like(x)
    lib().or_expm_apply(H.shape[0], _ptr(H), float(tau), int(nterms), _ptr(x), _ptr(out))
    return out.view(np.complex128).reshape(np.shape(psi))


def phase_apply(V: np.ndarray, theta: float, psi: np.ndarray) -> np.ndarray:
    """exp(-i theta V) psi, pointwise (a potential sub-step of the splittings)."""
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1)
    x = _real_view(np.array(psi, dtype=np.complex128, copy=True).reshape(-1))
    lib().or_phase_apply(V.size, _ptr(V), float(theta), _ptr(x))
    return x.view(np.complex128).reshape(np.shape(psi))


# --------------------------------------------------------------------------
# PCG (Sec. 3.2) and shifted inverse iteration (Sec. 4.1, 5.3.1)
# --------------------------------------------------------------------------

@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    relres: float          # recurrence residual ||r_k|| / ||f||
    true_relres: float     # ||f - A x|| / ||f|| recomputed with the stencil
    history: list


def inner(plan: Plan, x: np.ndarray, y: np.ndarray) -> float:
    """Inner product in which H1 is self-adjoint: Euclidean for FD plans, the
    mass-weighted sum_p (prod_k m_k) x_p y_p for SEM plans (H_k = M^{-1} S + F
    is symmetric with respect to M, not in the plain dot product)."""
    if plan.massed:
        return float(np.sum(_mass_root(plan, 1.0) * np.asarray(x).reshape(plan.shape)
                            * np.asarray(y).reshape(plan.shape)))
    return float(np.vdot(x, y))


def norm(plan: Plan, x: np.ndarray) -> float:
    return float(np.sqrt(inner(plan, x, x)))


def pcg(plan: Plan, V2, sigma: float, f: np.ndarray, x0=None, rtol: float = 1e-13,
        maxit: int = 500) -> PCGResult:
    """Textbook PCG for (H1 + diag V2 + sigma) x = f, preconditioner (H1 + sigma)^{-1},
    in the inner product of ``inner`` (for SEM plans this is CG on the
    symmetric weak form S + M (V + sigma)).

    The preconditioner is the oracle's own four-step solve in FP64.
    """
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(plan.shape)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64).reshape(plan.shape)
    nf = norm(plan, f)
    r = f - operator_apply(plan, x, V2, sigma)
    z = apply_inverse(plan, r, sigma)
    p = z.copy()
    rz = inner(plan, r, z)
    hist = [norm(plan, r) / nf]
    k = 0
    while hist[-1] > rtol and k < maxit:
        q = operator_apply(plan, p, V2, sigma)
        alpha = rz / inner(plan, p, q)
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        hist.append(norm(plan, r) / nf)
        if hist[-1] <= rtol:
            break
        z = apply_inverse(plan, r, sigma)
        rz_new = inner(plan, r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    true = norm(plan, f - operator_apply(plan, x, V2, sigma)) / nf
    return PCGResult(x=x, iters=k, relres=hist[-1], true_relres=true, history=hist)


def separable_ground_state(plan: Plan) -> np.ndarray:
    """Ground state of H1: the tensor product of each axis's lowest eigenvector
    (for SEM the column of T = M^{-1/2} Q), unit norm in ``inner``."""
    u = np.ones(())
    for k in range(plan.d):
        v = plan.Q[k][:, 0]
        if plan.massed:
            v = v / np.sqrt(plan.m[k])
        u = np.multiply.outer(u, v)
    return np.ascontiguousarray(u / norm(plan, u))


@dataclass
class InvIterResult:
    u: np.ndarray
    lam: list       # Rayleigh quotient after each step (index 0 = start vector)
    pcg_iters: list


def inverse_iteration(plan: Plan, V2, shift: float, steps: int = 20, u0=None,
                      pcg_rtol: float = 1e-13, maxit: int = 500, lam_tol: float = 0.0) -> InvIterResult:
    """Shifted inverse iteration for the lowest eigenpair of H = H1 + diag V2.

    Each step solves (H - shift) w = u by PCG preconditioned with
    (H1 - shift)^{-1}, warm-started from the previous step's solution w;
    then u <- w / ||w|| and lambda <- <u, H u> (norm and inner product of
    ``inner``).  With lam_tol > 0 the iteration stops early once
    |lambda_k - lambda_{k-1}| <= lam_tol |lambda_k|.
    """
    u = separable_ground_state(plan) if u0 is None else np.array(u0, dtype=np.float64)
    u = u / norm(plan, u)
    lam = [inner(plan, u, operator_apply(plan, u, V2, 0.0))]
    its = []
    w = None
    for _ in range(steps):
        res = pcg(plan, V2, -shift, u, x0=w, rtol=pcg_rtol, maxit=maxit)
        w = res.x
        its.append(res.iters)
        u = w / norm(plan, w)
        lam.append(inner(plan, u, operator_apply(plan, u, V2, 0.0)))
        if lam_tol > 0 and abs(lam[-1] - lam[-2]) <= lam_tol * abs(lam[-1]):
            break
    return InvIterResult(u=u, lam=lam, pcg_iters=its)


def interpolate(coarse: Plan, fine: Plan, u: np.ndarray) -> np.ndarray:
    """Tensor-product linear interpolation from the nodes of `coarse` to those
    of `fine` (Sec. 5.3.1), with the Dirichlet zeros at -L and L; one axis at a
    time with numpy's interp."""
    out = np.asarray(u, dtype=np.float64).reshape(coarse.shape)
    L = coarse.L
    for k in range(coarse.d):
        xc = np.concatenate([[-L], coarse.x[k], [L]])
        xf = fine.x[k]
        moved = np.moveaxis(out, k, -1)
        flat = moved.reshape(-1, moved.shape[-1])
        res = np.empty((flat.shape[0], xf.size))
        for r in range(flat.shape[0]):
            res[r] = np.interp(xf, xc, np.concatenate([[0.0], flat[r], [0.0]]))
        out = np.moveaxis(res.reshape(moved.shape[:-1] + (xf.size,)), -1, k)
    return np.ascontiguousarray(out)


@dataclass
class MultilevelResult:
    u: np.ndarray
    lam: float
    steps: list        # inverse-iteration steps per level
    pcg_iters: list    # PCG iterations per level (sum over its steps)
    lam_levels: list   # final lambda of each level


def multilevel_inverse_iteration(levels, lam_tol: float = 1e-13, max_steps: int = 100,
                                 pcg_rtol: float = 1e-12, maxit: int = 500) -> MultilevelResult:
    """Multi-level shifted inverse iteration (Sec. 5.3.1): `levels` is a list of
    (plan, V2, shift) from coarse to fine.  The first level starts from the
    separable ground state of its plan; each later level starts from the
    previous level's eigenvector, linearly interpolated."""
    u = None
    steps, its, lams = [], [], []
    prev = None
    for plan, V2, shift in levels:
        if prev is not None:
            u = interpolate(prev, plan, u)
        r = inverse_iteration(plan, V2, shift, steps=max_steps, u0=u, pcg_rtol=pcg_rtol, maxit=maxit,
                              lam_tol=lam_tol)
        u = r.u
        steps.append(len(r.lam) - 1)
        its.append(int(sum(r.pcg_iters)))
        lams.append(r.lam[-1])
        prev = plan
    return MultilevelResult(u=u, lam=lams[-1], steps=steps, pcg_iters=its, lam_levels=lams)


# --------------------------------------------------------------------------
# Splitting (Sec. 5.1): A = H1 (exact propagator), B = V2 (pointwise)
# --------------------------------------------------------------------------

YOSHIDA_G1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
YOSHIDA_G2 = -(2.0 ** (1.0 / 3.0)) / (2.0 - 2.0 ** (1.0 / 3.0))


def strang_step(plan: Plan, V2, psi, dt, form: str = "BAB"):
    """One Strang step.  BAB: e^{-iB dt/2} e^{-iA dt} e^{-iB dt/2};  ABA: A and B swapped."""
    if form == "BAB":
        psi = phase_apply(V2, dt / 2, psi)
        psi = apply_exp(plan, psi, dt)
        psi = phase_apply(V2, dt / 2, psi)
    elif form == "ABA":
        psi = apply_exp(plan, psi, dt / 2)
        psi = phase_apply(V2, dt, psi)
        psi = apply_exp(plan, psi, dt / 2)
    else:
        raise ValueError(form)
    return psi


def yoshida_step(plan: Plan, V2, psi, dt, form: str = "BAB"):
    """eq. (yoshida): Strang(g1 dt) Strang(g2 dt) Strang(g1 dt)."""
    for g in (YOSHIDA_G1, YOSHIDA_G2, YOSHIDA_G1):
        psi = strang_step(plan, V2, psi, g * dt, form)
    return psi


def split_propagate(plan: Plan, V2, psi0, dt, nsteps, scheme: str = "strang_bab"):
    """nsteps of the given scheme, as the literal product (no merging of factors)."""
    psi = np.array(psi0, dtype=np.complex128, copy=True).reshape(plan.shape)
    V2 = np.ascontiguousarray(V2, dtype=np.float64).reshape(plan.shape)
    for _ in range(int(nsteps)):
        if scheme == "strang_bab":
            psi = strang_step(plan, V2, psi, dt, "BAB")
        elif scheme == "strang_aba":
            psi = strang_step(plan, V2, psi, dt, "ABA")
        elif scheme == "yoshida_bab":
            psi = yoshida_step(plan, V2, psi, dt, "BAB")
        elif scheme == "yoshida_aba":
            psi = yoshida_step(plan, V2, psi, dt, "ABA")
        else:
            raise ValueError(scheme)
    return psi


# --------------------------------------------------------------------------
# Approximated qHOP (eq. (qhop_product)) and Magnus-2 via Yoshida composition
# --------------------------------------------------------------------------

def gauss_legendre(M: int, h: float):
    """Nodes s_k in [0, h] and normalised weights w_k (sum w_k = 1) of the
    M-point Gauss-Legendre rule (numpy's leggauss, mapped from [-1, 1])."""
    xi, om = np.polynomial.legendre.leggauss(int(M))
    return h * (xi + 1.0) / 2.0, om / 2.0


def qhop_step(plan: Plan, V2, psi, h, M: int):
    """One approximated qHOP step (Sec. 5.1):
    P(h) = e^{-iAh} prod_{k=1}^{M} e^{iA s_k} e^{-i w_k h B} e^{-iA s_k},
    the k = 1 factor acting first; A = H1, B = V2.  The literal product with
    2M + 1 propagations (no merging)."""
    s, w = gauss_legendre(M, h)
    for k in range(M):
        psi = apply_exp(plan, psi, s[k])
        psi = phase_apply(V2, w[k] * h, psi)
        psi = apply_exp(plan, psi, -s[k])
    return apply_exp(plan, psi, h)


def magnus2_step(plan: Plan, V2, psi, h, M: int):
    """eq. (yoshida) applied to the approximated qHOP step: P(g1 h) P(g2 h) P(g1 h)."""
    for g in (YOSHIDA_G1, YOSHIDA_G2, YOSHIDA_G1):
        psi = qhop_step(plan, V2, psi, g * h, M)
    return psi


def qhop_propagate(plan: Plan, V2, psi0, dt, nsteps, M: int, yoshida: bool = False):
    psi = np.array(psi0, dtype=np.complex128, copy=True).reshape(plan.shape)
    V2 = np.ascontiguousarray(V2, dtype=np.float64).reshape(plan.shape)
    for _ in range(int(nsteps)):
        psi = magnus2_step(plan, V2, psi, dt, M) if yoshida else qhop_step(plan, V2, psi, dt, M)
    return psi


# --------------------------------------------------------------------------
# GPE ground state by Riemannian gradient flows (Sec. 4.2, 4.3)
# --------------------------------------------------------------------------

def l2_weights(plan: Plan) -> np.ndarray:
    """Quadrature weights of the discrete L^2 inner product on the grid:
    prod_k m_k (Gauss-Lobatto mass) for SEM plans, h^d for FD plans."""
    if plan.massed:
        return _mass_root(plan, 1.0)
    return np.full(plan.shape, float(np.prod(plan.h)))


def gpe_energy(plan_lap: Plan, V, beta: float, u: np.ndarray) -> float:
    """eq. (gpe_energy): E(u) = 1/2 [(grad u, grad u) + (V u, u)] + beta/4 (u^4, 1),
    with (grad u, grad u) = (-Delta_h u, u) and the plan's L^2 weights.
    plan_lap discretises -Delta alone (f = 0); V is the full potential on the grid."""
    w = l2_weights(plan_lap)
    lap_u = operator_apply(plan_lap, u, None, 0.0)
    return float(0.5 * np.sum(w * u * lap_u) + 0.5 * np.sum(w * V * u * u) + 0.25 * beta * np.sum(w * u**4))


def gpe_eigenvalue(plan_lap: Plan, V, beta: float, u: np.ndarray) -> float:
    """lambda = ((-Delta + V + beta u^2) u, u) for ||u||_{L^2} = 1 (eq. (gpe))."""
    w = l2_weights(plan_lap)
    Hu = operator_apply(plan_lap, u, V + beta * u * u, 0.0)
    return float(np.sum(w * u * Hu))


def _riemannian_step(u, grad_g, normal_g, tau, w):
    """eq. (riemannian_update): project the metric gradient G^{-1} E'(u) onto the
    tangent space {v : (u, v) = 0} of the L^2 sphere along the metric normal
    G^{-1} u, step by tau and renormalise in L^2."""
    coef = np.sum(w * u * grad_g) / np.sum(w * u * normal_g)
    r = grad_g - coef * normal_g
    v = u - tau * r
    return v / np.sqrt(np.sum(w * v * v))


def h1_flow_step(plan_lap: Plan, V, beta: float, alpha: float, tau: float, u: np.ndarray) -> np.ndarray:
    """Modified H^1 flow, metric eq. (h1_metric) with G = -Delta + alpha: the two
    solves G^{-1} E'(u) and G^{-1} u, E'(u) = (-Delta + V + beta u^2) u."""
    Eprime = operator_apply(plan_lap, u, V + beta * u * u, 0.0)
    grad_g = apply_inverse(plan_lap, Eprime, alpha)
    normal_g = apply_inverse(plan_lap, u, alpha)
    return _riemannian_step(u, grad_g, normal_g, tau, l2_weights(plan_lap))


def au_flow_step(plan_v1: Plan, V2, beta: float, tau: float, u: np.ndarray, pcg_rtol: float = 1e-13):
    """a_u flow, metric eq. (au_metric) with G_u = -Delta + V + beta u^2: then
    G_u^{-1} E'(u) = u, and the normal G_u^{-1} u is one PCG solve with the
    preconditioner (-Delta + V1)^{-1} (plan_v1 holds V1; V2 the rest of V).
    Returns (u_new, pcg iterations)."""
    extra = beta * u * u if V2 is None else V2 + beta * u * u
    res = pcg(plan_v1, extra, 0.0, u, rtol=pcg_rtol)
    return _riemannian_step(u, u, res.x, tau, l2_weights(plan_v1)), res.iters


@dataclass
class GPEResult:
    u: np.ndarray
    energy: list
    eigenvalue: float
    iters: int


def gpe_ground_state(plan_lap: Plan, V, beta: float, u0: np.ndarray, method: str = "h1", alpha: float = 20.0,
                     tau: float = 0.1, tol: float = 1e-12, maxit: int = 2000, plan_v1: Plan = None,
                     V2=None) -> GPEResult:
    """Iterate a flow until |E_k - E_{k-1}| <= tol |E_k|.  The start is
    renormalised in L^2.  method 'h1' uses plan_lap (f = 0); 'au' uses plan_v1
    (f = V1) and V2 = V - V1 (None when V is separable)."""
    w = l2_weights(plan_lap)
    u = np.array(u0, dtype=np.float64).reshape(plan_lap.shape)
    u = u / np.sqrt(np.sum(w * u * u))
    E = [gpe_energy(plan_lap, V, beta, u)]
    k = 0
    while k < maxit:
        if method == "h1":
            u = h1_flow_step(plan_lap, V, beta, alpha, tau, u)
        else:
            u, _ = au_flow_step(plan_v1, V2, beta, tau, u)
        k += 1
        E.append(gpe_energy(plan_lap, V, beta, u))
        if abs(E[-1] - E[-2]) <= tol * abs(E[-1]):
            break
    return GPEResult(u=u, energy=E, eigenvalue=gpe_eigenvalue(plan_lap, V, beta, u), iters=k)
