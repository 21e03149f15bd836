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
_LIB = os.path.join(_HERE, "_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no fast-math)."""
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
    """
    shape: tuple
    L: float
    f: list
    h: list = field(default_factory=list)
    Q: list = field(default_factory=list)
    lam: list = field(default_factory=list)

    @property
    def d(self):
        return len(self.shape)

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
    return p


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
    """u = (H1 + sigma I)^{-1} b by the four-step solve (real FP64)."""
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(plan.shape)
    u = np.empty_like(b)
    work = np.empty_like(b)
    lib().or_apply_inverse(plan.d, _shape(plan.shape), _arrays_ptrs(plan.Q), _arrays_ptrs(plan.lam),
                           float(sigma), _ptr(b), _ptr(u), _ptr(work))
    return u


def apply_exp(plan: Plan, psi: np.ndarray, tau: float) -> np.ndarray:
    """psi' = exp(-i tau H1) psi (eq. (exact_prop)), complex128."""
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


def dense_operator(plan: Plan, V2=None, sigma: float = 0.0) -> np.ndarray:
    """Dense N x N matrix of H1 + diag V2 + sigma I built from the stencil rule."""
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


def pcg(plan: Plan, V2, sigma: float, f: np.ndarray, x0=None, rtol: float = 1e-13,
        maxit: int = 500) -> PCGResult:
    """Textbook PCG for (H1 + diag V2 + sigma) x = f, preconditioner (H1 + sigma)^{-1}.

    The preconditioner is the oracle's own four-step solve in FP64.
    """
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(plan.shape)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64).reshape(plan.shape)
    nf = np.linalg.norm(f)
    r = f - stencil_apply(plan, x, V2, sigma)
    z = apply_inverse(plan, r, sigma)
    p = z.copy()
    rz = float(np.vdot(r, z))
    hist = [np.linalg.norm(r) / nf]
    k = 0
    while hist[-1] > rtol and k < maxit:
        q = stencil_apply(plan, p, V2, sigma)
        alpha = rz / float(np.vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        hist.append(np.linalg.norm(r) / nf)
        if hist[-1] <= rtol:
            break
        z = apply_inverse(plan, r, sigma)
        rz_new = float(np.vdot(r, z))
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    true = np.linalg.norm(f - stencil_apply(plan, x, V2, sigma)) / nf
    return PCGResult(x=x, iters=k, relres=hist[-1], true_relres=true, history=hist)


def separable_ground_state(plan: Plan) -> np.ndarray:
    """Ground state of H1: the tensor product of each axis's lowest eigenvector."""
    u = np.ones(())
    for k in range(plan.d):
        u = np.multiply.outer(u, plan.Q[k][:, 0])
    return np.ascontiguousarray(u / np.linalg.norm(u))


@dataclass
class InvIterResult:
    u: np.ndarray
    lam: list       # Rayleigh quotient after each step (index 0 = start vector)
    pcg_iters: list


def inverse_iteration(plan: Plan, V2, shift: float, steps: int = 20, u0=None,
                      pcg_rtol: float = 1e-13, maxit: int = 500) -> InvIterResult:
    """Shifted inverse iteration for the lowest eigenpair of H = H1 + diag V2.

    Each step solves (H - shift) w = u by PCG preconditioned with
    (H1 - shift)^{-1}, warm-started from the previous step's solution w;
    then u <- w / ||w|| and lambda <- u^T H u.
    """
    u = separable_ground_state(plan) if u0 is None else np.array(u0, dtype=np.float64)
    u = u / np.linalg.norm(u)
    lam = [float(np.vdot(u, stencil_apply(plan, u, V2, 0.0)))]
    its = []
    w = None
    for _ in range(steps):
        res = pcg(plan, V2, -shift, u, x0=w, rtol=pcg_rtol, maxit=maxit)
        w = res.x
        its.append(res.iters)
        u = w / np.linalg.norm(w)
        lam.append(float(np.vdot(u, stencil_apply(plan, u, V2, 0.0))))
    return InvIterResult(u=u, lam=lam, pcg_iters=its)


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
