"""Python binding of libts.so, the MI355X separable tensor-product solver.

Thin marshalling over the C ABI declared in ``include/ts.h``: every function
has the name of the C entry point it calls and does no arithmetic of its own.
PyTorch provides device memory (tensors) and streams only.  There is no CPU
fallback: importing a function whose library is missing raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TS_LIBRARY selects another build of the library (for instance a copy whose
# host code is compiled with the address and undefined-behaviour sanitizers)
LIB_PATH = os.environ.get("TS_LIBRARY") or os.path.join(_HERE, "libts.so")

TS_OK, TS_ERR_INVALID, TS_ERR_NOT_SPD, TS_ERR_NOMEM, TS_ERR_DEVICE = 0, 1, 2, 3, 4
TS_ERR_NOCONV, TS_ERR_NONFINITE, TS_ERR_BUSY, TS_ERR_BREAKDOWN = 5, 6, 7, 8
STATUS_NAMES = {0: "TS_OK", 1: "TS_ERR_INVALID", 2: "TS_ERR_NOT_SPD", 3: "TS_ERR_NOMEM",
                4: "TS_ERR_DEVICE", 5: "TS_ERR_NOCONV", 6: "TS_ERR_NONFINITE", 7: "TS_ERR_BUSY",
                8: "TS_ERR_BREAKDOWN"}
TS_F64, TS_F32, TS_C128, TS_C64 = 0, 1, 2, 3
TS_PREC_FP64, TS_PREC_FP32, TS_PREC_BF16 = 0, 1, 2
TS_STRANG_BAB, TS_STRANG_ABA, TS_YOSHIDA_BAB, TS_YOSHIDA_ABA = 0, 1, 2, 3

PREC = {"fp64": TS_PREC_FP64, "fp32": TS_PREC_FP32, "bf16": TS_PREC_BF16}
SCHEME = {"strang_bab": TS_STRANG_BAB, "strang_aba": TS_STRANG_ABA,
          "yoshida_bab": TS_YOSHIDA_BAB, "yoshida_aba": TS_YOSHIDA_ABA}


class TSError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        self.code = code
        self.status = STATUS_NAMES.get(code, str(code))
        super().__init__("%s: %s (%s)" % (where, self.status, msg))


_lib = None
_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)


def lib():
    """Load libts.so (built by paper_2605_20491_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libts.so is not built (%s); run paper_2605_20491_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "ts_setup": [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_double,
                         ctypes.POINTER(_dp), ctypes.c_double, ctypes.POINTER(_vp)],
            "ts_destroy": [_vp],
            "ts_set_fold": [_vp, ctypes.c_int],
            "ts_set_bf16_tile": [_vp, ctypes.c_int],
            "ts_mode_pass": [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp],
            "ts_fold_butterfly": [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp],
            "ts_fold_axes": [_vp, _ip],
            "ts_setup_sem": [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_double,
                             ctypes.POINTER(_dp), ctypes.c_double, ctypes.POINTER(_vp)],
            "ts_sem_nodes": [ctypes.c_int, ctypes.c_int64, ctypes.c_double, _dp],
            "ts_sem_axis_eig": [ctypes.c_int, ctypes.c_int64, ctypes.c_double, _dp, _dp, _dp, _dp],
            "ts_setup_general": [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_dp),
                                 ctypes.POINTER(_dp), ctypes.POINTER(_dp), ctypes.POINTER(_dp), ctypes.c_double,
                                 ctypes.POINTER(_vp)],
            "ts_hermite_axis": [ctypes.c_int64, _dp, _dp, _dp],
            "ts_mass": [_vp, ctypes.c_int, _dp],
            "ts_apply_inverse": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp],
            "ts_apply_inverse_shift": [_vp, ctypes.c_double, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp],
            "ts_apply_inverse_noalloc": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp],
            "ts_apply_exp": [_vp, ctypes.c_double, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp],
            "ts_solve_refined": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _ip, _dp, _vp],
            "ts_pcg_solve": [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _ip, _dp, _vp],
            "ts_inverse_iteration": [_vp, _vp, ctypes.c_double, _vp, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, _dp, _ip, _vp],
            "ts_split_step": [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, _vp],
            "ts_qhop_step": [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, _vp],
            "ts_gauss_legendre": [ctypes.c_int, _dp, _dp],
            "ts_operator_apply": [_vp, _vp, ctypes.c_double, _vp, _vp, _vp],
            "ts_interpolate": [_vp, _vp, _vp, _vp, _vp],
            "ts_separable_ground_state": [_vp, _vp, _vp],
            "ts_multilevel_inverse_iteration": [ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _dp, _vp,
                                                ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                ctypes.c_int, _dp, _ip, _ip, _vp],
            "ts_gpe_h1_flow": [_vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp, ctypes.c_int,
                               ctypes.c_double, _dp, _ip, _dp, _dp, _vp],
            "ts_gpe_au_flow": [_vp, _vp, ctypes.c_double, ctypes.c_double, _vp, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _ip, _ip, _dp, _dp, _vp],
            "ts_eigvals": [_vp, ctypes.c_int, _dp],
            "ts_eigvecs": [_vp, ctypes.c_int, _dp],
            "ts_workspace_bytes": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
            "ts_tridiag_eig": [ctypes.c_int64, _dp, _dp, _dp, _dp],
            "ts_sym_eig": [ctypes.c_int64, _dp, _dp, _dp],
            "ts_tridiag_eig_even_odd": [ctypes.c_int64, _dp, _dp, _dp, _dp],
            "ts_bf16_round": [ctypes.c_int64, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint16)],
        }
        for name, argt in sig.items():
            fn = getattr(L, name)
            fn.argtypes = argt
            fn.restype = ctypes.c_int
        L.ts_last_error.argtypes = []
        L.ts_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def ts_last_error() -> str:
    return lib().ts_last_error().decode()


def _check(rc: int, where: str):
    if rc != TS_OK:
        raise TSError(rc, where, ts_last_error())


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


# ---------------------------------------------------------------- torch glue --

def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


_DTYPE_CODES = None


def _dtype_code(t) -> int:
    global _DTYPE_CODES
    torch = _torch()
    if _DTYPE_CODES is None:
        _DTYPE_CODES = {torch.float64: TS_F64, torch.float32: TS_F32,
                        torch.complex128: TS_C128, torch.complex64: TS_C64}
    if t.dtype not in _DTYPE_CODES:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return _DTYPE_CODES[t.dtype]


def _dev(t, plan, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if plan is not None and t.numel() != plan.N:
        raise ValueError("%s has %d elements, the grid has %d" % (name, t.numel(), plan.N))
    return _vp(t.data_ptr())


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


class Plan:
    """Owner of a ts_plan*; released by ts_destroy when collected."""

    def __init__(self, handle, shape, L, sigma):
        self._h = handle
        self.shape = tuple(int(s) for s in shape)
        self.d = len(self.shape)
        self.N = int(np.prod(self.shape))
        self.L = float(L)
        self.sigma = float(sigma)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.ts_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ entries --

def ts_setup(shape, L: float, f_list, sigma: float) -> Plan:
    d = len(shape)
    n = (ctypes.c_int64 * d)(*[int(s) for s in shape])
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in f_list]
    if len(fs) != d or any(f.shape != (int(s),) for f, s in zip(fs, shape)):
        raise ValueError("f_list must hold one array of n_k samples per axis")
    fp = (_dp * d)(*[_dptr(f) for f in fs])
    h = _vp()
    _check(lib().ts_setup(d, n, float(L), fp, float(sigma), ctypes.byref(h)), "ts_setup")
    return Plan(h, shape, L, sigma)


def ts_setup_sem(k: int, cells, L: float, f_list, sigma: float) -> Plan:
    """Q^k spectral-element plan; f_list[a] holds f_a at ts_sem_nodes(k, cells[a], L)."""
    d = len(cells)
    shape = tuple(int(k) * int(c) - 1 for c in cells)
    cc = (ctypes.c_int64 * d)(*[int(c) for c in cells])
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in f_list]
    if len(fs) != d or any(f.shape != (n,) for f, n in zip(fs, shape)):
        raise ValueError("f_list must hold one array of k * cells[a] - 1 samples per axis")
    fp = (_dp * d)(*[_dptr(f) for f in fs])
    h = _vp()
    _check(lib().ts_setup_sem(d, cc, int(k), float(L), fp, float(sigma), ctypes.byref(h)), "ts_setup_sem")
    return Plan(h, shape, L, sigma)


def ts_setup_general(K_list, m_list, f_list, sigma: float, x_list=None) -> Plan:
    """Plan of arbitrary per-axis operators: K_list[a] (n x n) self-adjoint in
    the weights m_list[a] (None: unit weights), f_list[a] the potential at the
    nodes x_list[a] (optional).  The plan has no interval: its L is 0."""
    d = len(K_list)
    Ks = [np.ascontiguousarray(K, dtype=np.float64) for K in K_list]
    shape = tuple(K.shape[0] for K in Ks)
    if any(K.ndim != 2 or K.shape[0] != K.shape[1] for K in Ks):
        raise ValueError("every K must be square")
    ms = [None if m is None else np.ascontiguousarray(m, dtype=np.float64) for m in (m_list or [None] * d)]
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in f_list]
    xs = None if x_list is None else [np.ascontiguousarray(x, dtype=np.float64) for x in x_list]
    for a, n in enumerate(shape):
        if fs[a].shape != (n,) or (ms[a] is not None and ms[a].shape != (n,)) or (xs is not None and xs[a].shape != (n,)):
            raise ValueError("axis %d: f, m and x must hold n = %d samples" % (a, n))
    nn = (ctypes.c_int64 * d)(*shape)
    Kp = (_dp * d)(*[_dptr(K) for K in Ks])
    mp = (_dp * d)(*[_dptr(m) if m is not None else None for m in ms])
    fp = (_dp * d)(*[_dptr(f) for f in fs])
    xp = None if xs is None else (_dp * d)(*[_dptr(x) for x in xs])
    h = _vp()
    _check(lib().ts_setup_general(d, nn, Kp, mp, xp, fp, float(sigma), ctypes.byref(h)), "ts_setup_general")
    return Plan(h, shape, 0.0, sigma)


def ts_hermite_axis(n: int):
    """(x, m, K) of n-point Hermite spectral collocation (host)."""
    n = int(n)
    x, m, K = np.empty(n), np.empty(n), np.empty((n, n))
    _check(lib().ts_hermite_axis(n, _dptr(x), _dptr(m), _dptr(K)), "ts_hermite_axis")
    return x, m, K


def ts_sem_nodes(k: int, cells: int, L: float) -> np.ndarray:
    x = np.empty(max(int(k) * int(cells) - 1, 1))
    _check(lib().ts_sem_nodes(int(k), int(cells), float(L), _dptr(x)), "ts_sem_nodes")
    return x



def ts_sem_axis_eig(k: int, cells: int, L: float, f):
    """Host eigenpairs of one Q^k SEM axis in the symmetric form
    M^{-1/2} S M^{-1/2} + diag(f), as ts_setup_sem computes them: (lam, Q, m)."""
    n = int(k) * int(cells) - 1
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.shape != (n,):
        raise ValueError("f must hold k * cells - 1 samples")
    lam = np.empty(n)
    Q = np.empty((n, n))
    m = np.empty(n)
    _check(lib().ts_sem_axis_eig(int(k), int(cells), float(L), _dptr(f), _dptr(lam), _dptr(Q), _dptr(m)),
           "ts_sem_axis_eig")
    return lam, Q, m

def ts_mass(plan: Plan, axis: int) -> np.ndarray:
    out = np.empty(plan.shape[axis])
    _check(lib().ts_mass(plan.handle, int(axis), _dptr(out)), "ts_mass")
    return out


def ts_set_fold(plan: Plan, enable):
    """enable: False / 0 off, True / 1 on, 2 on with the BF16 backward passes
    over full extents."""
    _check(lib().ts_set_fold(plan.handle, int(enable)), "ts_set_fold")


def ts_set_bf16_tile(plan: Plan, tile: int):
    _check(lib().ts_set_bf16_tile(plan.handle, int(tile)), "ts_set_bf16_tile")


def ts_mode_pass(plan: Plan, axis: int, forward: bool, x, out=None, prec="fp64", stream=None, folded=False):
    """folded=True: forward on input already folded along the axis (mode 2),
    backward without the butterfly (mode 3)."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    mode = (2 if forward else 3) if folded else (1 if forward else 0)
    _check(lib().ts_mode_pass(plan.handle, int(axis), mode, _dev(x, plan, "x"), _dev(out, plan, "out"),
                              _dtype_code(x), _prec(prec), _stream(stream)), "ts_mode_pass")
    return out


def ts_fold_butterfly(plan: Plan, axes: int, x, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty_like(x)
    _check(lib().ts_fold_butterfly(plan.handle, int(axes), _dev(x, plan, "x"), _dev(out, plan, "out"),
                                   _dtype_code(x), _stream(stream)), "ts_fold_butterfly")
    return out


def ts_fold_axes(plan: Plan) -> int:
    m = ctypes.c_int(0)
    _check(lib().ts_fold_axes(plan.handle, ctypes.byref(m)), "ts_fold_axes")
    return m.value


def ts_destroy(plan: Plan):
    plan.close()


def ts_apply_inverse(plan: Plan, b, u=None, prec="fp64", stream=None):
    torch = _torch()
    if u is None:
        u = torch.empty_like(b)
    _check(lib().ts_apply_inverse(plan.handle, _dev(b, plan, "b"), _dev(u, plan, "u"), _dtype_code(b),
                                  _prec(prec), _stream(stream)), "ts_apply_inverse")
    return u


def ts_apply_inverse_noalloc(plan: Plan, b, u, prec="fp64", stream=None):
    """ts_apply_inverse with the library's static scratch array (no device
    allocation inside the call); u must be given."""
    _check(lib().ts_apply_inverse_noalloc(plan.handle, _dev(b, plan, "b"), _dev(u, plan, "u"), _dtype_code(b),
                                          _prec(prec), _stream(stream)), "ts_apply_inverse_noalloc")
    return u


def ts_apply_inverse_shift(plan: Plan, s: float, b, u=None, prec="fp64", stream=None):
    torch = _torch()
    if u is None:
        u = torch.empty_like(b)
    _check(lib().ts_apply_inverse_shift(plan.handle, float(s), _dev(b, plan, "b"), _dev(u, plan, "u"),
                                        _dtype_code(b), _prec(prec), _stream(stream)),
           "ts_apply_inverse_shift")
    return u


def ts_apply_exp(plan: Plan, tau: float, psi, out=None, prec="fp64", stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty_like(psi)
    _check(lib().ts_apply_exp(plan.handle, float(tau), _dev(psi, plan, "psi"), _dev(out, plan, "out"),
                              _dtype_code(psi), _prec(prec), _stream(stream)), "ts_apply_exp")
    return out


def ts_solve_refined(plan: Plan, f, u=None, inner="fp32", rtol=1e-10, maxit=50, stream=None):
    torch = _torch()
    if u is None:
        u = torch.empty_like(f)
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    rc = lib().ts_solve_refined(plan.handle, _dev(f, plan, "f"), _dev(u, plan, "u"), _prec(inner),
                                float(rtol), int(maxit), ctypes.byref(it), ctypes.byref(rr),
                                _stream(stream))
    _check(rc, "ts_solve_refined")
    return u, it.value, rr.value


def ts_pcg_solve(plan: Plan, V2, f, u=None, rtol=1e-10, maxit=500, precond="fp64", stream=None,
                 raise_on_noconv=True):
    torch = _torch()
    if u is None:
        u = torch.zeros_like(f)
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    rc = lib().ts_pcg_solve(plan.handle, _dev(V2, plan, "V2"), _dev(f, plan, "f"), _dev(u, plan, "u"),
                            float(rtol), int(maxit), _prec(precond), ctypes.byref(it), ctypes.byref(rr),
                            _stream(stream))
    if rc == TS_ERR_NOCONV and not raise_on_noconv:
        return u, it.value, rr.value, rc
    _check(rc, "ts_pcg_solve")
    return u, it.value, rr.value, rc


def ts_inverse_iteration(plan: Plan, V2, shift: float, u, steps=20, pcg_rtol=1e-10, maxit=500,
                         precond="fp64", stream=None):
    lam = np.zeros(steps + 1)
    its = (ctypes.c_int * steps)()
    rc = lib().ts_inverse_iteration(plan.handle, _dev(V2, plan, "V2"), float(shift), _dev(u, plan, "u"),
                                    int(steps), float(pcg_rtol), int(maxit), _prec(precond), _dptr(lam),
                                    its, _stream(stream))
    _check(rc, "ts_inverse_iteration")
    return u, lam, list(its)


def ts_split_step(plan: Plan, V2, psi, dt: float, nsteps: int, scheme="strang_bab", prec="fp64",
                  stream=None):
    sch = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    _check(lib().ts_split_step(plan.handle, _dev(V2, plan, "V2"), _dev(psi, plan, "psi"), float(dt),
                               int(nsteps), sch, _dtype_code(psi), _prec(prec), _stream(stream)),
           "ts_split_step")
    return psi


def ts_qhop_step(plan: Plan, V2, psi, dt: float, nsteps: int, M: int, magnus2: bool = False, prec="fp64",
                 stream=None):
    _check(lib().ts_qhop_step(plan.handle, _dev(V2, plan, "V2"), _dev(psi, plan, "psi"), float(dt), int(nsteps),
                              int(M), int(bool(magnus2)), _dtype_code(psi), _prec(prec), _stream(stream)),
           "ts_qhop_step")
    return psi


def ts_gauss_legendre(M: int):
    nodes, weights = np.empty(max(int(M), 1)), np.empty(max(int(M), 1))
    _check(lib().ts_gauss_legendre(int(M), _dptr(nodes), _dptr(weights)), "ts_gauss_legendre")
    return nodes, weights


def ts_interpolate(coarse: Plan, fine: Plan, uc, uf=None, stream=None):
    torch = _torch()
    if uf is None:
        uf = torch.empty(fine.shape, dtype=torch.float64, device=uc.device)
    _check(lib().ts_interpolate(coarse.handle, fine.handle, _dev(uc, coarse, "uc"), _dev(uf, fine, "uf"),
                                _stream(stream)), "ts_interpolate")
    return uf


def ts_separable_ground_state(plan: Plan, u=None, stream=None):
    torch = _torch()
    if u is None:
        u = torch.empty(plan.shape, dtype=torch.float64, device="cuda")
    _check(lib().ts_separable_ground_state(plan.handle, _dev(u, plan, "u"), _stream(stream)),
           "ts_separable_ground_state")
    return u


def ts_multilevel_inverse_iteration(plans, V2s, shifts, u=None, max_steps=100, lam_tol=1e-13, pcg_rtol=1e-12,
                                    pcg_maxit=500, precond="fp64", stream=None):
    """Returns (u on the finest grid, lambda per level, steps per level, PCG iterations per level)."""
    torch = _torch()
    L = len(plans)
    if u is None:
        u = torch.empty(plans[-1].shape, dtype=torch.float64, device="cuda")
    ph = (_vp * L)(*[p.handle for p in plans])
    vh = (_vp * L)(*[_dev(v, p, "V2") for v, p in zip(V2s, plans)])
    sh = np.ascontiguousarray(shifts, dtype=np.float64)
    lam = np.zeros(L)
    steps = (ctypes.c_int * L)()
    its = (ctypes.c_int * L)()
    _check(lib().ts_multilevel_inverse_iteration(L, ph, vh, _dptr(sh), _dev(u, plans[-1], "u"), int(max_steps),
                                                 float(lam_tol), float(pcg_rtol), int(pcg_maxit), _prec(precond),
                                                 _dptr(lam), steps, its, _stream(stream)),
           "ts_multilevel_inverse_iteration")
    return u, lam, list(steps), list(its)


class GpeResult:
    def __init__(self, u, energy, eigenvalue, iters, history, linear_iters=None, status=0):
        self.u, self.energy, self.eigenvalue, self.iters = u, energy, eigenvalue, iters
        self.history, self.linear_iters, self.status = history, linear_iters, status


def ts_gpe_h1_flow(plan: Plan, V, beta: float, u, alpha: float = 20.0, tau: float = 0.1, maxit: int = 1000,
                   tol: float = 1e-12, stream=None, raise_on_noconv=True) -> GpeResult:
    hist = np.zeros(int(maxit) + 1)
    it, lam, E = ctypes.c_int(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().ts_gpe_h1_flow(plan.handle, _dev(V, plan, "V"), float(beta), float(alpha), float(tau),
                              _dev(u, plan, "u"), int(maxit), float(tol), _dptr(hist), ctypes.byref(it),
                              ctypes.byref(lam), ctypes.byref(E), _stream(stream))
    if not (rc == TS_ERR_NOCONV and not raise_on_noconv):
        _check(rc, "ts_gpe_h1_flow")
    return GpeResult(u, E.value, lam.value, it.value, hist[: it.value + 1].copy(), status=rc)


def ts_gpe_au_flow(plan: Plan, V2, beta: float, u, tau: float = 1.0, maxit: int = 500, tol: float = 1e-12,
                   pcg_rtol: float = 1e-12, pcg_maxit: int = 500, precond="fp64", stream=None,
                   raise_on_noconv=True) -> GpeResult:
    hist = np.zeros(int(maxit) + 1)
    it, lin = ctypes.c_int(0), ctypes.c_int(0)
    lam, E = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().ts_gpe_au_flow(plan.handle, _dev(V2, plan, "V2"), float(beta), float(tau), _dev(u, plan, "u"),
                              int(maxit), float(tol), float(pcg_rtol), int(pcg_maxit), _prec(precond),
                              _dptr(hist), ctypes.byref(it), ctypes.byref(lin), ctypes.byref(lam),
                              ctypes.byref(E), _stream(stream))
    if not (rc == TS_ERR_NOCONV and not raise_on_noconv):
        _check(rc, "ts_gpe_au_flow")
    return GpeResult(u, E.value, lam.value, it.value, hist[: it.value + 1].copy(), lin.value, rc)


def ts_operator_apply(plan: Plan, V2, s: float, u, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty_like(u)
    _check(lib().ts_operator_apply(plan.handle, _dev(V2, plan, "V2"), float(s), _dev(u, plan, "u"),
                                   _dev(out, plan, "out"), _stream(stream)), "ts_operator_apply")
    return out


def ts_eigvals(plan: Plan, axis: int) -> np.ndarray:
    out = np.empty(plan.shape[axis])
    _check(lib().ts_eigvals(plan.handle, int(axis), _dptr(out)), "ts_eigvals")
    return out


def ts_eigvecs(plan: Plan, axis: int) -> np.ndarray:
    n = plan.shape[axis]
    out = np.empty((n, n))
    _check(lib().ts_eigvecs(plan.handle, int(axis), _dptr(out)), "ts_eigvecs")
    return out


def ts_workspace_bytes(plan: Plan, dtype: int) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().ts_workspace_bytes(plan.handle, int(dtype), ctypes.byref(b)), "ts_workspace_bytes")
    return b.value


def ts_tridiag_eig(diag: np.ndarray, off: np.ndarray):
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.float64)
    n = diag.size
    lam = np.empty(n)
    Q = np.empty((n, n))
    offp = _dptr(off) if off.size else _dptr(np.zeros(1))
    _check(lib().ts_tridiag_eig(n, _dptr(diag), offp, _dptr(lam), _dptr(Q)), "ts_tridiag_eig")
    return lam, Q


def ts_tridiag_eig_even_odd(diag: np.ndarray, off: np.ndarray):
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.float64)
    n = diag.size
    lam = np.empty(n)
    Q = np.empty((n, n))
    _check(lib().ts_tridiag_eig_even_odd(n, _dptr(diag), _dptr(off), _dptr(lam), _dptr(Q)), "ts_tridiag_eig_even_odd")
    return lam, Q


def ts_sym_eig(A: np.ndarray):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    lam = np.empty(n)
    Q = np.empty((n, n))
    _check(lib().ts_sym_eig(n, _dptr(A), _dptr(lam), _dptr(Q)), "ts_sym_eig")
    return lam, Q


def ts_bf16_round(x: np.ndarray, route: int) -> np.ndarray:
    """BF16 bit patterns (uint16) of x as the library rounds them: route 0 =
    factor copies (FP64 rounded once), route 1 = data (FP64 -> FP32 -> BF16)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.empty(x.size, dtype=np.uint16)
    _check(lib().ts_bf16_round(x.size, _dptr(x), int(route), y.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))),
           "ts_bf16_round")
    return y


# ------------------------------------------------------------------ serving --

TS_REQ_INVERSE, TS_REQ_EXP = 0, 1


class TsRequest(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("d", ctypes.c_int), ("n", ctypes.c_int64 * 12), ("L", ctypes.c_double),
                ("f", ctypes.c_void_p * 12), ("sigma", ctypes.c_double), ("dtype", ctypes.c_int),
                ("prec", ctypes.c_int), ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("V2", ctypes.c_void_p), ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("rtol", ctypes.c_double), ("maxit", ctypes.c_int), ("tag", ctypes.c_uint64)]


class TsResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("relres", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("tag", ctypes.c_uint64)]


def _serve_lib():
    L = lib()
    if not hasattr(L, "_serve_ready"):
        L.ts_serve_create.argtypes = [ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(_vp)]
        L.ts_serve_submit.argtypes = [_vp, ctypes.POINTER(TsRequest), ctypes.POINTER(ctypes.c_uint64)]
        L.ts_serve_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(TsResult)]
        L.ts_serve_drain.argtypes = [_vp]
        L.ts_serve_destroy.argtypes = [_vp]
        L.ts_serve_clock.argtypes = [_vp]
        L.ts_serve_clock.restype = ctypes.c_double
        for name in ("ts_serve_create", "ts_serve_submit", "ts_serve_poll", "ts_serve_drain", "ts_serve_destroy"):
            getattr(L, name).restype = ctypes.c_int
        L._serve_ready = True
    return L


class Server:
    """ts_serve_*: requests are admitted by memory and run concurrently.

    Device tensors passed to submit() are kept referenced here until the
    request has finished (the library reads and writes them asynchronously).
    """

    def __init__(self, budget_bytes: int, n_streams: int = 4, max_active: int = 0, plan_reserve: int = 0):
        L = _serve_lib()
        h = _vp()
        _check(L.ts_serve_create(int(budget_bytes), int(plan_reserve), int(n_streams), int(max_active),
                                 ctypes.byref(h)), "ts_serve_create")
        self._h = h
        self._keep = {}

    def clock(self) -> float:
        return _serve_lib().ts_serve_clock(self._h)

    def submit(self, kind, shape, L, f_list, sigma, inp, out, prec="fp64", V2=None, tau=0.0, dt=0.0,
               rtol=1e-10, maxit=500, tag=0) -> int:
        r = TsRequest()
        r.kind = int(kind)
        r.d = len(shape)
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in f_list]
        for k, nk in enumerate(shape):
            r.n[k] = int(nk)
            r.f[k] = fs[k].ctypes.data
        r.L, r.sigma = float(L), float(sigma)
        r.dtype = _dtype_code(inp)
        r.prec = _prec(prec)
        r.in_ = inp.data_ptr()
        r.out = out.data_ptr()
        r.V2 = V2.data_ptr() if V2 is not None else None
        r.tau, r.dt, r.rtol, r.maxit, r.tag = float(tau), float(dt), float(rtol), int(maxit), int(tag)
        t = ctypes.c_uint64(0)
        _check(_serve_lib().ts_serve_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "ts_serve_submit")
        self._keep[t.value] = (inp, out, V2)
        return t.value

    def poll(self, ticket: int):
        done = ctypes.c_int(0)
        res = TsResult()
        _check(_serve_lib().ts_serve_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(res)),
               "ts_serve_poll")
        if done.value:
            self._keep.pop(ticket, None)
            return res
        return None

    def drain(self):
        _check(_serve_lib().ts_serve_drain(self._h), "ts_serve_drain")

    def close(self):
        if self._h is not None:
            _serve_lib().ts_serve_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ts_serve_create(budget_bytes, n_streams=4, max_active=0, plan_reserve=0) -> Server:
    return Server(budget_bytes, n_streams, max_active, plan_reserve)
