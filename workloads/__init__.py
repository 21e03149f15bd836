"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the solver: it only places the grid nodes,
samples potential functions at them and draws seeded random data.  Both the
oracle and the GPU library receive exactly the arrays produced here.

Grid: n interior nodes of [-L, L], x_j = -L + j h, h = 2L/(n+1), j = 1..n
(homogeneous Dirichlet; the paper's n interior grid points per direction).
Axis order is C order: axis d-1 is the fastest index (the paper's x).

Workload recipes (where the paper leaves a detail open, the choice is stated here):
* ``rhs_normal``: i.i.d. N(0, 1) right-hand side (numpy PCG64 from the seed).
* ``gaussian_wavepacket``: psi0(x) = exp(-|x - x0|^2 / (2 s^2) + i k0 . x),
  x0 ~ U[-2, 2]^d, s ~ U(0.5, 1.5), k0 ~ U[-2, 2]^d, normalised to unit 2-norm.
  It is a product of per-axis factors, returned as such by ``wavepacket_factors``.
* ``gaussian_bumps``: V2(x) = sum_b a_b exp(-|x - c_b|^2 / (2 w_b^2)), per bump
  a ~ U(-5, 5), w ~ U(0.5, 2), c ~ U[-4, 4]^d, drawn in that order.
* ``pairwise_v2``: V2(x) = sum_{i<j} 0.5 / (1 + (x_i - x_j)^2) over all axis pairs.
"""
from __future__ import annotations

import math

import numpy as np


def grid_nodes(n: int, L: float) -> np.ndarray:
    h = 2.0 * L / (n + 1)
    return -L + h * np.arange(1, n + 1, dtype=np.float64)


# ---- separable potential samples f_k(x_j) ------------------------------------
# Each sampler evaluates at the uniform FD nodes of (n, L), or at the nodes x
# passed in (for instance the Gauss-Lobatto nodes of a spectral-element grid).

def _nodes(n, L, x):
    return grid_nodes(n, L) if x is None else np.asarray(x, dtype=np.float64)


def f_harmonic(n: int, L: float, coef: float = 1.0, x=None) -> np.ndarray:
    """f(x) = coef * x^2."""
    x = _nodes(n, L, x)
    return coef * x * x


def f_harmonic_cos(n: int, L: float, x=None) -> np.ndarray:
    """f(x) = x^2 + 0.5 cos(2x) (the 1e9-DoF workload's per-axis potential)."""
    x = _nodes(n, L, x)
    return x * x + 0.5 * np.cos(2.0 * x)


def f_separable_v1(n: int, L: float, x=None) -> np.ndarray:
    """f(x) = x^2 + 100 sin^2(pi x / 4): per-axis term of eq. (separable_V1)."""
    x = _nodes(n, L, x)
    return x * x + 100.0 * np.sin(np.pi * x / 4.0) ** 2


def f_test_potential(n: int, L: float, c: float, x=None) -> np.ndarray:
    """f(x) = 1600 sin^2(pi x / 4) + c x^2: one axis of eq. (test_potential)."""
    x = _nodes(n, L, x)
    return 1600.0 * np.sin(np.pi * x / 4.0) ** 2 + c * x * x


def rational_sine(c: float, t: np.ndarray):
    """(g, g'') for g(t) = sin(c (t + 1)) / (1 + t^2): one factor of the exact
    solution of the Hermite test problem on R^3 (Appendix app:hermite)."""
    t = np.asarray(t, dtype=np.float64)
    s, sp, spp = np.sin(c * (t + 1)), c * np.cos(c * (t + 1)), -c * c * np.sin(c * (t + 1))
    q, qp = 1.0 + t * t, 2.0 * t
    g = s / q
    gpp = spp / q - 2.0 * sp * qp / q**2 - 2.0 * s / q**2 + 2.0 * s * qp**2 / q**3
    return g, gpp


# ---- random data -------------------------------------------------------------

def rhs_normal(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=tuple(shape))


def wavepacket_factors(shape, L: float, seed: int):
    """Per-axis complex factors g_k with psi0 = g_0 (x) g_1 (x) ... (outer product).

    The overall normalisation is folded into the factors so that the outer
    product has unit 2-norm.
    """
    d = len(shape)
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-2.0, 2.0, size=d)
    s = rng.uniform(0.5, 1.5)
    k0 = rng.uniform(-2.0, 2.0, size=d)
    facs = []
    for k in range(d):
        x = grid_nodes(shape[k], L)
        g = np.exp(-((x - x0[k]) ** 2) / (2.0 * s * s) + 1j * k0[k] * x)
        facs.append(g / np.linalg.norm(g))
    return facs


def outer(factors) -> np.ndarray:
    out = np.ones((), dtype=np.result_type(*factors))
    for g in factors:
        out = np.multiply.outer(out, g)
    return np.ascontiguousarray(out)


def gaussian_wavepacket(shape, L: float, seed: int) -> np.ndarray:
    return outer(wavepacket_factors(shape, L, seed))


def bump_params(d: int, nbumps: int, seed: int):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nbumps):
        a = rng.uniform(-5.0, 5.0)
        w = rng.uniform(0.5, 2.0)
        c = rng.uniform(-4.0, 4.0, size=d)
        out.append((a, w, c))
    return out


def gaussian_bumps(shape, L: float, nbumps: int, seed: int) -> np.ndarray:
    d = len(shape)
    params = bump_params(d, nbumps, seed)
    V = np.zeros(tuple(shape))
    axes = [grid_nodes(n, L) for n in shape]
    for a, w, c in params:
        # exp(-|x-c|^2/(2w^2)) = prod_k exp(-(x_k-c_k)^2/(2w^2))
        fac = [np.exp(-((axes[k] - c[k]) ** 2) / (2.0 * w * w)) for k in range(d)]
        V += a * outer(fac)
    return V


def pairwise_v2(shape, L: float) -> np.ndarray:
    d = len(shape)
    axes = [grid_nodes(n, L) for n in shape]
    V = np.zeros(tuple(shape))
    for i in range(d):
        for j in range(i + 1, d):
            xi = axes[i].reshape([-1 if k == i else 1 for k in range(d)])
            xj = axes[j].reshape([-1 if k == j else 1 for k in range(d)])
            V += 0.5 / (1.0 + (xi - xj) ** 2)
    return V


def complex_normal(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=tuple(shape)) + 1j * rng.standard_normal(size=tuple(shape))




__all__ = [n for n in dir() if not n.startswith("_") and n not in ("math", "np", "annotations")]


def lowest_separable_modes(lams, count: int):
    """Multi-indices of the `count` lowest separable eigenfunctions.

    Sorted by (eigenvalue sum rounded to 1e-9 relative, multi-index in
    lexicographic order), which breaks the degeneracies of identical axes
    deterministically.  lams[k]: ascending eigenvalues of axis k.
    """
    import itertools
    d = len(lams)
    cand = []
    depth = 3
    for idx in itertools.product(*[range(min(depth, len(l))) for l in lams]):
        s = sum(float(lams[k][idx[k]]) for k in range(d))
        cand.append((s, idx))
    top = max(abs(c[0]) for c in cand) or 1.0
    cand.sort(key=lambda c: (round(c[0] / (1e-9 * top)), c[1]))
    return [c[1] for c in cand[:count]]


def superposition_terms(Qs, lams, count: int, seed: int):
    """Seeded superposition of the `count` lowest separable eigenfunctions.

    Returns [(c_m, multi_index_m)] with c_m ~ CN(0,1) normalised so that
    sum |c_m|^2 = 1 (the eigenfunctions are orthonormal); Qs[k][:, j] is the
    j-th eigenvector of axis k.
    """
    modes = lowest_separable_modes(lams, count)
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(count) + 1j * rng.standard_normal(count)
    c /= np.linalg.norm(c)
    return list(zip(c, modes))


def superposition_grid(Qs, terms) -> np.ndarray:
    out = None
    for cm, idx in terms:
        t = cm * outer([Qs[k][:, j] for k, j in enumerate(idx)])
        out = t if out is None else out + t
    return out


# The serving mix: seeded Poisson arrivals over the request classes.
SERVE_SHAPES = [(2048, 2048), (128, 128, 128), (256, 256, 256), (512, 512, 512), (64,) * 4, (16,) * 6]
SERVE_KINDS = ["inverse_fp64", "inverse_mixed", "exp_c64"]


def serve_stream(seed: int, count: int, rate: float):
    """Requests with Poisson arrival times at `rate` per second; each draws a
    shape and a kind uniformly, V2 present with probability 1/2 and
    tau ~ U[1e-3, 1e-1] (used by the propagator kinds)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        reqs.append({"t": t, "shape": SERVE_SHAPES[rng.integers(len(SERVE_SHAPES))],
                     "kind": SERVE_KINDS[rng.integers(len(SERVE_KINDS))], "v2": bool(rng.integers(2)),
                     "tau": float(rng.uniform(1e-3, 1e-1))})
    return reqs
