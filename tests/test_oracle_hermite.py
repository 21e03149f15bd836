"""Pins of the oracle's generic per-axis operators and of Hermite spectral
collocation (Appendix app:hermite), CPU only.

* The nodes are the Gauss-Hermite nodes (numpy's hermgauss), and the weights
  m are its weights times e^{x^2} (the Gauss rule of the Hermite functions).
* D differentiates every Hermite function psi_0 .. psi_{n-1} exactly at the
  nodes (closed-form derivative psi_k' = sqrt(k/2) psi_{k-1} - sqrt((k+1)/2)
  psi_{k+1}, and psi_n vanishes at the nodes).
* K + diag(x^2) has the harmonic-oscillator eigenvalues 1, 3, ..., 2n - 3
  exactly (n - 1 of its n eigenvalues).
* A generic plan built from the FD or the Q^k SEM operator reproduces the FD
  and SEM plans.
* Applies, operator and PCG of a generic Hermite plan against the dense
  Kronecker-sum matrix and LU / expm.
* Table tab:hermite_accuracy at n = 199: both printed errors.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("n", [1, 2, 7, 40, 120])
def test_nodes_and_weights_are_gauss_hermite(n):
    x, m, K = oracle.hermite_axis(n)
    xr, wr = np.polynomial.hermite.hermgauss(n)
    assert np.max(np.abs(x - xr)) <= 1e-12 * max(1.0, np.abs(xr).max())
    assert np.max(np.abs(m - wr * np.exp(xr * xr)) / m) <= 1e-10
    # diag(m) K symmetric: K self-adjoint in the weights
    MK = m[:, None] * K
    assert np.max(np.abs(MK - MK.T)) <= 1e-11 * np.abs(MK).max() if n > 1 else True


def _deriv(psi, k):
    """psi_k' = sqrt(k/2) psi_{k-1} - sqrt((k+1)/2) psi_{k+1}, as coefficients."""
    out = {}
    if k > 0:
        out[k - 1] = np.sqrt(k / 2.0)
    out[k + 1] = -np.sqrt((k + 1) / 2.0)
    return out


@pytest.mark.parametrize("n", [5, 16, 60])
def test_differentiation_exact_on_hermite_functions(n):
    """-K psi_k = psi_k'' at the nodes for k <= n - 2 (psi_k'' lies in the span
    of psi_{k-2} .. psi_{k+2}, and psi_n vanishes at the nodes)."""
    x, m, K = oracle.hermite_axis(n)
    psi = oracle.hermite_functions(n + 1, x)
    assert np.max(np.abs(psi[n])) <= 1e-10
    for k in range(n - 1):
        d2 = np.zeros_like(x)
        for j, c in _deriv(psi, k).items():
            for i, c2 in _deriv(psi, j).items():
                d2 = d2 + c * c2 * psi[i]
        assert np.max(np.abs(-K @ psi[k] - d2)) <= 1e-9 * max(1.0, np.abs(d2).max())


@pytest.mark.parametrize("n", [8, 33, 90])
def test_harmonic_oscillator_spectrum(n):
    x, m, K = oracle.hermite_axis(n)
    plan = oracle.make_plan_general([K], [m], [x * x], [x])
    lam = plan.lam[0]
    exact = 2.0 * np.arange(n - 1) + 1.0
    # n - 1 eigenvalues are exact; the remaining one is the spurious top mode
    hit = [np.min(np.abs(lam - e)) for e in exact]
    assert max(hit) <= 1e-9 * (2 * n)


def test_generic_plan_reproduces_fd_and_sem():
    L = 3.0
    n = (9, 12, 7)
    f = [W.f_harmonic(k, L) for k in n]
    fd = oracle.make_plan(n, L, f)
    Ks = [oracle.fd_axis_matrix(k, L, np.zeros(k)) for k in n]
    ms = [np.full(k, 2 * L / (k + 1)) for k in n]
    gen = oracle.make_plan_general(Ks, ms, f)
    b = W.rhs_normal(n, 4)
    psi = W.complex_normal(n, 5)
    assert _rel(oracle.apply_inverse(gen, b, 0.7), oracle.apply_inverse(fd, b, 0.7)) <= 1e-12
    assert _rel(oracle.apply_exp(gen, psi, 0.03), oracle.apply_exp(fd, psi, 0.03)) <= 1e-12
    assert _rel(oracle.operator_apply(gen, b, None, 0.7), oracle.stencil_apply(fd, b, None, 0.7)) <= 1e-12
    k, cells = 3, (4, 5)
    sx = [oracle.sem_axis(k, c, L) for c in cells]
    fs = [W.f_harmonic(0, L, x=a[0]) for a in sx]
    sem = oracle.make_plan_sem(k, cells, L, fs)
    gen = oracle.make_plan_general([S / mm[:, None] for _, mm, S in sx], [mm for _, mm, _ in sx], fs)
    b = W.rhs_normal(sem.shape, 6)
    assert _rel(oracle.apply_inverse(gen, b, 0.2), oracle.apply_inverse(sem, b, 0.2)) <= 1e-12


def _hermite_plan(shape, seed=0):
    rng = np.random.default_rng(seed)
    axes = [oracle.hermite_axis(n) for n in shape]
    fs = [x * x + rng.uniform(0, 1, x.size) for x, _, _ in axes]
    return oracle.make_plan_general([K for _, _, K in axes], [m for _, m, _ in axes], fs,
                                    [x for x, _, _ in axes])


def test_hermite_applies_against_dense_matrix():
    plan = _hermite_plan((5, 6, 4))
    H = oracle.dense_operator(plan, None, 0.5)
    b = W.rhs_normal(plan.shape, 7)
    assert _rel(oracle.apply_inverse(plan, b, 0.5), oracle.lu_solve(H, b).reshape(plan.shape)) <= 1e-12
    psi = W.complex_normal(plan.shape, 8)
    H0 = oracle.dense_operator(plan, None, 0.0)
    ref = scipy.linalg.expm(-1j * 0.05 * H0) @ psi.ravel()
    assert _rel(oracle.apply_exp(plan, psi, 0.05), ref.reshape(plan.shape)) <= 1e-11
    u = W.rhs_normal(plan.shape, 9)
    V2 = W.rhs_normal(plan.shape, 10) ** 2
    assert _rel(oracle.operator_apply(plan, u, V2, 0.5), (oracle.dense_operator(plan, V2, 0.5) @ u.ravel()).reshape(plan.shape)) <= 1e-13


def test_hermite_pcg_against_dense_solve():
    plan = _hermite_plan((6, 5, 7), seed=1)
    V2 = 3.0 * W.rhs_normal(plan.shape, 11) ** 2
    f = W.rhs_normal(plan.shape, 12)
    r = oracle.pcg(plan, V2, 0.5, f, rtol=1e-13)
    ref = oracle.lu_solve(oracle.dense_operator(plan, V2, 0.5), f).reshape(plan.shape)
    assert _rel(r.x, ref) <= 1e-11


def _test_problem(n):
    x, m, K = oracle.hermite_axis(n)
    cs = [1.5 * np.pi, np.pi, 0.5 * np.pi]   # axis 0 = z, 1 = y, 2 = x
    fs = [W.f_test_potential(0, 0.0, c, x=x) for c in (3.0, 2.0, 1.0)]
    G = [W.rational_sine(c, x) for c in cs]
    ustar = W.outer([g for g, _ in G])
    rhs = np.zeros((n,) * 3)
    for a in range(3):
        fac = [g for g, _ in G]
        fac[a] = -G[a][1] + fs[a] * G[a][0]
        rhs += W.outer(fac)
    plan = oracle.make_plan_general([K] * 3, [m] * 3, fs, [x] * 3)
    return plan, x, ustar, rhs


def test_printed_hermite_accuracy_n199():
    row = GOLDEN["hermite_accuracy"]["rows"][0]
    n = row["n"]
    plan, x, ustar, rhs = _test_problem(n)
    u = oracle.apply_inverse(plan, rhs, 0.0)
    e = u - ustar
    l2 = np.linalg.norm(e) / np.linalg.norm(ustar)
    wgh = np.polynomial.hermite.hermgauss(n)[1]
    weighted = np.sqrt(np.sum(W.outer([wgh] * 3) * e * e))
    # printed to three digits: within half a unit of the last one
    assert abs(l2 - row["l2_rel"]) <= 0.005e-5
    assert abs(weighted - row["weighted_l2"]) <= 0.005e-5


def test_planted_mistake_is_caught():
    """Dropping the weights (treating K as symmetric) breaks the dense check."""
    plan = _hermite_plan((5, 4))
    bad = oracle.make_plan_general(plan.K, [None, None], plan.f, plan.x)
    H = oracle.dense_operator(plan, None, 0.5)
    b = W.rhs_normal(plan.shape, 13)
    ref = oracle.lu_solve(H, b).reshape(plan.shape)
    assert _rel(oracle.apply_inverse(bad, b, 0.5), ref) > 1e-3
