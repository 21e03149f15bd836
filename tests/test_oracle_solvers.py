"""Pins for the oracle's PCG, shifted inverse iteration and splitting (CPU only).

* PCG (Sec. 3.2): with V2 = 0 the preconditioner is the exact inverse, so one
  iteration suffices; with V2 it reaches the dense LU solution.
* inverse iteration (Sec. 4.1, 5.3.1): V2 = 0 gives the closed-form sum of the
  per-axis lowest eigenvalues; with V2 it reaches numpy's dense eigvalsh; the
  stirrer ground state of Table tab:multilevel is reached in the continuum limit.
* splitting (Sec. 5.1): V2 = 0 makes every scheme exact; constant V2 is a
  global phase; Strang is order 2 and Yoshida (eq. (yoshida)) order 4 against
  the dense exponential of the full operator; the Yoshida identities.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _plan(shape, L):
    return oracle.make_plan(shape, L, [W.f_harmonic(n, L) for n in shape])


def test_pcg_exact_preconditioner_one_iteration():
    shape, L = (7, 8, 9), 4.0
    plan = _plan(shape, L)
    f = W.rhs_normal(shape, 1)
    res = oracle.pcg(plan, None, 1.0, f, rtol=1e-12)
    assert res.iters == 1
    assert res.true_relres <= 1e-13


@pytest.mark.parametrize("shape", [(6, 6, 6), (5, 4, 3, 3)])
def test_pcg_matches_dense_lu(shape):
    L = 4.0
    plan = _plan(shape, L)
    V2 = W.gaussian_bumps(shape, L, 4, seed=3)
    sigma = 1.0 + max(0.0, -(sum(l[0] for l in plan.lam) + V2.min()) + 0.5)
    f = W.rhs_normal(shape, 2)
    res = oracle.pcg(plan, V2, sigma, f, rtol=1e-13)
    x = oracle.lu_solve(oracle.dense_operator(plan, V2, sigma), f).reshape(shape)
    assert res.true_relres <= 1e-12
    assert np.linalg.norm(res.x - x) <= 1e-11 * np.linalg.norm(x)
    assert 1 < res.iters < 60


def test_inverse_iteration_separable_closed_form():
    shape, L = (9, 7, 8), 3.0
    plan = oracle.make_plan(shape, L, [np.zeros(n) for n in shape])
    lam1 = sum((2 - 2 * np.cos(np.pi / (n + 1))) / (2 * L / (n + 1)) ** 2 for n in shape)
    V2 = np.zeros(shape)
    rng = np.random.default_rng(0)
    u0 = W.outer([np.ones(n) for n in shape]) + 0.1 * rng.standard_normal(shape)
    res = oracle.inverse_iteration(plan, V2, 0.9 * lam1, steps=20, u0=u0)
    assert abs(res.lam[-1] - lam1) <= 1e-12 * lam1
    assert all(res.lam[i + 1] <= res.lam[i] + 1e-12 for i in range(len(res.lam) - 1))


def test_inverse_iteration_dense_eigenvalue():
    shape, L = (6, 5, 6), 4.0
    plan = _plan(shape, L)
    V2 = np.abs(W.gaussian_bumps(shape, L, 3, seed=5))  # V2 >= 0: shift 0.9 lambda_min(A) is safe
    lamA = sum(l[0] for l in plan.lam)
    res = oracle.inverse_iteration(plan, V2, 0.9 * lamA, steps=40)
    Hd = oracle.dense_operator(plan, V2)
    ref = np.linalg.eigvalsh(Hd)[0]
    wj, _ = oracle.jacobi_eigh(Hd)
    assert abs(wj[0] - ref) <= 1e-12 * abs(ref)
    assert abs(res.lam[-1] - ref) <= 1e-10 * abs(ref)


def test_stirrer_ground_state_continuum():
    """Table tab:multilevel: lambda_1 = 5.286155366963 (stirrer, [-8,8]^3)."""
    g = GOLDEN["stirrer_lambda1"]
    L = g["L"]
    lams = []
    for n in (31, 63):
        x = W.grid_nodes(n, L)
        # C order: axis 0 = z (gamma_z = 2 -> 4 z^2), axis 1 = y, axis 2 = x
        plan = oracle.make_plan((n, n, n), L, [4 * x * x, x * x, x * x])
        V2 = np.broadcast_to(8.0 * np.exp(-((x[None, None, :] - 1.0) ** 2 + x[None, :, None] ** 2)),
                             (n, n, n)).copy()
        lamA = sum(l[0] for l in plan.lam)
        res = oracle.inverse_iteration(plan, V2, 0.9 * lamA, steps=20, pcg_rtol=1e-12)
        lams.append(res.lam[-1])
    extrap = (4 * lams[1] - lams[0]) / 3
    assert abs(extrap - g["value"]) / g["value"] < 5e-4
    ratio = (g["value"] - lams[0]) / (g["value"] - lams[1])
    assert 3.5 < ratio < 4.5


def test_yoshida_coefficients():
    g1, g2 = oracle.YOSHIDA_G1, oracle.YOSHIDA_G2
    assert abs(2 * g1 + g2 - 1) <= 1e-15
    assert abs(2 * g1**3 + g2**3) <= 1e-14
    assert g2 < 0


@pytest.mark.parametrize("scheme", ["strang_bab", "strang_aba", "yoshida_bab", "yoshida_aba"])
def test_split_exact_when_v2_vanishes(scheme):
    shape, L = (5, 6, 4), 3.0
    plan = _plan(shape, L)
    psi0 = W.complex_normal(shape, 1)
    out = oracle.split_propagate(plan, np.zeros(shape), psi0, 0.01, 7, scheme)
    ref = oracle.apply_exp(plan, psi0, 0.07)
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
    c = 1.7
    out_c = oracle.split_propagate(plan, np.full(shape, c), psi0, 0.01, 7, scheme)
    assert np.linalg.norm(out_c - np.exp(-1j * c * 0.07) * ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("shape,L", [((5, 6), 3.0), ((4, 4, 4), 3.0), ((3, 3, 3, 3, 3, 3), 6.0)])
def test_split_orders_against_dense_exponential(shape, L):
    plan = _plan(shape, L)
    V2 = W.pairwise_v2(shape, L) + W.gaussian_bumps(shape, L, 2, seed=1)
    psi0 = W.complex_normal(shape, 2)
    psi0 /= np.linalg.norm(psi0)
    T = 0.2
    ref = oracle.expm_apply(oracle.dense_operator(plan, V2), T, psi0.reshape(-1)).reshape(shape)
    for scheme, order in [("strang_bab", 2), ("strang_aba", 2), ("yoshida_bab", 4), ("yoshida_aba", 4)]:
        errs = [np.linalg.norm(oracle.split_propagate(plan, V2, psi0, T / m, m, scheme) - ref)
                for m in (4, 8, 16)]
        for a, b in zip(errs, errs[1:]):
            assert abs(np.log2(a / b) - order) < 0.1, (scheme, errs)
