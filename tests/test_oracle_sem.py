"""Pins of the oracle's Q^k spectral-element discretisation (Sec. 2,
eq. (eigen_decomp)), CPU only.

* Q^1 is the second-order FD scheme exactly (nodes, operator, applies).
* The Gauss-Lobatto rule integrates polynomials of degree <= 2k - 1 exactly,
  and not degree 2k.
* With the lumped mass, M^{-1} S reproduces -u'' exactly at the nodes for
  every polynomial u of degree <= k vanishing at +-L, on any mesh.
* The Q^2 error printed in Table tab:accuracy_gh200 (1.93e-9 at 550 cells,
  n = 1099), reached from 40 and 60 cells through the order-(k+2) scaling
  with a Richardson step on its O(h^2) relative correction.
* Low eigenvalues of Q^10 converge spectrally to (j pi / 2L)^2.
* Applies, operator, PCG (mass inner product) and inverse iteration against
  the dense Kronecker-sum matrix and LU / expm / eigh.
* A planted mistake (the mass scaling left out of T) is rejected.
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


@pytest.mark.parametrize("k", [1, 2, 3, 6, 10])
def test_gll_rule_exactness(k):
    x, w = oracle.gll_rule(k)
    assert x[0] == -1.0 and x[-1] == 1.0 and np.all(np.diff(x) > 0)
    for j in range(2 * k):
        exact = (1.0 - (-1.0) ** (j + 1)) / (j + 1)
        assert abs(np.dot(w, x**j) - exact) < 1e-13
    exact = 2.0 / (2 * k + 1)
    assert abs(np.dot(w, x ** (2 * k)) - exact) > 1e-6


def test_q1_is_finite_differences():
    n_cells, L = 12, 2.5
    x, m, S = oracle.sem_axis(1, n_cells, L)
    n = n_cells - 1
    assert np.allclose(x, W.grid_nodes(n, L), rtol=0, atol=1e-15)
    h = 2 * L / n_cells
    assert np.allclose(m, h, rtol=1e-15)
    K = S / m[:, None]
    assert np.max(np.abs(K - oracle.fd_axis_matrix(n, L, np.zeros(n)))) < 1e-12 / h**2
    f = [W.f_harmonic(n, L)] * 2
    sem = oracle.make_plan_sem(1, (n_cells, n_cells), L, f)
    fd = oracle.make_plan((n, n), L, f)
    b = W.rhs_normal((n, n), 3)
    assert _rel(oracle.apply_inverse(sem, b, 0.5), oracle.apply_inverse(fd, b, 0.5)) < 1e-13
    assert _rel(oracle.operator_apply(sem, b, None, 0.5), oracle.stencil_apply(fd, b, None, 0.5)) < 1e-13


@pytest.mark.parametrize("k", [2, 3, 5, 8])
@pytest.mark.parametrize("n_cells", [1, 3, 4])
def test_stiffness_over_mass_is_exact_second_derivative(k, n_cells):
    L = 1.3
    x, m, S = oracle.sem_axis(k, n_cells, L)
    K = S / m[:, None]
    # u = (L^2 - x^2) x^(k-2): degree k, zero at +-L
    u = np.polynomial.Polynomial([L**2, 0.0, -1.0]) * np.polynomial.Polynomial([0.0] * (k - 2) + [1.0])
    err = np.max(np.abs(K @ u(x) + u.deriv(2)(x)))
    assert err < 1e-12 * np.max(np.abs(K)) * np.max(np.abs(u(x))) + 1e-12


def test_printed_q2_accuracy():
    g = GOLDEN["sem_q2_3d_l2_error"]
    L, k = g["L"], g["k"]
    coef = {2: 1.0, 1: 2.0, 0: 3.0}  # x is the fastest axis (C order)

    def scaled_error(ne):
        x = oracle.sem_nodes(k, ne, L)
        f = [W.f_test_potential(0, L, coef[a], x=x) for a in range(3)]
        ustar = W.outer([np.sin(3 * np.pi * x), np.sin(2 * np.pi * x), np.sin(np.pi * x)])
        rhs = (14 * np.pi**2 + f[0][:, None, None] + f[1][None, :, None] + f[2][None, None, :]) * ustar
        plan = oracle.make_plan_sem(k, (ne,) * 3, L, f)
        e = _rel(oracle.apply_inverse(plan, rhs, 0.0), ustar)
        return e * (ne / g["n_cells"]) ** (k + 2)

    e40, e60 = scaled_error(40), scaled_error(60)
    # e(ne) = E (1 - a / ne^2): eliminate a
    E = (e60 * 60**2 - e40 * 40**2) / (60**2 - 40**2)
    assert abs(E - g["value"]) / g["value"] < 0.02, (e40, e60, E)
    assert abs(e60 - g["value"]) / g["value"] < 0.05


def test_q10_low_eigenvalues_are_spectrally_accurate():
    L, ne = 2.0, 6
    plan = oracle.make_plan_sem(10, (ne,), L, [np.zeros(10 * ne - 1)])
    j = np.arange(1, 9)
    exact = (j * np.pi / (2 * L)) ** 2
    assert np.max(np.abs(plan.lam[0][:8] - exact) / exact) < 1e-10


def _small_sem(k=3, cells=(2, 3, 2), L=1.5, seed=0):
    rng = np.random.default_rng(seed)
    shape = tuple(k * c - 1 for c in cells)
    f = [rng.uniform(0.0, 4.0, n) for n in shape]
    return oracle.make_plan_sem(k, cells, L, f)


def test_sem_applies_match_dense():
    plan = _small_sem()
    H = oracle.dense_operator(plan)
    b = W.rhs_normal(plan.shape, 1)
    u = oracle.apply_inverse(plan, b, 0.7)
    ref = oracle.lu_solve(H + 0.7 * np.eye(plan.N), b).reshape(plan.shape)
    assert _rel(u, ref) < 1e-12
    psi = W.complex_normal(plan.shape, 2)
    out = oracle.apply_exp(plan, psi, 0.03)
    ref = (scipy.linalg.expm(-0.03j * H) @ psi.reshape(-1)).reshape(plan.shape)
    assert _rel(out, ref) < 1e-11
    # the propagator is unitary in the mass inner product, not the plain one
    assert abs(oracle.norm(plan, out.real) ** 2 + oracle.norm(plan, out.imag) ** 2
               - oracle.norm(plan, psi.real) ** 2 - oracle.norm(plan, psi.imag) ** 2) < 1e-11 * np.linalg.norm(psi) ** 2
    V2 = np.random.default_rng(3).uniform(-1, 2, plan.shape)
    x = W.rhs_normal(plan.shape, 4)
    assert _rel(oracle.operator_apply(plan, x, V2, 0.2),
                ((H + np.diag(V2.reshape(-1) + 0.2)) @ x.reshape(-1)).reshape(plan.shape)) < 1e-13


def test_sem_pcg_and_inverse_iteration():
    plan = _small_sem(seed=1)
    rng = np.random.default_rng(5)
    V2 = rng.uniform(0.0, 6.0, plan.shape)
    f = W.rhs_normal(plan.shape, 6)
    res = oracle.pcg(plan, V2, 1.0, f, rtol=1e-13)
    H = oracle.dense_operator(plan, V2, 1.0)
    ref = oracle.lu_solve(H, f).reshape(plan.shape)
    assert res.true_relres < 1e-12 and _rel(res.x, ref) < 1e-11
    # H = M^{-1}(S + M V) has real spectrum; the lowest eigenvalue from the dense matrix
    lam1 = np.min(np.linalg.eigvals(oracle.dense_operator(plan, V2)).real)
    # V2 >= 0, so H1 - shift and H - shift are both >= 0.5
    shift = sum(l[0] for l in plan.lam) - 0.5
    out = oracle.inverse_iteration(plan, V2, shift, steps=40)
    assert abs(out.lam[-1] - lam1) < 1e-10 * lam1


def test_missing_mass_scaling_is_caught():
    plan = _small_sem(seed=2)
    b = W.rhs_normal(plan.shape, 1)
    ref = oracle.lu_solve(oracle.dense_operator(plan, None, 0.7), b).reshape(plan.shape)
    bad = oracle._apply_inverse_q(plan, b, 0.7)  # orthogonal Q used as if T were orthogonal
    assert _rel(bad, ref) > 1e-3
