"""Pins of the approximated qHOP and Magnus-2 drivers of the oracle (Sec. 5.1,
eq. (qhop_product), eq. (yoshida)), CPU only.

* The Gauss-Legendre rule is checked by what defines it: exact integration of
  polynomials up to degree 2M - 1 on [0, h].
* The printed errors of Table tab:splitting: for A = -Delta and a separable
  B = V1 every factor of the scheme is a Kronecker product of per-axis
  factors, so the 3D result for the product initial state is the outer product
  of three 1D results, and the 3D error follows from 1D inner products.  The
  1D runs use the FD discretisation at n = 255 (the paper uses Q^10 SEM at
  499^3; both are close to the continuum): the absolute errors agree within
  5 %, the ratios to Strang within 3 %.
* The remark that qHOP with M = 1 is Strang and Magnus-2 with M = 1 is Yoshida.
* The tensor factorisation itself, on a small 3D grid.
* Global orders 2 (qHOP) and 4 (Magnus-2).
* Planted mistakes (reversed product order, equal weights) fail the table pin.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("M", [1, 2, 3, 5, 7])
def test_gauss_legendre_exact_for_degree_2m_minus_1(M):
    h = 0.37
    s, w = oracle.gauss_legendre(M, h)
    assert np.all((s > 0) & (s < h)) and np.all(np.diff(s) > 0)
    assert abs(w.sum() - 1.0) < 1e-15
    for j in range(2 * M):
        exact = h**j / (j + 1)  # (1/h) * integral_0^h x^j dx
        assert abs(np.dot(w, s**j) - exact) <= 1e-14 * max(1.0, exact)
    # degree 2M is not integrated exactly (the rule has exactly that order)
    assert abs(np.dot(w, (s / h) ** (2 * M)) - 1.0 / (2 * M + 1)) > 1e-9


def _separable_1d(n, L):
    v = W.f_separable_v1(n, L)
    plan_a = oracle.make_plan((n,), L, [np.zeros(n)])
    plan_h = oracle.make_plan((n,), L, [v])
    x = W.grid_nodes(n, L)
    g = np.sin(np.pi * (x + L) / (2 * L)).astype(np.complex128)
    return v, plan_a, plan_h, g


def _rel3(y, ex, g):
    """||y x y x y - ex x ex x ex|| / ||g x g x g|| from 1D inner products."""
    a, b, c = np.vdot(y, y).real, np.vdot(ex, ex).real, np.vdot(ex, y)
    return np.sqrt(max(a**3 + b**3 - 2 * (c**3).real, 0.0)) / np.vdot(g, g).real ** 1.5


def _qhop_with_variant(plan, V, psi, h, M, variant):
    """A deliberately wrong qHOP step, assembled from the oracle's pieces."""
    s, w = oracle.gauss_legendre(M, h)
    order = range(M - 1, -1, -1) if variant == "reversed" else range(M)
    for k in order:
        wk = 1.0 / M if variant == "equal_weights" else w[k]
        psi = oracle.apply_exp(plan, psi, s[k])
        psi = oracle.phase_apply(V, wk * h, psi)
        psi = oracle.apply_exp(plan, psi, -s[k])
    return oracle.apply_exp(plan, psi, h)


def test_printed_qhop_errors_of_the_separable_example():
    g0 = GOLDEN["qhop_separable"]
    L, T = g0["L"], g0["T"]
    v, plan_a, plan_h, g = _separable_1d(255, L)
    ex = oracle.apply_exp(plan_h, g, T)
    for dt_s in ("0.1", "0.01", "0.005"):
        dt = float(dt_s)
        m = int(round(T / dt))
        printed = g0["rows"][dt_s]
        got = [_rel3(oracle.split_propagate(plan_a, v, g, dt, m, "strang_bab"), ex, g)]
        got += [_rel3(oracle.qhop_propagate(plan_a, v, g, dt, m, M), ex, g) for M in g0["M"][1:]]
        for e, p in zip(got, printed):
            assert abs(e - p) / p < 0.05, (dt_s, got, printed)
        for k in range(1, 4):
            assert abs((got[0] / got[k]) / (printed[0] / printed[k]) - 1) < 0.03, (dt_s, got, printed)


@pytest.mark.parametrize("variant", ["reversed", "equal_weights"])
def test_planted_qhop_mistakes_fail_the_printed_errors(variant):
    g0 = GOLDEN["qhop_separable"]
    L, T, dt = g0["L"], g0["T"], 0.01
    v, plan_a, plan_h, g = _separable_1d(127, L)
    ex = oracle.apply_exp(plan_h, g, T)
    y = g.copy()
    for _ in range(int(round(T / dt))):
        y = _qhop_with_variant(plan_a, v, y, dt, 3, variant)
    e = _rel3(y, ex, g)
    assert abs(e - g0["rows"]["0.01"][1]) / g0["rows"]["0.01"][1] > 0.5


def test_qhop_m1_is_strang_and_magnus2_m1_is_yoshida():
    shape, L = (9, 11), 3.0
    rng = np.random.default_rng(3)
    plan = oracle.make_plan(shape, L, [rng.uniform(0, 4, n) for n in shape])
    V = rng.uniform(-2, 5, shape)
    psi = W.complex_normal(shape, 4)
    dt = 0.07
    a = oracle.qhop_propagate(plan, V, psi, dt, 3, 1)
    b = oracle.split_propagate(plan, V, psi, dt, 3, "strang_aba")
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
    a = oracle.qhop_propagate(plan, V, psi, dt, 2, 1, yoshida=True)
    b = oracle.split_propagate(plan, V, psi, dt, 2, "yoshida_aba")
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


@pytest.mark.parametrize("yoshida", [False, True])
def test_tensor_factorisation_for_separable_b(yoshida):
    shape, L = (7, 9, 8), 4.0
    rng = np.random.default_rng(5)
    fa = [rng.uniform(0, 2, n) for n in shape]  # A may hold part of the potential too
    fb = [rng.uniform(0, 6, n) for n in shape]
    V = fb[0][:, None, None] + fb[1][None, :, None] + fb[2][None, None, :]
    phis = [W.complex_normal((n,), 10 + k) for k, n in enumerate(shape)]
    dt, m, M = 0.03, 2, 3
    full = oracle.qhop_propagate(oracle.make_plan(shape, L, fa), V, W.outer(phis), dt, m, M, yoshida)
    parts = [oracle.qhop_propagate(oracle.make_plan((n,), L, [fa[k]]), fb[k], phis[k], dt, m, M, yoshida)
             for k, n in enumerate(shape)]
    ref = W.outer(parts)
    assert np.linalg.norm(full - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("yoshida,order", [(False, 2), (True, 4)])
def test_global_order(yoshida, order):
    L, T = 8.0, 0.1
    v, plan_a, plan_h, g = _separable_1d(127, L)
    ex = oracle.apply_exp(plan_h, g, T)
    for M in (3, 5):
        e = [np.linalg.norm(oracle.qhop_propagate(plan_a, v, g, dt, int(round(T / dt)), M, yoshida) - ex)
             for dt in (0.01, 0.005)]
        rate = np.log2(e[0] / e[1])
        assert abs(rate - order) < 0.1, (M, e)
