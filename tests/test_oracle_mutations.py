"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case builds a deliberately wrong variant of one oracle step (transposed
operand, swapped axes, wrong grid spacing, dropped term, wrong sign) from the
oracle's own pieces and checks that the corresponding pin rejects it.
"""
import json
import os

import numpy as np

import oracle
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _small_plan():
    shape, L = (4, 5, 6), 2.0
    rng = np.random.default_rng(0)
    return oracle.make_plan(shape, L, [rng.uniform(0, 3, n) for n in shape])


def test_transposed_eigenvector_operand_is_caught():
    plan = _small_plan()
    b = W.rhs_normal(plan.shape, 1)
    ref = oracle.lu_solve(oracle.dense_operator(plan, sigma=1.0), b).reshape(plan.shape)
    bad = oracle.Plan(plan.shape, plan.L, plan.f, plan.h, [q.T.copy() for q in plan.Q], plan.lam)
    assert _rel(oracle.apply_inverse(plan, b, 1.0), ref) < 1e-12
    assert _rel(oracle.apply_inverse(bad, b, 1.0), ref) > 1e-3


def test_swapped_axes_are_caught_by_printed_accuracy():
    g = GOLDEN["fd_q1_3d_l2_error"]
    n, L = 63, g["L"]
    coef = {2: 1.0, 1: 2.0, 0: 3.0}
    f = [W.f_test_potential(n, L, coef[k]) for k in range(3)]
    x = W.grid_nodes(n, L)
    ustar = W.outer([np.sin(3 * np.pi * x), np.sin(2 * np.pi * x), np.sin(np.pi * x)])
    rhs = (14 * np.pi**2 + f[0][:, None, None] + f[1][None, :, None] + f[2][None, None, :]) * ustar
    scale = ((n + 1) / (g["n"] + 1)) ** 2
    good = oracle.make_plan((n, n, n), L, f)
    swapped = oracle.make_plan((n, n, n), L, f[::-1])
    e_good = _rel(oracle.apply_inverse(good, rhs, 0.0), ustar) * scale
    e_bad = _rel(oracle.apply_inverse(swapped, rhs, 0.0), ustar) * scale
    assert abs(e_good - g["value"]) / g["value"] < 0.01
    assert abs(e_bad - g["value"]) / g["value"] > 0.05


def test_wrong_grid_spacing_is_caught_by_closed_form():
    n, L = 10, 3.0
    j = np.arange(1, n + 1)
    lam = (2 - 2 * np.cos(j * np.pi / (n + 1))) / (2 * L / (n + 1)) ** 2
    # h = 2L/n instead of 2L/(n+1): same as the right formula on a smaller box
    w_bad, _ = oracle.jacobi_eigh(oracle.fd_axis_matrix(n, L * n / (n + 1), np.zeros(n)))
    assert np.max(np.abs(w_bad - lam)) > 1e-3 * lam.max()


def test_dropped_potential_and_shift_are_caught():
    plan = _small_plan()
    b = W.rhs_normal(plan.shape, 2)
    ref = oracle.lu_solve(oracle.dense_operator(plan, sigma=1.0), b).reshape(plan.shape)
    no_f = oracle.make_plan(plan.shape, plan.L, [np.zeros(n) for n in plan.shape])
    assert _rel(oracle.apply_inverse(no_f, b, 1.0), ref) > 1e-3
    assert _rel(oracle.apply_inverse(plan, b, 0.0), ref) > 1e-3


def test_sign_of_time_is_caught_by_dense_exponential():
    plan = _small_plan()
    psi = W.complex_normal(plan.shape, 3)
    ref = oracle.expm_apply(oracle.dense_operator(plan), 0.1, psi.reshape(-1)).reshape(plan.shape)
    assert _rel(oracle.apply_exp(plan, psi, 0.1), ref) < 1e-12
    assert _rel(oracle.apply_exp(plan, psi, -0.1), ref) > 1e-3
    assert _rel(np.conj(oracle.apply_exp(plan, np.conj(psi), 0.1)), ref) > 1e-3


def test_wrong_yoshida_weights_are_caught_by_order():
    shape, L = (4, 4, 4), 3.0
    plan = oracle.make_plan(shape, L, [W.f_harmonic(n, L) for n in shape])
    V2 = W.pairwise_v2(shape, L) + W.gaussian_bumps(shape, L, 2, seed=1)
    psi0 = W.complex_normal(shape, 2)
    T = 0.2
    ref = oracle.expm_apply(oracle.dense_operator(plan, V2), T, psi0.reshape(-1)).reshape(shape)

    def run(m, g1, g2):
        psi = psi0.copy()
        for _ in range(m):
            for g in (g1, g2, g1):
                psi = oracle.strang_step(plan, V2, psi, g * T / m, "BAB")
        return np.linalg.norm(psi - ref)

    # Strang with thirds (2 g1 + g2 = 1 still holds, 2 g1^3 + g2^3 = 0 does not): order 2, not 4
    e = [run(m, 1 / 3, 1 / 3) for m in (4, 8)]
    assert abs(np.log2(e[0] / e[1]) - 2) < 0.2
