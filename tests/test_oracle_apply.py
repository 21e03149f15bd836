"""Pins for the oracle's separable apply (inverse and propagator), CPU only.

* brute force: dense operator assembled entry by entry from the stencil, solved
  by the oracle's LU; cross-checked with an independent Kronecker-sum assembly
  (numpy.kron) and numpy.linalg.solve / scipy.linalg.expm (library routines).
* closed form: eigenfunction inputs built from the analytic sine eigenvectors
  of the FD Laplacian map to 1/(Lambda+sigma) and exp(-i tau Lambda) multiples.
* printed value: FD accuracy of Table tab:accuracy_gh200 (FP64, 3D, Q^1), scaled
  by h^2 to smaller n.
* invariants: symmetry, positivity, norm conservation, group law, tau = 0,
  rank-one separability of the propagator.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

SHAPES = [(6,), (5, 6), (4, 5, 6), (3, 2, 3, 2), (2, 2, 2, 2, 2, 2)]


def _plan(shape, L=2.0, seed=0):
    rng = np.random.default_rng(seed)
    f = [rng.uniform(0.0, 3.0, size=n) for n in shape]
    return oracle.make_plan(shape, L, f)


def _kron_sum(plan):
    N = plan.N
    H = np.zeros((N, N))
    for k in range(plan.d):
        Hk = oracle.fd_axis_matrix(plan.shape[k], plan.L, plan.f[k])
        left = np.eye(int(np.prod(plan.shape[:k])))
        right = np.eye(int(np.prod(plan.shape[k + 1:])))
        H += np.kron(np.kron(left, Hk), right)
    return H


@pytest.mark.parametrize("shape", SHAPES)
def test_stencil_dense_equals_kron_sum(shape):
    plan = _plan(shape)
    assert np.max(np.abs(oracle.dense_operator(plan) - _kron_sum(plan))) <= 1e-12


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("sigma", [1.0, 0.0, -0.3])
def test_inverse_matches_dense_lu(shape, sigma):
    plan = _plan(shape, seed=len(shape))
    b = W.rhs_normal(shape, 7)
    u = oracle.apply_inverse(plan, b, sigma)
    Hd = oracle.dense_operator(plan, sigma=sigma)
    ulu = oracle.lu_solve(Hd, b).reshape(shape)
    unp = np.linalg.solve(_kron_sum(plan) + sigma * np.eye(plan.N), b.reshape(-1)).reshape(shape)
    assert np.linalg.norm(u - ulu) <= 1e-12 * np.linalg.norm(ulu)
    assert np.linalg.norm(ulu - unp) <= 1e-12 * np.linalg.norm(unp)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tau", [0.01, 0.3, -0.2])
def test_exp_matches_dense_expm(shape, tau):
    plan = _plan(shape, seed=3)
    psi = W.complex_normal(shape, 11)
    out = oracle.apply_exp(plan, psi, tau)
    Hd = oracle.dense_operator(plan)
    ref = oracle.expm_apply(Hd, tau, psi.reshape(-1)).reshape(shape)
    ref2 = (scipy.linalg.expm(-1j * tau * _kron_sum(plan)) @ psi.reshape(-1)).reshape(shape)
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(ref - ref2) <= 1e-12 * np.linalg.norm(ref2)


def test_eigenfunction_inputs_closed_form():
    """V = 0: analytic eigenvectors per axis (distinct n and mode per axis pin axis order)."""
    shape, L, sigma, tau = (5, 7, 9), 3.0, 0.7, 0.05
    plan = oracle.make_plan(shape, L, [np.zeros(n) for n in shape])
    modes = (2, 5, 3)
    facs, lam = [], 0.0
    for n, j in zip(shape, modes):
        i = np.arange(1, n + 1)
        facs.append(np.sqrt(2.0 / (n + 1)) * np.sin(i * j * np.pi / (n + 1)))
        h = 2 * L / (n + 1)
        lam += (2 - 2 * np.cos(j * np.pi / (n + 1))) / h**2
    b = W.outer(facs)
    u = oracle.apply_inverse(plan, b, sigma)
    assert np.max(np.abs(u - b / (lam + sigma))) <= 1e-13
    psi = oracle.apply_exp(plan, b.astype(np.complex128), tau)
    assert np.max(np.abs(psi - np.exp(-1j * tau * lam) * b)) <= 1e-13


def test_fd_accuracy_matches_printed_value():
    """Table tab:accuracy_gh200, FP64 3D Q^1: 3.66e-6 at n = 1099, error ~ h^2."""
    g = GOLDEN["fd_q1_3d_l2_error"]
    L = g["L"]
    coef = {2: 1.0, 1: 2.0, 0: 3.0}     # C order: axis 2 = x, axis 1 = y, axis 0 = z
    for n in (63, 99):
        shape = (n, n, n)
        f = [W.f_test_potential(n, L, coef[k]) for k in range(3)]
        plan = oracle.make_plan(shape, L, f)
        x = W.grid_nodes(n, L)
        ustar = W.outer([np.sin(3 * np.pi * x), np.sin(2 * np.pi * x), np.sin(np.pi * x)])
        Vsum = f[0][:, None, None] + f[1][None, :, None] + f[2][None, None, :]
        rhs = (14 * np.pi**2 + Vsum) * ustar     # -Laplacian of u* is 14 pi^2 u*
        u = oracle.apply_inverse(plan, rhs, 0.0)
        err = np.linalg.norm(u - ustar) / np.linalg.norm(ustar)
        scaled = err * ((n + 1) / (g["n"] + 1)) ** 2
        assert abs(scaled - g["value"]) / g["value"] < 0.01, (n, err, scaled)


def test_symmetry_positivity_norm_group_identity():
    shape = (6, 5, 7)
    plan = _plan(shape, L=4.0, seed=5)
    u = W.rhs_normal(shape, 1)
    v = W.rhs_normal(shape, 2)
    Su, Sv = oracle.apply_inverse(plan, u, 1.0), oracle.apply_inverse(plan, v, 1.0)
    assert abs(np.vdot(v, Su) - np.vdot(Sv, u)) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(Sv)
    assert np.vdot(u, Su) > 0
    psi = W.complex_normal(shape, 3)
    p1 = oracle.apply_exp(plan, psi, 0.37)
    assert abs(np.linalg.norm(p1) - np.linalg.norm(psi)) <= 1e-13 * np.linalg.norm(psi)
    p12 = oracle.apply_exp(plan, oracle.apply_exp(plan, psi, 0.1), 0.27)
    assert np.linalg.norm(p12 - p1) <= 1e-12 * np.linalg.norm(psi)
    back = oracle.apply_exp(plan, p1, -0.37)
    assert np.linalg.norm(back - psi) <= 1e-12 * np.linalg.norm(psi)
    same = oracle.apply_exp(plan, psi, 0.0)
    assert np.linalg.norm(same - psi) <= 1e-13 * np.linalg.norm(psi)


def test_exp_rank_one_separability():
    shape, L, tau = (9, 8, 10), 5.0, 0.02
    f = [W.f_harmonic_cos(n, L) for n in shape]
    plan = oracle.make_plan(shape, L, f)
    facs = W.wavepacket_factors(shape, L, seed=4)
    out = oracle.apply_exp(plan, W.outer(facs), tau)
    per_axis = [oracle.expm_apply(oracle.fd_axis_matrix(n, L, fk), tau, g)
                for n, fk, g in zip(shape, f, facs)]
    ref = W.outer(per_axis)
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)


def test_mode_product_directions():
    """Forward applies Q^T along the axis, backward applies Q (checked with einsum)."""
    rng = np.random.default_rng(0)
    shape = (3, 4, 5)
    X = rng.standard_normal(shape)
    for axis in range(3):
        Q = rng.standard_normal((shape[axis], shape[axis]))
        fwd = oracle.mode_product(shape, axis, Q, X, transpose=True)
        bwd = oracle.mode_product(shape, axis, Q, X, transpose=False)
        Xm = np.moveaxis(X, axis, 0)
        ref_f = np.moveaxis(np.tensordot(Q.T, Xm, axes=1), 0, axis)
        ref_b = np.moveaxis(np.tensordot(Q, Xm, axes=1), 0, axis)
        assert np.allclose(fwd, ref_f, rtol=0, atol=1e-13)
        assert np.allclose(bwd, ref_b, rtol=0, atol=1e-13)
