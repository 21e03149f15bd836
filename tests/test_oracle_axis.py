"""Pins for the oracle's per-axis operator and Jacobi eigensolver (CPU only).

What pins what:
* closed form of the 1D FD Laplacian spectrum (Sec. 2.1, K = h^-2 tridiag(-1,2,-1)):
  lambda_j = (2 - 2 cos(j pi/(n+1))) / h^2, q_j(i) = sqrt(2/(n+1)) sin(i j pi/(n+1)).
* special case that reduces to a library routine: numpy.linalg.eigh.
* continuum limits: harmonic oscillator levels 2j+1; the ground-state eigenvalue
  printed in Table tab:inverse_iter (eq. (separable_V1) on [-8,8]^3) via
  Richardson extrapolation of the 1D FD eigenvalue.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("n,L", [(1, 1.0), (2, 3.0), (7, 8.0), (16, 1.0), (33, 10.0)])
def test_jacobi_closed_form_laplacian(n, L):
    H = oracle.fd_axis_matrix(n, L, np.zeros(n))
    w, V = oracle.jacobi_eigh(H)
    h = 2 * L / (n + 1)
    j = np.arange(1, n + 1)
    lam = (2 - 2 * np.cos(j * np.pi / (n + 1))) / h**2
    assert np.max(np.abs(w - lam)) <= 1e-13 * lam.max()
    i = np.arange(1, n + 1)
    Qc = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, j) * np.pi / (n + 1))
    # equal up to the sign of each column
    for c in range(n):
        s = np.sign(np.dot(Qc[:, c], V[:, c]))
        assert np.max(np.abs(V[:, c] - s * Qc[:, c])) <= 1e-12


def test_constant_potential_shifts_spectrum():
    n, L = 20, 5.0
    w0, _ = oracle.jacobi_eigh(oracle.fd_axis_matrix(n, L, np.zeros(n)))
    w1, _ = oracle.jacobi_eigh(oracle.fd_axis_matrix(n, L, np.full(n, 3.25)))
    assert np.max(np.abs(w1 - (w0 + 3.25))) <= 1e-12 * w1.max()


@pytest.mark.parametrize("n,seed", [(5, 0), (20, 1), (50, 2)])
def test_jacobi_matches_numpy_eigh(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A + A.T
    w, V = oracle.jacobi_eigh(A)
    wr, Vr = np.linalg.eigh(A)
    assert np.max(np.abs(w - wr)) <= 1e-12 * np.abs(wr).max()
    for c in range(n):
        s = np.sign(np.dot(Vr[:, c], V[:, c]))
        assert np.max(np.abs(V[:, c] - s * Vr[:, c])) <= 1e-9


def test_jacobi_residual_orthogonality_sign():
    n, L = 120, 10.0
    H = oracle.fd_axis_matrix(n, L, W.f_harmonic_cos(n, L))
    w, V = oracle.jacobi_eigh(H)
    nH = np.linalg.norm(H, 2)
    assert np.all(np.diff(w) > 0)
    assert np.linalg.norm(H @ V - V * w) <= 1e-13 * nH * np.sqrt(n)
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 1e-13
    # sign convention: largest-magnitude entry of each column is positive
    idx = np.argmax(np.abs(V), axis=0)
    assert np.all(V[idx, np.arange(n)] > 0)


def test_harmonic_oscillator_levels():
    # f = x^2 on a wide box: lambda_j -> 2j + 1 with O(h^2) error
    n, L = 400, 8.0
    w, _ = oracle.jacobi_eigh(oracle.fd_axis_matrix(n, L, W.f_harmonic(n, L)))
    h = 2 * L / (n + 1)
    for j in range(5):
        assert abs(w[j] - (2 * j + 1)) <= 2.0 * (2 * j + 1) ** 2 * h**2


def test_continuum_ground_state_separable_v1():
    """Table tab:inverse_iter: lambda_1 = 23.2878438176 = 3 mu_1 (separable)."""
    ref = GOLDEN["separable_v1_lambda1"]["value"]
    L = GOLDEN["separable_v1_lambda1"]["L"]
    mus = []
    for n in (127, 255, 511):  # h halves each time
        w, _ = oracle.jacobi_eigh(oracle.fd_axis_matrix(n, L, W.f_separable_v1(n, L)))
        mus.append(w[0])
    r1 = [(4 * mus[i + 1] - mus[i]) / 3 for i in range(2)]
    r2 = (16 * r1[1] - r1[0]) / 15
    assert abs(3 * r2 - ref) / ref <= 2e-7
    # the raw second-order values approach from below at rate ~4
    e = [abs(3 * m - ref) for m in mus]
    assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5


@pytest.mark.parametrize("n,kind", [(200, "cos"), (333, "sepv1")])
def test_jacobi_accuracy_against_lapack_tridiagonal(n, kind):
    """LAPACK's tridiagonal eigensolver (scipy) as the library-routine special case."""
    import scipy.linalg
    L = 8.0
    f = {"cos": W.f_harmonic_cos, "sepv1": W.f_separable_v1}[kind](n, L)
    h = 2 * L / (n + 1)
    ref = scipy.linalg.eigh_tridiagonal(2 / h**2 + f, np.full(n - 1, -1 / h**2), eigvals_only=True)
    w, _ = oracle.jacobi_eigh(oracle.fd_axis_matrix(n, L, f))
    assert np.max(np.abs(w - ref)) <= 1e-14 * np.abs(ref).max()
