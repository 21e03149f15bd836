"""Pins of the oracle's multi-level inverse iteration (Sec. 5.3.1, Table
tab:multilevel), CPU only.

* Tensor-product linear interpolation: the identity on the same grid, exact
  for products of per-axis linear functions between the outermost nodes,
  zero Dirichlet values honoured.
* The multi-level iteration reaches the same eigenpair as a single-level run
  on the finest grid, with fewer steps there.
* The printed ground-state eigenvalue of the stirrer problem, 5.286155366963
  (Q^20 SEM at 499^3), reached by Q^10 SEM on 6 cells per axis (n = 59)
  within 1e-8: eq. (stirrer) with gamma = (1, 1, 2), w0 = 4, delta = 1,
  r0 = 1 on [-8,8]^3, shift 0.9 lambda_min(-Delta + V1).
"""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _stirrer(k, cells, L=8.0):
    x = oracle.sem_nodes(k, cells, L)
    # C order (z, y, x): V1 = x^2 + y^2 + 4 z^2, V2 = 2 w0 exp(-((x - r0)^2 + y^2))
    plan = oracle.make_plan_sem(k, (cells,) * 3, L, [4.0 * x * x, x * x, x * x])
    V2 = 8.0 * np.exp(-(((x - 1.0) ** 2)[None, None, :] + (x**2)[None, :, None])) * np.ones((x.size, 1, 1))
    shift = 0.9 * sum(float(l[0]) for l in plan.lam)
    return plan, V2, shift


def test_interpolation():
    L = 3.0
    rng = np.random.default_rng(0)
    a = oracle.make_plan_sem(3, (2, 3), L, [np.zeros(5), np.zeros(8)])
    b = oracle.make_plan_sem(4, (3, 4), L, [np.zeros(11), np.zeros(15)])
    u = rng.standard_normal(a.shape)
    assert np.array_equal(oracle.interpolate(a, a, u), u)
    # product of linear functions, checked between the outermost coarse nodes
    c = rng.standard_normal(4)
    ua = np.multiply.outer(c[0] + c[1] * a.x[0], c[2] + c[3] * a.x[1])
    ub = oracle.interpolate(a, b, ua)
    inner0 = (b.x[0] >= a.x[0][0]) & (b.x[0] <= a.x[0][-1])
    inner1 = (b.x[1] >= a.x[1][0]) & (b.x[1] <= a.x[1][-1])
    exact = np.multiply.outer(c[0] + c[1] * b.x[0], c[2] + c[3] * b.x[1])
    assert np.max(np.abs((ub - exact)[np.ix_(inner0, inner1)])) < 1e-13
    # below the first coarse node of axis 1: linear towards the zero value at -L
    j = np.nonzero(b.x[1] < a.x[1][0])[0]
    t = (b.x[1][j] + L) / (a.x[1][0] + L)
    first = np.interp(b.x[0][inner0], a.x[0], ua[:, 0])  # axis 0 between its outermost nodes
    assert np.max(np.abs(ub[np.ix_(inner0, j)] - first[:, None] * t[None, :])) < 1e-13


def test_multilevel_matches_single_level():
    levels = [_stirrer(8, 3), _stirrer(8, 5)]
    ml = oracle.multilevel_inverse_iteration(levels, lam_tol=1e-13, max_steps=60)
    plan, V2, shift = levels[-1]
    single = oracle.inverse_iteration(plan, V2, shift, steps=60, lam_tol=1e-13)
    assert abs(ml.lam - single.lam[-1]) < 1e-12 * ml.lam
    s = np.sign(oracle.inner(plan, ml.u, single.u))
    assert oracle.norm(plan, s * ml.u - single.u) < 1e-6
    assert ml.steps[-1] < len(single.lam) - 1


def test_printed_stirrer_eigenvalue():
    g = GOLDEN["stirrer_lambda1"]
    ml = oracle.multilevel_inverse_iteration([_stirrer(10, 3), _stirrer(10, 6)], lam_tol=1e-14, max_steps=80)
    assert abs(ml.lam - g["value"]) < 1e-8 * g["value"], ml.lam_levels
