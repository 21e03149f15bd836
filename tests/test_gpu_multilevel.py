"""Multi-level inverse iteration on the GPU (Sec. 5.3.1, Table tab:multilevel)
through ts_interpolate, ts_separable_ground_state and
ts_multilevel_inverse_iteration.

* Interpolation between FD and SEM grids against the oracle's (bitwise up to
  rounding: two-tap linear combinations).
* The separable ground state against the oracle's.
* The multi-level iteration on small grids against the oracle's: eigenvalue
  per level and the final eigenvector.
* Full size: the stirrer problem of Table tab:multilevel with Q^20 SEM on
  99^3 -> 199^3 -> 499^3, shift 0.9 lambda_min(-Delta + V1), PCG tolerance
  1e-12: the eigenvalue against the printed 5.286155366963.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _fd(shape, L, seed=0):
    rng = np.random.default_rng(seed)
    f = [rng.uniform(0, 3, n) for n in shape]
    return ts.ts_setup(shape, L, f, 1.0), oracle.make_plan(shape, L, f)


def _sem(k, cells, L, seed=0):
    rng = np.random.default_rng(seed)
    f = [rng.uniform(0, 3, k * c - 1) for c in cells]
    return ts.ts_setup_sem(k, cells, L, f, 1.0), oracle.make_plan_sem(k, cells, L, f)


def test_interpolation_matches_oracle():
    L = 5.0
    pairs = [(_fd((9, 12, 7), L), _fd((19, 25, 30), L)),
             (_sem(4, (3, 5), L), _sem(6, (5, 7), L)),
             (_fd((15, 15), L), _sem(5, (6, 4), L))]
    for (ca, co), (fa, fo) in pairs:
        u = W.rhs_normal(ca.shape, 3)
        got = to_host(ts.ts_interpolate(ca, fa, to_dev(u)))
        ref = oracle.interpolate(co, fo, u)
        e = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        announce("interp %s -> %s: %.2e" % (ca.shape, fa.shape, e))
        assert e <= 1e-14


def test_separable_ground_state_matches_oracle():
    for plan, oplan in (_fd((20, 17, 40), 4.0), _sem(6, (3, 4, 2), 4.0)):
        got = to_host(ts.ts_separable_ground_state(plan))
        ref = oracle.separable_ground_state(oplan)
        s = np.sign(np.sum(got * ref))
        got = s * got / np.sqrt(oracle.inner(oplan, got, got))
        assert rel(got, ref) <= 1e-12


def _stirrer(k, cells, L=8.0, lib_nodes=True):
    x = ts.ts_sem_nodes(k, cells, L)
    f = [4.0 * x * x, x * x, x * x]  # C order (z, y, x): gamma = (1, 1, 2)
    V2 = 8.0 * np.exp(-(((x - 1.0) ** 2)[None, None, :] + (x**2)[None, :, None])) * np.ones((x.size, 1, 1))
    plan = ts.ts_setup_sem(k, (cells,) * 3, L, f, 1.0)
    shift = 0.9 * sum(float(ts.ts_eigvals(plan, a)[0]) for a in range(3))
    return plan, f, V2, shift


def test_multilevel_matches_oracle():
    L = 8.0
    levels = [_stirrer(8, 3), _stirrer(8, 5)]
    olevels = [(oracle.make_plan_sem(8, (c,) * 3, L, f), V2, s) for (p, f, V2, s), c in zip(levels, (3, 5))]
    ref = oracle.multilevel_inverse_iteration(olevels, lam_tol=1e-13, max_steps=60, pcg_rtol=1e-12)
    u, lam, steps, its = ts.ts_multilevel_inverse_iteration([l[0] for l in levels], [to_dev(l[2]) for l in levels],
                                                            [l[3] for l in levels], max_steps=60, lam_tol=1e-13,
                                                            pcg_rtol=1e-12)
    announce("multilevel: lambda %s (oracle %s), steps %s (%s), PCG %s (%s)"
             % (lam, ref.lam_levels, steps, ref.steps, its, ref.pcg_iters))
    for a, b in zip(lam, ref.lam_levels):
        assert abs(a - b) <= 1e-11 * abs(b)
    uh = to_host(u)
    op = olevels[-1][0]
    s = np.sign(oracle.inner(op, uh, ref.u))
    assert oracle.norm(op, s * uh - ref.u) <= 1e-6


@pytest.mark.timeout(900)
def test_printed_multilevel_stirrer_full_size():
    g = GOLDEN["stirrer_lambda1"]
    levels = []
    for cells in (5, 10, 25):  # Q^20: 99^3, 199^3, 499^3
        announce("multilevel: setup Q^20 with %d cells" % cells)
        levels.append(_stirrer(20, cells))
    V2s = [to_dev(l[2]) for l in levels]
    u, lam, steps, its = ts.ts_multilevel_inverse_iteration([l[0] for l in levels], V2s, [l[3] for l in levels],
                                                            max_steps=60, lam_tol=1e-13, pcg_rtol=1e-12)
    announce("multilevel stirrer: lambda per level %s (printed %.12f), steps %s, PCG per step %s"
             % (["%.12f" % v for v in lam], g["value"], steps,
                ["%.1f" % (i / max(s, 1)) for i, s in zip(its, steps)]))
    assert abs(lam[-1] - g["value"]) <= 1e-11 * g["value"]
