"""Approximated qHOP and Magnus-2 (Sec. 5.1, eq. (qhop_product), eq. (yoshida))
on the GPU through ts_qhop_step.

* Parity with the oracle's literal product (2M + 1 propagations per qHOP
  step, no merging) on grouped (all n <= 32) and MFMA grids, for
  A = -Delta + V1, B = V2 and for A = -Delta, B = V1 + V2; complex128 with
  FP64 transforms and complex64 with FP32 transforms.
* M = 1 is bitwise the Strang ABA / Yoshida ABA schedule of ts_split_step.
* The separable example at full size (499^3, complex128, T = 0.1,
  A = -Delta, B = V1 of eq. (separable_V1), product initial state): the 3D
  result is the outer product of three 1D results, so sampled entries are
  checked against the oracle's 1D runs, and the relative error against the
  exact propagator is compared with the value printed in Table tab:splitting.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, make_pair, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _n_apply(M, magnus2, nsteps):
    """A propagations of the merged schedule."""
    return nsteps * M * (3 if magnus2 else 1) + 1


def _bars(n_apply):
    # FP64: each apply is unitary to a few eps and the factor times are
    # rounded once; measured ~1e-14 per apply.  FP32: ~1e-7 per apply (the
    # FP32-rounded eigenvectors are orthogonal to that level).
    return max(1e-12, 2e-14 * n_apply), 2e-7 * n_apply


CASES = [
    ((5, 5, 5, 5, 5, 5), 3, False), ((5, 5, 5, 5, 5, 5), 3, True),
    ((20, 24, 18), 7, False), ((20, 24, 18), 5, True),
    ((33, 40), 1, False), ((33, 40), 3, False), ((33, 40), 7, True),
    ((48, 40, 36), 3, False),
]


@pytest.mark.parametrize("shape,M,magnus2", CASES)
@pytest.mark.parametrize("a_is_laplacian", [False, True])
def test_qhop_matches_oracle_product(shape, M, magnus2, a_is_laplacian):
    L, dt, nsteps = 6.0, 1e-2, 4
    plan, oplan, f = make_pair(shape, L, "harm", sigma=1.0)
    V2 = W.pairwise_v2(shape, L)
    if a_is_laplacian:  # A = -Delta, the whole potential in B
        zeros = [np.zeros(n) for n in shape]
        plan = ts.ts_setup(shape, L, zeros, 1.0)
        oplan = oracle.make_plan(shape, L, zeros)
        V1 = f[0]
        for fk in f[1:]:
            V1 = np.add.outer(V1, fk)  # sum_k f_k(x_k) on the grid
        V2 = V2 + V1
    psi0 = W.complex_normal(shape, 7)
    psi0 /= np.linalg.norm(psi0)
    ref = oracle.qhop_propagate(oplan, V2, psi0, dt, nsteps, M, magnus2)
    t = to_dev(psi0)
    ts.ts_qhop_step(plan, to_dev(V2), t, dt, nsteps, M, magnus2)
    got = to_host(t)
    n_apply = _n_apply(M, magnus2, nsteps)
    bar128, bar64 = _bars(n_apply)
    e = rel(got, ref)
    t64 = to_dev(psi0).to(torch.complex64)
    ts.ts_qhop_step(plan, to_dev(V2).to(torch.float32), t64, dt, nsteps, M, magnus2, prec="fp32")
    e64 = rel(to_host(t64).astype(np.complex128), ref)
    announce("qhop %s M=%d magnus2=%s A=%s: c128 %.2e (bar %.1e), c64 %.2e (bar %.1e), %d A applies"
             % (shape, M, magnus2, "-lap" if a_is_laplacian else "H1", e, bar128, e64, bar64, n_apply))
    assert e <= bar128
    assert e64 <= bar64


def test_m1_is_the_strang_and_yoshida_schedule():
    shape, L = (33, 40), 6.0
    plan, _, _ = make_pair(shape, L, "harm", sigma=1.0)
    V2 = to_dev(W.pairwise_v2(shape, L))
    psi0 = to_dev(W.complex_normal(shape, 8))
    for magnus2, scheme in ((False, "strang_aba"), (True, "yoshida_aba")):
        a, b = psi0.clone(), psi0.clone()
        ts.ts_qhop_step(plan, V2, a, 0.01, 5, 1, magnus2)
        ts.ts_split_step(plan, V2, b, 0.01, 5, scheme)
        torch.cuda.synchronize()
        assert torch.equal(a, b), scheme


def test_qhop_argument_errors():
    shape, L = (16, 16), 6.0
    plan, _, _ = make_pair(shape, L, "harm", sigma=1.0)
    V2 = torch.zeros(shape, dtype=torch.float64, device=DEV)
    psi = torch.zeros(shape, dtype=torch.complex128, device=DEV)
    for M in (0, 65):
        with pytest.raises(ts.TSError) as e:
            ts.ts_qhop_step(plan, V2, psi, 0.01, 1, M)
        assert e.value.code == ts.TS_ERR_INVALID
    with pytest.raises(ts.TSError):
        ts.ts_qhop_step(plan, V2, psi, 0.01, -1, 3)
    with pytest.raises(ts.TSError):  # real data
        ts.ts_qhop_step(plan, V2, V2.clone(), 0.01, 1, 3)
    # nsteps = 0 leaves psi unchanged
    x = to_dev(W.complex_normal(shape, 1))
    y = x.clone()
    ts.ts_qhop_step(plan, V2, y, 0.01, 0, 3)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def _separable_1d(n, L):
    v = W.f_separable_v1(n, L)
    x = W.grid_nodes(n, L)
    g = np.sin(np.pi * (x + L) / (2 * L)).astype(np.complex128)
    return v, g


@pytest.mark.timeout(400)
def test_separable_example_full_size():
    """499^3 complex128, M = 3, dt = 0.01, T = 0.1 (31 propagations)."""
    g0 = GOLDEN["qhop_separable"]
    n, L, T, dt, M = 499, g0["L"], g0["T"], 0.01, 3
    m = int(round(T / dt))
    v, g = _separable_1d(n, L)
    announce("oracle 1D runs at n = %d" % n)
    oa = oracle.make_plan((n,), L, [np.zeros(n)])
    oh = oracle.make_plan((n,), L, [v])
    y1 = oracle.qhop_propagate(oa, v, g, dt, m, M)
    ex1 = oracle.apply_exp(oh, g, T)

    announce("GPU qHOP at %d^3" % n)
    plan = ts.ts_setup((n, n, n), L, [np.zeros(n)] * 3, 1.0)
    vd = to_dev(v)
    V = (vd[:, None, None] + vd[None, :, None] + vd[None, None, :]).contiguous()
    gd = to_dev(g)
    psi = (gd[:, None, None] * gd[None, :, None] * gd[None, None, :]).contiguous()
    ts.ts_qhop_step(plan, V, psi, dt, m, M)
    torch.cuda.synchronize()
    del V
    # sampled entries against the outer product of the oracle's 1D results
    rng = np.random.default_rng(0)
    idx = rng.integers(0, n, size=(3, 200000))
    got = psi[tuple(torch.from_numpy(i).to(DEV) for i in idx)].cpu().numpy()
    want = y1[idx[0]] * y1[idx[1]] * y1[idx[2]]
    scale = np.max(np.abs(y1)) ** 3
    err = np.max(np.abs(got - want)) / scale
    # relative error against the exact propagator, from the full 3D array
    e1 = to_dev(ex1)
    exact = (e1[:, None, None] * e1[None, :, None] * e1[None, None, :])
    rel_err = float(torch.linalg.vector_norm(psi - exact) / torch.linalg.vector_norm(gd) ** 3)
    printed = g0["rows"]["0.01"][1]
    announce("499^3 qHOP M=3: sampled max err %.2e, rel err vs exact %.4e (printed %.3e)" % (err, rel_err, printed))
    assert err <= 1e-11
    assert abs(rel_err - printed) / printed < 0.05
