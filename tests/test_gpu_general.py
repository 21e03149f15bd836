"""Generic per-axis operators on the GPU (ts_setup_general), with Hermite
spectral collocation (Appendix app:hermite) as the main case.

* Applies (inverse, shifted inverse, propagator; FP64, FP32, BF16) against the
  oracle's generic plan built from the same K, m and f (the oracle's Hermite
  construction feeds both sides).
* A generic plan from the FD operator against the oracle's FD plan.
* Operator apply with a dense K (band of half-width n - 1), PCG in the mass
  inner product, one step of each GPE flow.
* Reflection-symmetric Hermite axes fold; folded and plain passes agree.
* Rejections: K not self-adjoint in m; interpolation of a plan with no interval.
* Full size: Table tab:hermite_accuracy (n = 199, 399, 599) with the library's
  own ts_hermite_axis, against both printed error columns.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, exp_tol, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def hermite_pair(shape, seed=0, symmetric=False, sigma=0.5):
    """Library and oracle plans of sum_a (-d^2/dx_a^2 + f_a) on Hermite nodes."""
    rng = np.random.default_rng(seed)
    axes = [oracle.hermite_axis(n) for n in shape]
    if symmetric:
        # the oracle's nodes (eigvalsh) are symmetric only to rounding: reflect-average
        # the axis data so that it qualifies for the half-extent passes
        axes = [(0.5 * (x - x[::-1]), 0.5 * (m + m[::-1]), 0.5 * (K + K[::-1, ::-1])) for x, m, K in axes]
        fs = [x * x + 0.5 * np.cos(2 * x) for x, _, _ in axes]
    else:
        fs = [x * x + rng.uniform(0, 1, x.size) for x, _, _ in axes]
    Ks = [K for _, _, K in axes]
    ms = [m for _, m, _ in axes]
    xs = [x for x, _, _ in axes]
    return (ts.ts_setup_general(Ks, ms, fs, sigma, xs), oracle.make_plan_general(Ks, ms, fs, xs))


@pytest.mark.parametrize("shape", [(20, 24, 18), (33, 40), (12, 10, 9, 11), (70,)])
def test_hermite_applies_match_oracle(shape):
    plan, oplan = hermite_pair(shape, seed=1)
    b = W.rhs_normal(shape, 2)
    psi = W.complex_normal(shape, 3)
    tau = 0.02
    e_inv = rel(to_host(ts.ts_apply_inverse(plan, to_dev(b))), oracle.apply_inverse(oplan, b, 0.5))
    e_sh = rel(to_host(ts.ts_apply_inverse_shift(plan, 1.5, to_dev(b))), oracle.apply_inverse(oplan, b, 1.5))
    e_exp = rel(to_host(ts.ts_apply_exp(plan, tau, to_dev(psi))), oracle.apply_exp(oplan, psi, tau))
    ref = oracle.apply_inverse(oplan, b, 0.5)
    e32 = rel(to_host(ts.ts_apply_inverse(plan, to_dev(b).float(), prec="fp32")).astype(np.float64), ref)
    e16 = rel(to_host(ts.ts_apply_inverse(plan, to_dev(b).float(), prec="bf16")).astype(np.float64), ref)
    announce("hermite %s: inv %.2e shift %.2e exp %.2e (tol %.1e) fp32 %.2e bf16 %.2e"
             % (shape, e_inv, e_sh, e_exp, exp_tol(oplan, tau), e32, e16))
    assert e_inv <= 1e-12 and e_sh <= 1e-12
    assert e_exp <= exp_tol(oplan, tau)
    assert e32 <= 2e-5 and e16 <= 1.5e-2   # BF16 measured 3.3e-3 .. 4.6e-3


def test_generic_fd_operator_matches_fd_oracle():
    shape, L = (30, 26, 35), 4.0
    f = [W.f_harmonic(n, L) for n in shape]
    Ks = [oracle.fd_axis_matrix(n, L, np.zeros(n)) for n in shape]
    ms = [np.full(n, 2 * L / (n + 1)) for n in shape]
    plan = ts.ts_setup_general(Ks, ms, f, 1.0)
    assert ts.ts_fold_axes(plan) == 0  # all n < 64
    oplan = oracle.make_plan(shape, L, f)
    b = W.rhs_normal(shape, 4)
    assert rel(to_host(ts.ts_apply_inverse(plan, to_dev(b))), oracle.apply_inverse(oplan, b, 1.0)) <= 1e-12
    V2 = W.rhs_normal(shape, 5) ** 2
    got = to_host(ts.ts_operator_apply(plan, to_dev(V2), 1.0, to_dev(b)))
    assert rel(got, oracle.stencil_apply(oplan, b, V2, 1.0)) <= 1e-13
    np.testing.assert_allclose(ts.ts_mass(plan, 1), ms[1], rtol=0, atol=0)


def test_hermite_operator_pcg_and_gpe_step():
    shape = (18, 22, 20)
    plan, oplan = hermite_pair(shape, seed=6, sigma=1.0)
    V2 = 3.0 * W.rhs_normal(shape, 7) ** 2
    u = W.rhs_normal(shape, 8)
    got = to_host(ts.ts_operator_apply(plan, to_dev(V2), 0.25, to_dev(u)))
    assert rel(got, oracle.operator_apply(oplan, u, V2, 0.25)) <= 1e-13
    rhs = W.rhs_normal(shape, 9)
    ref = oracle.pcg(oplan, V2, 1.0, rhs, rtol=1e-13)
    for prec in ("fp64", "fp32", "bf16"):
        x = torch.zeros(shape, dtype=torch.float64, device=DEV)
        _, its, rr, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(rhs), x, rtol=1e-10, maxit=300, precond=prec)
        xh = to_host(x)
        true = oracle.norm(oplan, rhs - oracle.operator_apply(oplan, xh, V2, 1.0)) / oracle.norm(oplan, rhs)
        announce("hermite pcg %s: %d its, relres %.2e, true %.2e, err %.2e" % (prec, its, rr, true, rel(xh, ref.x)))
        assert true <= 2e-10 and rel(xh, ref.x) <= 1e-8
    # one modified H^1 flow step (-Delta plan: f = 0) against the oracle's step
    axes = [oracle.hermite_axis(n) for n in shape]
    zeros = [np.zeros(n) for n in shape]
    lap = ts.ts_setup_general([a[2] for a in axes], [a[1] for a in axes], zeros, 1.0)
    olap = oracle.make_plan_general([a[2] for a in axes], [a[1] for a in axes], zeros)
    V = sum(np.reshape(a[0] ** 2, [-1 if i == k else 1 for i in range(3)]) for k, a in enumerate(axes))
    V = np.ascontiguousarray(np.broadcast_to(V, shape))
    w = oracle.l2_weights(olap)
    u0 = np.abs(W.rhs_normal(shape, 10)) + 0.1
    u0 = u0 / np.sqrt(np.sum(w * u0 * u0))
    ref = oracle.h1_flow_step(olap, V, 50.0, 10.0, 0.1, u0)
    ud = to_dev(u0)
    r = ts.ts_gpe_h1_flow(lap, to_dev(V), 50.0, ud, alpha=10.0, tau=0.1, maxit=1, tol=0.0, raise_on_noconv=False)
    assert r.iters == 1
    assert rel(to_host(ud), ref) <= 1e-12


@pytest.mark.parametrize("shape", [(70,), (40, 90), (36, 50, 41)])
def test_hermite_dense_operator_and_pcg(shape):
    """Hermite axes with n > 33: the operator apply runs as per-axis FP64 MFMA
    passes plus a combine kernel (the band would be n - 1 wide); both the
    public operator and PCG (symmetric form) against the oracle."""
    plan, oplan = hermite_pair(shape, seed=13, sigma=1.0)
    V2 = 2.0 * W.rhs_normal(shape, 14) ** 2
    u = W.rhs_normal(shape, 15)
    got = to_host(ts.ts_operator_apply(plan, to_dev(V2), 0.25, to_dev(u)))
    e_op = rel(got, oracle.operator_apply(oplan, u, V2, 0.25))
    got0 = to_host(ts.ts_operator_apply(plan, None, 0.0, to_dev(u)))
    e_op0 = rel(got0, oracle.operator_apply(oplan, u, None, 0.0))
    rhs = W.rhs_normal(shape, 16)
    ref = oracle.pcg(oplan, V2, 1.0, rhs, rtol=1e-13)
    x = torch.zeros(shape, dtype=torch.float64, device=DEV)
    _, its, rr, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(rhs), x, rtol=1e-10, maxit=300)
    xh = to_host(x)
    true = oracle.norm(oplan, rhs - oracle.operator_apply(oplan, xh, V2, 1.0)) / oracle.norm(oplan, rhs)
    announce("hermite dense %s: operator %.2e / %.2e, pcg %d its relres %.2e true %.2e err %.2e"
             % (shape, e_op, e_op0, its, rr, true, rel(xh, ref.x)))
    assert e_op <= 1e-13 and e_op0 <= 1e-13
    assert true <= 2e-10 and rel(xh, ref.x) <= 1e-8


def test_hermite_dense_gpe_steps():
    """One step of each GPE flow on Hermite axes with n > 33 (E'(u) from the
    dense operator passes) against the oracle's steps."""
    shape = (36, 40, 34)
    axes = [oracle.hermite_axis(n) for n in shape]
    Ks, ms, xs = [a[2] for a in axes], [a[1] for a in axes], [a[0] for a in axes]
    zeros = [np.zeros(n) for n in shape]
    v = [x * x for x in xs]
    lap = ts.ts_setup_general(Ks, ms, zeros, 1.0, xs)
    pv1 = ts.ts_setup_general(Ks, ms, v, 1.0, xs)
    olap = oracle.make_plan_general(Ks, ms, zeros, xs)
    opv1 = oracle.make_plan_general(Ks, ms, v, xs)
    V = np.ascontiguousarray(v[0][:, None, None] + v[1][None, :, None] + v[2][None, None, :])
    w = oracle.l2_weights(olap)
    u0 = oracle.separable_ground_state(opv1) * (1.0 + 0.2 * np.cos(W.outer(xs)))
    u0 = u0 / np.sqrt(np.sum(w * u0 * u0))
    ref = oracle.h1_flow_step(olap, V, 80.0, 10.0, 0.1, u0)
    ud = to_dev(u0)
    r = ts.ts_gpe_h1_flow(lap, to_dev(V), 80.0, ud, alpha=10.0, tau=0.1, maxit=1, tol=0.0, raise_on_noconv=False)
    e_h1 = rel(to_host(ud), ref)
    ref_a, _ = oracle.au_flow_step(opv1, None, 80.0, 1.0, u0)
    ud = to_dev(u0)
    ts.ts_gpe_au_flow(pv1, None, 80.0, ud, tau=1.0, maxit=1, tol=0.0, pcg_rtol=1e-13, raise_on_noconv=False)
    e_au = rel(to_host(ud), ref_a)
    announce("hermite dense gpe: h1 step %.2e, au step %.2e, E %.10f" % (e_h1, e_au, r.energy))
    assert r.iters == 1 and e_h1 <= 1e-12 and e_au <= 1e-10


def test_symmetric_hermite_axes_fold():
    shape = (80, 66, 30)
    plan, oplan = hermite_pair(shape, symmetric=True)
    assert ts.ts_fold_axes(plan) == 3
    b = W.rhs_normal(shape, 11)
    psi = W.complex_normal(shape, 12)
    out = {}
    for fold in (True, False):
        ts.ts_set_fold(plan, fold)
        out[fold] = (to_host(ts.ts_apply_inverse(plan, to_dev(b))), to_host(ts.ts_apply_exp(plan, 0.01, to_dev(psi))))
    assert rel(out[True][0], out[False][0]) <= 1e-13 and rel(out[True][1], out[False][1]) <= 1e-13
    assert rel(out[True][0], oracle.apply_inverse(oplan, b, 0.5)) <= 1e-12
    assert rel(out[True][1], oracle.apply_exp(oplan, psi, 0.01)) <= exp_tol(oplan, 0.01)


def test_rejections():
    x, m, K = oracle.hermite_axis(12)
    with pytest.raises(ts.TSError) as e:
        ts.ts_setup_general([K], [None], [x * x], 1.0)  # K is self-adjoint in m, not in unit weights
    assert e.value.code == ts.TS_ERR_INVALID
    with pytest.raises(ts.TSError):
        ts.ts_setup_general([K + np.triu(np.ones_like(K), 1)], [m], [x * x], 1.0)
    g = ts.ts_setup_general([K], [m], [x * x], 1.0)
    fd = ts.ts_setup((12,), 3.0, [np.zeros(12)], 1.0)
    with pytest.raises(ts.TSError):
        ts.ts_interpolate(g, fd, torch.zeros(12, dtype=torch.float64, device=DEV))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("row", [0, 1, 2])
def test_printed_hermite_accuracy(row):
    g = GOLDEN["hermite_accuracy"]["rows"][row]
    n = g["n"]
    announce("hermite accuracy: setup n = %d" % n)
    x, m, K = ts.ts_hermite_axis(n)
    coef = (3.0, 2.0, 1.0)  # axis 0 = z, 1 = y, 2 = x
    cs = (1.5 * np.pi, np.pi, 0.5 * np.pi)
    fs = [W.f_test_potential(0, 0.0, c, x=x) for c in coef]
    plan = ts.ts_setup_general([K] * 3, [m] * 3, fs, 0.0, [x] * 3)
    G = [W.rational_sine(c, x) for c in cs]
    gd = [to_dev(gg) for gg, _ in G]
    rhs = torch.zeros((n,) * 3, dtype=torch.float64, device=DEV)
    for a in range(3):
        fac = list(gd)
        fac[a] = to_dev(-G[a][1] + fs[a] * G[a][0])
        rhs += fac[0][:, None, None] * fac[1][None, :, None] * fac[2][None, None, :]
    ustar = gd[0][:, None, None] * gd[1][None, :, None] * gd[2][None, None, :]
    u = ts.ts_apply_inverse(plan, rhs)
    e = u - ustar
    l2 = float(torch.linalg.norm(e) / torch.linalg.norm(ustar))
    wgh = to_dev(m * np.exp(-x * x))  # the Gauss-Hermite weights of e^{-x^2}
    w3 = wgh[:, None, None] * wgh[None, :, None] * wgh[None, None, :]
    weighted = float(torch.sqrt(torch.sum(w3 * e * e)))
    announce("hermite n=%d: l2 rel %.3e (printed %.2e), weighted %.3e (printed %.2e)"
             % (n, l2, g["l2_rel"], weighted, g["weighted_l2"]))
    # the printed three digits: within one unit of the last one
    assert abs(l2 - g["l2_rel"]) <= 0.01 * g["l2_rel"]
    assert abs(weighted - g["weighted_l2"]) <= 0.01 * g["weighted_l2"]
