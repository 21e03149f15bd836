"""Parity of the HIP separable apply (inverse and propagator) with the oracle.

FP64 bar: ||x_gpu - x_oracle||_2 / ||x_oracle||_2 <= 1e-12 (the tolerance of
the FP64 path); for the propagator at large tau ||H1|| the bar widens to the
conditioning bound of ``gpu_common.exp_tol``.  Shapes span several 128-wide MFMA tiles with ragged tails,
1 to 9 axes, extents of 1, and the 64^3 workload (L = 8, f = x^2, sigma = 1,
N(0,1) right-hand side from seed 1, complex128 Gaussian wavepacket, tau = 0.01).
FP32 results are compared at the FP32 rounding level (error reported).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, exp_tol, inv_tol, make_pair, maxrel, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [
    (64, 64, 64),
    (130, 70, 150),
    (257, 129),
    (1000,),
    (20, 17, 24, 19),
    (7, 6, 5, 8, 4, 6),
    (1, 5, 1, 7),
    (3, 3, 3, 3, 3, 3, 3, 3, 3),
    (200, 144, 176),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_inverse_fp64_parity(shape):
    announce("inverse fp64 %s" % (shape,))
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 1)
    u = to_host(ts.ts_apply_inverse(plan, to_dev(b)))
    ref = oracle.apply_inverse(oplan, b, 1.0)
    e, em = rel(u, ref), maxrel(u, ref)
    announce("  rel err %.3e, max-norm rel err %.3e" % (e, em))
    assert e <= 1e-12 and em <= 1e-12


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("tau", [0.01, -0.3])
def test_exp_fp64_parity(shape, tau):
    announce("exp fp64 %s tau=%g" % (shape, tau))
    plan, oplan, _ = make_pair(shape, 8.0, "cos", sigma=1.0)
    psi = W.complex_normal(shape, 2)
    out = to_host(ts.ts_apply_exp(plan, tau, to_dev(psi)))
    ref = oracle.apply_exp(oplan, psi, tau)
    e, em = rel(out, ref), maxrel(out, ref)
    tol = exp_tol(oplan, tau)
    announce("  rel err %.3e, max-norm rel err %.3e (tol %.1e)" % (e, em, tol))
    assert e <= tol and em <= tol


def test_config0_workload_inverse_and_exp():
    """64^3 on [-8,8]^3, f = x^2, sigma = 1: N(0,1) RHS (seed 1) and wavepacket (tau = 0.01)."""
    shape, L = (64, 64, 64), 8.0
    plan, oplan, _ = make_pair(shape, L, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 1)
    assert rel(to_host(ts.ts_apply_inverse(plan, to_dev(b))), oracle.apply_inverse(oplan, b, 1.0)) <= 1e-12
    psi = W.gaussian_wavepacket(shape, L, 1)
    out = to_host(ts.ts_apply_exp(plan, 0.01, to_dev(psi)))
    assert rel(out, oracle.apply_exp(oplan, psi, 0.01)) <= 1e-12
    assert abs(np.linalg.norm(out) - 1.0) <= 1e-13


def test_in_place_and_tau_zero():
    shape = (33, 65, 17)
    plan, oplan, _ = make_pair(shape, 5.0, "rand", sigma=0.5, seed=3)
    b = W.rhs_normal(shape, 4)
    t = to_dev(b)
    ts.ts_apply_inverse(plan, t, t)
    assert rel(to_host(t), oracle.apply_inverse(oplan, b, 0.5)) <= 1e-12
    psi = W.complex_normal(shape, 5)
    tp = to_dev(psi)
    ts.ts_apply_exp(plan, 0.0, tp, tp)
    assert rel(to_host(tp), psi) <= 1e-13


def test_shifted_inverse_and_not_spd():
    shape = (40, 30, 20)
    plan, oplan, _ = make_pair(shape, 6.0, "harm", sigma=1.0)
    lam1 = sum(ts.ts_eigvals(plan, k)[0] for k in range(3))
    s = -(lam1 - 1e-3)  # denominators as small as 1e-3: formed in FP64
    b = W.rhs_normal(shape, 6)
    u = to_host(ts.ts_apply_inverse_shift(plan, s, to_dev(b)))
    e, tol = rel(u, oracle.apply_inverse(oplan, b, s)), inv_tol(oplan, s)
    announce("shifted inverse rel err %.3e (tol %.1e)" % (e, tol))
    assert e <= tol
    with pytest.raises(ts.TSError) as e:
        ts.ts_apply_inverse_shift(plan, -lam1 - 1.0, to_dev(b))
    assert e.value.code == ts.TS_ERR_NOT_SPD


@pytest.mark.parametrize("shape", [(64, 64, 64), (130, 70, 150), (20, 17, 24, 19)])
def test_fp32_transforms(shape):
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 7)
    ref = oracle.apply_inverse(oplan, b, 1.0)
    for dt in (torch.float64, torch.float32):
        u = to_host(ts.ts_apply_inverse(plan, to_dev(b).to(dt), prec="fp32")).astype(np.float64)
        e = rel(u, ref)
        announce("fp32 inverse %s in=%s rel err %.3e" % (shape, dt, e))
        assert e <= 2e-6
    psi = W.complex_normal(shape, 8)
    refp = oracle.apply_exp(oplan, psi, 0.01)
    for dt in (torch.complex128, torch.complex64):
        out = to_host(ts.ts_apply_exp(plan, 0.01, to_dev(psi).to(dt), prec="fp32")).astype(np.complex128)
        e = rel(out, refp)
        announce("fp32 exp %s in=%s rel err %.3e" % (shape, dt, e))
        assert e <= 2e-6


def test_operator_matches_oracle_stencil():
    shape = (31, 40, 27)
    plan, oplan, _ = make_pair(shape, 4.0, "rand", sigma=0.0, seed=9)
    u = W.rhs_normal(shape, 10)
    V2 = W.gaussian_bumps(shape, 4.0, 5, seed=11)
    out = to_host(ts.ts_operator_apply(plan, to_dev(V2), 0.75, to_dev(u)))
    ref = oracle.stencil_apply(oplan, u, V2, 0.75)
    assert rel(out, ref) <= 1e-14
    out0 = to_host(ts.ts_operator_apply(plan, None, 0.0, to_dev(u)))
    assert rel(out0, oracle.stencil_apply(oplan, u, None, 0.0)) <= 1e-14


def test_eigvals_match_oracle():
    shape = (50, 37)
    plan, oplan, _ = make_pair(shape, 8.0, "cos", sigma=1.0)
    for k in range(2):
        lam = ts.ts_eigvals(plan, k)
        assert np.max(np.abs(lam - oplan.lam[k])) <= 1e-13 * np.abs(lam).max()
        Q = ts.ts_eigvecs(plan, k)
        assert np.max(np.abs(Q.T @ Q - np.eye(shape[k]))) <= 1e-13


@pytest.mark.parametrize("shape", [(64, 64, 64), (130, 70, 150), (20, 40, 24, 19), (257, 129), (96, 64, 128)])
def test_bf16_transforms_error_reported(shape):
    """BF16 operands, FP32 accumulation: no exact value exists (parity unpinned);
    the error against the FP64 oracle is reported and must sit at the BF16
    rounding level (the paper's BF16 rows show 1.6e-2)."""
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 7)
    ref = oracle.apply_inverse(oplan, b, 1.0)
    for dt in (torch.float64, torch.float32):
        u = to_host(ts.ts_apply_inverse(plan, to_dev(b).to(dt), prec="bf16")).astype(np.float64)
        e, em = rel(u, ref), maxrel(u, ref)
        announce("bf16 inverse %s in=%s rel err %.3e, max-norm %.3e" % (shape, dt, e, em))
        # measured 4.8e-3 .. 7.2e-3: BF16 operands through 2d passes; the max-norm bar
        # catches a few corrupted outputs that the 2-norm would average away
        assert 1e-3 < e <= 1.5e-2 and em <= 5e-2
    psi = W.complex_normal(shape, 8)
    refp = oracle.apply_exp(oplan, psi, 0.01)
    for dt in (torch.complex128, torch.complex64):
        out = to_host(ts.ts_apply_exp(plan, 0.01, to_dev(psi).to(dt), prec="bf16")).astype(np.complex128)
        e, em = rel(out, refp), maxrel(out, refp)
        announce("bf16 exp %s in=%s rel err %.3e, max-norm %.3e" % (shape, dt, e, em))
        assert 1e-3 < e <= 1.5e-2 and em <= 5e-2


@pytest.mark.parametrize("shape", [(100, 99, 128), (99, 101, 7), (64, 96)])
def test_bf16_input_rounding_sweep_and_in_place(shape):
    """BF16 applies of FP64 data round the input to BF16 in one sweep into the
    output buffer when input and output differ (and N % 4 == 0); in place, or
    for other N, the first pass rounds while loading, the same way (FP64 ->
    FP32 -> BF16).  Both forms sit at the BF16 level against the oracle and are
    bitwise equal; the out-of-place form leaves its input unchanged."""
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 9)
    ref = oracle.apply_inverse(oplan, b, 1.0)
    bd = to_dev(b)
    u_out = to_host(ts.ts_apply_inverse(plan, bd, prec="bf16"))
    assert np.array_equal(to_host(bd), b)
    ts.ts_apply_inverse(plan, bd, bd, prec="bf16")
    u_in = to_host(bd)
    e_out, e_in, e_pair = rel(u_out, ref), rel(u_in, ref), rel(u_out, u_in)
    announce("bf16 inverse %s: out of place %.3e, in place %.3e, between %.3e" % (shape, e_out, e_in, e_pair))
    assert e_out <= 1.5e-2 and e_in <= 1.5e-2
    assert np.array_equal(u_out, u_in)
    psi = W.complex_normal(shape, 10)
    refp = oracle.apply_exp(oplan, psi, 0.01)
    pd = to_dev(psi)
    o = to_host(ts.ts_apply_exp(plan, 0.01, pd, prec="bf16"))
    assert np.array_equal(to_host(pd), psi)
    assert rel(o, refp) <= 1.5e-2


@pytest.mark.parametrize("n", [100, 257, 1000])
def test_bf16_factor_copies_are_rne_of_fp64(n):
    """The BF16 factor copies are FP64 Q rounded once to nearest even: a BF16
    pass over the identity (FP32 data, FP32 accumulation of one product)
    returns the BF16 factor entries exactly, which must equal the host
    rounding of ts_eigvecs bit for bit (route 0 of ts_bf16_round, itself
    checked against exact RNE on the CPU)."""
    rng = np.random.default_rng(n)
    f = [rng.uniform(0.0, 3.0, n), rng.uniform(0.0, 3.0, n)]   # not symmetric: natural order, no fold
    plan = ts.ts_setup((n, n), 4.0, f, 1.0)
    assert ts.ts_fold_axes(plan) == 0
    eye = torch.eye(n, dtype=torch.float32, device=DEV)
    for axis in (0, 1):
        Q = ts.ts_eigvecs(plan, axis)
        want = ts.ts_bf16_round(Q, 0).reshape(n, n)
        for forward in (True, False):
            y = to_host(ts.ts_mode_pass(plan, axis, forward, eye, prec="bf16"))
            # axis 0: forward gives Q^T, backward Q; axis 1: forward Q, backward Q^T
            transposed = (axis == 0) == forward
            got = (y.T if transposed else y).copy().view(np.uint32) >> 16
            assert np.all((y.view(np.uint32) & 0xffff) == 0)
            bad = int(np.count_nonzero(got.astype(np.uint16) != want))
            announce("bf16 factor copy n=%d axis %d forward %s: %d of %d entries differ" % (n, axis, forward, bad, n * n))
            assert bad == 0


@pytest.mark.parametrize("shape", [(64, 64, 64), (130, 70, 150), (20, 17, 24, 19), (12, 10, 11, 9, 8, 7)])
def test_fp32_data_fp64_transforms(shape):
    """FP32 / complex64 data with FP64 transforms (FP64 factors and arithmetic
    inside each pass, FP32 between passes): the error against the oracle is
    the FP32 rounding of the data (a few 1e-8 per pass), well below the FP32
    transforms' error."""
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 7)
    ref = oracle.apply_inverse(oplan, b, 1.0)
    u = to_host(ts.ts_apply_inverse(plan, to_dev(b).float(), prec="fp64")).astype(np.float64)
    e = rel(u, ref)
    psi = W.complex_normal(shape, 8)
    refp = oracle.apply_exp(oplan, psi, 0.01)
    out = to_host(ts.ts_apply_exp(plan, 0.01, to_dev(psi).to(torch.complex64), prec="fp64")).astype(np.complex128)
    ep = rel(out, refp)
    announce("fp32 data, fp64 transforms %s: inverse %.2e, exp %.2e" % (shape, e, ep))
    assert e <= 5e-7 and ep <= 5e-7


@pytest.mark.parametrize("shape", [(1000,), (70, 90), (31, 40, 27), (33, 25, 128, 64), (6, 5, 7, 4, 3),
                                   (16, 16, 16, 16, 16, 16)])
def test_operator_matches_oracle_stencil_any_d(shape):
    """The tiled operator kernel on 1D-6D grids, including grids where one
    block marches through several planes across the ends of the slower axes
    (33 x 25 x 128 x 64: three planes per block along an axis of 25; 16^6:
    32 planes per block along an axis of 16)."""
    L = 5.0
    rng = np.random.default_rng(21)
    f = [rng.uniform(0.0, 5.0, size=n) for n in shape]
    plan = ts.ts_setup(shape, L, f, 0.0)
    oplan = oracle.Plan(shape=shape, L=L, f=f, h=[oracle.grid_spacing(n, L) for n in shape])
    u = W.rhs_normal(shape, 22)
    V2 = W.gaussian_bumps(shape, L, 3, seed=23)
    out = to_host(ts.ts_operator_apply(plan, to_dev(V2), 0.5, to_dev(u)))
    ref = oracle.stencil_apply(oplan, u, V2, 0.5)
    e, em = rel(out, ref), maxrel(out, ref)
    announce("operator %s vs oracle stencil: %.2e (max-norm %.2e)" % (shape, e, em))
    assert e <= 1e-14 and em <= 1e-14
