"""Half-extent passes on reflection-symmetric axes (ts_set_fold): with f_k
symmetric every eigenvector is even or odd and the passes contract half the
extent.  The folded and plain passes must agree to rounding, and both must
match the oracle; axes with non-symmetric f_k, or n_k < 64, are not folded.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, exp_tol, make_pair, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(64,), (65,), (200,), (128, 96), (97, 64), (100, 99, 130), (64, 65, 66, 67), (33, 130, 80)]


@pytest.mark.parametrize("shape", SHAPES)
def test_fold_matches_plain_and_oracle(shape):
    plan, oplan, f = make_pair(shape, 6.0, "cos", sigma=1.0)  # x^2 + 0.5 cos 2x: symmetric
    mask = ts.ts_fold_axes(plan)
    expect = sum(1 << k for k, n in enumerate(shape) if n >= 64)
    assert mask == expect, (mask, expect)
    b = W.rhs_normal(shape, 1)
    psi = W.complex_normal(shape, 2)
    out = {}
    for fold in (True, False):
        ts.ts_set_fold(plan, fold)
        out[fold] = (to_host(ts.ts_apply_inverse(plan, to_dev(b))),
                     to_host(ts.ts_apply_inverse_shift(plan, 2.5, to_dev(b))),
                     to_host(ts.ts_apply_exp(plan, 0.05, to_dev(psi))),
                     to_host(ts.ts_apply_inverse(plan, to_dev(b).float(), prec="fp32")).astype(np.float64),
                     to_host(ts.ts_apply_exp(plan, 0.05, to_dev(psi).to(torch.complex64), prec="fp32")),
                     to_host(ts.ts_apply_inverse(plan, to_dev(b).float(), prec="bf16")).astype(np.float64),
                     to_host(ts.ts_apply_exp(plan, 0.05, to_dev(psi).to(torch.complex64), prec="bf16")))
    refs = (oracle.apply_inverse(oplan, b, 1.0), oracle.apply_inverse(oplan, b, 2.5), oracle.apply_exp(oplan, psi, 0.05))
    d = [rel(a, c) for a, c in zip(out[True], out[False])]
    e = [rel(out[True][i], refs[i]) for i in range(3)]
    e32 = rel(out[True][3], refs[0])
    e64c = rel(out[True][4].astype(np.complex128), refs[2])
    # BF16 transforms: both variants at the BF16 rounding level of the oracle
    e16 = [rel(out[fold][5], refs[0]) for fold in (True, False)]
    e16c = [rel(out[fold][6].astype(np.complex128), refs[2]) for fold in (True, False)]
    announce("fold %s mask %d: fold vs plain %s; vs oracle %s; fp32 %.2e c64 %.2e; bf16 fold/plain %s, c64 %s"
             % (shape, mask, ["%.1e" % x for x in d], ["%.1e" % x for x in e], e32, e64c,
                ["%.2e" % x for x in e16], ["%.2e" % x for x in e16c]))
    assert max(d[:3]) <= 1e-13 and max(d[3:5]) <= 2e-6
    assert e[0] <= 1e-12 and e[1] <= 1e-12 and e[2] <= exp_tol(oplan, 0.05)
    assert e32 <= 2e-6 and e64c <= 2e-6
    # (the two variants round different quantities, so their errors are two samples
    # of the BF16 rounding noise; in 1D a few low modes dominate and the ratio varies)
    assert max(e16 + e16c) <= 1.5e-2   # measured 2.9e-3 .. 7.5e-3


def test_non_symmetric_axes_are_not_folded():
    shape = (80, 70)
    plan, oplan, f = make_pair(shape, 6.0, "rand", sigma=1.0)
    assert ts.ts_fold_axes(plan) == 0
    shape = (80, 70)
    rng = np.random.default_rng(0)
    fs = [W.f_harmonic(80, 6.0), rng.uniform(0, 2, 70)]
    plan = ts.ts_setup(shape, 6.0, fs, 1.0)
    assert ts.ts_fold_axes(plan) == 1
    oplan = oracle.make_plan(shape, 6.0, fs)
    b = W.rhs_normal(shape, 3)
    assert rel(to_host(ts.ts_apply_inverse(plan, to_dev(b))), oracle.apply_inverse(oplan, b, 1.0)) <= 1e-12


def test_fold_in_solvers_and_sem():
    """PCG with a folded preconditioner, and a symmetric SEM plan (mass-scaled factors)."""
    shape, L = (96, 80, 72), 8.0
    plan, oplan, f = make_pair(shape, L, "harm", sigma=1.0)
    assert ts.ts_fold_axes(plan) == 7
    V2 = W.gaussian_bumps(shape, L, 4, seed=5)
    V2 = V2 - min(0.0, V2.min())
    rhs = W.rhs_normal(shape, 6)
    u = torch.zeros(shape, dtype=torch.float64, device=DEV)
    _, its, rr, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(rhs), u, rtol=1e-10, maxit=200)
    true = np.linalg.norm(rhs - oracle.stencil_apply(oplan, to_host(u), V2, 1.0)) / np.linalg.norm(rhs)
    assert true <= 2e-10
    k, cells = 4, (20, 18)
    fs = [W.f_harmonic(0, L, x=ts.ts_sem_nodes(k, c, L)) for c in cells]
    sp = ts.ts_setup_sem(k, cells, L, fs, 1.0)
    assert ts.ts_fold_axes(sp) == 3
    osp = oracle.make_plan_sem(k, cells, L, fs)
    b = W.rhs_normal(sp.shape, 7)
    assert rel(to_host(ts.ts_apply_inverse(sp, to_dev(b))), oracle.apply_inverse(osp, b, 1.0)) <= 1e-12
    u16 = to_host(ts.ts_apply_inverse(sp, to_dev(b).float(), prec="bf16")).astype(np.float64)
    assert rel(u16, oracle.apply_inverse(osp, b, 1.0)) <= 1.5e-2


@pytest.mark.parametrize("shape", [(100, 99, 130), (70, 81)])
def test_single_pass_round_trip(shape):
    """ts_mode_pass: backward after forward is the identity on every axis,
    folded or not, and the folded forward pass equals the plain one."""
    plan, _, _ = make_pair(shape, 6.0, "cos", sigma=1.0)
    x = to_dev(W.rhs_normal(shape, 4))
    for axis in range(len(shape)):
        y = ts.ts_mode_pass(plan, axis, True, x)
        z = ts.ts_mode_pass(plan, axis, False, y)
        assert rel(to_host(z), to_host(x)) <= 1e-13
        ts.ts_set_fold(plan, False)
        y0 = ts.ts_mode_pass(plan, axis, True, x)
        ts.ts_set_fold(plan, True)
        assert rel(to_host(y), to_host(y0)) <= 1e-14


@pytest.mark.parametrize("shape", [(100, 99, 130), (70, 81), (64, 96)])
def test_single_pass_bf16_fold(shape):
    """BF16 single passes (FP64 data in and out), folded and plain, against the
    FP64 pass: relative error at the BF16 rounding level on every axis and
    direction; the folded BF16 backward pass includes the butterfly."""
    plan, _, _ = make_pair(shape, 6.0, "cos", sigma=1.0)
    x = to_dev(W.rhs_normal(shape, 5))
    for axis in range(len(shape)):
        for fwd in (True, False):
            ref = to_host(ts.ts_mode_pass(plan, axis, fwd, x))
            errs = []
            for fold in (True, False):
                ts.ts_set_fold(plan, fold)
                errs.append(rel(to_host(ts.ts_mode_pass(plan, axis, fwd, x, prec="bf16")), ref))
            ts.ts_set_fold(plan, True)
            announce("bf16 pass %s axis %d %s: fold %.2e plain %.2e"
                     % (shape, axis, "fwd" if fwd else "bwd", errs[0], errs[1]))
            assert max(errs) <= 5e-3   # measured 2.2e-3 .. 2.4e-3


def _butterfly_ref(x, axes):
    """out_i = x_i + x_{n-1-i}, out_{n-1-i} = x_i - x_{n-1-i} (i < n // 2) per axis."""
    y = x.copy()
    for a in axes:
        n, h = y.shape[a], y.shape[a] // 2
        yf = np.flip(y, a)
        idx = np.arange(n).reshape([-1 if k == a else 1 for k in range(y.ndim)])
        y = np.where(idx < h, y + yf, np.where(idx >= n - h, yf - y, y))
    return y


@pytest.mark.parametrize("shape,mask", [((100, 99, 130), 7), ((70, 81), 2), ((12, 13, 10, 11, 9), 31),
                                        ((33, 130, 80), 5), ((7, 64, 5, 3), 11), ((64, 66, 100), 7),
                                        ((20, 12), 2), ((9, 7, 5, 3, 8), 31), ((50, 1000), 3)])
def test_fold_butterfly(shape, mask):
    """ts_fold_butterfly against the per-axis definition: out of place, in place,
    complex and FP32 data, up to five axes (two sweeps); real data whose
    fastest axis folds with n % 4 == 0 move in pairs (the mirror pair swapped),
    complex data one element per access."""
    plan = ts.ts_setup(shape, 6.0, [W.f_harmonic(n, 6.0) for n in shape], 1.0)
    axes = [k for k in range(len(shape)) if mask >> k & 1]
    x = W.rhs_normal(shape, 8)
    ref = _butterfly_ref(x, axes)
    assert rel(to_host(ts.ts_fold_butterfly(plan, mask, to_dev(x))), ref) <= 1e-15
    xd = to_dev(x)
    ts.ts_fold_butterfly(plan, mask, xd, xd)
    assert rel(to_host(xd), ref) <= 1e-15
    # twice: 2x per axis, except on the middle row of an odd extent (copied)
    ts.ts_fold_butterfly(plan, mask, xd, xd)
    scale = np.ones(shape)
    for a in axes:
        w = np.full(shape[a], 2.0)
        if shape[a] % 2:
            w[shape[a] // 2] = 1.0
        scale = scale * w.reshape([-1 if k == a else 1 for k in range(len(shape))])
    assert rel(to_host(xd), scale * x) <= 1e-15
    psi = W.complex_normal(shape, 9)
    refc = _butterfly_ref(psi, axes)
    assert rel(to_host(ts.ts_fold_butterfly(plan, mask, to_dev(psi))), refc) <= 1e-15
    got32 = to_host(ts.ts_fold_butterfly(plan, mask, to_dev(psi).to(torch.complex64)))
    assert rel(got32.astype(np.complex128), refc) <= 1e-6
    got32 = to_host(ts.ts_fold_butterfly(plan, mask, to_dev(x).float()))
    assert rel(got32.astype(np.float64), ref) <= 1e-6
    with pytest.raises(ts.TSError):
        ts.ts_fold_butterfly(plan, 1 << len(shape), to_dev(x))
    with pytest.raises(ts.TSError):
        ts.ts_fold_butterfly(plan, 0, to_dev(x))


@pytest.mark.parametrize("shape", [(100, 99, 130), (70, 81), (65, 64)])
def test_single_pass_on_folded_data(shape):
    """ts_mode_pass modes 2 and 3 (the passes inside an apply with several
    folded axes): the forward pass on butterflied input equals the forward pass
    on the input, and the backward pass without its butterfly, butterflied,
    equals the backward pass; FP64, FP32 and complex data."""
    plan, _, _ = make_pair(shape, 6.0, "cos", sigma=1.0)
    mask = ts.ts_fold_axes(plan)
    assert mask == sum(1 << k for k in range(len(shape)))
    xr = to_dev(W.rhs_normal(shape, 4))
    xc = to_dev(W.complex_normal(shape, 5))
    cases = [(xr, "fp64", 1e-13), (xr.float(), "fp32", 2e-6), (xc, "fp64", 1e-13),
             (xc.to(torch.complex64), "fp32", 2e-6)]
    for axis in range(len(shape)):
        for x, prec, tol in cases:
            xf = ts.ts_fold_butterfly(plan, 1 << axis, x)
            y1 = ts.ts_mode_pass(plan, axis, True, x, prec=prec)
            y2 = ts.ts_mode_pass(plan, axis, True, xf, prec=prec, folded=True)
            z0 = ts.ts_mode_pass(plan, axis, False, y1, prec=prec)
            z3 = ts.ts_fold_butterfly(plan, 1 << axis, ts.ts_mode_pass(plan, axis, False, y1, prec=prec, folded=True))
            e_f, e_b = rel(to_host(y2), to_host(y1)), rel(to_host(z3), to_host(z0))
            announce("folded-data passes %s axis %d %s %s: forward %.2e backward %.2e"
                     % (shape, axis, x.dtype, prec, e_f, e_b))
            assert e_f <= tol and e_b <= tol
    with pytest.raises(ts.TSError):
        ts.ts_mode_pass(plan, 0, True, xr.float(), prec="bf16", folded=True)


def test_five_folded_axes_two_sweeps():
    """64^5 (every axis folds): the apply folds and unfolds in two butterfly
    sweeps each (four axes, then one); it must equal the plain apply, whose
    parity with the oracle is checked on smaller grids.  Compared on the device
    (1.07e9 values per array)."""
    shape = (64,) * 5
    plan = ts.ts_setup(shape, 6.0, [W.f_harmonic_cos(64, 6.0)] * 5, 1.0)
    assert ts.ts_fold_axes(plan) == 31
    gen = torch.Generator(device=DEV)
    gen.manual_seed(11)
    b = torch.randn(shape, dtype=torch.float64, device=DEV, generator=gen)
    u_fold = ts.ts_apply_inverse(plan, b)
    ts.ts_set_fold(plan, False)
    u_plain = ts.ts_apply_inverse(plan, b)
    ts.ts_set_fold(plan, True)
    e = float(torch.linalg.vector_norm(u_fold - u_plain) / torch.linalg.vector_norm(u_plain))
    del u_plain
    # the inverse undone by the operator: a check of the folded result on its own
    r = ts.ts_operator_apply(plan, None, 1.0, u_fold)
    r.sub_(b)
    res = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))
    announce("64^5 fold vs plain %.2e, relative residual %.2e" % (e, res))
    assert e <= 1e-13 and res <= 1e-12


@pytest.mark.parametrize("rel_pert,folds", [(2.0e-16, True), (5.0e-14, False)])
def test_nearly_symmetric_f(rel_pert, folds):
    """f perturbed on one side: within a few ulps the axis still folds (the
    solver averages the mirrored pair); at 5e-14 relative it takes the plain
    path.  Either way the result matches the oracle, which uses the samples as
    given, to the FP64 bar (the 1e9-DoF potential f = x^2 + 0.5 cos 2x on
    [-10, 10] has max|f| ~ 100)."""
    n, L = 200, 10.0
    f0 = W.f_harmonic_cos(n, L)
    fmax = np.abs(f0).max()
    f1 = f0.copy()
    f1[: n // 2] += rel_pert * fmax * np.linspace(0.2, 1.0, n // 2)
    shape = (n, 96)
    fs = [f1, W.f_harmonic_cos(96, L)]
    plan = ts.ts_setup(shape, L, fs, 1.0)
    assert bool(ts.ts_fold_axes(plan) & 1) == folds
    oplan = oracle.make_plan(shape, L, fs)
    b = W.rhs_normal(shape, 12)
    e = rel(to_host(ts.ts_apply_inverse(plan, to_dev(b))), oracle.apply_inverse(oplan, b, 1.0))
    psi = W.complex_normal(shape, 13)
    ep = rel(to_host(ts.ts_apply_exp(plan, 0.01, to_dev(psi))), oracle.apply_exp(oplan, psi, 0.01))
    announce("near-symmetric f (%.0e): folds %s, inverse %.2e, exp %.2e" % (rel_pert, folds, e, ep))
    assert e <= 1e-12 and ep <= exp_tol(oplan, 0.01)
