"""BF16 passes on 256 x 256 output tiles (ts_set_bf16_tile).

The larger tile halves the operand traffic from L2 but consumes K in the same
order (64-wide k-tiles, two 32-wide MFMA steps each) as the 128 x 128 kernel,
so without folding every BF16 apply must give bitwise equal results under
both tiles: the plain, scaling and last passes, BF16 / FP32 / FP64 outputs,
ragged tiles (n = 200, 264 against 256-wide tiles) and factor rows beyond the
stored padding (n = 264 keeps 384 padded rows against 512 tile rows).  The
default choice is checked against the FP64 oracle at the BF16 level (parity
unpinned: BF16 operands have no exact value, the bar is the one of the other
BF16 tests), and the PCG with a BF16 preconditioner on the large tiles still
reaches the FP64 residual bar.

On reflection-symmetric axes the large tiles also run the forward passes on
data folded by the input sweep (half the extent; the odd half of an axis with
h = n / 2 = 4 mod 8 is read from n - h - 4 against a factor shifted by 4):
checked against the oracle and against the same apply with folding off, with
even and odd extents, ragged half-tiles and the shifted case.

With every slower axis folded and even (2D, 3D) the backward passes over them
also run on half extents and the last pass unfolds in registers (rows gathered
by reflection orbits); that pass also adds the refinement's corrections.
Checked against the oracle, against the same apply with full backward passes
(ts_set_fold mode 2), and through the refined inverse (true residual by the
oracle's stencil); PCG on such a shape is the 256^3 test above.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, make_pair, maxrel, rel

pytestmark = pytest.mark.gpu


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("shape", [(200, 256, 264), (264, 200, 256), (256, 64, 200), (512, 2048)])
def test_large_and_small_tiles_bitwise_equal(shape):
    # library plan only: no oracle value is needed for a comparison of two kernels
    plan = ts.ts_setup(shape, 8.0, [W.f_harmonic(n, 8.0) for n in shape], 1.0)
    ts.ts_set_fold(plan, 0)  # folded passes exist only on the large tiles
    b = to_dev(W.rhs_normal(shape, 21))
    for dt in (torch.float64, torch.float32):
        x = b.to(dt)
        outs = {}
        for tile in (128, 256):
            ts.ts_set_bf16_tile(plan, tile)
            outs[tile] = to_host(ts.ts_apply_inverse(plan, x, prec="bf16"))
        ts.ts_set_bf16_tile(plan, 0)
        auto = to_host(ts.ts_apply_inverse(plan, x, prec="bf16"))
        same = np.array_equal(outs[128], outs[256])
        announce("bf16 tiles %s %s: 128 vs 256 bitwise equal %s" % (shape, dt, same))
        assert same and np.array_equal(auto, outs[128])
        assert np.isfinite(outs[256]).all() and np.abs(outs[256]).max() > 0


def test_tile_knob_rejects_other_values():
    plan = ts.ts_setup((8, 8), 4.0, [W.f_harmonic(8, 4.0)] * 2, 1.0)
    with pytest.raises(ts.TSError):
        ts.ts_set_bf16_tile(plan, 64)


@pytest.mark.parametrize("shape", [(256, 256, 256), (512, 512, 64)])
def test_default_tiles_against_oracle(shape):
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 22)
    ref = oracle.apply_inverse(oplan, b, 1.0)
    u = to_host(ts.ts_apply_inverse(plan, to_dev(b), prec="bf16"))
    e, em = rel(u, ref), maxrel(u, ref)
    announce("bf16 inverse %s (default tiles): rel err %.3e, max-norm %.3e" % (shape, e, em))
    assert 1e-3 < e <= 1.5e-2 and em <= 5e-2


def test_pcg_bf16_preconditioner_on_large_tiles():
    shape = (256, 256, 256)
    L = 8.0
    f = [W.f_harmonic(n, L) for n in shape]
    V2 = W.gaussian_bumps(shape, L, 16, seed=3)
    sigma = max(1.0, 0.5 - sum(float(min(fk)) for fk in f) - float(V2.min()))
    plan = ts.ts_setup(shape, L, f, sigma)
    rhs = W.rhs_normal(shape, 23)
    u = torch.zeros(shape, dtype=torch.float64, device=DEV)
    _, its, relres, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(rhs), u, rtol=1e-10, maxit=200, precond="bf16")
    op = oracle.Plan(shape=shape, L=L, f=f, h=[oracle.grid_spacing(n, L) for n in shape])
    true = np.linalg.norm(rhs - oracle.stencil_apply(op, to_host(u), V2, sigma)) / np.linalg.norm(rhs)
    announce("PCG bf16 preconditioner 256^3: %d iterations, recurrence %.2e, true residual %.2e" % (its, relres, true))
    assert true <= 1.05e-10


@pytest.mark.parametrize("shape", [(200, 256, 264), (257, 200, 256), (400, 264)])
def test_folded_forward_passes(shape):
    """BF16 inverse of FP64 data on symmetric axes: the input sweep folds along
    every axis whose forward pass reads folded data and those passes contract
    half the extent.  n = 200, 264: h = 4 mod 8 (the shifted odd half); 257:
    odd extent on a column axis (the middle value stays unfolded), 256: h = 0
    mod 8; ragged half-tiles against 256-wide tiles everywhere.  Against the
    oracle at the BF16 level, and against the same apply with folding off (a
    different rounding of the same products)."""
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    b = W.rhs_normal(shape, 23)
    ref = oracle.apply_inverse(oplan, b, 1.0)
    bd = to_dev(b)
    u = to_host(ts.ts_apply_inverse(plan, bd, prec="bf16"))
    ush = to_host(ts.ts_apply_inverse_shift(plan, 2.5, bd, prec="bf16"))
    ref_sh = oracle.apply_inverse(oplan, b, 2.5)
    ts.ts_set_fold(plan, 0)
    u0 = to_host(ts.ts_apply_inverse(plan, bd, prec="bf16"))
    ts.ts_set_fold(plan, 1)
    e, em, e_sh, e0, ed = rel(u, ref), maxrel(u, ref), rel(ush, ref_sh), rel(u0, ref), rel(u, u0)
    announce("bf16 folded %s: rel err %.3e (max-norm %.3e), shifted %.3e, unfolded %.3e, between %.3e"
             % (shape, e, em, e_sh, e0, ed))
    assert 1e-3 < e <= 1.5e-2 and em <= 5e-2 and e_sh <= 1.5e-2
    assert ed <= 1.5e-2 and not np.array_equal(u, u0)
    assert np.array_equal(to_host(bd), b)


def test_pcg_folded_residual_update():
    """PCG with a BF16 preconditioner on an operator whose preconditioner folds
    its input (n = 257 on axis 0: odd, the middle plane unfolded; 264: h = 4
    mod 8): the residual update writes the folded BF16 input itself.  With
    folding on and off the true residual (oracle stencil) meets the FP64 bar,
    and the two solutions agree far below it."""
    shape = (257, 264, 256)
    L = 8.0
    f = [W.f_harmonic(n, L) for n in shape]
    V2 = W.gaussian_bumps(shape, L, 16, seed=4)
    sigma = max(1.0, 0.5 - sum(float(min(fk)) for fk in f) - float(V2.min()))
    plan = ts.ts_setup(shape, L, f, sigma)
    rhs = W.rhs_normal(shape, 24)
    op = oracle.Plan(shape=shape, L=L, f=f, h=[oracle.grid_spacing(n, L) for n in shape])
    sols = []
    for fold in (1, 0):
        ts.ts_set_fold(plan, fold)
        u = torch.zeros(shape, dtype=torch.float64, device=DEV)
        _, its, relres, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(rhs), u, rtol=1e-10, maxit=200, precond="bf16")
        uh = to_host(u)
        true = np.linalg.norm(rhs - oracle.stencil_apply(op, uh, V2, sigma)) / np.linalg.norm(rhs)
        announce("PCG bf16 %s fold=%d: %d iterations, recurrence %.2e, true residual %.2e"
                 % (shape, fold, its, relres, true))
        assert true <= 1.05e-10
        sols.append(uh)
    assert rel(sols[0], sols[1]) <= 1e-8


def test_refined_bf16_adds_in_last_pass():
    """BF16-refined direct inverse: on the large tiles each correction is added
    to u inside the last pass of its apply (no separate update sweep).  With
    folding off the large and small tiles are bitwise equal per pass, so the
    refined solutions with the large tiles (adding in the pass) and the small
    ones (correction, then a separate update) must be bitwise equal too; the
    true residual meets the bar."""
    shape = (256, 200, 264)
    L = 8.0
    f = [W.f_harmonic(n, L) for n in shape]
    plan = ts.ts_setup(shape, L, f, 1.0)
    ts.ts_set_fold(plan, 0)
    b = to_dev(W.rhs_normal(shape, 25))
    outs = {}
    for tile in (256, 128):
        ts.ts_set_bf16_tile(plan, tile)
        u = torch.empty_like(b)
        _, its, relres = ts.ts_solve_refined(plan, b, u, inner="bf16", rtol=1e-10, maxit=60)
        outs[tile] = (to_host(u), its, relres)
    announce("refined bf16 %s: %d / %d sweeps, relres %.2e / %.2e, bitwise equal %s"
             % (shape, outs[256][1], outs[128][1], outs[256][2], outs[128][2],
                np.array_equal(outs[256][0], outs[128][0])))
    assert outs[256][1] == outs[128][1] and np.array_equal(outs[256][0], outs[128][0])
    assert outs[256][2] <= 1e-10


@pytest.mark.parametrize("shape,tile", [((256, 264, 256), 0), ((202, 200, 200), 256), ((400, 256), 256)])
def test_folded_backward_passes(shape, tile):
    """BF16 inverse of FP64 data with every slower axis folded and of even
    extent (2D and 3D): the backward passes over the slower axes also contract
    half the extent and leave their output folded, and the last pass (the
    fastest axis, FP64 output) gathers the rows of each reflection orbit into
    one lane and unfolds them before storing.  n = 264, 200: h = 4 mod 8 (the
    shifted odd half); 202: h = 101, 5 mod 8; orbits per tile 64 (3D) or 128
    (2D), with ragged last tiles (10100 orbits for 202 x 200, 200 for 400).
    Against the oracle at the BF16 level (every output stored: the output starts
    as NaN), and against the same apply with full backward passes (ts_set_fold
    mode 2: a different rounding of the same products)."""
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    ts.ts_set_bf16_tile(plan, tile)
    b = W.rhs_normal(shape, 26)
    ref = oracle.apply_inverse(oplan, b, 1.0)
    bd = to_dev(b)
    out = torch.full(shape, float("nan"), dtype=torch.float64, device=DEV)
    u = to_host(ts.ts_apply_inverse(plan, bd, out, prec="bf16"))
    ts.ts_set_fold(plan, 2)
    u2 = to_host(ts.ts_apply_inverse(plan, bd, prec="bf16"))
    ts.ts_set_fold(plan, 1)
    e, em, e2, ed = rel(u, ref), maxrel(u, ref), rel(u2, ref), rel(u, u2)
    announce("bf16 folded backward %s tile %d: rel err %.3e (max-norm %.3e), full backward %.3e, between %.3e"
             % (shape, tile, e, em, e2, ed))
    assert np.isfinite(u).all()
    assert 1e-3 < e <= 1.5e-2 and em <= 5e-2
    assert ed <= 1.5e-2 and not np.array_equal(u, u2)
    with pytest.raises(ts.TSError):
        ts.ts_set_fold(plan, 3)


def test_refined_bf16_folded_backward():
    """The BF16-refined direct inverse on a shape that takes the folded
    backward passes: each correction is added to u by the unfolding last pass.
    The true residual (oracle stencil) meets the bar, and the solution agrees
    with the refined solve whose BF16 applies run full backward passes."""
    shape = (256, 264, 256)
    L = 8.0
    f = [W.f_harmonic(n, L) for n in shape]
    plan = ts.ts_setup(shape, L, f, 1.0)
    b = W.rhs_normal(shape, 27)
    op = oracle.Plan(shape=shape, L=L, f=f, h=[oracle.grid_spacing(n, L) for n in shape])
    sols = []
    for mode in (1, 2):
        ts.ts_set_fold(plan, mode)
        u = torch.empty(shape, dtype=torch.float64, device=DEV)
        _, its, relres = ts.ts_solve_refined(plan, to_dev(b), u, inner="bf16", rtol=1e-10, maxit=60)
        uh = to_host(u)
        true = np.linalg.norm(b - oracle.stencil_apply(op, uh, None, 1.0)) / np.linalg.norm(b)
        announce("refined bf16 %s fold mode %d: %d sweeps, relres %.2e, true residual %.2e" % (shape, mode, its, relres, true))
        assert relres <= 1e-10 and true <= 1.05e-10
        sols.append(uh)
    assert rel(sols[0], sols[1]) <= 1e-8

