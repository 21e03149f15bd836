"""PCG (Sec. 3.2), mixed-precision iterative refinement and shifted inverse
iteration (Sec. 4.1, 5.3.1) on the GPU, against the oracle.

Bars: every solve must reach a true relative residual <= 1e-10 (recomputed by
the oracle's stencil on the host); the error against the oracle's solution is
bounded by the conditioning of the system times that residual.  PCG with the
FP64 preconditioner and V2 = 0 converges in one iteration (exact
preconditioner).  Inverse iteration: per-step eigenvalue estimates track the
oracle's run of the same 20 steps, and the final value matches numpy's dense
eigvalsh on a small grid.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import announce, make_pair, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _sigma_c14(plan_lam_min, V2min):
    # sigma = 1, raised so that lambda_min(H1) + min(V2) + sigma >= 0.5
    return max(1.0, 0.5 - plan_lam_min - V2min)


def test_pcg_exact_preconditioner_one_iteration():
    shape, L = (40, 33, 48), 8.0
    plan, oplan, _ = make_pair(shape, L, "harm", sigma=1.0)
    f = W.rhs_normal(shape, 3)
    u, it, rr, _ = ts.ts_pcg_solve(plan, None, to_dev(f), rtol=1e-12, precond="fp64")
    assert it == 1 and rr <= 1e-12
    assert rel(to_host(u), oracle.apply_inverse(oplan, f, 1.0)) <= 1e-12


@pytest.mark.parametrize("precond", ["fp64", "fp32"])
def test_pcg_bumps_matches_oracle(precond):
    shape, L = (48, 40, 56), 8.0
    f_list = [W.f_harmonic(n, L) for n in shape]
    V2 = W.gaussian_bumps(shape, L, 16, seed=3)
    lam_min = sum(l[0] for l in oracle.make_plan(shape, L, f_list).lam)
    sigma = _sigma_c14(lam_min, V2.min())
    plan = ts.ts_setup(shape, L, f_list, sigma)
    oplan = oracle.make_plan(shape, L, f_list)
    f = W.rhs_normal(shape, 3)
    u, it, rr, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(f), rtol=1e-10, precond=precond)
    uh = to_host(u)
    true = np.linalg.norm(f - oracle.stencil_apply(oplan, uh, V2, sigma)) / np.linalg.norm(f)
    ref = oracle.pcg(oplan, V2, sigma, f, rtol=1e-13)
    e = rel(uh, ref.x)
    announce("pcg %s: iters %d (oracle %d), relres %.2e (oracle-stencil %.2e), err vs oracle %.2e"
             % (precond, it, ref.iters, rr, true, e))
    assert rr <= 1e-10 and true <= 1.05e-10
    assert abs(true - rr) <= 0.05 * rr + 1e-14
    assert e <= 1e-8
    assert it <= ref.iters + 3


@pytest.mark.parametrize("n", [256, 512])
def test_pcg_config2_fp64_vs_mixed(n):
    """3D n = 256 and 512, V1 = sum x^2 on [-8,8]^3, 16 bumps (seed 3), f ~ N(0,1):
    rtol 1e-10 with the FP64, FP32 and BF16 preconditioners; the true residual
    of each result is recomputed on the host by the oracle's stencil."""
    L = 8.0
    shape = (n, n, n)
    f_list = [W.f_harmonic(n, L) for _ in range(3)]
    V2 = W.gaussian_bumps(shape, L, 16, seed=3)
    h = 2 * L / (n + 1)
    lam_min = 3 * float(np.linalg.eigvalsh(np.diag(2 / h**2 + f_list[0]) + np.diag(np.full(n - 1, -1 / h**2), 1)
                                            + np.diag(np.full(n - 1, -1 / h**2), -1))[0])
    sigma = _sigma_c14(lam_min, V2.min())
    plan = ts.ts_setup(shape, L, f_list, sigma)
    oplan = oracle.Plan(shape=shape, L=L, f=f_list, h=[oracle.grid_spacing(n, L)] * 3)
    f = W.rhs_normal(shape, 3)
    fd, V2d = to_dev(f), to_dev(V2)
    sols = {}
    for pc in ("fp64", "fp32", "bf16"):
        u, it, rr, _ = ts.ts_pcg_solve(plan, V2d, fd, rtol=1e-10, precond=pc)
        uh = to_host(u)
        del u
        true = np.linalg.norm(f - oracle.stencil_apply(oplan, uh, V2, sigma)) / np.linalg.norm(f)
        err = rel(uh, sols["fp64"][0]) if sols else 0.0
        announce("n=%d pcg %s: iters %d relres %.2e oracle-stencil %.2e, vs the FP64-preconditioned solution %.2e"
                 % (n, pc, it, rr, true, err))
        assert true <= 1.05e-10
        sols[pc] = (uh, it)
    for pc in ("fp32", "bf16"):
        assert rel(sols[pc][0], sols["fp64"][0]) <= 1e-8
        assert abs(sols[pc][1] - sols["fp64"][1]) <= 3


@pytest.mark.parametrize("shape", [(64, 64, 64), (100, 90, 80)])
def test_refined_mixed_inverse(shape):
    plan, oplan, _ = make_pair(shape, 8.0, "harm", sigma=1.0)
    f = W.rhs_normal(shape, 5)
    ref = oracle.apply_inverse(oplan, f, 1.0)
    u, it, rr = ts.ts_solve_refined(plan, to_dev(f), inner="fp32", rtol=1e-10, maxit=50)
    uh = to_host(u)
    true = np.linalg.norm(f - oracle.stencil_apply(oplan, uh, None, 1.0)) / np.linalg.norm(f)
    e = rel(uh, ref)
    announce("refined fp32 %s: sweeps %d relres %.2e (oracle-stencil %.2e) err %.2e" % (shape, it, rr, true, e))
    assert true <= 1.05e-10 and e <= 1e-9


def test_inverse_iteration_matches_oracle():
    shape, L = (24, 20, 28), 6.0
    plan, oplan, f_list = make_pair(shape, L, "harm", sigma=1.0)
    V2 = np.abs(W.gaussian_bumps(shape, L, 6, seed=7))   # V2 >= 0: shift 0.9 lambda_min(A)
    lamA = sum(l[0] for l in oplan.lam)
    shift = 0.9 * lamA
    u0 = oracle.separable_ground_state(oplan)
    u = to_dev(u0)
    _, lam, its = ts.ts_inverse_iteration(plan, to_dev(V2), shift, u, steps=20, pcg_rtol=1e-10)
    ref = oracle.inverse_iteration(oplan, V2, shift, steps=20, u0=u0, pcg_rtol=1e-10)
    dense = np.linalg.eigvalsh(oracle.dense_operator(oplan, V2))[0]
    announce("inverse iteration: lam %.12f oracle %.12f dense %.12f; pcg iters %s"
             % (lam[-1], ref.lam[-1], dense, its))
    assert np.max(np.abs(np.array(lam) - np.array(ref.lam)) / np.abs(ref.lam)) <= 1e-9
    assert abs(lam[-1] - dense) <= 1e-9 * abs(dense)
    uh = to_host(u)
    assert abs(np.linalg.norm(uh) - 1) <= 1e-12
    assert abs(abs(np.vdot(uh, ref.u)) - 1) <= 1e-8


def test_inverse_iteration_separable_closed_form():
    shape, L = (30, 26, 22), 5.0
    plan = ts.ts_setup(shape, L, [np.zeros(n) for n in shape], 1.0)
    lam1 = sum((2 - 2 * np.cos(np.pi / (n + 1))) / (2 * L / (n + 1)) ** 2 for n in shape)
    rng = np.random.default_rng(1)
    u = to_dev(np.ones(shape) + 0.1 * rng.standard_normal(shape))
    _, lam, _ = ts.ts_inverse_iteration(plan, None, 0.9 * lam1, u, steps=20, pcg_rtol=1e-12)
    assert abs(lam[-1] - lam1) <= 1e-11 * lam1


def test_error_paths_forced_from_host():
    shape = (20, 24, 16)
    plan, oplan, _ = make_pair(shape, 6.0, "harm", sigma=1.0)
    V2 = W.gaussian_bumps(shape, 6.0, 8, seed=2)
    f = W.rhs_normal(shape, 1)
    # iteration limit -> TS_ERR_NOCONV, residual still reported
    u, it, rr, rc = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(f), rtol=1e-14, maxit=1, precond="fp64",
                                    raise_on_noconv=False)
    assert rc == ts.TS_ERR_NOCONV and it == 1 and 0 < rr < 1
    # non-finite right-hand side -> TS_ERR_NONFINITE
    fb = f.copy()
    fb[3, 4, 5] = np.nan
    with pytest.raises(ts.TSError) as e:
        ts.ts_pcg_solve(plan, to_dev(V2), to_dev(fb), rtol=1e-10)
    assert e.value.code == ts.TS_ERR_NONFINITE
    # a strongly negative V2 makes the operator indefinite -> breakdown (or no convergence)
    with pytest.raises(ts.TSError) as e:
        ts.ts_pcg_solve(plan, to_dev(np.full(shape, -1e3)), to_dev(f), rtol=1e-10, maxit=50)
    assert e.value.code in (ts.TS_ERR_BREAKDOWN, ts.TS_ERR_NOCONV)
    # shift above lambda_min(H1) -> TS_ERR_NOT_SPD
    with pytest.raises(ts.TSError) as e:
        ts.ts_inverse_iteration(plan, None, 1e4, to_dev(f), steps=1)
    assert e.value.code == ts.TS_ERR_NOT_SPD


def test_mixed_bf16_solvers_reach_fp64_tolerance():
    """BF16 transforms inside refinement / flexible PCG still reach 1e-10 in FP64."""
    shape, L = (64, 72, 80), 8.0
    f_list = [W.f_harmonic(n, L) for n in shape]
    plan = ts.ts_setup(shape, L, f_list, 1.0)
    oplan = oracle.make_plan(shape, L, f_list)
    f = W.rhs_normal(shape, 9)
    u, it, rr = ts.ts_solve_refined(plan, to_dev(f), inner="bf16", rtol=1e-10, maxit=60)
    uh = to_host(u)
    true = np.linalg.norm(f - oracle.stencil_apply(oplan, uh, None, 1.0)) / np.linalg.norm(f)
    announce("refined bf16: %d iterations, relres %.2e (oracle-stencil %.2e)" % (it, rr, true))
    assert true <= 1.05e-10
    V2 = W.gaussian_bumps(shape, L, 16, seed=3)
    sigma = max(1.0, 0.5 - sum(l[0] for l in oplan.lam) - V2.min())
    plan2 = ts.ts_setup(shape, L, f_list, sigma)
    u, it, rr, _ = ts.ts_pcg_solve(plan2, to_dev(V2), to_dev(f), rtol=1e-10, precond="bf16")
    uh = to_host(u)
    true = np.linalg.norm(f - oracle.stencil_apply(oplan, uh, V2, sigma)) / np.linalg.norm(f)
    announce("pcg bf16 preconditioner: %d iterations, relres %.2e (oracle-stencil %.2e)" % (it, rr, true))
    assert true <= 1.05e-10


@pytest.mark.parametrize("shape,precond", [((33, 25, 128, 64), "fp64"), ((16, 16, 16, 16, 16, 16), "bf16"),
                                           ((700, 600), "fp32")])
def test_pcg_higher_d_true_residual(shape, precond):
    """PCG (with the direction update fused into the operator sweep) on 2D, 4D
    and 6D grids: the true residual of the result, recomputed by the oracle's
    stencil, meets the tolerance."""
    L = 6.0
    f_list = [W.f_harmonic(n, L) for n in shape]
    V2 = np.abs(W.gaussian_bumps(shape, L, 6, seed=31))
    plan = ts.ts_setup(shape, L, f_list, 1.0)
    oplan = oracle.Plan(shape=shape, L=L, f=f_list, h=[oracle.grid_spacing(n, L) for n in shape])
    f = W.rhs_normal(shape, 32)
    u, it, rr, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(f), rtol=1e-10, precond=precond)
    true = np.linalg.norm(f - oracle.stencil_apply(oplan, to_host(u), V2, 1.0)) / np.linalg.norm(f)
    announce("pcg %s %s: %d iterations, relres %.2e, oracle-stencil %.2e" % (shape, precond, it, rr, true))
    assert rr <= 1e-10 and true <= 1.05e-10
