"""Q^k spectral elements on the GPU (Sec. 2, eq. (eigen_decomp)) through
ts_setup_sem.

* Applies (inverse, shifted inverse, propagator) against the oracle's SEM
  plan on grouped (all n <= 32) and MFMA grids, k = 1..10, FP64 and FP32.
* The operator M^{-1} S + F + V2 against the oracle's mode products.
* PCG, refinement and inverse iteration against the oracle's solvers in the
  mass inner product.
* Full size: the FP64 rows of Table tab:accuracy_gh200 (3D Q^2 and Q^10 at
  1099^3, 4D Q^10 at 179^4, 6D Q^2 at 33^6): the l2 error of the computed
  solution against the printed value, and at sampled points the residual of
  the discrete equation evaluated by the oracle's own per-axis operators.
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


def sem_pair(k, cells, L=6.0, seed=0, kind="harm"):
    """Library and oracle SEM plans on the same f samples (taken at the
    library's nodes)."""
    rng = np.random.default_rng(seed)
    f = []
    for c in cells:
        x = ts.ts_sem_nodes(k, c, L)
        f.append(W.f_harmonic(0, L, x=x) if kind == "harm" else rng.uniform(0.0, 5.0, x.size))
    return ts.ts_setup_sem(k, cells, L, f, 1.0), oracle.make_plan_sem(k, cells, L, f), f


CASES = [(1, (9, 7)), (2, (6, 5, 4)), (3, (5,) * 4), (6, (3, 2, 3)), (10, (2, 3)),
         (2, (40, 33)), (3, (22, 17, 15)), (6, (12, 10)), (10, (7,)), (4, (30, 12, 9))]


@pytest.mark.parametrize("k,cells", CASES)
def test_sem_apply_parity(k, cells):
    plan, oplan, _ = sem_pair(k, cells)
    b = W.rhs_normal(plan.shape, 1)
    e_inv = rel(to_host(ts.ts_apply_inverse(plan, to_dev(b))), oracle.apply_inverse(oplan, b, 1.0))
    e_sh = rel(to_host(ts.ts_apply_inverse_shift(plan, 3.5, to_dev(b))), oracle.apply_inverse(oplan, b, 3.5))
    psi = W.complex_normal(plan.shape, 2)
    tau = 0.02
    e_exp = rel(to_host(ts.ts_apply_exp(plan, tau, to_dev(psi))), oracle.apply_exp(oplan, psi, tau))
    u32 = to_host(ts.ts_apply_inverse(plan, to_dev(b).float(), prec="fp32")).astype(np.float64)
    e32 = rel(u32, oracle.apply_inverse(oplan, b, 1.0))
    u16 = to_host(ts.ts_apply_inverse(plan, to_dev(b).float(), prec="bf16")).astype(np.float64)
    e16 = rel(u16, oracle.apply_inverse(oplan, b, 1.0))
    announce("sem k=%d cells=%s n=%s: inv %.2e shift %.2e exp %.2e (tol %.1e) fp32 %.2e bf16 %.2e"
             % (k, cells, plan.shape, e_inv, e_sh, e_exp, exp_tol(oplan, tau), e32, e16))
    assert e_inv <= 1e-12 and e_sh <= 1e-12
    assert e_exp <= exp_tol(oplan, tau)
    assert e32 <= 2e-5
    # BF16 operands (8-bit mantissa) through 2d passes; the grouped small path computes in FP32
    assert e16 <= 1.5e-2


@pytest.mark.parametrize("k,cells", [(2, (6, 5, 4)), (6, (3, 2, 3)), (3, (22, 17, 15)), (10, (2, 3))])
def test_sem_operator_matches_oracle(k, cells):
    plan, oplan, _ = sem_pair(k, cells, kind="rand", seed=3)
    rng = np.random.default_rng(4)
    V2 = rng.uniform(-1.0, 3.0, plan.shape)
    u = W.rhs_normal(plan.shape, 5)
    got = to_host(ts.ts_operator_apply(plan, to_dev(V2), 0.25, to_dev(u)))
    ref = oracle.operator_apply(oplan, u, V2, 0.25)
    assert rel(got, ref) <= 1e-13


@pytest.mark.parametrize("k,cells", [(2, (10, 9, 8)), (6, (5, 4, 4)), (3, (22, 17, 15))])
def test_sem_pcg_refine_and_inverse_iteration(k, cells):
    L = 6.0
    plan, oplan, f = sem_pair(k, cells, L=L)
    nodes = [ts.ts_sem_nodes(k, c, L) for c in cells]
    rng = np.random.default_rng(7)
    # a Gaussian bump V2 >= 0 at the SEM nodes
    c0 = rng.uniform(-2, 2, 3)
    g = [np.exp(-((x - c) ** 2) / 2.0) for x, c in zip(nodes, c0)]
    V2 = 4.0 * W.outer(g)
    rhs = W.rhs_normal(plan.shape, 8)
    ref = oracle.pcg(oplan, V2, 1.0, rhs, rtol=1e-13)
    for prec in ("fp64", "fp32", "bf16"):
        u = torch.zeros(plan.shape, dtype=torch.float64, device=DEV)
        _, its, rr, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(rhs), u, rtol=1e-10, maxit=300, precond=prec)
        uh = to_host(u)
        true = oracle.norm(oplan, rhs - oracle.operator_apply(oplan, uh, V2, 1.0)) / oracle.norm(oplan, rhs)
        announce("sem pcg k=%d %s: %d its, relres %.2e, true %.2e, err %.2e"
                 % (k, prec, its, rr, true, rel(uh, ref.x)))
        assert true <= 2e-10 and rel(uh, ref.x) <= 1e-8
    u, its, rr = ts.ts_solve_refined(plan, to_dev(rhs), inner="fp32", rtol=1e-10, maxit=60)
    direct = oracle.apply_inverse(oplan, rhs, 1.0)
    assert rel(to_host(u), direct) <= 1e-8
    # inverse iteration: V2 >= 0 so H1 - shift and H - shift are >= 0.5
    shift = sum(float(ts.ts_eigvals(plan, a)[0]) for a in range(plan.d)) - 0.5
    u0 = oracle.separable_ground_state(oplan)
    out = oracle.inverse_iteration(oplan, V2, shift, steps=20, u0=u0)
    ud = to_dev(u0)
    _, lam, _ = ts.ts_inverse_iteration(plan, to_dev(V2), shift, ud, steps=20, pcg_rtol=1e-12, maxit=300)
    uh = to_host(ud)
    announce("sem invit k=%d: lambda %.12f oracle %.12f" % (k, lam[-1], out.lam[-1]))
    assert abs(lam[-1] - out.lam[-1]) <= 1e-10 * abs(out.lam[-1])
    s = np.sign(oracle.inner(oplan, uh, out.u))
    assert rel(s * uh, out.u) <= 1e-6
    assert abs(oracle.norm(oplan, uh) - 1.0) <= 1e-12


def _sampled_residual(k, cells_list, L, f_list, V_extra, u_dev, rhs_fn, npts=4000, seed=0):
    """Max over sampled points of |f_p - (H u)_p|, relative to the largest
    magnitude sum |K||u| + |diag u| + |f| met among the samples (rounding in u
    is absolute, so a point-local scale would blow up where u* is tiny), with
    the oracle's dense per-axis K = M^{-1} S rows."""
    d = len(cells_list)
    axes = [oracle.sem_axis(k, c, L) for c in cells_list]
    Ks = [S / m[:, None] for (_, m, S) in axes]
    shape = u_dev.shape
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, n, npts) for n in shape])
    worst = 0.0
    scale = 0.0
    u_flat = u_dev.reshape(-1)
    strides = [int(np.prod(shape[a + 1:])) for a in range(d)]
    for p in range(npts):
        i = idx[:, p]
        base = int(sum(int(i[a]) * strides[a] for a in range(d)))
        acc = 0.0
        mag = 0.0
        for a in range(d):
            row = Ks[a][i[a]]
            nz = np.nonzero(row)[0]
            offs = torch.from_numpy(base + (nz - i[a]) * strides[a]).to(DEV)
            vals = u_flat[offs].cpu().numpy()
            acc += float(np.dot(row[nz], vals))
            mag += float(np.dot(np.abs(row[nz]), np.abs(vals)))
        up = float(u_flat[base].item())
        diag = sum(f_list[a][i[a]] for a in range(d)) + V_extra
        fp = rhs_fn(i)
        r = fp - (acc + diag * up)
        worst = max(worst, abs(r))
        scale = max(scale, mag + abs(diag * up) + abs(fp))
    return worst / scale


FULL = [
    # (name, dim, k, cells, printed l2 error, tolerance on the ratio to it)
    ("3d_q2", 3, 2, 550, 1.93e-9, 0.03),
    ("3d_q10", 3, 10, 110, 7.66e-13, None),   # FP64 rounding floor
    ("4d_q10", 4, 10, 18, 1.29e-13, None),    # FP64 rounding floor
    ("6d_q2", 6, 2, 17, 2.95e-2, 0.02),       # mesh too coarse: a discretisation error
]
# Where the printed error is the FP64 rounding floor it depends on how exactly
# the axis operators are formed and diagonalised, not on the discretisation:
# with the operator assembled in double and a decomposition that is only
# backward stable, a 1D Q^10 solve on 110 cells misses u* by 1e-11
# (|A| / lam_min ~ 5e5).  The library assembles in long double and refines the
# eigenvectors against that operator; measured 2.2e-15 (3D) and 6.2e-15 (4D),
# below the printed floors.  The bar is twice the larger of the two.
FLOOR_BAR = 1.25e-14


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,d,k,cells,printed,tol", FULL)
def test_accuracy_table_full_size(name, d, k, cells, printed, tol):
    L = 1.0
    x = ts.ts_sem_nodes(k, cells, L)
    n = x.size
    if d == 3:  # eq. (test_potential); the paper's x is the fastest axis
        coef = {2: 1.0, 1: 2.0, 0: 3.0}
        f = [W.f_test_potential(0, L, coef[a], x=x) for a in range(3)]
        modes = [3, 2, 1]
    else:       # V = sum x_k^2, u* = prod sin(k pi x_k), k = 1 on the fastest axis
        f = [W.f_harmonic(0, L, x=x) for _ in range(d)]
        modes = list(range(d, 0, -1))
    announce("%s: setup %d^%d" % (name, n, d))
    plan = ts.ts_setup_sem(k, (cells,) * d, L, f, 0.0)
    xd = to_dev(x)
    fac = [torch.sin(mm * np.pi * xd) for mm in modes]
    fd = [to_dev(fa) for fa in f]
    lap = float(sum((mm * np.pi) ** 2 for mm in modes))

    def outer(vs):
        out = vs[0]
        for v in vs[1:]:
            out = out.unsqueeze(-1) * v
        return out.contiguous()

    ustar = outer(fac)
    Vsum = fd[0]
    for a in range(1, d):
        Vsum = Vsum.unsqueeze(-1) + fd[a]
    rhs = ((lap + Vsum) * ustar).contiguous()
    del Vsum
    u = ts.ts_apply_inverse(plan, rhs)
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm(u - ustar) / torch.linalg.vector_norm(ustar))
    announce("%s: l2 rel err %.3e (printed %.3e)" % (name, err, printed))
    xs = x

    def rhs_fn(i):
        val = lap + sum(f[a][i[a]] for a in range(d))
        for a in range(d):
            val *= np.sin(modes[a] * np.pi * xs[i[a]])
        return val

    res = _sampled_residual(k, [cells] * d, L, f, 0.0, u, rhs_fn, npts=2000)
    announce("%s: sampled residual %.2e" % (name, res))
    assert res <= 1e-11
    if tol is None:
        assert err <= FLOOR_BAR
    else:
        assert abs(err - printed) / printed <= tol


def test_sem_banded_operator_passes():
    """A plan with an axis of n >= 128 applies its operator as FP64 matrix-core
    passes restricted to the band (|i - j| <= k): the public operator, the
    symmetric-form operator inside PCG and the GPE step against the oracle."""
    k, cells, L = 3, (50, 44, 12), 6.0  # n = 149, 131, 35
    plan, oplan, f = sem_pair(k, cells, L=L, kind="rand", seed=9)
    rng = np.random.default_rng(10)
    V2 = rng.uniform(0.0, 3.0, plan.shape)
    u = W.rhs_normal(plan.shape, 11)
    got = to_host(ts.ts_operator_apply(plan, to_dev(V2), 0.5, to_dev(u)))
    e_op = rel(got, oracle.operator_apply(oplan, u, V2, 0.5))
    rhs = W.rhs_normal(plan.shape, 12)
    x = torch.zeros(plan.shape, dtype=torch.float64, device=DEV)
    _, its, rr, _ = ts.ts_pcg_solve(plan, to_dev(V2), to_dev(rhs), x, rtol=1e-10, maxit=300)
    xh = to_host(x)
    true = oracle.norm(oplan, rhs - oracle.operator_apply(oplan, xh, V2, 1.0)) / oracle.norm(oplan, rhs)
    # GPE: one modified H^1 step on a -Delta plan of the same mesh
    lap = ts.ts_setup_sem(k, cells, L, [np.zeros_like(a) for a in f], 1.0)
    olap = oracle.make_plan_sem(k, cells, L, [np.zeros_like(a) for a in f])
    Vg = V2
    w = oracle.l2_weights(olap)
    u0 = np.abs(W.rhs_normal(plan.shape, 13)) + 0.1
    u0 = u0 / np.sqrt(np.sum(w * u0 * u0))
    ref = oracle.h1_flow_step(olap, Vg, 30.0, 10.0, 0.1, u0)
    ud = to_dev(u0)
    ts.ts_gpe_h1_flow(lap, to_dev(Vg), 30.0, ud, alpha=10.0, tau=0.1, maxit=1, tol=0.0, raise_on_noconv=False)
    e_gpe = rel(to_host(ud), ref)
    announce("sem banded passes %s: operator %.2e, pcg %d its true %.2e, gpe step %.2e"
             % (plan.shape, e_op, its, true, e_gpe))
    assert e_op <= 1e-13
    assert true <= 2e-10
    assert e_gpe <= 1e-12
