"""Serving loop (ts_serve_*): a mix of requests of different d, n and kind,
admitted by memory and run concurrently, must give every request the result
it gets alone through the plain entry points (bitwise: same kernels, same
task code, deterministic reductions), and a sample is checked against the
oracle.  Memory admission is exercised with a budget that fits only a few
requests at a time, FIFO mode with max_active = 1, and a request larger than
the budget.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _requests(seed=0):
    """(kind, shape, L, f_list, sigma, inp, prec, V2, tau, dt) tuples of a mixed workload."""
    rng = np.random.default_rng(seed)
    out = []
    specs = [
        ("inv", (48, 40, 56), "fp64", False), ("inv", (33, 47), "fp32", False), ("inv", (40, 36, 44), "bf16", False),
        ("inv", (32, 30, 28), "fp64", True), ("inv", (36, 40, 32), "bf16", True), ("inv", (16,) * 4, "fp32", True),
        ("exp", (200, 130), "fp64", False), ("exp", (24, 24, 24), "fp32", False), ("exp", (6,) * 6, "fp64", True),
        ("exp", (40, 36, 30), "fp32", True), ("inv", (12,) * 5, "fp64", False), ("exp", (64, 70), "fp32", True),
    ]
    for i, (kind, shape, prec, withv2) in enumerate(specs * 2):
        L = 6.0
        f = [W.f_harmonic(n, L) for n in shape]
        if kind == "inv":
            V2 = W.gaussian_bumps(shape, L, 8, seed=10 + i) if withv2 else None
            lam_min = sum(float(np.min(fk)) for fk in f)  # lambda_min(H1) >= sum of min f_k
            sigma = 1.0 if V2 is None else max(1.0, 0.5 - lam_min - V2.min())
            inp = W.rhs_normal(shape, 100 + i)
            out.append(dict(kind=ts.TS_REQ_INVERSE, shape=shape, L=L, f=f, sigma=sigma, inp=inp, prec=prec,
                            V2=V2, tau=0.0, dt=0.0))
        else:
            V2 = W.pairwise_v2(shape, L) if withv2 else None
            psi = W.complex_normal(shape, 200 + i)
            psi /= np.linalg.norm(psi)
            tau = float(rng.uniform(1e-3, 1e-1))
            out.append(dict(kind=ts.TS_REQ_EXP, shape=shape, L=L, f=f, sigma=1.0, inp=psi, prec=prec,
                            V2=V2, tau=tau, dt=1e-2))
    return out


def _device_inputs(r):
    if r["kind"] == ts.TS_REQ_INVERSE:
        x = to_dev(r["inp"])
        V2 = None if r["V2"] is None else to_dev(r["V2"])
    else:
        dt = torch.complex128 if r["prec"] == "fp64" else torch.complex64
        x = to_dev(r["inp"]).to(dt)
        V2 = None if r["V2"] is None else to_dev(r["V2"]).to(torch.float64 if dt == torch.complex128 else torch.float32)
    return x, V2


def _alone(r, x, V2):
    """The same request through the plain entry points."""
    plan = ts.ts_setup(r["shape"], r["L"], r["f"], r["sigma"])
    if r["kind"] == ts.TS_REQ_INVERSE:
        if V2 is not None:
            u = torch.zeros_like(x)
            ts.ts_pcg_solve(plan, V2, x, u, rtol=1e-10, maxit=500, precond=r["prec"])
            return u
        if r["prec"] == "fp64":
            return ts.ts_apply_inverse(plan, x)
        u, _, _ = ts.ts_solve_refined(plan, x, inner=r["prec"], rtol=1e-10, maxit=60)
        return u
    if V2 is not None:
        nsteps = max(1, int(np.ceil(abs(r["tau"]) / r["dt"])))
        psi = x.clone()
        ts.ts_split_step(plan, V2, psi, r["tau"] / nsteps, nsteps, "strang_bab", prec=r["prec"])
        return psi
    return ts.ts_apply_exp(plan, r["tau"], x, prec=r["prec"])


def _run_server(reqs, budget, n_streams, max_active, plan_reserve=0):
    srv = ts.Server(budget, n_streams, max_active, plan_reserve)
    tickets, outs, ins = [], [], []
    for i, r in enumerate(reqs):
        x, V2 = _device_inputs(r)
        out = torch.empty_like(x)
        t = srv.submit(r["kind"], r["shape"], r["L"], r["f"], r["sigma"], x, out, prec=r["prec"], V2=V2,
                       tau=r["tau"], dt=r["dt"], rtol=1e-10, maxit=500 if V2 is not None else 60, tag=i)
        tickets.append(t)
        outs.append(out)
        ins.append((x, V2))
    srv.drain()
    results = [srv.poll(t) for t in tickets]
    torch.cuda.synchronize()
    srv.close()
    return results, outs, ins


def test_mix_matches_requests_alone_bitwise():
    reqs = _requests()
    announce("serving %d requests on 4 streams" % len(reqs))
    results, outs, ins = _run_server(reqs, 2 << 30, 4, 0)
    for i, (r, res, out, (x, V2)) in enumerate(zip(reqs, results, outs, ins)):
        assert res is not None and res.status == ts.TS_OK, (i, res.status if res else None)
        assert res.t_submit <= res.t_admit <= res.t_done
        alone = _alone(r, x, V2)
        torch.cuda.synchronize()
        same = torch.equal(out, alone)
        if not same:
            announce("request %d differs: %.3e" % (i, rel(to_host(out), to_host(alone))))
        assert same, i
    # a sample against the oracle
    for i in (0, 6, 10):
        r = reqs[i]
        op = oracle.make_plan(r["shape"], r["L"], r["f"])
        got = to_host(outs[i])
        ref = oracle.apply_inverse(op, r["inp"], r["sigma"]) if r["kind"] == ts.TS_REQ_INVERSE else \
            oracle.apply_exp(op, r["inp"], r["tau"])
        assert rel(got, ref) <= 1e-12


def test_admission_by_memory_and_fifo():
    reqs = _requests(seed=1)[:12]
    # the largest of these requests needs ~3 MB of scratch; a 4 MB arena holds one to three at once
    # (the other 20 MB of the budget hold the twelve plans)
    results, outs, _ = _run_server(reqs, 24 << 20, 3, 0, plan_reserve=20 << 20)
    assert all(r is not None and r.status == ts.TS_OK for r in results)
    admits = sorted(r.t_admit for r in results)
    dones = sorted(r.t_done for r in results)
    assert admits[-1] > dones[0]  # some requests waited for memory freed by others
    fifo, outs2, _ = _run_server(reqs, 2 << 30, 1, 1)
    for a, b in zip(outs, outs2):
        assert torch.equal(a, b)
    # FIFO: each request is admitted after the previous one finished
    order = sorted(fifo, key=lambda r: r.t_admit)
    for prev, nxt in zip(order, order[1:]):
        assert nxt.t_admit >= prev.t_done - 1e-6


def test_oversized_request_rejected():
    srv = ts.Server(2 << 20, 2, 0, plan_reserve=1 << 20)
    shape, L = (64, 64, 64), 6.0
    x = torch.zeros(shape, dtype=torch.float64, device=DEV)
    with pytest.raises(ts.TSError) as e:
        srv.submit(ts.TS_REQ_INVERSE, shape, L, [W.f_harmonic(64, L)] * 3, 1.0, x, torch.empty_like(x))
    assert e.value.code == ts.TS_ERR_NOMEM
    srv.close()


def test_plan_cache_within_reserve_and_busy():
    """Plans are keyed without the shift (one cached plan serves requests of
    different sigma); the plan reserve is honoured by evicting plans that no
    request uses, and a submit whose plan cannot fit while running requests
    hold the others returns TS_ERR_BUSY."""
    L = 6.0
    shapes = [(40, 36, 44), (44, 40, 36), (36, 44, 40)]   # three distinct axes each: ~1.4 MB of factors
    srv = ts.Server(64 << 20, 2, 0, plan_reserve=3 << 20)
    outs, refs = [], []
    for i, shape in enumerate(shapes[:2]):
        f = [W.f_harmonic(n, L) for n in shape]
        for sigma in (1.0, 2.5):
            x = to_dev(W.rhs_normal(shape, 30 + i))
            out = torch.empty_like(x)
            srv.submit(ts.TS_REQ_INVERSE, shape, L, f, sigma, x, out)
            outs.append(out)
            refs.append((shape, f, sigma, x))
    srv.drain()
    for out, (shape, f, sigma, x) in zip(outs, refs):
        alone = ts.ts_apply_inverse(ts.ts_setup(shape, L, f, sigma), x)
        torch.cuda.synchronize()
        assert torch.equal(out, alone)
    # two plans resident (~2.8 MB); a third evicts the least recently used idle one
    shape = shapes[2]
    f = [W.f_harmonic(n, L) for n in shape]
    x = to_dev(W.rhs_normal(shape, 40))
    out = torch.empty_like(x)
    srv.submit(ts.TS_REQ_INVERSE, shape, L, f, 1.0, x, out)
    srv.drain()
    srv.close()
    # a reserve that holds one 256^3 plan (~3.2 MB with its half factors) but not
    # that and a 1.4 MB plan: a submit made while a long 256^3 PCG holds its plan
    # is told to come back later, and succeeds once that request has finished
    srv = ts.Server(2 << 30, 2, 0, plan_reserve=13 << 18)
    big = (256, 256, 256)
    fb = [W.f_harmonic(n, L) for n in big]
    V2b = torch.from_numpy(W.gaussian_bumps(big, L, 8, seed=5)).to(DEV).abs()
    xb = torch.randn(big, dtype=torch.float64, device=DEV)
    ob = torch.empty_like(xb)
    srv.submit(ts.TS_REQ_INVERSE, big, L, fb, 1.0, xb, ob, V2=V2b, rtol=1e-12, maxit=500)
    shape = shapes[0]
    f = [W.f_harmonic(n, L) for n in shape]
    x = to_dev(W.rhs_normal(shape, 41))
    out = torch.empty_like(x)
    with pytest.raises(ts.TSError) as e:
        srv.submit(ts.TS_REQ_INVERSE, shape, L, f, 1.0, x, out)
    assert e.value.code == ts.TS_ERR_BUSY
    srv.drain()
    srv.submit(ts.TS_REQ_INVERSE, shape, L, f, 1.0, x, out)
    srv.drain()
    torch.cuda.synchronize()
    assert torch.equal(out, ts.ts_apply_inverse(ts.ts_setup(shape, L, f, 1.0), x))
    srv.close()
