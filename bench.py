#!/usr/bin/env python3
"""Benchmark of the separable tensor-product apply on one MI355X.

Headline: DoF/s of the FP64 separable inverse apply (H1 + sigma)^{-1} b on the
3D grid of n = 1000 points per axis (1e9 DoFs): second-order FD on [-10,10]^3,
V1 = sum_k (x_k^2 + 0.5 cos 2x_k), sigma = 1, N(0,1) right-hand side drawn on
the device from a seeded generator.  One step = one apply (forward transforms,
fused diagonal scaling, backward transforms), inputs resident in HBM.

Also reported (not part of `value`): FP32 / BF16 transform variants, the
propagator exp(-i tau H1) on complex128 / complex64 wavepackets (tau = 0.01),
setup time, the FP64 residual of the timed result, the roofline of the
dominant kernel (the FP64 MFMA mode-product pass) and the oracle timed on a
bounded sample on the host cores.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # TFLOP/s, dense MFMA, MI355X
HBM_PEAK = 8000.0                                      # GB/s
METRIC = "DoF/s of separable inverse apply at 3D 1e9 DoFs; mixed vs FP64 PCG solve time"


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic_modeprod_fp64_n1000.json")
TRAFFIC_SOURCES = ["paper_2605_20491_amd/csrc/modeprod.hip", "paper_2605_20491_amd/csrc/modeprod_common.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(root, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size);
    None when absent or when the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, None
    with open(TRAFFIC_FILE) as f:
        d = json.load(f)
    if d.get("source_sha256") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return d["bytes_per_launch"], d


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def bumps_on_device(W, torch, dev, shape, L, nbumps, seed):
    """The Gaussian-bump V2 of the workload recipe, evaluated on the device."""
    axes = [torch.from_numpy(W.grid_nodes(n, L)).to(dev) for n in shape]
    V = torch.zeros(shape, dtype=torch.float64, device=dev)
    for a, w, c in W.bump_params(len(shape), nbumps, seed):
        g = [torch.exp(-(axes[k] - c[k]) ** 2 / (2.0 * w * w)) for k in range(len(shape))]
        t = g[0]
        for k in range(1, len(shape)):
            t = t.unsqueeze(-1) * g[k]
        V += a * t
    return V


def pcg_section(ts, W, torch, dev, n, precs):
    """Non-separable PCG workload: 3D n^3 on [-8,8]^3, V1 = sum x^2, 16 bumps (seed 3),
    f ~ N(0,1) (seed 3), preconditioner (H1 + sigma)^-1 in each precision, rtol 1e-10."""
    L = 8.0
    shape = (n, n, n)
    f_list = [W.f_harmonic(n, L) for _ in range(3)]
    V2 = bumps_on_device(W, torch, dev, shape, L, 16, 3)
    plan = ts.ts_setup(shape, L, f_list, 1.0)
    lam_min = sum(float(ts.ts_eigvals(plan, k)[0]) for k in range(3))
    sigma = max(1.0, 0.5 - lam_min - float(V2.min()))
    if sigma != 1.0:
        plan = ts.ts_setup(shape, L, f_list, sigma)
    gen = torch.Generator(device=dev)
    gen.manual_seed(3)
    f = torch.randn(shape, dtype=torch.float64, device=dev, generator=gen)
    out = {"n": n, "sigma": sigma}
    for prec in precs:
        try:
            u = torch.zeros_like(f)
            ts.ts_pcg_solve(plan, V2, f, u, rtol=1e-10, precond=prec)   # warm-up
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, it, rr, _ = ts.ts_pcg_solve(plan, V2, f, u, rtol=1e-10, precond=prec)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            N = n ** 3
            # per-iteration roofline: one preconditioner apply (4 N sum n_k flops at the MFMA peak of its
            # precision, or its 16 B/point of FP64 in/out at the HBM peak) plus the FP64 vector work of
            # one PCG iteration (operator 24 B/point, x and r updates 48, <z,r> 16, p update 24)
            t_pre = max(12.0 * N * n / (PEAK[prec] * 1e12), 16.0 * N / (HBM_PEAK * 1e9))
            t_vec = 112.0 * N / (HBM_PEAK * 1e9)
            t_iter = ms / max(it, 1)
            out[prec] = {"solve_ms": ms, "iters": it, "relres": rr, "ms_per_iter": t_iter,
                         "roofline_ms_per_iter": (t_pre + t_vec) * 1e3,
                         "roofline_frac_per_iter": (t_pre + t_vec) * 1e3 / t_iter}
            log("pcg n=%d %s: %.1f ms, %d iters, relres %.2e, %.2f ms/iter = %.0f%% of its roofline"
                % (n, prec, ms, it, rr, t_iter, 100 * out[prec]["roofline_frac_per_iter"]))
        except ts.TSError as e:
            out[prec] = "unavailable: %s" % e.status
    if isinstance(out.get("fp64"), dict):
        for prec in precs[1:]:
            if isinstance(out.get(prec), dict):
                out["speedup_%s_vs_fp64" % prec] = out["fp64"]["solve_ms"] / out[prec]["solve_ms"]
    return out


def invit_section(ts, W, torch, dev, n, precs, steps=20):
    """20 steps of shifted inverse iteration on the same workload (shift per the recipe)."""
    L = 8.0
    shape = (n, n, n)
    f_list = [W.f_harmonic(n, L) for _ in range(3)]
    V2 = bumps_on_device(W, torch, dev, shape, L, 16, 3)
    plan = ts.ts_setup(shape, L, f_list, 1.0)
    lam1 = sum(float(ts.ts_eigvals(plan, k)[0]) for k in range(3))
    shift = lam1 + min(0.0, float(V2.min())) - 1e-4
    Q = [torch.from_numpy(ts.ts_eigvecs(plan, k)[:, 0].copy()).to(dev) for k in range(3)]
    out = {"n": n, "shift": shift, "steps": steps}
    for prec in precs:
        try:
            u = ((Q[0][:, None, None] * Q[1][None, :, None]) * Q[2][None, None, :]).contiguous()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, lam, its = ts.ts_inverse_iteration(plan, V2, shift, u, steps=steps, pcg_rtol=1e-10, precond=prec)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            # eigen-residual ||H u - lambda u|| / |lambda| of the final unit vector (H = H1 + V2)
            r = ts.ts_operator_apply(plan, V2, 0.0, u)
            r.sub_(u, alpha=float(lam[-1]))
            eres = float(torch.linalg.vector_norm(r)) / abs(float(lam[-1])) / float(torch.linalg.vector_norm(u))
            del r
            out[prec] = {"ms": ms, "lambda": float(lam[-1]), "lambda_history": [float(x) for x in lam],
                         "pcg_iters": [int(x) for x in its], "pcg_iters_total": int(sum(its)),
                         "eigen_residual": eres}
            log("inverse iteration n=%d %s: %.1f ms, lambda %.10f, %d PCG iters, eigen-residual %.2e"
                % (n, prec, ms, lam[-1], sum(its), eres))
        except ts.TSError as e:
            out[prec] = "unavailable: %s" % e.status
    return out


def pairwise_on_device(W, torch, dev, shape, L, dtype):
    """V2 = sum_{i<j} 0.5 / (1 + (x_i - x_j)^2), evaluated on the device."""
    d = len(shape)
    ax = [torch.from_numpy(W.grid_nodes(n, L)).to(dev) for n in shape]
    V = torch.zeros(shape, dtype=torch.float64, device=dev)
    for i in range(d):
        for j in range(i + 1, d):
            vi = ax[i].reshape([-1 if k == i else 1 for k in range(d)])
            vj = ax[j].reshape([-1 if k == j else 1 for k in range(d)])
            V += 0.5 / (1.0 + (vi - vj) ** 2)
    return V.to(dtype)


def split_section(ts, W, torch, dev, d, n, steps=100, dt=1e-3):
    """Splitting workload: V1 = sum x^2 on [-6,6]^d, pairwise V2, psi0 = seeded
    superposition of the 4 lowest separable eigenfunctions, 100 steps of 1e-3."""
    import numpy as np
    L = 6.0
    shape = (n,) * d
    N = n ** d
    f = [W.f_harmonic(n, L) for _ in range(d)]
    plan = ts.ts_setup(shape, L, f, 1.0)
    Q = ts.ts_eigvecs(plan, 0)
    w = ts.ts_eigvals(plan, 0)
    terms = W.superposition_terms([Q] * d, [w] * d, 4, seed=4)
    out = {"d": d, "n": n, "dofs": N, "steps": steps, "dt": dt}
    for dtype, prec in ((torch.complex64, "fp32"), (torch.complex64, "fp64"), (torch.complex128, "fp64")):
        V2 = pairwise_on_device(W, torch, dev, shape, L, torch.float32 if dtype == torch.complex64 else torch.float64)
        psi0 = torch.zeros(shape, dtype=dtype, device=dev)
        for cm, idx in terms:
            t = torch.ones((), dtype=dtype, device=dev)
            for k, j in enumerate(idx):
                t = t.unsqueeze(-1) * torch.from_numpy(Q[:, j].copy()).to(dev).to(dtype)
            psi0 += complex(cm) * t
        for scheme in ("strang_bab", "yoshida_bab"):
            psi = psi0.clone()
            ts.ts_split_step(plan, V2, psi, dt, 2, scheme, prec=prec)   # warm-up
            psi = psi0.clone()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            ts.ts_split_step(plan, V2, psi, dt, steps, scheme, prec=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            n_apply = steps + 1 if scheme == "strang_bab" else 3 * steps + 1
            drift = abs(float(torch.linalg.vector_norm(psi)) / float(torch.linalg.vector_norm(psi0)) - 1.0)
            key = "%s_%s" % (scheme, "c128" if dtype == torch.complex128 else
                             ("c64" if prec == "fp32" else "c64_fp64_transforms"))
            sz = 8 if dtype == torch.complex64 else 16
            # algorithmic bytes of one propagation: read and write the state once (2 N s); flops 8 N sum n_k
            gbs = 2.0 * N * sz / (ms / n_apply * 1e-3) / 1e9
            tfl = 8.0 * N * n * d / (ms / n_apply * 1e-3) / 1e12
            out[key] = {"ms_per_step": ms / steps, "ms_per_apply": ms / n_apply, "norm_drift": drift,
                        "dof_s_per_apply": N / (ms / n_apply * 1e-3), "alg_gb_s": gbs, "alg_tflops": tfl,
                        "roofline_ms_per_apply": max(8.0 * N * n * d / (PEAK[prec] * 1e12),
                                                     2.0 * N * sz / (HBM_PEAK * 1e9)) * 1e3}
            out[key]["roofline_frac"] = out[key]["roofline_ms_per_apply"] / (ms / n_apply)
            log("split %dD n=%d %s: %.2f ms/step, %.2f ms/apply (%.0f%% of roofline), drift %.1e"
                % (d, n, key, ms / steps, ms / n_apply, 100 * out[key]["roofline_frac"], drift))
        del V2, psi0, psi
        torch.cuda.empty_cache()
    return out


def qhop_section(ts, W, torch, dev, n=499, T=0.1, dt=0.01, Ms=(3, 5, 7)):
    """The separable splitting example: A = -Delta, B = V1 of eq. (separable_V1)
    on [-8,8]^3, psi0 = prod sin(pi (x_k + L) / 2L), complex128, T = 0.1.
    Strang (BAB) and approximated qHOP with M nodes; error relative to ||psi0||
    against the exact propagator of -Delta + V1."""
    import numpy as np
    L = 8.0
    shape = (n, n, n)
    m = int(round(T / dt))
    v = W.f_separable_v1(n, L)
    x = W.grid_nodes(n, L)
    g = torch.from_numpy(np.sin(np.pi * (x + L) / (2 * L))).to(dev)
    vd = torch.from_numpy(v).to(dev)
    V = (vd[:, None, None] + vd[None, :, None] + vd[None, None, :]).contiguous()
    psi0 = (g[:, None, None] * g[None, :, None] * g[None, None, :]).to(torch.complex128).contiguous()
    norm0 = float(torch.linalg.vector_norm(psi0))
    plan_h = ts.ts_setup(shape, L, [v] * 3, 1.0)
    exact = ts.ts_apply_exp(plan_h, T, psi0)
    del plan_h
    plan = ts.ts_setup(shape, L, [np.zeros(n)] * 3, 1.0)
    out = {"n": n, "dofs": n ** 3, "T": T, "dt": dt,
           "paper_gh200_s": {"strang": 0.9, "M3": 3.0, "M5": 4.8, "M7": 6.7},
           "paper_error": {"strang": 5.22e-3, "M3": 1.02e-3, "M5": 4.11e-4, "M7": 2.21e-4}}
    runs = [("strang", None)] + [("M%d" % M, M) for M in Ms]
    for key, M in runs:
        psi = psi0.clone()
        if M is None:  # warm-up, then the timed run
            ts.ts_split_step(plan, V, psi, dt, 1, "strang_bab")
        else:
            ts.ts_qhop_step(plan, V, psi, dt, 1, M)
        psi.copy_(psi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if M is None:
            ts.ts_split_step(plan, V, psi, dt, m, "strang_bab")
            n_apply = m + 1
        else:
            ts.ts_qhop_step(plan, V, psi, dt, m, M)
            n_apply = m * M + 1
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        err = float(torch.linalg.vector_norm(psi - exact)) / norm0
        out[key] = {"s": sec, "error": err, "propagations": n_apply, "ms_per_propagation": 1e3 * sec / n_apply}
        log("qhop %s at %d^3: %.3f s, error %.3e" % (key, n, sec, err))
        del psi
    del plan, V, psi0, exact
    torch.cuda.empty_cache()
    return out


# Rows of Table tab:accuracy_gh200: (label, precision, dim, k, cells, printed error, GH200 setup s, solve s)
ACCURACY_ROWS = [
    ("fp64_3d_q1", "fp64", 3, 1, 1100, 3.66e-6, 5.2, 0.508),
    ("fp64_3d_q2", "fp64", 3, 2, 550, 1.93e-9, 5.1, 0.512),
    ("fp64_3d_q10", "fp64", 3, 10, 110, 7.66e-13, 6.4, 0.510),
    ("fp64_4d_q10", "fp64", 4, 10, 18, 1.29e-13, 6.2, 0.195),
    ("fp64_6d_q2", "fp64", 6, 2, 17, 2.95e-2, 5.9, 0.258),
    ("fp32_3d_q2", "fp32", 3, 2, 500, 7.17e-7, 5.4, 0.270),
    ("fp32_4d_q10", "fp32", 4, 10, 15, 4.99e-7, 5.8, 0.058),
    ("fp32_4d_q10_199", "fp32", 4, 10, 20, 6.20e-7, 5.8, 0.188),
    ("fp32_6d_q10", "fp32", 6, 10, 3, 4.75e-4, 5.7, 0.052),
    ("bf16_3d_q2", "bf16", 3, 2, 500, 1.65e-2, 5.4, 0.088),
    ("bf16_3d_q2_1599", "bf16", 3, 2, 800, 1.64e-2, 5.6, 0.517),
]


def accuracy_section(ts, W, torch, dev, steps=3):
    """Direct inverse of the paper's test problems with Q^k SEM on [-1,1]^d:
    eq. (test_potential) with u* = sin(pi x) sin(2 pi y) sin(3 pi z) in 3D,
    V = sum x_k^2 with u* = prod sin(k pi x_k) in 4D and 6D.  Reports setup
    and per-solve time and the l2 relative error beside the printed values."""
    import numpy as np
    L = 1.0
    out = {}
    for label, prec, d, k, cells, printed, p_setup, p_solve in ACCURACY_ROWS:
        x = ts.ts_sem_nodes(k, cells, L)
        n = x.size
        if d == 3:
            coef = {2: 1.0, 1: 2.0, 0: 3.0}
            f = [W.f_test_potential(0, L, coef[a], x=x) for a in range(3)]
            modes = [3, 2, 1]
        else:
            f = [W.f_harmonic(0, L, x=x) for _ in range(d)]
            modes = list(range(d, 0, -1))
        t0 = time.perf_counter()
        plan = ts.ts_setup_sem(k, (cells,) * d, L, f, 0.0)
        setup = time.perf_counter() - t0
        dt = torch.float64 if prec == "fp64" else torch.float32
        xd = torch.from_numpy(x).to(dev)
        fac = [torch.sin(mm * np.pi * xd) for mm in modes]
        fd = [torch.from_numpy(fa).to(dev) for fa in f]
        lap = float(sum((mm * np.pi) ** 2 for mm in modes))
        ustar = fac[0]
        rhs = fd[0]
        for a in range(1, d):
            ustar = ustar.unsqueeze(-1) * fac[a]
            rhs = rhs.unsqueeze(-1) + fd[a]
        rhs.add_(lap).mul_(ustar)          # (-Delta + V) u* at the nodes, in place
        if dt != torch.float64:
            rhs = rhs.to(dt)
        u = torch.empty_like(rhs)
        ms, _ = timed(lambda: ts.ts_apply_inverse(plan, rhs, u, prec=prec), steps, 1)
        num = den = 0.0
        for i in range(n):                 # error norms slab by slab (no full-size temporaries)
            num += float(torch.sum((u[i].to(torch.float64) - ustar[i]) ** 2))
            den += float(torch.sum(ustar[i] ** 2))
        err = (num / den) ** 0.5
        out[label] = {"n": n, "d": d, "k": k, "cells": cells, "dofs": n ** d, "setup_s": setup,
                      "solve_s": ms * 1e-3, "l2_rel_err": err, "paper_err": printed,
                      "paper_gh200_setup_s": p_setup, "paper_gh200_solve_s": p_solve}
        log("accuracy %s: %d^%d setup %.2f s solve %.4f s err %.3e (printed %.3e, GH200 %.3f s)"
            % (label, n, d, setup, ms * 1e-3, err, printed, p_solve))
        del plan, rhs, u, ustar, fac
        torch.cuda.empty_cache()
    return out


def small_section(ts, W, torch, dev, reps=200, per_graph=10):
    """Latency-bound case: 3D n = 64 (2.6e5 DoFs, 2 MB; L = 8, f = x^2,
    sigma = 1, N(0,1) right-hand side seed 1, complex128 wavepacket seed 1,
    tau = 0.01): microseconds per FP64 inverse and complex128 propagator apply,
    launched one by one and replayed from a HIP graph of per_graph applies."""
    n, L = 64, 8.0
    shape = (n,) * 3
    plan = ts.ts_setup(shape, L, [W.f_harmonic(n, L)] * 3, 1.0)
    b = torch.from_numpy(W.rhs_normal(shape, 1)).to(dev)
    u = torch.empty_like(b)
    psi = torch.from_numpy(W.gaussian_wavepacket(shape, L, 1)).to(dev)
    out = torch.empty_like(psi)
    res = {"n": n, "dofs": n ** 3}
    for name, fn, y in (("inverse_fp64", lambda: ts.ts_apply_inverse(plan, b, u), u),
                        ("exp_c128", lambda: ts.ts_apply_exp(plan, 0.01, psi, out), out)):
        ms, _ = timed(fn, reps, 5)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(per_graph):
                fn()
        g.replay()
        torch.cuda.synchronize()
        got = y.clone()
        fn()
        torch.cuda.synchronize()
        same = bool(torch.equal(got, y))
        ms_g, _ = timed(g.replay, max(1, reps // per_graph), 2)
        res[name] = {"us_per_apply_eager": ms * 1e3, "us_per_apply_graph": ms_g * 1e3 / per_graph,
                     "graph_equals_eager": same}
        log("64^3 %s: %.1f us/apply eager, %.1f us/apply from a graph (replay == eager: %s)"
            % (name, ms * 1e3, ms_g * 1e3 / per_graph, same))
        del g
    return res


HERMITE_ROWS = [(199, 1.53e-5, 6.31e-5, 2.7, 0.002), (399, 4.05e-6, 2.20e-5, 3.2, 0.024),
                (599, 1.87e-6, 1.20e-5, 3.2, 0.117)]


def hermite_section(ts, W, torch, dev, steps=3):
    """Table tab:hermite_accuracy: (-Delta + V)^{-1} of eq. (test_potential)
    on R^3 by Hermite collocation (ts_hermite_axis + ts_setup_general), exact
    solution prod sin(c (t + 1)) / (1 + t^2); setup and per-solve time, the
    l2 relative error and the weighted L2 error (Gauss-Hermite weights of
    e^{-|x|^2}) beside the printed values."""
    import numpy as np
    out = {}
    for n, p_w, p_l2, p_setup, p_solve in HERMITE_ROWS:
        t0 = time.perf_counter()
        x, m, K = ts.ts_hermite_axis(n)
        fs = [W.f_test_potential(0, 0.0, c, x=x) for c in (3.0, 2.0, 1.0)]
        plan = ts.ts_setup_general([K] * 3, [m] * 3, fs, 0.0, [x] * 3)
        setup = time.perf_counter() - t0
        G = [W.rational_sine(c, x) for c in (1.5 * np.pi, np.pi, 0.5 * np.pi)]
        gd = [torch.from_numpy(g).to(dev) for g, _ in G]
        rhs = torch.zeros((n,) * 3, dtype=torch.float64, device=dev)
        for a in range(3):
            fac = list(gd)
            fac[a] = torch.from_numpy(-G[a][1] + fs[a] * G[a][0]).to(dev)
            rhs += fac[0][:, None, None] * fac[1][None, :, None] * fac[2][None, None, :]
        ustar = gd[0][:, None, None] * gd[1][None, :, None] * gd[2][None, None, :]
        u = torch.empty_like(rhs)
        ms, _ = timed(lambda: ts.ts_apply_inverse(plan, rhs, u), steps, 1)
        e = u - ustar
        wd = torch.from_numpy(m * np.exp(-x * x)).to(dev)
        w3 = wd[:, None, None] * wd[None, :, None] * wd[None, None, :]
        l2 = float(torch.linalg.norm(e) / torch.linalg.norm(ustar))
        weighted = float(torch.sqrt(torch.sum(w3 * e * e)))
        out["n%d" % n] = {"n": n, "dofs": n ** 3, "setup_s": setup, "solve_s": ms * 1e-3, "l2_rel_err": l2,
                          "weighted_l2_err": weighted, "paper_l2_rel_err": p_l2, "paper_weighted_l2_err": p_w,
                          "paper_a100_setup_s": p_setup, "paper_a100_solve_s": p_solve}
        log("hermite %d^3: setup %.2f s solve %.4f s l2 %.3e (printed %.2e) weighted %.3e (printed %.2e, A100 %.3f s)"
            % (n, setup, ms * 1e-3, l2, p_l2, weighted, p_w, p_solve))
        del plan, rhs, u, ustar, e, w3
        torch.cuda.empty_cache()
    return out


def gpe_section(ts, W, torch, dev, betas=(10.0, 100.0), cells=30, k=20, tol=1e-14, maxit=3000):
    """Modified H^1 flow of Table tab:h1_flow: V1 of eq. (separable_V1) on
    [-8,8]^3, Q^20 SEM at 599^3, alpha = 20, tau = 0.1, linear-ground-state
    start; stops when the successive energy change is below tol (relative)."""
    import numpy as np
    L = 8.0
    x = ts.ts_sem_nodes(k, cells, L)
    v = W.f_separable_v1(0, L, x=x)
    t0 = time.perf_counter()
    lap = ts.ts_setup_sem(k, (cells,) * 3, L, [np.zeros_like(x)] * 3, 1.0)
    pv1 = ts.ts_setup_sem(k, (cells,) * 3, L, [v] * 3, 1.0)
    setup = time.perf_counter() - t0
    vd = torch.from_numpy(v).to(dev)
    V = (vd[:, None, None] + vd[None, :, None] + vd[None, None, :]).contiguous()
    out = {"n": x.size, "k": k, "setup_s": setup,
           "paper": {"beta10": {"iters": 175, "total_s": 34.8, "energy": 14.1965761916},
                     "beta100": {"iters": 405, "total_s": 71.9, "energy": 20.6824463703}}}
    for beta in betas:
        u = ts.ts_separable_ground_state(pv1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ts.ts_gpe_h1_flow(lap, V, beta, u, alpha=20.0, tau=0.1, maxit=maxit, tol=tol, raise_on_noconv=False)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        key = "beta%g" % beta
        out[key] = {"iters": r.iters, "s": sec, "s_per_iter": sec / max(r.iters, 1), "energy": r.energy,
                    "eigenvalue": r.eigenvalue}
        log("gpe h1 %s: %d steps %.2f s, E %.12f lambda %.10f" % (key, r.iters, sec, r.energy, r.eigenvalue))
        del u
    del lap, pv1, V
    torch.cuda.empty_cache()
    return out


def gpe1600_section(ts, W, torch, dev, cells=30, k=20):
    """Table tab:au_vs_h1: beta = 1600, V1 of eq. (separable_V1) on [-8,8]^3,
    Q^20 SEM at 599^3, constant initial guess; the a_u flow (tau = 1, PCG with
    (-Delta + V1)^{-1}) and the modified H^1 flow (alpha = 20, tau = 0.1).  The
    flows run until the successive energy change is below 1e-15 (relative);
    the iteration at which |E_k - E*| / E* < 1e-12 (the table's criterion,
    E* = 33.80227900547423) is read off the energy history."""
    import numpy as np
    L, beta, Estar = 8.0, 1600.0, 33.80227900547423
    x = ts.ts_sem_nodes(k, cells, L)
    v = W.f_separable_v1(0, L, x=x)
    lap = ts.ts_setup_sem(k, (cells,) * 3, L, [np.zeros_like(x)] * 3, 1.0)
    pv1 = ts.ts_setup_sem(k, (cells,) * 3, L, [v] * 3, 1.0)
    vd = torch.from_numpy(v).to(dev)
    V = (vd[:, None, None] + vd[None, :, None] + vd[None, None, :]).contiguous()
    shape = (x.size,) * 3
    out = {"n": x.size, "beta": beta, "E_star": Estar,
           "paper_gh200": {"au": {"iters": 66, "linear_solves": 790, "s": 72.8, "energy": 33.80227900550},
                           "h1": {"iters": 272, "linear_solves": 544, "s": 42.6, "energy": 33.80227900551}}}
    for method in ("au", "h1"):
        u = torch.ones(shape, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if method == "au":
            r = ts.ts_gpe_au_flow(pv1, None, beta, u, tau=1.0, maxit=300, tol=1e-15, pcg_rtol=1e-12,
                                  raise_on_noconv=False)
        else:
            r = ts.ts_gpe_h1_flow(lap, V, beta, u, alpha=20.0, tau=0.1, maxit=800, tol=1e-15,
                                  raise_on_noconv=False)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        err = np.abs(r.history - Estar) / Estar
        hit = np.nonzero(err < 1e-12)[0]
        k12 = int(hit[0]) if hit.size else None
        res = {"iters": r.iters, "s": sec, "s_per_iter": sec / max(r.iters, 1), "energy": r.energy,
               "iters_to_1e-12": k12, "s_to_1e-12": None if k12 is None else sec * k12 / max(r.iters, 1)}
        if method == "au":
            res["linear_solves"] = r.linear_iters
        out[method] = res
        log("gpe beta=1600 %s flow: %d steps %.2f s, E %.13f, |E-E*|/E* < 1e-12 after %s steps (~%s s)"
            % (method, r.iters, sec, r.energy, k12, None if k12 is None else "%.1f" % res["s_to_1e-12"]))
        del u
    del lap, pv1, V
    torch.cuda.empty_cache()
    return out


def multilevel_section(ts, W, torch, dev, k=20, cells=(5, 10, 25)):
    """Table tab:multilevel: the stirrer potential, Q^20 SEM 99^3 -> 199^3 -> 499^3."""
    import numpy as np
    L = 8.0
    t0 = time.perf_counter()
    plans, V2s, shifts = [], [], []
    for c in cells:
        x = ts.ts_sem_nodes(k, c, L)
        plan = ts.ts_setup_sem(k, (c,) * 3, L, [4.0 * x * x, x * x, x * x], 1.0)
        xd = torch.from_numpy(x).to(dev)
        V2 = (8.0 * torch.exp(-((xd - 1.0) ** 2)[None, None, :] - (xd ** 2)[None, :, None])
              * torch.ones(x.size, 1, 1, dtype=torch.float64, device=dev)).contiguous()
        plans.append(plan)
        V2s.append(V2)
        shifts.append(0.9 * sum(float(ts.ts_eigvals(plan, a)[0]) for a in range(3)))
    setup = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, lam, steps, its = ts.ts_multilevel_inverse_iteration(plans, V2s, shifts, max_steps=60, lam_tol=1e-13,
                                                            pcg_rtol=1e-12)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    log("multilevel stirrer: lambda %.12f, steps %s, PCG %s, %.1f s (+ %.1f s setup)" % (lam[-1], steps, its, sec,
                                                                                        setup))
    out = {"levels_n": [k * c - 1 for c in cells], "lambda": list(lam), "steps": steps, "pcg_iters": its,
           "solve_s": sec, "setup_s": setup, "paper_lambda": 5.286155366963,
           "paper_a100": {"inverse_iters": [30, 21, 11], "pcg_per_iter": [75, 24, 21], "total_s": 62}}
    del plans, V2s, u
    torch.cuda.empty_cache()
    return out


def serve_run(ts, W, torch, dev, reqs, mode, inputs):
    """Replay the stream against a server.  mode: 'batch' (4 streams, no cap),
    'fp64' (same, every request in plain FP64), 'fifo' (1 stream, 1 request),
    'saturate' (as batch, every request submitted at once: saturation throughput).
    Output tensors come from per-class pools of at most ~16 GB each (a request
    whose pool is empty is submitted once a buffer returns; its latency still
    counts from its arrival)."""
    import numpy as np
    n_streams, max_active = (1, 1) if mode == "fifo" else (4, 0)
    srv = ts.Server(64 << 30, n_streams, max_active)
    L = 8.0
    pools, made = {}, {}

    def request_args(r):
        shape = r["shape"]
        V2 = inputs["v2"][shape] if r["v2"] else None
        if r["kind"].startswith("inverse"):
            prec = "fp64" if (mode == "fp64" or r["kind"] == "inverse_fp64") else "bf16"
            return ts.TS_REQ_INVERSE, inputs["rhs"][shape], prec, V2, inputs["sigma"][shape]
        c128 = mode == "fp64"
        x = inputs["psi128" if c128 else "psi64"][shape]
        V2 = None if V2 is None else (V2 if c128 else inputs["v2f"][shape])
        return ts.TS_REQ_EXP, x, "fp64" if c128 else "fp32", V2, 1.0

    def take_out(x):
        key = (tuple(x.shape), x.dtype)
        lst = pools.setdefault(key, [])
        if lst:
            return lst.pop()
        cap = max(2, min(256, int(16e9 // (x.numel() * x.element_size()))))
        if made.get(key, 0) < cap:
            made[key] = made.get(key, 0) + 1
            return torch.empty_like(x)
        return None

    def submit(r, tag):
        kind, x, prec, V2, sigma = request_args(r)
        out = take_out(x)
        if out is None:
            return None, None
        try:
            if kind == ts.TS_REQ_INVERSE:
                t = srv.submit(kind, r["shape"], L, inputs["f"][r["shape"]], sigma, x, out, prec=prec, V2=V2,
                               rtol=1e-10, maxit=500 if V2 is not None else 60, tag=tag)
            else:
                t = srv.submit(kind, r["shape"], L, inputs["f"][r["shape"]], sigma, x, out, prec=prec, V2=V2,
                               tau=r["tau"], dt=1e-2, tag=tag)
        except ts.TSError as e:
            pools[(tuple(out.shape), out.dtype)].append(out)
            if e.code != ts.TS_ERR_BUSY:   # plan reserve held by running requests: retry later
                raise
            return None, None
        return t, out

    # warm the plan cache and the kernels with one request per (shape, kind, V2)
    seen = set()
    for r in reqs:
        k = (r["shape"], r["kind"], r["v2"])
        if k not in seen:
            seen.add(k)
            t, out = submit(r, 0)
            srv.drain()
            pools[(tuple(out.shape), out.dtype)].append(out)
    torch.cuda.synchronize()
    t0 = srv.clock()
    tickets = {}
    waiting = []                      # arrived, not yet submitted (no free output buffer)
    upcoming = list(enumerate(reqs))
    results = {}
    while upcoming or waiting or tickets:
        now = srv.clock() - t0
        while upcoming and (mode == "saturate" or upcoming[0][1]["t"] <= now):
            waiting.append(upcoming.pop(0))
        still = []
        for i, r in waiting:
            t, out = submit(r, i)
            if t is None:
                still.append((i, r))
            else:
                tickets[i] = (t, out)
        waiting = still
        for i in list(tickets):
            t, out = tickets[i]
            res = srv.poll(t)
            if res is not None:
                results[i] = (res, t0 + reqs[i]["t"])
                pools[(tuple(out.shape), out.dtype)].append(out)
                del tickets[i]
        time.sleep(0.0005)
    if mode == "saturate":
        results = {i: (res, t0) for i, (res, _) in results.items()}
    makespan = max(res.t_done for res, _ in results.values()) - t0
    lat = np.array([res.t_done - arr for res, arr in results.values()])
    ok = sum(1 for res, _ in results.values() if res.status == 0)
    dofs = sum(int(np.prod(r["shape"])) for r in reqs)
    srv.close()
    del pools
    torch.cuda.empty_cache()
    by = {}
    for i, (res, arr) in results.items():
        key = "%dD_n%d_%s%s" % (len(reqs[i]["shape"]), reqs[i]["shape"][0], reqs[i]["kind"],
                                 "_v2" if reqs[i]["v2"] else "")
        by.setdefault(key, []).append(res.t_done - arr)
    by = {k: {"count": len(v), "p50_ms": float(np.percentile(v, 50) * 1e3), "p99_ms": float(np.percentile(v, 99) * 1e3)}
          for k, v in sorted(by.items())}
    return {"by_class": by,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "makespan_s": makespan, "dof_s": dofs / makespan, "ok": ok, "requests": len(reqs)}


def serve_section(ts, W, torch, dev, count, rate=200.0):
    """Serving mix: Poisson 200 req/s over {2D 2048; 3D 128/256/512; 4D 64; 6D 16}
    x {inverse FP64, inverse mixed (BF16 + refinement / BF16-preconditioned PCG),
    exp complex64 tau ~ U[1e-3, 1e-1]}, V2 zero or 8 seeded bumps."""
    L = 8.0
    reqs = W.serve_stream(5, count, rate)
    inputs = {"f": {}, "v2": {}, "v2f": {}, "rhs": {}, "psi64": {}, "psi128": {}, "sigma": {}}
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    for shape in W.SERVE_SHAPES:
        inputs["f"][shape] = [W.f_harmonic(n, L) for n in shape]
        V2 = bumps_on_device(W, torch, dev, shape, L, 8, 5)
        inputs["v2"][shape] = V2
        inputs["v2f"][shape] = V2.to(torch.float32)
        inputs["rhs"][shape] = torch.randn(shape, dtype=torch.float64, device=dev, generator=gen)
        facs = W.wavepacket_factors(shape, L, 5)
        psi = torch.ones((), dtype=torch.complex128, device=dev)
        for g in facs:
            psi = psi.unsqueeze(-1) * torch.from_numpy(g).to(dev)
        inputs["psi128"][shape] = psi.contiguous()
        inputs["psi64"][shape] = psi.to(torch.complex64)
        # sigma: 1, raised so that H1 + V2 + sigma >= 0.5 (lambda_min(H1) >= sum of min f_k)
        lam_lb = sum(float(min(f)) for f in inputs["f"][shape])
        inputs["sigma"][shape] = max(1.0, 0.5 - lam_lb - float(V2.min()))
    out = {"requests": count, "rate_per_s": rate, "arrival_span_s": reqs[-1]["t"]}
    for mode in ("batch", "fp64", "fifo", "saturate"):
        out[mode] = serve_run(ts, W, torch, dev, reqs, mode, inputs)
        log("serve %s: p50 %.1f ms p99 %.1f ms, %.3e DoF/s, %d/%d ok" % (
            mode, out[mode]["p50_ms"], out[mode]["p99_ms"], out[mode]["dof_s"], out[mode]["ok"], count))
    return out


def cpu_baseline(n, depth):
    """The oracle's six mode products on slabs holding `depth` x n full fibres per axis."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((n, n))   # stand-in factor: the loops' cost does not depend on values
    X = rng.standard_normal((depth, n, n))
    total = 0.0
    for axis, shape in ((2, (depth, n, n)), (1, (depth, n, n)), (0, (n, n, depth))):
        Xs = X.reshape(shape)
        for transpose in (True, False):
            t0 = time.perf_counter()
            oracle.mode_product(shape, axis, Q, Xs, transpose)
            total += (time.perf_counter() - t0) * (n / depth)
    N = float(n) ** 3
    return {"value": N / total, "unit": "DoF/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "oracle mode products (3 axes x forward/backward) over %d x %d full-length fibres "
                      "per axis of the %d^3 grid (slabs of depth %d), scaled by %d/%d to the full apply; "
                      "a random %dx%d matrix stands in for Q (the loop cost is value-independent); the "
                      "O(N) diagonal scaling is not timed" % (depth, n, n, depth, n, depth, n, n)}


SECTIONS = ["headline", "variants", "bf16", "vendor_gemm", "small64", "pcg", "split", "qhop", "table", "hermite", "gpe",
            "serve", "cpu"]


def apply_rooflines(N, n, d, t_ms, prec, flops_exec=None):
    """Roofline of one apply: the algorithmic flops 4 N sum(n_k) (real data) over
    the time, against the MFMA peak of the transform precision; flops_exec, if
    given, is what the kernels execute (half on folded axes)."""
    alg = 4.0 * N * n * d
    out = {"alg_flops": alg, "alg_tflops": alg / (t_ms * 1e-3) / 1e12, "peak_tflops": PEAK[prec]}
    out["alg_frac"] = out["alg_tflops"] / PEAK[prec]
    if flops_exec is not None:
        out["executed_flops"] = flops_exec
        out["executed_tflops"] = flops_exec / (t_ms * 1e-3) / 1e12
        out["executed_frac"] = out["executed_tflops"] / PEAK[prec]
    return out


def headline_section(ts, W, torch, dev, args):
    """The 1e9-DoF FP64 inverse apply (the headline value) and its dominant kernel."""
    n, L, sigma = args.n, 10.0, 1.0
    shape = (n, n, n)
    N = n ** 3
    f = [W.f_harmonic_cos(n, L) for _ in range(3)]
    t0 = time.perf_counter()
    plan = ts.ts_setup(shape, L, f, sigma)
    setup_s = time.perf_counter() - t0
    log("setup %.2f s" % setup_s)
    gen = torch.Generator(device=dev)
    gen.manual_seed(2)
    b = torch.randn(shape, dtype=torch.float64, device=dev, generator=gen)
    u = torch.empty_like(b)
    ms, wall = timed(lambda: ts.ts_apply_inverse(plan, b, u, prec="fp64"), args.steps, args.warmup)
    value = N / (ms * 1e-3)
    log("fp64 inverse %.2f ms/apply -> %.3e DoF/s" % (ms, value))
    # FP64 residual of the timed result (self-check; parity lives in tests/)
    r = ts.ts_operator_apply(plan, None, sigma, u)
    r.sub_(b)
    resid = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))
    del r

    # dominant kernel: the forward pass on axis 1 (a column pass, half extent on a symmetric axis,
    # on input folded beforehand as inside the apply), timed on its own with HIP events on the
    # stream the library launches on
    fmask = ts.ts_fold_axes(plan)
    folded = bool(fmask & 2)
    deferred = folded and bin(fmask).count("1") >= 2
    hh, cc = n // 2, n % 2
    flops_alg = 2.0 * N * n                      # per pass, dense (any f_k)
    flops_exec = 2.0 * (N / n) * ((hh + cc) ** 2 + hh ** 2) if folded else flops_alg
    work = torch.empty_like(b)
    t_pass, _ = timed(lambda: ts.ts_mode_pass(plan, 1, True, b, work, folded=deferred), args.steps, 1)
    t_back, _ = timed(lambda: ts.ts_mode_pass(plan, 1, False, b, work, folded=deferred), args.steps, 1)
    t_bfly = None
    if deferred:
        t_bfly, _ = timed(lambda: ts.ts_fold_butterfly(plan, fmask, b, work), args.steps, 1)
        log("single launches: forward pass %.2f ms, backward pass %.2f ms, %d-axis butterfly %.2f ms"
            % (t_pass, t_back, bin(fmask).count("1"), t_bfly))
    # the same apply and pass with the half-extent passes off: what a potential
    # without reflection symmetry runs
    ts.ts_set_fold(plan, False)
    ms_plain, _ = timed(lambda: ts.ts_apply_inverse(plan, b, u, prec="fp64"), max(2, args.steps // 2), 1)
    t_plain, _ = timed(lambda: ts.ts_mode_pass(plan, 1, True, b, work), max(2, args.steps // 2), 1)
    ts.ts_set_fold(plan, True)
    log("plain passes: apply %.2f ms (%.3e DoF/s), forward column pass %.2f ms = %.1f%% of the FP64 peak"
        % (ms_plain, N / (ms_plain * 1e-3), t_plain, 100 * flops_alg / (t_plain * 1e-3) / 1e12 / PEAK["fp64"]))
    del work
    achieved = flops_alg / (t_pass * 1e-3) / 1e12
    executed = flops_exec / (t_pass * 1e-3) / 1e12
    traffic, tinfo = measured_traffic()
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp64"], "traffic": traffic, "traffic_unit": "bytes per launch",
                "traffic_algorithmic": 2 * 8 * N,
                "achieved_basis": "algorithmic flops 2 N n per pass (dense mode product), per the work count of "
                                  "the method; the folded kernel executes %.3g of them" % (flops_exec / flops_alg),
                "executed_flops_per_launch": flops_exec, "executed_achieved": executed,
                "executed_frac": executed / PEAK["fp64"], "fold_factor": flops_exec / flops_alg,
                "traffic_note": (tinfo if isinstance(tinfo, str) else
                                 (None if tinfo is None else {k: tinfo[k] for k in ("fetch_bytes", "write_bytes",
                                                                                     "copy_scale", "profile")})),
                "kernel": ("k_mode_mfma<double, cols, FOLD=3>: FP64 16x16x4 MFMA forward pass over half the extent "
                           "on folded data (even/odd halves of a symmetric axis)" if deferred else
                           "k_mode_mfma<double, cols, FOLD=1>: FP64 16x16x4 MFMA forward pass over half the extent "
                           "(even/odd halves of a symmetric axis)" if folded else
                           "k_mode_mfma<double, cols>: FP64 16x16x4 MFMA forward pass"),
                "per_launch_flops": flops_alg, "avg_launch_ms": t_pass,
                "backward_pass_ms": t_back, "butterfly_ms": t_bfly, "apply_ms": ms, "folded": folded,
                "plain": {"kernel": "k_mode_mfma<double, cols>: FP64 16x16x4 MFMA forward pass, full extent",
                          "avg_launch_ms": t_plain,
                          "achieved": flops_alg / (t_plain * 1e-3) / 1e12,
                          "frac": flops_alg / (t_plain * 1e-3) / 1e12 / PEAK["fp64"],
                          "apply_ms": ms_plain, "apply_dof_s": N / (ms_plain * 1e-3),
                          "apply": apply_rooflines(N, n, 3, ms_plain, "fp64")}}
    roofline["apply"] = apply_rooflines(N, n, 3, ms, "fp64", flops_exec * 6)
    extra = {"setup_s": setup_s, "fp64_relres": resid, "wall_s_timed": wall}
    state = {"plan": plan, "b": b, "shape": shape, "N": N, "n": n, "L": L, "flops_exec": flops_exec,
             "flops_alg": flops_alg}
    return value, ms, roofline, extra, state


def variants_section(ts, W, torch, dev, args, st):
    """FP32 / BF16 transforms, the mixed inverse refined to 1e-10, propagators."""
    import numpy as np
    plan, b, shape, N, n, L = st["plan"], st["b"], st["shape"], st["N"], st["n"], st["L"]
    tau = 0.01
    extra = {}
    u = torch.empty_like(b)
    for prec in ("fp32", "bf16"):
        try:
            msx, _ = timed(lambda: ts.ts_apply_inverse(plan, b, u, prec=prec), args.steps, 1)
            extra["inverse_%s_dof_s" % prec] = N / (msx * 1e-3)
            extra["inverse_%s_ms" % prec] = msx
            extra["inverse_%s_roofline" % prec] = apply_rooflines(
                N, n, 3, msx, prec, st["flops_exec"] * 6 if prec == "fp32" else None)
            if prec == "bf16":
                # HBM side: one BF16 apply moves 2 N s_io + (passes) x 2 N x 2 B at the least
                extra["inverse_bf16_roofline"]["hbm_alg_bytes"] = 2.0 * N * 8
                extra["inverse_bf16_roofline"]["hbm_alg_ms"] = 2.0 * N * 8 / HBM_PEAK / 1e6
            log("%s inverse %.2f ms/apply (%.1f%% of the %s MFMA peak on the algorithmic flops)"
                % (prec, msx, 100 * extra["inverse_%s_roofline" % prec]["alg_frac"], prec))
        except ts.TSError as e:
            extra["inverse_%s" % prec] = "unavailable: %s" % e.status
    # mixed-precision direct inverse refined to 1e-10 (FP64 residuals, FP32 / BF16 inner applies)
    for inner in ("fp32", "bf16"):
        ur = torch.empty_like(b)
        it_rr = {}

        def run_refined():
            _, it_rr["it"], it_rr["rr"] = ts.ts_solve_refined(plan, b, ur, inner=inner, rtol=1e-10, maxit=60)
        msr, _ = timed(run_refined, max(1, args.steps // 4), 1)
        extra["refined_%s" % inner] = {"ms": msr, "iters": it_rr["it"], "relres": it_rr["rr"],
                                      "dof_s": N / (msr * 1e-3)}
        log("%s inverse refined to 1e-10: %.1f ms, %d iterations, relres %.2e"
            % (inner, msr, it_rr["it"], it_rr["rr"]))
        del ur
    del u
    facs = W.wavepacket_factors(shape, L, 2)
    g = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in facs]
    psi = (g[0][:, None, None] * g[1][None, :, None]) * g[2][None, None, :]
    out = torch.empty_like(psi)
    msx, _ = timed(lambda: ts.ts_apply_exp(plan, tau, psi, out, prec="fp64"), max(1, args.steps // 2), 1)
    extra["exp_c128_fp64_dof_s"] = N / (msx * 1e-3)
    extra["exp_c128_fp64_ms"] = msx
    log("c128 exp %.2f ms/apply" % msx)
    del out
    psi64 = psi.to(torch.complex64)
    del psi
    out64 = torch.empty_like(psi64)
    msx, _ = timed(lambda: ts.ts_apply_exp(plan, tau, psi64, out64, prec="fp32"), args.steps, 1)
    extra["exp_c64_fp32_dof_s"] = N / (msx * 1e-3)
    extra["exp_c64_fp32_ms"] = msx
    log("c64 exp %.2f ms/apply" % msx)
    del psi64, out64
    return extra


def bf16_section(ts, W, torch, dev, args):
    """The BF16 inverse apply of the 1e9-DoF workload alone (for counter runs):
    setup, then `steps` timed applies of FP64 data with BF16 transforms."""
    n, L = args.n, 10.0
    shape = (n, n, n)
    plan = ts.ts_setup(shape, L, [W.f_harmonic_cos(n, L) for _ in range(3)], 1.0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(2)
    b = torch.randn(shape, dtype=torch.float64, device=dev, generator=gen)
    u = torch.empty_like(b)
    ms, _ = timed(lambda: ts.ts_apply_inverse(plan, b, u, prec="bf16"), args.steps, 1)
    log("bf16 inverse %.2f ms/apply" % ms)
    return {"inverse_bf16_ms": ms, "roofline": apply_rooflines(n ** 3, n, 3, ms, "bf16")}


def vendor_gemm_section(torch, dev, n, reps=10):
    """Yardstick only (not the library): the vendor BF16 GEMM (torch.matmul /
    torch.bmm on random BF16 tensors) on the shapes of the BF16 passes of the
    n^3 apply: the row passes' [n^2 x n] x [n x n], the column passes' n batched
    [n x n] x [n x n], and axis 0 as one [n x n] x [n x n^2] product; one warm-up,
    then `reps` timed products each."""
    def t(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3
    N = n ** 3
    X = torch.randn(N // n, n, device=dev, dtype=torch.bfloat16)
    Q = torch.randn(n, n, device=dev, dtype=torch.bfloat16)
    Qb = Q.t().contiguous().expand(n, n, n)
    out = {"n": n}
    for key, fn in (("rows_ms", lambda: torch.matmul(X, Q)), ("cols_batched_ms", lambda: torch.bmm(Qb, X.view(n, n, n))),
                    ("axis0_ms", lambda: torch.matmul(Q, X.view(n, n * n)))):
        ms = t(fn)
        out[key] = ms
        log("vendor BF16 GEMM n=%d %s: %.3f ms = %.0f TFLOP/s" % (n, key, ms, 2.0 * N * n / ms / 1e9))
    del X, Q, Qb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1000, help="points per axis (1000 is the headline workload)")
    ap.add_argument("--only", default="",
                    help="comma-separated sections to run (%s); the headline value is then omitted unless "
                         "'headline' is listed" % ",".join(SECTIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-depth", type=int, default=96)
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--no-table", action="store_true", help="skip the Table tab:accuracy_gh200 rows")
    ap.add_argument("--no-gpe", action="store_true", help="skip the GPE and multi-level sections")
    ap.add_argument("--split-steps", type=int, default=100)
    ap.add_argument("--pcg-sizes", default="256,512")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB device copy three times first (reference for HBM byte counters)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path in this build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_20491_amd as ts
    import workloads as W

    if args.only:
        run = set(x.strip() for x in args.only.split(",") if x.strip())
        unknown = run - set(SECTIONS)
        if unknown:
            print("unknown sections: %s" % sorted(unknown), file=sys.stderr)
            sys.exit(2)
    else:
        run = set(SECTIONS)
        if args.no_extras:
            run -= {"variants", "small64"}
        if args.no_pcg:
            run.discard("pcg")
        if args.no_split:
            run -= {"split", "qhop"}
        if args.no_table:
            run -= {"table", "hermite"}
        if args.no_gpe:
            run.discard("gpe")
        if args.serve_requests <= 0:
            run.discard("serve")
        if args.no_cpu_baseline:
            run.discard("cpu")

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        # 2^27 doubles: each copy reads and writes exactly 1 GiB
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 copies of 1 GiB")
    n = args.n
    N = n ** 3
    value = ms = roofline = None
    extra = {}
    if "headline" in run or "variants" in run:
        value, ms, roofline, extra, st = headline_section(ts, W, torch, dev, args)
        if "headline" not in run:
            value = ms = roofline = None
        if "variants" in run:
            extra.update(variants_section(ts, W, torch, dev, args, st))
        del st
        torch.cuda.empty_cache()
    if "bf16" in run and args.only:
        extra["bf16_only"] = bf16_section(ts, W, torch, dev, args)
        torch.cuda.empty_cache()
    if "vendor_gemm" in run and args.only:
        extra["vendor_gemm"] = vendor_gemm_section(torch, dev, n)
        torch.cuda.empty_cache()
    if "small64" in run:
        extra["small_64"] = small_section(ts, W, torch, dev)
    if "pcg" in run:
        precs = ["fp64", "fp32", "bf16"]
        for m in [int(x) for x in args.pcg_sizes.split(",") if x]:
            extra["pcg_n%d" % m] = pcg_section(ts, W, torch, dev, m, precs)
            extra["inverse_iteration_n%d" % m] = invit_section(ts, W, torch, dev, m, precs)
            torch.cuda.empty_cache()
    if "split" in run:
        extra["split_6d_n24"] = split_section(ts, W, torch, dev, 6, 24, steps=args.split_steps)
        extra["split_9d_n8"] = split_section(ts, W, torch, dev, 9, 8, steps=args.split_steps)
    if "qhop" in run:
        extra["qhop_separable_499"] = qhop_section(ts, W, torch, dev)
    if "table" in run:
        extra["accuracy_table"] = accuracy_section(ts, W, torch, dev)
    if "hermite" in run:
        extra["hermite_table"] = hermite_section(ts, W, torch, dev)
    if "gpe" in run:
        extra["gpe_h1_flow_599"] = gpe_section(ts, W, torch, dev)
        extra["gpe_beta1600_599"] = gpe1600_section(ts, W, torch, dev)
        extra["multilevel_stirrer"] = multilevel_section(ts, W, torch, dev)
    if "serve" in run:
        extra["serving"] = serve_section(ts, W, torch, dev, args.serve_requests)
        torch.cuda.empty_cache()
    extra["paper_context"] = ("FP64 direct inverse, 1099^3 (Q^1 = FD), NVIDIA GH200: 0.508 s = 2.61e9 DoF/s "
                              "(Table tab:accuracy_gh200); not the same workload or hardware")
    extra["sections"] = sorted(run)
    torch.cuda.synchronize()

    cpu = None
    if "cpu" in run:
        t0 = time.perf_counter()
        cpu = cpu_baseline(n, args.cpu_depth)
        log("cpu baseline %.3e DoF/s (%.1f s)" % (cpu["value"], time.perf_counter() - t0))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D separable inverse apply (H1+sigma)^-1 b, n=%d per axis (%.3g DoFs), "
                               "FD on [-10,10]^3, V1=sum(x^2+0.5cos 2x), sigma=1, N(0,1) RHS" % (n, N),
                   "n": n, "d": 3, "dofs": N, "precision": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
    # Every GPU result is synchronised and the line is printed: leave at once
    # rather than through the interpreter's teardown (the caching allocator and
    # the runtime release tens of GB of device memory there), so the process is
    # gone when the caller's clock stops.  Under rocprofv3 (which writes its
    # records from exit handlers) the normal teardown runs.
    sys.stdout.flush()
    sys.stderr.flush()
    if "ROCPROF_OUTPUT_PATH" not in os.environ:
        os._exit(0)
