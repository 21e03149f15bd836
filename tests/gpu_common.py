"""Helpers shared by the GPU tests: build the library plan and the oracle plan
from the same seeded per-axis samples, and compare results."""
import numpy as np
import torch

import oracle
import paper_2605_20491_amd as ts
import workloads as W

DEV = "cuda:0"


def make_pair(shape, L, kind="harm", sigma=1.0, seed=0):
    """Library plan and oracle plan of the same operator."""
    if kind == "harm":
        f = [W.f_harmonic(n, L) for n in shape]
    elif kind == "cos":
        f = [W.f_harmonic_cos(n, L) for n in shape]
    elif kind == "rand":
        rng = np.random.default_rng(seed)
        f = [rng.uniform(0.0, 5.0, size=n) for n in shape]
    else:
        raise ValueError(kind)
    plan = ts.ts_setup(shape, L, f, sigma)
    oplan = oracle.make_plan(shape, L, f)
    return plan, oplan, f


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def maxrel(a, b):
    """max|a - b| / max|b|: the elementwise companion of rel()."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return t if dtype is None else t.to(dtype)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def announce(msg):
    print("[gpu-test]", msg, flush=True)


EPS = np.finfo(np.float64).eps


def exp_tol(oplan, tau):
    """FP64 parity tolerance of the propagator.

    exp(-i tau H) moves by at most |tau| ||dH|| when H moves by dH.  Two
    backward-stable eigensolvers (the library's QL, the oracle's Jacobi) each
    reproduce H only up to a few eps ||H||, so two correct results differ by
    ~ |tau| eps ||H1|| times a modest constant (50 covers the sqrt(n) growth
    measured at n = 1000).  Below tau ||H1|| ~ 200 the 1e-12 target binds.
    """
    normH = sum(float(l[-1]) for l in oplan.lam)
    return max(1e-12, 50.0 * abs(tau) * EPS * normH)


def inv_tol(oplan, shift):
    """FP64 parity tolerance of (H1 + shift)^{-1}.

    Each eigensolver returns eigenvalues within a few eps ||H1|| of the exact
    ones, and a mode's coefficient b_j / (Lambda_j + shift) moves relatively
    by dLambda / (Lambda_j + shift); the lowest mode is the most sensitive.
    Two correct results therefore differ by up to ~4 eps ||H1|| /
    (lambda_min + shift); for shifts far from -lambda_min the 1e-12 target binds.
    """
    normH = sum(float(l[-1]) for l in oplan.lam)
    lam_min = sum(float(l[0]) for l in oplan.lam)
    return max(1e-12, 4.0 * EPS * normH / (lam_min + shift))
