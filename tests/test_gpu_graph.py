"""The applies under HIP graph capture: torch.cuda.graph records the library's
launches on the capturing stream (no allocation, copy, fill or host wait sits
on the apply path once its workspace exists).  Each graph is replayed several
times with eager work of the program in between, and every replay must equal
the eager result bit for bit (the kernels are deterministic).  Cases: the FP64
inverse and the complex128 propagator on the MFMA path (64^3, symmetric axes:
half-extent passes), a Q^k SEM plan (mass scaling) and the grouped small-extent
path (6D n = 8), and the BF16 inverse."""
import numpy as np
import pytest
import torch

import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce

pytestmark = pytest.mark.gpu


def _capture_and_check(fn, y, reps=3, per_graph=4):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()  # workspace allocation happens here, outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    fn()
    torch.cuda.synchronize()
    eager = y.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            fn()
    for r in range(reps):
        y.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, eager), "replay %d differs from the eager result" % r
        fn()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(y, eager)
    return True


@pytest.mark.parametrize("case", ["fd64", "sem", "small6d"])
def test_apply_graph_replays_equal_eager(case):
    if case == "fd64":
        n, L = 64, 8.0
        plan = ts.ts_setup((n,) * 3, L, [W.f_harmonic_cos(n, L)] * 3, 1.0)
        assert ts.ts_fold_axes(plan) == 7
    elif case == "sem":
        k, cells, L = 4, (12, 10, 9), 6.0
        fs = [W.f_harmonic(0, L, x=ts.ts_sem_nodes(k, c, L)) for c in cells]
        plan = ts.ts_setup_sem(k, cells, L, fs, 1.0)
    else:
        n, L = 8, 4.0
        plan = ts.ts_setup((n,) * 6, L, [W.f_harmonic(n, L)] * 6, 1.0)
    b = torch.from_numpy(W.rhs_normal(plan.shape, 1)).to(DEV)
    u = torch.empty_like(b)
    _capture_and_check(lambda: ts.ts_apply_inverse(plan, b, u), u)
    psi = torch.from_numpy(W.complex_normal(plan.shape, 2)).to(DEV)
    out = torch.empty_like(psi)
    _capture_and_check(lambda: ts.ts_apply_exp(plan, 0.02, psi, out), out)
    if case == "fd64":
        b32 = b.float()
        u32 = torch.empty_like(b32)
        _capture_and_check(lambda: ts.ts_apply_inverse(plan, b32, u32, prec="bf16"), u32)
    announce("graph %s: replays equal eager" % case)
