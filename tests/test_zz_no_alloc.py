"""ts_apply_inverse_noalloc: the inverse apply with its scratch in the
library's static device array.  Through the C ABI it must give exactly what
ts_apply_inverse gives (same kernels, deterministic), on two calls in a row
with the second smaller than the first (the array keeps the first call's
contents), for the MFMA passes and the grouped small-extent passes, and it
must refuse an apply whose scratch exceeds the array.
"""
import numpy as np
import pytest
import torch

import paper_2605_20491_amd as ts
import workloads as W
from gpu_common import DEV, announce, to_dev

pytestmark = pytest.mark.gpu


def _plan(shape, L=8.0):
    return ts.ts_setup(shape, L, [W.f_harmonic_cos(n, L) for n in shape], 1.0)


@pytest.mark.parametrize("shapes,prec,dtype", [
    (((160, 150, 144), (96, 80, 72)), "fp64", torch.float64),
    (((160, 150, 144), (64, 40, 33)), "fp32", torch.float32),
    (((130, 128, 100), (70, 66, 64)), "bf16", torch.float64),
    (((20, 18, 16, 14, 12), (12, 10, 9, 8)), "fp64", torch.float64),
])
def test_noalloc_equals_apply_inverse(shapes, prec, dtype):
    for i, shape in enumerate(shapes):
        announce("no-alloc inverse %s %s, call %d" % (shape, prec, i + 1))
        plan = _plan(shape)
        b = to_dev(W.rhs_normal(shape, 20 + i)).to(dtype)
        u = torch.full_like(b, float("nan"))
        ts.ts_apply_inverse_noalloc(plan, b, u, prec=prec)
        ref = ts.ts_apply_inverse(plan, b, prec=prec)
        torch.cuda.synchronize()
        same = bool(torch.equal(u, ref))
        if not same:
            d = float((u.double() - ref.double()).norm() / ref.double().norm())
            announce("  differs from ts_apply_inverse: %.3e" % d)
        assert same


def test_noalloc_rejects_oversized_apply():
    shape = (340, 340, 340)   # 3.9e7 points: 314 MB of FP64 workspace > 256 MiB
    plan = _plan(shape)
    b = torch.zeros(shape, dtype=torch.float64, device=DEV)
    u = torch.empty_like(b)
    with pytest.raises(ts.TSError) as e:
        ts.ts_apply_inverse_noalloc(plan, b, u)
    assert e.value.code == ts.TS_ERR_INVALID
    announce("oversized no-alloc apply refused: %s" % e.value)
    # the plain entry point still serves it
    ts.ts_apply_inverse(plan, b, u)
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0.0
