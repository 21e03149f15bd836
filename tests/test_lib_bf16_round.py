"""The library's BF16 rounding, run on the host through ts_bf16_round (the
same inline code the kernels use), against an exact round-to-nearest-even
written with rational arithmetic.

Route 0 (factor copies: FP64 rounded once) must equal exact RNE everywhere.
Route 1 (data: FP64 -> FP32 -> BF16, each RNE) must equal exact RNE of the
FP32-rounded value, and so differs from route 0 exactly where the FP32
rounding lands on a BF16 midpoint (double rounding); the crafted cases below
show both kinds.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import paper_2605_20491_amd as ts


def exact_bf16_bits(v: float) -> int:
    """Round v to BF16 (8-bit exponent, 7 fraction bits, subnormals kept),
    nearest with ties to even, by exact rational arithmetic."""
    if math.isnan(v):
        return 0x7fc0
    sign = 0x8000 if math.copysign(1.0, v) < 0 else 0
    a = abs(v)
    if math.isinf(a):
        return sign | 0x7f80
    if a == 0.0:
        return sign
    _, ex = math.frexp(a)          # a = m 2^ex, 0.5 <= m < 1
    e = max(ex - 1, -126)          # exponent of the binade (subnormals share -126)
    ulp = Fraction(2) ** (e - 7)
    q = Fraction(a) / ulp
    lo = math.floor(q)
    rem = q - lo
    k = lo + 1 if (rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1)) else lo
    val = k * ulp
    if val >= Fraction(2) ** 128:
        return sign | 0x7f80
    f32 = np.float32(float(val))   # a BF16 value is exact in FP32 (and in FP64)
    assert Fraction(float(f32)) == val
    return sign | int(f32.view(np.uint32) >> np.uint32(16))


def bf16_value(bits: int) -> float:
    return float(np.uint32(bits << 16).view(np.float32))


def crafted_values():
    """BF16 midpoints and their FP64 neighbours (1 ulp either side), over
    normal and subnormal binades and both signs; values exactly at BF16
    points; the largest finite and overflow neighbourhood."""
    rng = np.random.default_rng(0)
    out = []
    for _ in range(600):
        e = int(rng.integers(-133, 127))
        frac = int(rng.integers(0, 128))
        b = max(e, -126)
        base = (1 + frac / 128.0) * 2.0 ** e if e >= -126 else frac * 2.0 ** -133
        mid = base + 2.0 ** (b - 8)
        for v in (mid, np.nextafter(mid, np.inf), np.nextafter(mid, -np.inf), base):
            out.append(float(v))
            out.append(-float(v))
    big = bf16_value(0x7f7f)
    out += [big, big + 2.0 ** 119, np.nextafter(big + 2.0 ** 119, 0.0), 1e300, -1e300, 0.0, -0.0,
            np.inf, -np.inf, 5e-324, 2.0 ** -134, 2.0 ** -133, 3 * 2.0 ** -134]
    return np.array(out, dtype=np.float64)


def test_exact_reference_on_known_values():
    """The rational reference itself, on values whose BF16 encoding is known."""
    assert exact_bf16_bits(1.0) == 0x3f80
    assert exact_bf16_bits(-2.0) == 0xc000
    assert exact_bf16_bits(1.0 + 2.0 ** -8) == 0x3f80           # tie -> even (down)
    assert exact_bf16_bits(1.0 + 3 * 2.0 ** -8) == 0x3f82       # tie -> even (up)
    assert exact_bf16_bits(1.0 + 2.0 ** -8 + 2.0 ** -40) == 0x3f81
    assert exact_bf16_bits(2.0 ** -133) == 0x0001               # smallest subnormal
    assert exact_bf16_bits(2.0 ** -134) == 0x0000               # tie -> even zero
    assert exact_bf16_bits(3 * 2.0 ** -134) == 0x0002
    assert exact_bf16_bits(3.3895313892515355e38) == 0x7f7f     # largest finite
    assert exact_bf16_bits(1e39) == 0x7f80


@pytest.mark.parametrize("sample", ["crafted", "random"])
def test_factor_route_is_exact_rne(sample):
    if sample == "crafted":
        x = crafted_values()
    else:
        rng = np.random.default_rng(1)
        x = rng.standard_normal(4000) * np.exp(rng.uniform(-80, 80, 4000))
    got = ts.ts_bf16_round(x, 0)
    want = np.array([exact_bf16_bits(float(v)) for v in x], dtype=np.uint16)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(x[i], hex(got[i]), hex(want[i])) for i in bad[:5]]


def test_data_route_rounds_through_fp32():
    x = np.concatenate([crafted_values(), np.random.default_rng(2).standard_normal(4000)])
    got = ts.ts_bf16_round(x, 1)
    want = np.array([exact_bf16_bits(float(np.float32(v))) for v in x], dtype=np.uint16)
    assert np.array_equal(got, want)
    # double rounding: a value 1 FP64 ulp above a BF16 midpoint rounds to the
    # midpoint in FP32 and then to even, which can be the lower neighbour
    direct = ts.ts_bf16_round(x, 0)
    differ = np.nonzero(got != direct)[0]
    assert differ.size > 0
    for i in differ:
        f32 = float(np.float32(x[i]))
        # (the BF16 neighbour above the largest finite value is 2^128, encoded as Inf)
        lo, hi = sorted(min(bf16_value(int(b) & 0x7fff), 2.0 ** 128) for b in (got[i], direct[i]))
        assert abs(f32) == (lo + hi) / 2          # the FP32 value sits on the midpoint


def test_bad_arguments():
    with pytest.raises(ts.TSError):
        ts.ts_bf16_round(np.zeros(3), 2)
