"""Pins of the oracle's error bound, quantizer and decoding rule against exact
rational arithmetic and the paper's worked example (Sec. IV-A, Sec. IV-E)."""
import math
from fractions import Fraction

import numpy as np
import pytest


def rnd_half_even(q: Fraction) -> int:
    return round(q)  # Fraction.__round__ rounds half to even


def q_exact(y: float, inv: float) -> int:
    return rnd_half_even(Fraction(y) * Fraction(inv))


def test_inv_is_smallest_double_with_product_at_least_one(ref):
    rng = np.random.default_rng(1)
    epss = [0.1, 1e-3, 3.0, 1.0 / 3, 7e-300, 2.0 ** -30, 0.7]
    epss += list(10.0 ** rng.uniform(-12, 12, 200))
    for eps in epss:
        x = np.array([[0.0, 1.0]])
        e, inv = ref.error_params(x, float(eps), ref.ABS)
        assert e == eps
        assert Fraction(inv) * Fraction(eps) >= 1
        prev = math.nextafter(inv, 0.0)
        assert Fraction(prev) * Fraction(eps) < 1


def test_noa_bound_is_eb_times_range(ref):
    rng = np.random.default_rng(2)
    for dt in (np.float32, np.float64):
        x = rng.uniform(-3, 5, (17, 9)).astype(dt)
        eb = 1e-3
        eps, _ = ref.error_params(x, eb, ref.NOA)
        lo, hi = float(x.min()), float(x.max())
        # binary64 product of eb and the binary64 range (Sec. IV-A: R = max - min)
        assert eps == eb * (hi - lo)
    # a field spanning exactly [0, 1]: eps = eb
    x = np.array([[0.0, 0.25], [1.0, 0.5]])
    assert ref.error_params(x, 0.01, ref.NOA)[0] == 0.01


def test_quantizer_matches_exact_rational_rounding(ref):
    rng = np.random.default_rng(3)
    cases = []
    for _ in range(4000):
        inv = float(10.0 ** rng.uniform(-6, 8))
        y = float(rng.standard_normal() * 10.0 ** rng.integers(-6, 6))
        cases.append((y, inv))
        # products near half-integers (the ties that decide the bin)
        k = math.floor(y * inv)
        cases.append(((k + 0.5) / inv, inv))
        cases.append((math.nextafter((k + 0.5) / inv, math.inf), inv))
        cases.append((math.nextafter((k + 0.5) / inv, -math.inf), inv))
    # exact ties at the real-number level: integer + 1/2 with inv a power of 2
    for k in range(-20, 20):
        cases.append((k + 0.5, 1.0))
        cases.append(((k + 0.5) / 8, 8.0))
    # signed zeros, subnormals, large magnitudes
    cases += [(0.0, 3.0), (-0.0, 3.0), (5e-324, 1e300), (-5e-324, 1e300),
              (2.0 ** 61 + 3.0, 1.0), (-(2.0 ** 60) - 1.0, 2.0), (1e15 + 0.5, 3.0)]
    for y, inv in cases:
        exp = q_exact(y, inv)
        if abs(exp) > 2 ** 62:
            with pytest.raises(ref.OracleError):
                ref.quantize(y, inv, 1)
            continue
        assert ref.quantize(y, inv, 1) == exp, (y, inv)


def test_paper_example_bin_10(ref):
    """Sec. IV-A: with an ABS bound of 0.1 every value between 0.95 and 1.05
    falls in bin 10.  Real-number level: the doubles inside the closed real
    interval [0.95, 1.05] map to 10, the doubles just outside do not."""
    x = np.array([[0.0, 1.0]])
    eps, inv = ref.error_params(x, 0.1, ref.ABS)
    lo = math.nextafter(0.95, 1.0) if Fraction(0.95) < Fraction(95, 100) else 0.95
    hi = math.nextafter(1.05, 0.0) if Fraction(1.05) > Fraction(105, 100) else 1.05
    assert Fraction(lo) >= Fraction(95, 100) and Fraction(hi) <= Fraction(105, 100)
    for y in (lo, 0.97, 1.0, 1.03, hi):
        assert ref.quantize(y, inv, 1) == 10
    assert ref.quantize(math.nextafter(lo, 0.0), inv, 1) == 9
    assert ref.quantize(math.nextafter(hi, 2.0), inv, 1) == 11


def test_bin_range_limits(ref):
    inv = 1.0
    assert ref.quantize(2147483646.0, inv, 0) == 2147483646
    with pytest.raises(ref.OracleError) as e:
        ref.quantize(2147483647.0, inv, 0)
    assert e.value.code == ref.E_RANGE
    assert ref.quantize(2.0 ** 62, inv, 1) == 2 ** 62
    with pytest.raises(ref.OracleError):
        ref.quantize(2.0 ** 62 + 2.0 ** 11, inv, 1)


@pytest.mark.parametrize("dtype_code", [0, 1])
def test_bin_floor_is_lowest_value_of_bin(ref, dtype_code):
    """Sec. IV-E: subbin 0 decodes to the lowest representable value of the
    bin.  Checked against exact rational bins of the value and its
    predecessor."""
    rng = np.random.default_rng(4 + dtype_code)
    ftype = np.float32 if dtype_code == 0 else np.float64
    for _ in range(1500):
        eps = float(10.0 ** rng.uniform(-5, 1))
        _, inv = ref.error_params(np.array([[0.0, 1.0]]), eps, ref.ABS)
        y = float(ftype(rng.standard_normal() * 10.0 ** rng.integers(-2, 3)))
        b = q_exact(y, inv)
        lo = ref.bin_floor(b, inv, dtype_code)
        assert float(ftype(lo)) == lo
        assert q_exact(lo, inv) == b
        prev = float(np.nextafter(ftype(lo), ftype(-np.inf)))
        if prev == 0.0 and lo == 0.0:
            prev = float(np.nextafter(ftype(0.0), ftype(-1.0)))
        assert q_exact(prev, inv) < b
        assert lo <= y


@pytest.mark.parametrize("dtype_code", [0, 1])
def test_reconstruct_steps_through_representable_values(ref, dtype_code):
    ftype = np.float32 if dtype_code == 0 else np.float64
    _, inv = ref.error_params(np.array([[0.0, 1.0]]), 0.01, ref.ABS)
    for b in (-7, 0, 3, 250):
        lo = ref.bin_floor(b, inv, dtype_code)
        v = ftype(lo)
        for s in range(6):
            assert ref.reconstruct(b, s, inv, dtype_code) == float(v)
            v = np.nextafter(v, ftype(np.inf))
            if v == 0:
                v = np.nextafter(v, ftype(np.inf))  # -0 and +0 are one value
    # a subbin that leaves the bin is rejected
    with pytest.raises(ref.OracleError):
        ref.reconstruct(0, 2 ** 63, inv, dtype_code)


def test_zero_is_one_value(ref):
    """-0 and +0 are equal values: both in bin 0, one step apart from the
    smallest negative and positive subnormals, and the decoder emits +0."""
    _, inv = ref.error_params(np.array([[0.0, 1.0]]), 1.0, ref.ABS)
    assert ref.quantize(-0.0, inv, 1) == 0
    lo = ref.bin_floor(0, inv, 1)
    assert lo == -0.5
    steps = 0x3FE0000000000000  # representable values from -0.5 up to 0
    z = ref.reconstruct(0, steps, inv, 1)
    assert z == 0.0 and not math.copysign(1.0, z) < 0
    assert ref.reconstruct(0, steps - 1, inv, 1) == -5e-324
    assert ref.reconstruct(0, steps + 1, inv, 1) == 5e-324


@pytest.mark.parametrize("dtype_code", [0, 1])
def test_bin_floor_walk_is_short(ref, dtype_code):
    """The bin floor of any bin b in range, at any bound: found exactly when
    some value of the dtype lies in the bin (exact rationals), and equal to
    the lowest such value.  The search starts at the rounded edge
    (b - 1/2)/inv and may take at most 8 steps; this pins that a non-empty
    bin is always within reach (across bin magnitudes up to the limits,
    bounds from subnormal to huge, so bins both much wider and much narrower
    than the spacing of representable values)."""
    rng = np.random.default_rng(40 + dtype_code)
    ftype = np.float32 if dtype_code == 0 else np.float64
    lim = 2 ** 31 - 2 if dtype_code == 0 else 2 ** 62
    lo_e, hi_e = (-40, 30) if dtype_code == 0 else (-300, 30)
    seen_empty = seen_full = 0
    for _ in range(1500):
        eps = float(10.0 ** rng.uniform(lo_e, hi_e))
        try:
            _, inv = ref.error_params(np.array([[0.0, 1.0]]), eps, ref.ABS)
        except ref.OracleError:
            continue
        b = int(rng.choice([-1, 1])) * int(10 ** rng.uniform(0, math.log10(lim)))
        edge = (Fraction(b) - Fraction(1, 2)) / Fraction(inv)
        with np.errstate(over="ignore"):
            c = float(ftype(float(edge)))
        if not math.isfinite(c):
            continue
        # the exact floor: walk with exact bins from the edge's neighbourhood
        y = c
        while True:
            p = float(np.nextafter(ftype(y), ftype(-np.inf)))
            if p == 0.0 and y == 0.0:
                p = float(np.nextafter(ftype(0.0), ftype(-1.0)))
            if not math.isfinite(p) or q_exact(p, inv) < b:
                break
            y = p
        while math.isfinite(y) and q_exact(y, inv) < b:
            y = float(np.nextafter(ftype(y), ftype(np.inf)))
        nonempty = math.isfinite(y) and q_exact(y, inv) == b
        if nonempty:
            seen_full += 1
            assert ref.bin_floor(b, inv, dtype_code) == y, (b, inv)
        else:
            seen_empty += 1
            with pytest.raises(ref.OracleError):
                ref.bin_floor(b, inv, dtype_code)
    assert seen_full > 100 and seen_empty > 100
