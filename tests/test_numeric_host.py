"""The library's quantizer (lopc_numeric.h, the same source the kernels use)
compiled for the host and checked against exact rational rounding on
adversarial inputs: products within a few ulps of half-integers of both
signs, around zero, near 2^52 and 2^62, subnormal inputs (Sec. IV-A)."""
import math
import os
import shutil
import struct
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SAT = 2 ** 62 + 1


def bits(d):
    return struct.unpack("<Q", struct.pack("<d", d))[0]


def exact(y, inv):
    q = round(Fraction(y) * Fraction(inv))
    return max(-SAT, min(SAT, q))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("numeric") / "host_numeric")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-ffp-contract=off",
                    "-fno-fast-math", "-o", exe, os.path.join(HERE, "host_numeric.cpp")],
                   check=True, capture_output=True)
    return exe


def cases():
    rng = np.random.default_rng(17)
    out = []
    invs = [10.0, 1.0, 3.0, 1 / 0.3, 8.0, 1e3, 12345.678, 1e-3, 2.0 ** 40, 1e15]
    invs += list(10.0 ** rng.uniform(-8, 12, 40))
    for inv in invs:
        for k in list(range(-3, 3)) + list(rng.integers(-10 ** 6, 10 ** 6, 6)):
            for sgn in (1.0, -1.0):
                c = sgn * (int(k) + 0.5) / inv
                y = c
                for _ in range(3):
                    y = math.nextafter(y, -math.inf)
                for _ in range(7):
                    out.append((y, inv))
                    y = math.nextafter(y, math.inf)
        for _ in range(20):
            out.append((float(rng.standard_normal() * 10.0 ** rng.integers(-12, 12)), inv))
    # magnitudes around 2^52 and 2^62
    for base in (2.0 ** 52, 2.0 ** 53, 2.0 ** 61, 2.0 ** 62):
        for sgn in (1.0, -1.0):
            for inv in (1.0, 0.5, 0.25, 1.5, 0.1, 3.0):
                y = sgn * base / inv
                for _ in range(4):
                    y = math.nextafter(y, -math.inf)
                for _ in range(9):
                    out.append((y, inv))
                    y = math.nextafter(y, math.inf)
    # products near the float32 bin limit 2^31 - 2
    for sgn in (1.0, -1.0):
        for base in (2.0 ** 31 - 2.5, 2.0 ** 31 - 1.5, 2.0 ** 31 - 0.5, 2.0 ** 31):
            for inv in (1.0, 0.5, 3.0):
                y = sgn * base / inv
                for _ in range(2):
                    y = math.nextafter(y, -math.inf)
                for _ in range(5):
                    out.append((y, inv))
                    y = math.nextafter(y, math.inf)
    # subnormal inputs, zeros
    for y in (5e-324, -5e-324, 1e-310, -1e-310, 0.0, -0.0, 2.2250738585072014e-308):
        for inv in (1.0, 1e300, 1e308, 3.0):
            out.append((y, inv))
    return out


def test_quantizer_source_matches_exact_rounding(harness):
    cs = cases()
    inp = "".join(f"{bits(y):x} {bits(i):x}\n" for y, i in cs)
    res = subprocess.run([harness], input=inp, capture_output=True, text=True, check=True)
    vals = [int(v) for v in res.stdout.split()]
    got, got32 = vals[0::2], vals[1::2]
    assert len(got) == len(cs)
    bad = [(y, i, g, exact(y, i)) for (y, i), g in zip(cs, got) if g != exact(y, i)]
    assert not bad, bad[:5]
    # the float32 variant: exact inside the float32 bin range, out of range outside
    lim = 2 ** 31 - 2
    for (y, i), g in zip(cs, got32):
        e = exact(y, i)
        if abs(e) <= lim:
            assert g == e, (y, i, g, e)
        else:
            assert abs(g) > lim, (y, i, g, e)
