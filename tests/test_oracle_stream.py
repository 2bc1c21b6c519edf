"""Whole-stream pins of the oracle: the guarantees the paper states for the
reconstruction (Sec. IV-A error bound, Sec. IV-B/IV-E local order and
critical points, CPU/GPU-identical output), error handling, corrupt-stream
safety, and the golden streams that freeze the container layout."""
import json
import os
import struct
from fractions import Fraction

import numpy as np
import pytest

import topo
from paper_2603_26968_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fields():
    rng = np.random.default_rng(21)
    yield "bumps2d", synth.gaussian_bumps((40, 52), seed=3)
    yield "bumps3d", synth.gaussian_bumps((14, 12, 17), seed=4, sigma_range=(2, 8))
    yield "turb3d", synth.turbulence_field((16, 16, 16), seed=5)
    yield "lognormal3d", synth.lognormal_field((16, 16, 16), seed=6)
    yield "fronts2d", synth.fronts_field((45, 90), seed=7)
    yield "ties2d", (rng.integers(0, 5, (33, 29)) / 4.0).astype(np.float32)
    yield "noise64", rng.standard_normal((30, 31)).astype(np.float64)


FIELDS = list(fields())


@pytest.mark.parametrize("name,x", FIELDS, ids=[f[0] for f in FIELDS])
@pytest.mark.parametrize("eb", [1e-1, 1e-2, 1e-4])
def test_guarantees(ref, name, x, eb):
    s = ref.compress(x, eb, ref.NOA)
    y = ref.decompress(s)
    assert y.dtype == x.dtype and y.shape == x.shape
    info = ref.stream_info(s)
    eps, inv = info["eps"], info["inv"]
    # error bound (Sec. IV-A), exact rational check
    fx = x.ravel().tolist()
    fy = y.ravel().tolist()
    eps_q = Fraction(eps)
    assert all(abs(Fraction(a) - Fraction(b)) <= eps_q for a, b in zip(fx, fy))
    # every decoded value lies in its bin at or below the original
    for a, b in zip(fx[:400], fy[:400]):
        assert ref.quantize(a, inv, 1) == ref.quantize(b, inv, 1)
        assert b <= a
    # local order on every edge, ties broken by index (Sec. IV-B)
    for ex, ey in zip(topo.edge_orders(x), topo.edge_orders(y)):
        assert np.array_equal(ex, ey)
    # critical points and their types (Sec. II, Sec. IV-E)
    assert np.array_equal(topo.critical_points(x), topo.critical_points(y))


def test_noa_equals_abs_with_derived_bound(ref):
    x = synth.gaussian_bumps((20, 30), seed=8)
    s1 = ref.compress(x, 1e-3, ref.NOA)
    eps = ref.stream_info(s1)["eps"]
    s2 = ref.compress(x, eps, ref.ABS)
    assert np.array_equal(ref.decompress(s1), ref.decompress(s2))
    assert s1[64:] == s2[64:]  # identical apart from the recorded mode and bound


def test_deterministic(ref):
    x = synth.turbulence_field((12, 12, 12), seed=1)
    assert ref.compress(x, 1e-2) == ref.compress(x.copy(), 1e-2)


def test_error_codes(ref):
    x = np.ones((4, 4), np.float32)
    with pytest.raises(ref.OracleError) as e:
        ref.compress(x, 1e-3, ref.NOA)  # constant field: zero range
    assert e.value.code == ref.E_BOUND
    x = np.arange(16, dtype=np.float32).reshape(4, 4)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(ref.OracleError) as e:
            ref.compress(x, bad, ref.ABS)
        assert e.value.code == ref.E_BOUND
    y = x.copy()
    y[1, 2] = np.nan
    with pytest.raises(ref.OracleError) as e:
        ref.compress(y, 0.1, ref.ABS)
    assert e.value.code == ref.E_NONFINITE
    y[1, 2] = np.inf
    with pytest.raises(ref.OracleError) as e:
        ref.compress(y, 0.1, ref.ABS)
    assert e.value.code == ref.E_NONFINITE
    with pytest.raises(ref.OracleError) as e:
        ref.compress(np.array([[3e9, 0.0]], np.float32), 1.0, ref.ABS)
    assert e.value.code == ref.E_RANGE
    with pytest.raises(ref.OracleError) as e:
        ref.compress(np.zeros(5, np.float32), 0.1, ref.ABS)  # 1D
    assert e.value.code == ref.E_ARG


def test_bound_holds_and_capacity(ref):
    rng = np.random.default_rng(3)
    for dt in (np.float32, np.float64):
        x = rng.standard_normal((70, 80)).astype(dt)  # incompressible noise
        s = ref.compress(x, 1e-7, ref.NOA)
        assert len(s) <= ref.compress_bound(x.shape, dt)


def test_corrupt_streams_never_crash(ref):
    x = synth.gaussian_bumps((70, 61), seed=2)
    s = ref.compress(x, 1e-3)
    rng = np.random.default_rng(0)
    for cut in (0, 10, 63, 64, 70, len(s) - 1):
        with pytest.raises(ref.OracleError):
            ref.decompress(s[:cut])
    with pytest.raises(ref.OracleError):
        ref.decompress(s + b"\0\0\0\0")
    bad_header = bytearray(s)
    bad_header[0] ^= 1
    with pytest.raises(ref.OracleError):
        ref.decompress(bytes(bad_header))
    bad_inv = bytearray(s)
    bad_inv[56] ^= 1  # inv no longer the rounded-up reciprocal of eps
    with pytest.raises(ref.OracleError):
        ref.decompress(bytes(bad_inv))
    n_ok = 0
    for t in range(300):
        c = bytearray(s)
        pos = int(rng.integers(64, len(c)))
        c[pos] ^= 1 << int(rng.integers(0, 8))
        try:
            y = ref.decompress(bytes(c))
            assert y.shape == x.shape
            n_ok += 1
        except ref.OracleError as e:
            assert e.code == ref.E_FORMAT
    assert n_ok < 300


def _golden_cases():
    with open(os.path.join(GOLDEN, "index.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", sorted(_golden_cases()))
def test_golden_streams(ref, name):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    x, eb, mode = mg.golden_inputs()[name]
    with open(os.path.join(GOLDEN, name + ".hex")) as f:
        want = bytes.fromhex("".join(line.strip() for line in f))
    assert ref.compress(x, eb, mode) == want
    assert np.array_equal(ref.decompress(want), ref.decompress(ref.compress(x, eb, mode)))


def test_header_layout(ref):
    x = np.arange(12, dtype=np.float64).reshape(3, 4)
    s = ref.compress(x, 0.5, ref.ABS)
    magic, ver, dt, nd = struct.unpack_from("<IHBB", s, 0)
    assert magic == 0x43504F4C and ver == 1 and dt == 1 and nd == 2
    assert struct.unpack_from("<3Q", s, 8) == (3, 4, 1)
    assert s[32] == 0 and struct.unpack_from("<I", s, 36)[0] == 16384
    eb, eps, inv = struct.unpack_from("<3d", s, 40)
    assert eb == 0.5 and eps == 0.5 and inv == 2.0
    (rec,) = struct.unpack_from("<I", s, 64)
    assert len(s) == 64 + 4 + rec
