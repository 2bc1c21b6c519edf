"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Streams must be byte-identical and reconstructions bit-identical (integer,
bit-exact work: no tolerance).  Every case prints its name before it runs
on the GPU."""
import numpy as np
import pytest
import torch

from paper_2603_26968_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_26968_amd as P
    return P


def gpu_compress(P, x, eb, mode="noa"):
    s = P.compress(torch.from_numpy(np.ascontiguousarray(x)).cuda(), eb, mode)
    torch.cuda.synchronize()
    return s.cpu().numpy().tobytes()


def gpu_decompress(P, stream: bytes):
    t = torch.from_numpy(np.frombuffer(stream, np.uint8).copy()).cuda()
    y = P.decompress(t)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def same_bits(a, b):
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(
        a.view(np.uint8), b.view(np.uint8))


def check(P, ref, x, eb, mode="noa", name=""):
    _say(name, x.shape, x.dtype, eb, mode)
    try:
        want = ref.compress(x, eb, ref.NOA if mode == "noa" else ref.ABS)
    except ref.OracleError as e:
        # the GPU must reject the same input with the same status
        with pytest.raises(P.LopcError) as g:
            gpu_compress(P, x, eb, mode)
        assert g.value.code == e.code, (name, g.value.code, e.code)
        return
    got = gpu_compress(P, x, eb, mode)
    if got != want:
        # locate the first differing byte for the report
        n = min(len(got), len(want))
        d = next((i for i in range(n) if got[i] != want[i]), n)
        pytest.fail(f"{name}: stream differs at byte {d} (gpu {len(got)} B, oracle {len(want)} B)")
    y = gpu_decompress(P, want)
    z = ref.decompress(want)
    if not same_bits(y, z):
        b, sb = ref.decode_codes(want)
        u = np.uint32 if x.dtype == np.float32 else np.uint64
        bad = np.flatnonzero(y.view(u).ravel() != z.view(u).ravel())
        rows = [f"i={i} bin={b.flat[i]} sub={sb.flat[i]} gpu={y.view(u).flat[i]:#x} "
                f"oracle={z.view(u).flat[i]:#x}" for i in bad[:6]]
        pytest.fail(f"{name}: {bad.size} reconstructed values differ\n" + "\n".join(rows))


SMALL = [
    ("bumps2d", lambda: synth.gaussian_bumps((40, 52), seed=3)),
    ("bumps3d", lambda: synth.gaussian_bumps((14, 12, 17), seed=4, sigma_range=(2, 8))),
    ("turb3d", lambda: synth.turbulence_field((32, 32, 32), seed=5)),
    ("turb3d_f64", lambda: synth.turbulence_field((20, 24, 36), seed=5, dtype=np.float64)),
    ("lognormal3d", lambda: synth.lognormal_field((32, 32, 32), seed=6)),
    ("fronts2d", lambda: synth.fronts_field((90, 180), seed=7)),
    ("ties2d", lambda: (np.random.default_rng(21).integers(0, 5, (70, 61)) / 4.0).astype(np.float32)),
    ("noise64", lambda: np.random.default_rng(22).standard_normal((65, 67))),
]


@pytest.mark.parametrize("name,gen", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("eb", [1e-1, 1e-2, 1e-4])
def test_small_fields(P, ref, name, gen, eb):
    check(P, ref, gen(), eb, "noa", name)


SHAPES = [(1, 1), (1, 2), (2, 1), (1, 4097), (4097, 1), (3, 1, 5), (2, 2, 2), (1, 1, 9),
          (64, 64), (65, 63), (4096, 2), (9, 17, 33), (8, 8, 32), (17, 9, 65), (33, 65)]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(s) for s in SHAPES])
@pytest.mark.parametrize("dt", [np.float32, np.float64], ids=["f32", "f64"])
def test_shapes_and_ragged_chunks(P, ref, shape, dt):
    rng = np.random.default_rng(sum(shape))
    x = np.cumsum(rng.standard_normal(shape), axis=0).astype(dt)
    check(P, ref, x, 0.3, "abs", f"shape{shape}")
    if x.size > 1 and x.max() > x.min():
        check(P, ref, x, 1e-2, "noa", f"shape{shape}")


def test_golden_streams(P, ref):
    import json
    import os
    import importlib.util
    g = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(g, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    with open(os.path.join(g, "index.json")) as f:
        names = sorted(json.load(f))
    for name in names:
        x, eb, mode = mg.golden_inputs()[name]
        with open(os.path.join(g, name + ".hex")) as f:
            want = bytes.fromhex("".join(line.strip() for line in f))
        _say("golden", name)
        assert gpu_compress(P, x, eb, "noa" if mode == ref.NOA else "abs") == want, name
        assert same_bits(gpu_decompress(P, want), ref.decompress(want)), name


def test_special_values(P, ref):
    x = np.array([[-0.0, 0.0, 1e-45, -1e-45, 3e-39, -3e-39],
                  [1.0, -1.0, 0.5, -0.5, 0.0, 1e-40]], np.float32)
    check(P, ref, x, 1e-3, "abs", "subnormals_f32")
    check(P, ref, x, 1e-40, "abs", "subnormals_tiny_bound")
    y = np.array([[5e-324, -5e-324, 0.0, -0.0], [1e-310, -1e-310, 2.0, -2.0]])
    check(P, ref, y, 1e-3, "noa", "subnormals_f64")
    big = np.array([[1e15, 1e15 + 0.5, 1e15 + 1.0, 1e15 - 7.0]])
    check(P, ref, big, 0.25, "abs", "large_bins_f64")


def test_wide_bin_range_f64(P, ref):
    # float64 tiles whose bins span far more than 2^31, with neighbours whose
    # bins agree in their low 32 bits but differ; the left half of the 3D
    # field keeps a narrow range, so narrow and wide tiles meet
    rng = np.random.default_rng(31)
    for shape in [(12, 20, 70), (70, 140), (6, 9, 300)]:
        hi = rng.integers(0, 3, shape).astype(np.float64)
        if len(shape) == 3:
            hi[..., : shape[-1] // 2] = 0
        x = hi * 2.0**32 + rng.integers(0, 3, shape) + rng.random(shape)
        check(P, ref, x, 2.0, "abs", f"wide{shape}")  # bins up to 2^32 + 1
        check(P, ref, x, 2e-10, "noa", f"wide{shape}")


def _code(fn):
    import paper_2603_26968_amd as P
    try:
        fn()
    except P.LopcError as e:
        return e.code
    return 0


def test_error_codes(P, ref):
    import paper_2603_26968_amd as P2
    _say("errors")
    x = np.arange(20, dtype=np.float32).reshape(4, 5)
    assert _code(lambda: gpu_compress(P, np.ones((4, 4), np.float32), 1e-3)) == P2.lopc.LOPC_E_BOUND
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        assert _code(lambda: gpu_compress(P, x, bad, "abs")) == P2.lopc.LOPC_E_BOUND
    y = x.copy()
    y[2, 3] = np.nan
    assert _code(lambda: gpu_compress(P, y, 0.1, "noa")) == P2.lopc.LOPC_E_NONFINITE
    y[2, 3] = -np.inf
    assert _code(lambda: gpu_compress(P, y, 0.1, "abs")) == P2.lopc.LOPC_E_NONFINITE
    z = np.array([[3e9, 0.0]], np.float32)
    assert _code(lambda: gpu_compress(P, z, 1.0, "abs")) == P2.lopc.LOPC_E_RANGE


def test_capacity(P, ref):
    import paper_2603_26968_amd as P2
    from paper_2603_26968_amd import lopc
    _say("capacity")
    x = synth.gaussian_bumps((70, 61), seed=3)
    want = ref.compress(x, 1e-3)
    t = torch.from_numpy(x).cuda()
    ctx = lopc.context(0)
    ws = torch.empty(lopc.lopc_workspace_size(ctx, x.shape, t.dtype, 0), dtype=torch.uint8,
                     device="cuda")
    for cap in (len(want) - 1, 64, 10):
        out = torch.zeros(len(want), dtype=torch.uint8, device="cuda")
        st, size, _ = lopc.lopc_compress(ctx, t.data_ptr(), 0, x.shape, 1e-3, 1, out.data_ptr(),
                                         cap, ws.data_ptr(), ws.numel(), 0)
        torch.cuda.synchronize()
        assert st == P2.lopc.LOPC_E_CAPACITY and size == len(want)
        assert not out[cap:].any().item()  # nothing written beyond the capacity
    st, size, _ = lopc.lopc_compress(ctx, t.data_ptr(), 0, x.shape, 1e-3, 1, out.data_ptr(),
                                     len(want), ws.data_ptr(), ws.numel(), 0)
    torch.cuda.synchronize()
    assert st == 0 and out.cpu().numpy().tobytes() == want


def test_corrupt_streams_match_oracle(P, ref):
    _say("corrupt")
    x = synth.gaussian_bumps((70, 61), seed=2)
    s = ref.compress(x, 1e-3)
    rng = np.random.default_rng(0)
    for t in range(120):
        c = bytearray(s)
        pos = int(rng.integers(64, len(c)))
        c[pos] ^= 1 << int(rng.integers(0, 8))
        c = bytes(c)
        try:
            want = ref.decompress(c)
        except ref.OracleError:
            want = None
        try:
            got = gpu_decompress(P, c)
        except Exception:
            got = None
        if want is None:
            assert got is None, f"flip at {pos}: oracle rejects, GPU accepts"
        else:
            assert got is not None and same_bits(got, want), f"flip at {pos}"


CORRUPT = [
    # binary64: items of 8 bytes in the subbin stage, 2048 values a chunk
    ("turb3d_f64", lambda: synth.turbulence_field((12, 20, 36), seed=9, dtype=np.float64), 1e-3),
    # a loose bound: long same-bin runs, so most bytes of the stream belong
    # to the subbin part (RZE_K levels and payload)
    ("turb3d_f32_loose", lambda: synth.turbulence_field((16, 24, 40), seed=10), 1e-1),
]


@pytest.mark.parametrize("name,gen,eb", CORRUPT, ids=[c[0] for c in CORRUPT])
def test_corrupt_streams_more_match_oracle(P, ref, name, gen, eb):
    """Single-bit flips anywhere past the header of binary64 and
    subbin-heavy streams: the GPU accepts exactly what the oracle accepts
    and decodes it to the same values."""
    _say("corrupt", name)
    s = ref.compress(gen(), eb)
    rng = np.random.default_rng(1)
    for t in range(100):
        c = bytearray(s)
        pos = int(rng.integers(64, len(c)))
        c[pos] ^= 1 << int(rng.integers(0, 8))
        c = bytes(c)
        try:
            want = ref.decompress(c)
        except ref.OracleError:
            want = None
        try:
            got = gpu_decompress(P, c)
        except Exception:
            got = None
        if want is None:
            assert got is None, f"{name}: flip at {pos}: oracle rejects, GPU accepts"
        else:
            assert got is not None and same_bits(got, want), f"{name}: flip at {pos}"


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_turb3d_full_size(P, ref, eb):
    x = synth.turbulence_field()
    check(P, ref, x, eb, "noa", "turb3d 256^3")


def test_more_chunks_than_one_offset_pass(P, ref):
    """binary64, 4160 chunks: the record-offset scan takes 4096 chunks per
    pass, so the second pass and its carry are exercised (ragged tail of 64
    chunks)."""
    x = synth.turbulence_field((130, 256, 256), seed=5, dtype=np.float64)
    check(P, ref, x, 1e-3, "noa", "turb3d f64 130x256x256")


def test_smooth2d_full_size(P, ref):
    check(P, ref, synth.smooth_field(), 1e-3, "noa", "smooth2d 512^2")


def test_fronts2d_full_size(P, ref):
    check(P, ref, synth.fronts_field(), 1e-3, "noa", "fronts2d 1800x3600")


def test_adversarial_bin_edges(P, ref):
    """Values one to three ulps around the real bin edges (k + 1/2) * eps, both
    signs, including bin 0 and large bins: the quantizer and the bin floor
    must agree with the oracle's exact arithmetic."""
    import math
    for dt, eps in [(np.float64, 0.1), (np.float64, 1 / 3), (np.float32, 0.1),
                    (np.float32, 0.007), (np.float64, 1e-7)]:
        _, inv = ref.error_params(np.array([[0.0, 1.0]]), eps, ref.ABS)
        vals = []
        for k in (-4, -3, -2, -1, 0, 1, 2, 3, 50, -77, 12345):
            for sgn in (1.0, -1.0):
                c = sgn * (k + 0.5) / inv
                y = dt(c)
                for _ in range(3):
                    y = np.nextafter(y, dt(-np.inf))
                for _ in range(7):
                    vals.append(y)
                    y = np.nextafter(y, dt(np.inf))
        x = np.array(vals, dt)
        x = np.resize(x, (len(x) // 7, 7))
        check(P, ref, x, eps, "abs", f"edges {dt.__name__} eps={eps}")


def test_header_passthrough(P, ref):
    """lopc_ctx_last_header returns the stream's header; lopc_decompress_h
    with it equals lopc_decompress; a mismatched header is rejected or gives
    wrong values but stays inside the buffers."""
    from paper_2603_26968_amd import lopc
    _say("header passthrough")
    x = synth.gaussian_bumps((70, 61), seed=9)
    t = torch.from_numpy(x).cuda()
    s, hdr = P.compress(t, 1e-3, "noa", header=True)
    assert hdr == s[:64].cpu().numpy().tobytes()
    y1 = P.decompress(s).cpu().numpy()
    y2 = P.decompress(s, header=hdr).cpu().numpy()
    assert same_bits(y1, y2) and same_bits(y1, ref.decompress(s.cpu().numpy().tobytes()))
    # a header of another shape with the same number of chunks
    other = bytearray(hdr)
    other[8:16] = (61).to_bytes(8, "little")
    other[16:24] = (70).to_bytes(8, "little")
    out = torch.zeros((61, 70), dtype=torch.float32, device="cuda")
    try:
        P.decompress(s, header=bytes(other), out=out)
    except P.LopcError as e:
        assert e.code == lopc.LOPC_E_FORMAT
    torch.cuda.synchronize()


def test_phase_timing_mask(P, ref):
    """Phase timing: the phases in the mask report positive times, the others
    0; outputs are those of an untimed call; a mask with unknown bits is
    refused."""
    from paper_2603_26968_amd import lopc
    _say("phase timing mask")
    x = synth.gaussian_bumps((40, 33, 29), seed=4)
    t = torch.from_numpy(x).cuda()
    ctx = lopc.lopc_ctx_create(0)
    try:
        want = ref.compress(x, 1e-3, ref.NOA)
        for phases in (True, ("encode", "decode"), ("range", "repair", "offsets")):
            lopc.lopc_ctx_set_timing(ctx, phases)
            s = P.compress(t, 1e-3, "noa", ctx=ctx)
            ms_c = lopc.lopc_ctx_last_timings(ctx)
            y = P.decompress(s, ctx=ctx)
            ms_d = lopc.lopc_ctx_last_timings(ctx)
            torch.cuda.synchronize()
            assert s.cpu().numpy().tobytes() == want
            assert same_bits(y.cpu().numpy(), ref.decompress(want))
            on = set(lopc.PHASES) if phases is True else set(phases)
            for p in lopc.PHASES:
                v = (ms_d if p in ("offsets", "decode") else ms_c)[p]
                assert (v > 0) == (p in on), (phases, p, v)
        lopc.lopc_ctx_set_timing(ctx, False)
        assert lopc.load().lopc_ctx_set_timing(ctx, 1 << 6) == lopc.LOPC_E_ARG
    finally:
        lopc.lopc_ctx_destroy(ctx)
