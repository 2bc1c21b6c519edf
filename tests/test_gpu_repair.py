"""GPU parity of the repair schedulers and of the enqueued (host-free)
compression, through the C ABI, against the CPU oracle.

* Long same-bin chains whose value falls as the index rises: the worst case
  of Sec. IV-E, where the least fixed point is s = n-1, ..., 0 and the
  dependency crosses every tile of the field.
* The schedulers of the single-field repair (host-driven sweeps, work-list
  sweeps then a device work queue, the queue alone, and the default, which
  restarts on the queue after many sweeps) give the same bytes.
* lopc_compress with h_stream_size NULL: sizes and status codes arrive in
  device words, and the call can be captured into a graph and replayed.
"""
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


def same_bits(a, b):
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(
        a.view(np.uint8), b.view(np.uint8))


def _falling(shape, dt):
    n = int(np.prod(shape))
    # n, n-1, ..., 1 over n: exact in either dtype for n <= 2^23, strictly
    # falling with the index, all in bin 0 at an absolute bound of 10
    return (np.arange(n, 0, -1, dtype=np.float64) / n).astype(dt).reshape(shape)


CHAINS = [((1, 1 << 20), np.float32), ((1 << 20, 1), np.float32), ((1, 1 << 23), np.float32),
          ((1, 1, 1 << 20), np.float64), ((1 << 18, 1, 1), np.float32)]


@pytest.mark.parametrize("shape,dt", CHAINS, ids=[f"{s}-{d.__name__}" for s, d in CHAINS])
def test_falling_chain_crosses_every_tile(P, ref, shape, dt):
    x = _falling(shape, dt)
    _say("falling chain", shape, dt.__name__)
    want = ref.compress(x, 10.0, ref.ABS)
    t = torch.from_numpy(x).cuda()
    s, st = P.compress(t, 10.0, "abs", stats=True)
    got = s.cpu().numpy().tobytes()
    assert got == want, (len(got), len(want))
    if x.size <= 1 << 20:
        # the host-driven sweeps in checkerboard order (the default for
        # fields of many tiles) up to their limit, then the queue
        from paper_2603_26968_amd import lopc
        ctx = lopc.lopc_ctx_create(0)
        try:
            lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_SWEEP_ORDER, 1)
            assert P.compress(t, 10.0, "abs", ctx=ctx).cpu().numpy().tobytes() == want
        finally:
            lopc.lopc_ctx_destroy(ctx)
    b, sub = ref.decode_codes(got)
    n = x.size
    assert not b.any()
    assert np.array_equal(sub.ravel().astype(np.int64), np.arange(n - 1, -1, -1))
    assert same_bits(P.decompress(s).cpu().numpy(), ref.decompress(want))
    _say("  tile runs", st["active_tiles_total"], "chain depth", st["repair_sweeps"])


FIELDS = [
    ("turb3d", lambda: synth.turbulence_field((48, 40, 72), seed=3), 1e-2),
    ("lognormal3d", lambda: synth.lognormal_field((40, 48, 64), seed=4), 1e-3),
    ("fronts2d", lambda: synth.fronts_field((200, 330), seed=5), 1e-3),
    ("bumps2d_f64", lambda: synth.gaussian_bumps((150, 170), seed=6).astype(np.float64), 1e-2),
]


@pytest.mark.parametrize("name,gen,eb", FIELDS, ids=[f[0] for f in FIELDS])
def test_schedulers_agree(P, ref, name, gen, eb):
    from paper_2603_26968_amd import lopc
    x = gen()
    _say("schedulers", name, x.shape)
    want = ref.compress(x, eb, ref.NOA)
    t = torch.from_numpy(x).cuda()
    ctx = lopc.lopc_ctx_create(0)
    try:
        for mode in (lopc.LOPC_REPAIR_SWEEPS, lopc.LOPC_REPAIR_QUEUE, lopc.LOPC_REPAIR_HYBRID,
                     lopc.LOPC_REPAIR_HYBRID, lopc.LOPC_REPAIR_AUTO, lopc.LOPC_REPAIR_POINTS,
                     lopc.LOPC_REPAIR_SWEEPS):
            for order in (1, 2):
                lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_REPAIR, mode)
                lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_SWEEP_ORDER, order)
                s = P.compress(t, eb, "noa", ctx=ctx)
                assert s.cpu().numpy().tobytes() == want, (name, mode, order)
    finally:
        lopc.lopc_ctx_destroy(ctx)


TILES = [(0, 0), (0, 1), (0, 2), (1, 0)]


@pytest.mark.parametrize("t2,t3", TILES, ids=[f"t2_{a}-t3_{b}" for a, b in TILES])
def test_tile_shapes_agree(P, ref, t2, t3):
    """Every repair tile shape, under every scheduler, gives the oracle's
    bytes (ragged tiles on every side, both dtypes, 2D and 3D), and so does
    a falling chain along z, which crosses every tile plane."""
    from paper_2603_26968_amd import lopc
    cases = [(synth.turbulence_field((37, 45, 70), seed=8), 1e-2, "noa"),
             (synth.lognormal_field((20, 33, 100), seed=9), 1e-3, "noa"),
             (synth.fronts_field((150, 290), seed=10), 1e-3, "noa"),
             (synth.gaussian_bumps((90, 260), seed=11).astype(np.float64), 1e-2, "noa"),
             (_falling((96, 3, 5), np.float32), 10.0, "abs")]
    ctx = lopc.lopc_ctx_create(0)
    try:
        lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_TILE_2D, t2)
        lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_TILE_3D, t3)
        for x, eb, mode in cases:
            _say("tiles", t2, t3, x.shape, x.dtype)
            want = ref.compress(x, eb, ref.NOA if mode == "noa" else ref.ABS)
            t = torch.from_numpy(x).cuda()
            for m, order in ((lopc.LOPC_REPAIR_AUTO, 0), (lopc.LOPC_REPAIR_AUTO, 1),
                             (lopc.LOPC_REPAIR_QUEUE, 0), (lopc.LOPC_REPAIR_HYBRID, 0),
                             (lopc.LOPC_REPAIR_SWEEPS, 1), (lopc.LOPC_REPAIR_SWEEPS, 2),
                             (lopc.LOPC_REPAIR_POINTS, 0)):
                lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_REPAIR, m)
                lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_SWEEP_ORDER, order)
                s = P.compress(t, eb, mode, ctx=ctx)
                assert s.cpu().numpy().tobytes() == want, (x.shape, m, order)
            lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_REPAIR, lopc.LOPC_REPAIR_AUTO)
            lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_SWEEP_ORDER, 0)
            out, size, status = P.compress_enqueue(t, eb, mode, ctx=ctx)
            torch.cuda.synchronize()
            assert status.item() == 0 and out[:size.item()].cpu().numpy().tobytes() == want
    finally:
        lopc.lopc_ctx_destroy(ctx)


@pytest.mark.parametrize("shape,dt", [((1, 5000), np.float32), ((300, 1, 1), np.float64),
                                      ((20, 30, 7), np.float32)],
                         ids=["row", "column", "block"])
def test_point_worklists_on_falling_chains(P, ref, shape, dt):
    """The point-worklist scheduler on the worst case (one more iteration per
    point of the chain) gives the oracle's bytes, and s = n-1 .. 0 along a
    single chain."""
    from paper_2603_26968_amd import lopc
    x = _falling(shape, dt)
    _say("point worklists, falling chain", shape)
    want = ref.compress(x, 10.0, ref.ABS)
    t = torch.from_numpy(x).cuda()
    ctx = lopc.lopc_ctx_create(0)
    try:
        lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_REPAIR, lopc.LOPC_REPAIR_POINTS)
        s, st = P.compress(t, 10.0, "abs", stats=True, ctx=ctx)
        assert s.cpu().numpy().tobytes() == want
        assert st["repair_sweeps"] >= 2
        if sum(d > 1 for d in shape) == 1:  # a single chain through every point
            _, sub = ref.decode_codes(want)
            assert np.array_equal(sub.ravel().astype(np.int64), np.arange(x.size - 1, -1, -1))
        # host-driven: not for enqueued calls
        with pytest.raises(lopc.LopcError):
            P.compress_enqueue(t, 10.0, "abs", ctx=ctx)
    finally:
        lopc.lopc_ctx_destroy(ctx)


def test_enqueued_compress_reports_on_device(P, ref):
    """Enqueued calls: size and status words against the synchronous call
    and the oracle, also for the failure cases."""
    from paper_2603_26968_amd import lopc
    _say("enqueued compress")
    cases = [(synth.gaussian_bumps((70, 61), seed=3), 1e-3, "noa"),
             (synth.turbulence_field((24, 20, 28), seed=2, dtype=np.float64), 1e-2, "noa"),
             (synth.lognormal_field((32, 32, 32), seed=6), 1e-3, "noa"),
             (np.arange(20, dtype=np.float32).reshape(4, 5), 0.5, "abs")]
    for x, eb, mode in cases:
        want = ref.compress(x, eb, ref.NOA if mode == "noa" else ref.ABS)
        t = torch.from_numpy(x).cuda()
        out, size, status = P.compress_enqueue(t, eb, mode)
        torch.cuda.synchronize()
        assert status.item() == 0 and size.item() == len(want)
        assert out[:len(want)].cpu().numpy().tobytes() == want
    # a NaN: status NONFINITE, size 0
    y = np.arange(20, dtype=np.float32).reshape(4, 5)
    y[1, 2] = np.nan
    out, size, status = P.compress_enqueue(torch.from_numpy(y).cuda(), 0.1, "abs")
    torch.cuda.synchronize()
    assert status.item() == lopc.LOPC_E_NONFINITE and size.item() == 0
    # zero range under NOA: status BOUND
    out, size, status = P.compress_enqueue(torch.ones((8, 8), device="cuda"), 1e-3, "noa")
    torch.cuda.synchronize()
    assert status.item() == lopc.LOPC_E_BOUND and size.item() == 0
    # a short stream buffer: CAPACITY, with the size needed
    x = synth.gaussian_bumps((70, 61), seed=3)
    want = ref.compress(x, 1e-3, ref.NOA)
    t = torch.from_numpy(x).cuda()
    ctx = lopc.context(0)
    ws = torch.empty(lopc.lopc_workspace_size(ctx, x.shape, t.dtype, 0), dtype=torch.uint8,
                     device="cuda")
    out = torch.zeros(len(want), dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    st, _, _ = lopc.lopc_compress(ctx, t.data_ptr(), 0, x.shape, 1e-3, 1, out.data_ptr(),
                                  len(want) - 1, ws.data_ptr(), ws.numel(),
                                  torch.cuda.current_stream().cuda_stream, False,
                                  size.data_ptr(), status.data_ptr(), enqueue_only=True)
    assert st == 0
    torch.cuda.synchronize()
    assert status.item() == lopc.LOPC_E_CAPACITY and size.item() == len(want)
    assert not out[len(want) - 1:].any().item()
    # enqueued calls need the device size word and no host statistics; the
    # host-driven sweeps cannot run enqueued
    assert lopc.lopc_compress(ctx, t.data_ptr(), 0, x.shape, 1e-3, 1, out.data_ptr(),
                              len(want), ws.data_ptr(), ws.numel(), 0, False,
                              enqueue_only=True)[0] == lopc.LOPC_E_ARG
    c2 = lopc.lopc_ctx_create(0)
    try:
        lopc.lopc_ctx_set_option(c2, lopc.LOPC_OPT_REPAIR, lopc.LOPC_REPAIR_SWEEPS)
        assert lopc.lopc_compress(c2, t.data_ptr(), 0, x.shape, 1e-3, 1, out.data_ptr(),
                                  len(want), ws.data_ptr(), ws.numel(), 0, False,
                                  size.data_ptr(), None, enqueue_only=True)[0] == lopc.LOPC_E_ARG
    finally:
        lopc.lopc_ctx_destroy(c2)


@pytest.mark.parametrize("dt,shape", [(np.float32, (40, 36, 52)), (np.float64, (150, 170))],
                         ids=["f32-3d", "f64-2d"])
def test_enqueued_compress_in_a_graph(P, ref, dt, shape):
    """The enqueued compression captured once and replayed on new field
    values, with eager device work and synchronisations between replays:
    every replay's stream equals the oracle's for the values it saw."""
    _say("graph capture", dt.__name__, shape)
    from paper_2603_26968_amd import lopc
    ctx = lopc.context(0)
    tdt = torch.float32 if dt == np.float32 else torch.float64
    fields = [synth.turbulence_field(shape, seed=s, dtype=dt) if len(shape) == 3 else
              synth.gaussian_bumps(shape, seed=s).astype(dt) for s in range(4)]
    x = torch.from_numpy(fields[0]).cuda()
    cap, wsz, _ = lopc.lopc_compress_bound(shape, tdt), \
        lopc.lopc_workspace_size(ctx, shape, tdt, 0), None
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.compress_enqueue(x, 1e-3, "noa", out=out, workspace=ws, size=size, status=status)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.compress_enqueue(x, 1e-3, "noa", out=out, workspace=ws, size=size, status=status)
    torch.cuda.synchronize()
    for rep, f in enumerate(fields[1:] + fields[:1] + fields[1:2]):
        want = ref.compress(f, 1e-3, ref.NOA)
        x.copy_(torch.from_numpy(f))
        out.fill_(0xAB)
        size.fill_(-1)
        g.replay()
        junk = torch.randn(1 << 18, device="cuda").cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        assert status.item() == 0 and size.item() == len(want), rep
        assert out[:len(want)].cpu().numpy().tobytes() == want, rep
        del junk


REPEATS = [
    ("turb3d_1e0", lambda: synth.turbulence_field((64, 96, 96), seed=7), 1.0, "noa"),
    ("fronts2d_1e-1", lambda: synth.fronts_field((300, 500), seed=8), 1e-1, "noa"),
    ("falling_chain", lambda: _falling((1, 1 << 16), np.float32), 10.0, "abs"),
]


@pytest.mark.parametrize("name,gen,eb,mode", REPEATS, ids=[r[0] for r in REPEATS])
def test_repeated_compressions_on_one_context(P, ref, name, gen, eb, mode):
    """A context learns from each compression how many sweeps to enqueue
    before its first read on the next; call after call, in both sweep
    orders, the bytes stay the oracle's."""
    from paper_2603_26968_amd import lopc
    x = gen()
    _say("repeated compressions", name, x.shape)
    want = ref.compress(x, eb, ref.ABS if mode == "abs" else ref.NOA)
    t = torch.from_numpy(x).cuda()
    ctx = lopc.lopc_ctx_create(0)
    try:
        lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_REPAIR, lopc.LOPC_REPAIR_SWEEPS)
        for order in (1, 2):
            lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_SWEEP_ORDER, order)
            sweeps = []
            for _ in range(3):
                s, st = P.compress(t, eb, mode, stats=True, ctx=ctx)
                assert s.cpu().numpy().tobytes() == want, (name, order)
                sweeps.append(st["repair_sweeps"])
            assert min(sweeps) > 1, sweeps
    finally:
        lopc.lopc_ctx_destroy(ctx)
