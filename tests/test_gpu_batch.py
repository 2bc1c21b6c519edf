"""GPU batch calls through the C ABI.

Fields in a batch never interact, so every field's stream from
lopc_compress_batch must equal its lopc_compress stream byte for byte (and
the oracle's), and every field from lopc_decompress_batch its
lopc_decompress output bit for bit -- whether the launch sequence is a graph
replay or direct launches, whatever the persistent grid size, and also when
the repair needs more sweeps than the captured graph holds.  Every case
prints its name before it runs on the GPU."""
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


def mixed_batch():
    """Both dtypes, both dimensionalities, ragged chunks and tiles, NOA and
    ABS, a single point."""
    rng = np.random.default_rng(5)
    g = synth.power_law_grf((40, 40, 40), 3.0, seed=2)
    out = [
        (synth.gaussian_bumps((40, 52), seed=3), 1e-3, "noa"),
        (synth.gaussian_bumps((14, 12, 17), seed=4, sigma_range=(2, 8)), 1e-2, "noa"),
        (synth.gaussian_bumps((70, 61), seed=2, dtype=np.float64), 1e-4, "noa"),
        (rng.standard_normal((9, 10, 11)), 1e-2, "abs"),
        (np.array([[0.25]], np.float32), 1e-3, "abs"),
        (rng.standard_normal((3, 5, 7)), 1e-3, "noa"),
        (rng.standard_normal((1, 4097)).astype(np.float32), 1e-2, "noa"),
        (synth.gaussian_bumps((130, 300), seed=6), 1e-2, "noa"),
        ((g - g.min()).astype(np.float32), 1e-3, "noa"),
        (synth.fronts_field((180, 360)), 1e-3, "noa"),
        (np.round(rng.standard_normal((33, 65)) * 3).astype(np.float32), 0.5, "abs"),
        (rng.standard_normal((1, 40, 70)).astype(np.float32), 1e-2, "noa"),
        (rng.standard_normal((2, 3, 300)), 1e-2, "noa"),
    ]
    return out


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def single_streams(P, batch):
    out = []
    for x, eb, mode in batch:
        s = P.compress(to_dev(x), eb, mode)
        torch.cuda.synchronize()
        out.append(s.cpu().numpy().tobytes())
    return out


def batch_streams(P, batch, **kw):
    xs = [to_dev(x) for x, _, _ in batch]
    res = P.compress_batch(xs, [eb for _, eb, _ in batch], [m for _, _, m in batch], **kw)
    torch.cuda.synchronize()
    if isinstance(res, tuple):
        return [s.cpu().numpy().tobytes() for s in res[0]], res[1]
    return [s.cpu().numpy().tobytes() for s in res], None


def first_diff(a, b):
    n = min(len(a), len(b))
    return next((i for i in range(n) if a[i] != b[i]), n)


def assert_same_streams(got, want, label):
    for i, (g, w) in enumerate(zip(got, want)):
        if g != w:
            pytest.fail(f"{label}: field {i} stream differs at byte {first_diff(g, w)} "
                        f"({len(g)} B vs {len(w)} B)")


def test_batch_streams_equal_single_and_oracle(P, ref):
    _say("mixed batch: batch vs single vs oracle")
    batch = mixed_batch()
    want = single_streams(P, batch)
    for (x, eb, mode), w in zip(batch, want):
        assert w == ref.compress(x, eb, ref.NOA if mode == "noa" else ref.ABS)
    got, st = batch_streams(P, batch, stats=True)
    assert_same_streams(got, want, "batch")
    assert st["status"] == [0] * len(batch)
    assert st["repair_sweeps"] >= 1
    hdrs = P.lopc_ctx_last_batch_headers(P.context(0), len(batch))
    assert [h for h in hdrs] == [w[:64] for w in want]


def test_batch_decompress_equals_single(P, ref):
    _say("mixed batch: decompress_batch vs single vs oracle")
    batch = mixed_batch()
    streams = single_streams(P, batch)
    ts = [torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda() for s in streams]
    ys = P.decompress_batch(ts)
    torch.cuda.synchronize()
    for i, (y, s, t) in enumerate(zip(ys, streams, ts)):
        z = P.decompress(t)
        torch.cuda.synchronize()
        a, b = y.cpu().numpy(), z.cpu().numpy()
        assert a.dtype == b.dtype and a.shape == b.shape, i
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), i
        r = ref.decompress(s)
        assert np.array_equal(a.view(np.uint8), r.view(np.uint8)), i


def test_graph_replays_and_direct_launches_agree(P):
    """Replays of the captured sequence, with other device work and
    synchronisations between them, each give the bytes of direct launches."""
    batch = mixed_batch()
    ctx = P.context(0)
    _say("direct launches")
    P.lopc_ctx_set_option(ctx, P.LOPC_OPT_BATCH_GRAPH, 0)
    try:
        want, st = batch_streams(P, batch, stats=True)
        assert st["graph"] == 0
    finally:
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_BATCH_GRAPH, 1)
    x0 = to_dev(batch[0][0])
    for r in range(4):
        _say("graph replay", r)
        got, st = batch_streams(P, batch, stats=True)
        assert st["graph"] == 1
        assert_same_streams(got, want, f"replay {r}")
        # eager work between replays
        P.compress(x0, 1e-2, "noa")
        torch.cuda.synchronize()
    for r in range(3):
        _say("decompress graph replay", r)
        ts = [torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda() for s in want]
        ys = P.decompress_batch(ts)
        torch.cuda.synchronize()
        for (x, _, _), y, t in zip(batch, ys, ts):
            z = P.decompress(t)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy().view(np.uint8), z.cpu().numpy().view(np.uint8))


@pytest.mark.parametrize("pct", [0, 100])
def test_sweeps_beyond_the_graph_continue(P, pct):
    """With one sweep captured, fields that need more continue with direct
    launches and still give the single-field streams."""
    batch = mixed_batch()
    want = single_streams(P, batch)
    ctx = P.context(0)
    P.lopc_ctx_set_option(ctx, P.LOPC_OPT_GRAPH_SWEEPS, 1)
    P.lopc_ctx_set_option(ctx, P.LOPC_OPT_PERSIST_PCT, pct)
    try:
        _say("graph with 1 sweep, grid mode", pct)
        got, st = batch_streams(P, batch, stats=True)
        assert st["continued"] == 1 and st["repair_sweeps"] > 2
        assert_same_streams(got, want, "continued")
    finally:
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_GRAPH_SWEEPS, 0)
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_PERSIST_PCT, 0)


def test_autotuner_keeps_results(P):
    batch = mixed_batch()
    want = single_streams(P, batch)
    xs = [to_dev(x) for x, _, _ in batch]
    ctx = P.context(0)
    _say("autotune")
    try:
        pct = P.autotune_compress_batch(xs, [eb for _, eb, _ in batch],
                                        [m for _, _, m in batch], reps=1)
        assert pct in (0, 50, 100, 200)
        assert P.lopc_ctx_get_option(ctx, P.LOPC_OPT_PERSIST_PCT) == pct
        t2 = P.lopc_ctx_get_option(ctx, P.LOPC_OPT_TILE_2D)
        t3 = P.lopc_ctx_get_option(ctx, P.LOPC_OPT_TILE_3D)
        assert 0 <= t2 < 2 and 0 <= t3 < 3
        got, _ = batch_streams(P, batch)
        assert_same_streams(got, want, f"tuned {pct}% tiles {t2} {t3}")
    finally:
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_PERSIST_PCT, 0)
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_TILE_2D, 0)
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_TILE_3D, 0)


@pytest.mark.parametrize("t2,t3", [(0, 1), (1, 2), (1, 0)])
@pytest.mark.parametrize("pct", [0, 100])
def test_tile_shapes_give_the_same_batch_streams(P, t2, t3, pct):
    """The repair tile shape changes the schedule, not the fixed point: the
    batch streams under every shape equal the default single-field ones."""
    batch = mixed_batch()
    want = single_streams(P, batch)
    ctx = P.context(0)
    try:
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_TILE_2D, t2)
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_TILE_3D, t3)
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_PERSIST_PCT, pct)
        _say("batch tiles", t2, t3, "grid", pct)
        got, _ = batch_streams(P, batch)
        assert_same_streams(got, want, f"tiles {t2} {t3} grid {pct}")
    finally:
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_PERSIST_PCT, 0)
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_TILE_2D, 0)
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_TILE_3D, 0)


@pytest.mark.parametrize("pct", [1, 25, 100, 300])
def test_persistent_grid_size_does_not_matter(P, pct):
    batch = mixed_batch()
    want = single_streams(P, batch)
    ctx = P.context(0)
    P.lopc_ctx_set_option(ctx, P.LOPC_OPT_PERSIST_PCT, pct)
    try:
        _say("persistent grid", pct, "%")
        got, _ = batch_streams(P, batch)
        assert_same_streams(got, want, f"grid {pct}%")
        ts = [torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda() for s in want]
        ys = P.decompress_batch(ts)
        for i, (y, t) in enumerate(zip(ys, ts)):
            z = P.decompress(t)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy().view(np.uint8), z.cpu().numpy().view(np.uint8)), i
    finally:
        P.lopc_ctx_set_option(ctx, P.LOPC_OPT_PERSIST_PCT, 0)


def test_per_field_status_and_device_words(P, ref):
    """A failing field does not disturb the others; sizes and statuses reach
    the caller's device words and lopc_ctx_last_batch."""
    from paper_2603_26968_amd import lopc
    good = synth.gaussian_bumps((70, 61), seed=9)
    nan = good.copy()
    nan[3, 4] = np.nan
    const = np.full((20, 30), 1.5, np.float32)
    fields = [to_dev(good), to_dev(nan), to_dev(const), to_dev(good), to_dev(good)]
    caps = [P.lopc_compress_bound(f.shape, f.dtype) for f in fields]
    caps[3] = 100  # too small
    outs = [torch.zeros(max(c, 256), dtype=torch.uint8, device="cuda") for c in caps]
    words = torch.full((len(fields),), -77, dtype=torch.int64, device="cuda")
    sts = torch.full((len(fields),), 99, dtype=torch.int32, device="cuda")
    jobs = (P.Job * len(fields))()
    for i, (f, o) in enumerate(zip(fields, outs)):
        j = jobs[i]
        j.d_in, j.d_out, j.out_cap = f.data_ptr(), o.data_ptr(), caps[i]
        j.dtype, j.ndim = 0, 2
        j.dims[0], j.dims[1] = f.shape
        j.error_bound, j.mode = 1e-3, lopc.LOPC_EB_NOA
        j.d_out_size = words.data_ptr() + 8 * i
        j.d_status = sts.data_ptr() + 4 * i
    ctx = P.context(0)
    wsz = P.lopc_batch_workspace_size(ctx, 0, jobs)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    _say("per-field statuses")
    st, _ = P.lopc_compress_batch(ctx, jobs, ws.data_ptr(), wsz,
                                  torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    sizes, codes = P.lopc_ctx_last_batch(ctx, len(fields))
    want_codes = [0, lopc.LOPC_E_NONFINITE, lopc.LOPC_E_BOUND, lopc.LOPC_E_CAPACITY, 0]
    assert codes == want_codes
    assert st == lopc.LOPC_E_NONFINITE
    assert sts.cpu().tolist() == want_codes
    want = ref.compress(good, 1e-3, ref.NOA)
    assert sizes[0] == sizes[4] == len(want)
    assert sizes[3] == len(want)  # required size reported with CAPACITY
    assert words.cpu().tolist()[0] == len(want)
    for i in (0, 4):
        assert outs[i][:sizes[i]].cpu().numpy().tobytes() == want


def test_decompress_batch_flags_bad_streams(P, ref):
    from paper_2603_26968_amd import lopc
    x = synth.gaussian_bumps((130, 300), seed=6)
    s = ref.compress(x, 1e-3, ref.NOA)
    good = torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda()
    bad = bytearray(s)
    bad[64] ^= 0x04  # first record size: the sizes no longer add up to the body
    corrupt = torch.from_numpy(np.frombuffer(bytes(bad), np.uint8).copy()).cuda()
    streams = [good, corrupt, good]
    outs = [torch.empty(x.shape, dtype=torch.float32, device="cuda") for _ in streams]
    jobs = (P.Job * 4)()
    for i, (t, y) in enumerate(zip(streams, outs)):
        j = jobs[i]
        j.d_in, j.in_bytes, j.d_out, j.out_cap = t.data_ptr(), t.numel(), y.data_ptr(), y.numel() * 4
        j.dtype, j.ndim = 0, 2
        j.dims[0], j.dims[1] = x.shape
    # a job whose shape disagrees with its header
    y3 = torch.empty(x.size, dtype=torch.float32, device="cuda")
    j = jobs[3]
    j.d_in, j.in_bytes, j.d_out, j.out_cap = good.data_ptr(), good.numel(), y3.data_ptr(), x.size * 4
    j.dtype, j.ndim = 0, 2
    j.dims[0], j.dims[1] = x.shape[1], x.shape[0]
    ctx = P.context(0)
    wsz = P.lopc_batch_workspace_size(ctx, 1, jobs)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    _say("decompress statuses")
    st = P.lopc_decompress_batch(ctx, jobs, ws.data_ptr(), wsz,
                                 torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    _, codes = P.lopc_ctx_last_batch(ctx, 4)
    want = ref.decompress(s)
    try:
        ref.decompress(bytes(bad))
        corrupt_code = 0
    except ref.OracleError as e:
        corrupt_code = e.code
    assert codes == [0, corrupt_code, 0, lopc.LOPC_E_FORMAT]
    assert corrupt_code == lopc.LOPC_E_FORMAT
    assert st == lopc.LOPC_E_FORMAT
    for i in (0, 2):
        assert np.array_equal(outs[i].cpu().numpy().view(np.uint32), want.view(np.uint32))


def test_uneven_batch_matches_single(P, ref):
    """The batched workload at reduced scale (fields of 2D side 32..512, 3D
    side 16..96): every stream equals the single-field stream; the smallest
    fields also the oracle's; the round trip through decompress_batch equals
    single decompression."""
    _say("uneven batch, 64 fields, scale 0.5")
    batch = [(x, eb, "noa") for x, eb in synth.batch_fields(64, seed=0, scale=0.5)]
    want = single_streams(P, batch)
    got, st = batch_streams(P, batch, stats=True)
    assert_same_streams(got, want, "uneven batch")
    small = sorted(range(len(batch)), key=lambda i: batch[i][0].size)[:3]
    for i in small:
        x, eb, _ = batch[i]
        assert want[i] == ref.compress(x, eb, ref.NOA), i
    ts = [torch.from_numpy(np.frombuffer(s, np.uint8).copy()).cuda() for s in want]
    ys = P.decompress_batch(ts)
    torch.cuda.synchronize()
    for i, (y, t) in enumerate(zip(ys, ts)):
        z = P.decompress(t)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint8), z.cpu().numpy().view(np.uint8)), i


def test_batch_with_a_chain_across_many_tiles(P, ref):
    """A field whose same-bin chain falls with the index across 4096 tiles
    (Sec. IV-E worst case) next to ordinary fields: past 64 sweeps the batch
    compresses that field on its own (the repair restarts on the device
    queue); every stream still equals the oracle's, and the chain's subbins
    are n-1, ..., 0."""
    _say("batch with a long falling chain")
    n = 1 << 18
    chain = (np.arange(n, 0, -1, dtype=np.float64) / n).astype(np.float32).reshape(1, n)
    batch = [(synth.gaussian_bumps((40, 52), seed=3), 1e-3, "noa"),
             (chain, 10.0, "abs"),
             (synth.turbulence_field((24, 20, 28), seed=2, dtype=np.float64), 1e-2, "noa")]
    want = [ref.compress(x, eb, ref.NOA if m == "noa" else ref.ABS) for x, eb, m in batch]
    got, st = batch_streams(P, batch, stats=True)
    assert_same_streams(got, want, "batch with chain")
    assert st["status"] == [0] * len(batch)
    _, sub = ref.decode_codes(got[1])
    assert np.array_equal(sub.ravel().astype(np.int64), np.arange(n - 1, -1, -1))
