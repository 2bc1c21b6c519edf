"""The serving loop on the GPU: requests served concurrently on several slots
(each with its own context and HIP stream) give exactly the bytes the same
request gives when it runs alone and the bytes of the CPU oracle (streams and
reconstructions, float32 and float64, 2D and 3D, 1 MiB up to a few hundred
MiB), the HBM budget holds with the kept workspaces counted, and a request
whose data a kernel still writes when it is submitted reads it only after
that kernel."""
import numpy as np
import pytest
import torch

from paper_2603_26968_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_26968_amd as P
    return P


def templates(P, n, max_bytes):
    """n request templates drawn like the serving workload (sizes 1 MiB up
    to max_bytes), with payloads mirror-tiled from two generated fields, and
    each template's result when it runs alone."""
    base2 = torch.from_numpy(synth.smooth_field()).cuda()
    base3 = torch.from_numpy(synth.turbulence_field((64, 64, 64))).cuda()
    out = []
    for spec in synth.serving_requests(n, seed=7, min_bytes=1 << 20, max_bytes=max_bytes):
        base = base2 if len(spec["shape"]) == 2 else base3
        x = synth.reflect_tile(base, spec["shape"])
        x = x.to(torch.float32 if spec["dtype"] == np.float32 else torch.float64).contiguous()
        s, hdr = P.compress(x, spec["eb"], "noa", header=True)
        s = s.clone()
        if spec["op"] == "compress":
            out.append(dict(op="compress", data=x, eb=spec["eb"], want=s))
        else:
            y = P.decompress(s, header=hdr)
            out.append(dict(op="decompress", data=s, header=hdr, want=y))
    torch.cuda.synchronize()
    return out


def test_served_results_equal_alone(P):
    from paper_2603_26968_amd import serve
    print("[case] serving: 12 templates, 48 requests, 3 slots", flush=True)
    T = templates(P, 12, 8 << 20)
    budget = 96 << 20
    srv = serve.Server(budget, slots=3)
    try:
        def make(i):
            t = T[i % len(T)]
            return serve.Request(t["op"], t["data"], eb=t.get("eb", 0.0),
                                 header=t.get("header"), tag=i % len(T))
        offs = serve.poisson_arrivals(48, rate=4000.0, seed=11)
        reqs = serve.run_arrivals(srv, make, offs)
    finally:
        srv.close()
    for r in reqs:
        assert r.error is None, (r.tag, r.error)
        want = T[r.tag]["want"]
        got = r.result
        torch.cuda.synchronize()
        assert got.dtype == want.dtype and got.shape == want.shape, r.tag
        assert torch.equal(got.view(torch.uint8) if got.dtype != torch.uint8 else got,
                           want.view(torch.uint8) if want.dtype != torch.uint8 else want), r.tag
    assert srv.admission.peak <= budget and srv.admission.in_use == 0
    st = serve.latency_stats(reqs, lambda r: 1)
    assert st["failed"] == 0 and st["p99_ms"] >= st["p50_ms"] > 0


def _host(t):
    return t.cpu().numpy()


def test_served_results_equal_oracle(P, ref):
    """Templates of both dtypes and ranks plus two large requests (a 160 MiB
    float64 3D compression and a 128 MiB float32 2D decompression), served
    concurrently: every stream equals the oracle's stream of the same field
    and every decoded field the oracle's reconstruction."""
    from paper_2603_26968_amd import serve
    print("[case] serving vs oracle", flush=True)
    T = templates(P, 10, 6 << 20)
    base3 = torch.from_numpy(synth.turbulence_field((64, 64, 64), seed=4)).cuda()
    big = synth.reflect_tile(base3, (160, 256, 512)).to(torch.float64).contiguous()
    T.append(dict(op="compress", data=big, eb=3e-3))
    base2 = torch.from_numpy(synth.smooth_field(seed=5)).cuda()
    x2 = synth.reflect_tile(base2, (4096, 8192)).contiguous()
    s2, h2 = P.compress(x2, 1e-3, "noa", header=True)
    T.append(dict(op="decompress", data=s2.clone(), header=h2, field=x2))
    torch.cuda.synchronize()
    kinds = set()
    for t in T:
        if t["op"] == "compress":
            xh = _host(t["data"])
            t["want_oracle"] = ref.compress(xh, t["eb"], ref.NOA)
            kinds.add((xh.dtype.name, xh.ndim))
        else:
            t["want_oracle"] = ref.decompress(_host(t["data"]).tobytes())
            kinds.add((t["want_oracle"].dtype.name, t["want_oracle"].ndim))
    assert len({d for d, _ in kinds}) == 2 and len({r for _, r in kinds}) == 2
    budget = 2 << 30
    srv = serve.Server(budget, slots=3)
    try:
        def make(i):
            t = T[i % len(T)]
            return serve.Request(t["op"], t["data"], eb=t.get("eb", 0.0),
                                 header=t.get("header"), tag=i % len(T))
        offs = serve.poisson_arrivals(2 * len(T), rate=2000.0, seed=13)
        reqs = serve.run_arrivals(srv, make, offs)
    finally:
        srv.close()
    for r in reqs:
        assert r.error is None, (r.tag, r.error)
        t = T[r.tag]
        got = _host(r.result)
        if t["op"] == "compress":
            assert got.tobytes() == t["want_oracle"], r.tag
        else:
            w = t["want_oracle"]
            assert got.dtype == w.dtype and got.shape == w.shape, r.tag
            assert np.array_equal(got.view(np.uint8), w.view(np.uint8)), r.tag
    assert srv.peak_total <= budget and srv.admission.in_use == 0


def test_submit_orders_after_unsynchronised_producer(P, ref):
    """The caller writes the field with kernels on its own stream and submits
    at once, without synchronising: the slot's stream waits for them, so the
    stream is the oracle's stream of the final values."""
    from paper_2603_26968_amd import serve
    print("[case] serving: unsynchronised producer", flush=True)
    x = synth.turbulence_field((96, 96, 96), seed=8)
    want = ref.compress(x, 1e-3, ref.NOA)
    prod = torch.cuda.Stream()
    with serve.Server(1 << 30, slots=2) as srv:
        for rep in range(3):
            with torch.cuda.stream(prod):
                d = torch.zeros(x.shape, dtype=torch.float32, device="cuda")
                torch.cuda._sleep(20_000_000)  # keep the stream busy before the copy
                d.copy_(torch.from_numpy(x).pin_memory(), non_blocking=True)
                r = srv.submit(serve.Request("compress", d, eb=1e-3))
            got = r.wait(60)
            torch.cuda.synchronize()
            assert got.cpu().numpy().tobytes() == want, rep
