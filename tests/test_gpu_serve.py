"""The serving loop on the GPU: requests served concurrently on several slots
(each with its own context and HIP stream) give exactly the bytes the same
request gives when it runs alone, and the HBM budget holds."""
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
