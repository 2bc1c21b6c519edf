"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (default scheduler, synchronous calls):

* the 3D float64 512^3 lognormal field (1 GiB, NOA 1e-3): the whole stream
  and the whole reconstruction against one oracle run;
* the 256-field float32 batch: one batch compression and decompression of
  all fields, every 16th field's stream and reconstruction against the
  oracle, and every field's stream against its own single-field stream.

Each step prints what it does (the oracle's 1 GiB run takes a minute or
two)."""
import hashlib

import numpy as np
import pytest
import torch

from paper_2603_26968_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_26968_amd as P
    return P


@pytest.mark.timeout(900)
def test_lognormal3d_512_whole_field(P, ref):
    _say("lognormal3d 512^3 f64: generating")
    x = synth.lognormal_field((512, 512, 512), seed=0)
    _say("GPU compress + decompress")
    t = torch.from_numpy(x).cuda()
    s, hdr = P.compress(t, 1e-3, "noa", header=True)
    y = P.decompress(s, header=hdr)
    torch.cuda.synchronize()
    got_s = s.cpu().numpy().tobytes()
    got_y = hashlib.sha256(y.cpu().numpy().view(np.uint8).tobytes()).hexdigest()
    del t, y, s
    _say("oracle compress (whole field)")
    want = ref.compress(x, 1e-3, ref.NOA)
    _say("oracle decompress")
    assert len(got_s) == len(want) and got_s == want
    z = ref.decompress(want)
    assert got_y == hashlib.sha256(z.view(np.uint8).tobytes()).hexdigest()


@pytest.mark.timeout(900)
def test_batch_256_fields(P, ref):
    _say("batch of 256 fields: generating")
    fields = synth.batch_fields(256, seed=0)
    xs = [torch.from_numpy(x).cuda() for x, _ in fields]
    ebs = [eb for _, eb in fields]
    _say("GPU batch compress + decompress")
    streams, hdrs = P.compress_batch(xs, ebs, "noa", headers=True)
    ys = P.decompress_batch(streams, headers=hdrs)
    torch.cuda.synchronize()
    for i in range(0, len(fields), 16):
        x, eb = fields[i]
        _say("field", i, x.shape, eb)
        want = ref.compress(x, eb, ref.NOA)
        assert streams[i].cpu().numpy().tobytes() == want, i
        assert np.array_equal(ys[i].cpu().numpy().view(np.uint8),
                              ref.decompress(want).view(np.uint8)), i
    _say("every batch stream against its single-field stream")
    for i, (x, s) in enumerate(zip(xs, streams)):
        assert torch.equal(P.compress(x, ebs[i], "noa"), s), i
