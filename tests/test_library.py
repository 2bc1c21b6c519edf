"""CPU checks of the C ABI library: it loads, exports every function that
include/lopc.h declares, and its host-only calls (bounds, header parsing)
agree with the oracle.  No compute call is made without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lopc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lopc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    from paper_2603_26968_amd import lopc
    lib = ctypes.CDLL(lopc.LIB_PATH)
    names = declared_functions()
    assert "lopc_compress" in names and "lopc_decompress" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(lopc.EXPORTS) | set(names)


def test_binding_names_mirror_the_abi():
    import paper_2603_26968_amd as P
    for name in ("lopc_compress", "lopc_decompress", "lopc_compress_bound",
                 "lopc_workspace_size", "lopc_stream_info", "lopc_ctx_create"):
        assert callable(getattr(P, name))


@pytest.mark.parametrize("shape", [(1, 1), (512, 512), (70, 61), (256, 256, 256),
                                   (1800, 3600), (3, 5, 7), (4096, 1), (1, 4097)])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_compress_bound_matches_oracle(ref, shape, dt):
    import paper_2603_26968_amd as P
    tdt = torch.float32 if dt == np.float32 else torch.float64
    assert P.lopc_compress_bound(shape, tdt) == ref.compress_bound(shape, dt)


def test_stream_info_agrees_with_oracle(ref):
    import paper_2603_26968_amd as P
    rng = np.random.default_rng(0)
    for dt in (np.float32, np.float64):
        for shape in ((9, 13), (4, 5, 6)):
            x = rng.standard_normal(shape).astype(dt)
            s = ref.compress(x, 1e-2)
            a = P.lopc_stream_info(s[:64])
            b = ref.stream_info(s)
            assert a["shape"] == b["shape"] and a["eps"] == b["eps"]
            assert a["field_bytes"] == x.nbytes
            bad = bytearray(s)
            bad[56] ^= 1
            with pytest.raises(P.LopcError):
                P.lopc_stream_info(bytes(bad[:64]))


def test_workspace_sizes():
    import paper_2603_26968_amd as P
    from paper_2603_26968_amd import lopc
    for shape in ((512, 512), (256, 256, 256)):
        c = lopc.lopc_workspace_size(None, shape, torch.float32, 0)
        d = lopc.lopc_workspace_size(None, shape, torch.float32, 1)
        n = int(np.prod(shape))
        assert c >= n * 10 and 0 < d < n
    with pytest.raises(P.LopcError):
        lopc.lopc_workspace_size(None, (2 ** 20, 2 ** 13), torch.float32, 0)  # >= 2^32 points


def _job(P, shape, dtype=0, eb=1e-3, mode=1, d_in=1 << 20, d_out=1 << 21, in_bytes=0,
         out_cap=1 << 30):
    j = P.Job()
    j.d_in, j.d_out, j.in_bytes, j.out_cap = d_in, d_out, in_bytes, out_cap
    j.dtype, j.ndim = dtype, len(shape)
    for i, s in enumerate(shape[:3]):
        j.dims[i] = s
    j.error_bound, j.mode = eb, mode
    return j


def _batch_ws(P, op, jobs):
    arr = (P.Job * len(jobs))(*jobs)
    n = ctypes.c_size_t()
    st = P.lopc.load().lopc_batch_workspace_size(None, op, len(jobs), arr, ctypes.byref(n))
    return st, n.value


def test_batch_workspace_size_and_validation():
    """Host-only plan of the batch calls: sizes grow with the jobs, every
    invalid job is rejected with the documented status before any launch."""
    import paper_2603_26968_amd as P
    from paper_2603_26968_amd import lopc
    ok = [_job(P, (70, 61)), _job(P, (9, 10, 11), dtype=1, mode=0)]
    st, a = _batch_ws(P, 0, ok)
    assert st == 0 and a > 0 and a % 256 == 0
    st, b = _batch_ws(P, 0, ok + [_job(P, (300, 200))])
    assert st == 0 and b > a
    # at least the bins, flags and subbins of every field
    assert a >= 70 * 61 * (4 + 2 + 4) + 9 * 10 * 11 * (8 + 2 + 4)
    cases = [
        ([_job(P, (4, 4), dtype=2)], 0, lopc.LOPC_E_ARG),
        ([_job(P, (4, 4, 4, 4))], 0, lopc.LOPC_E_ARG),
        ([_job(P, (0, 4))], 0, lopc.LOPC_E_ARG),
        ([_job(P, (4, 4), eb=0.0)], 0, lopc.LOPC_E_BOUND),
        ([_job(P, (4, 4), eb=float("nan"))], 0, lopc.LOPC_E_BOUND),
        ([_job(P, (4, 4), eb=float("inf"))], 0, lopc.LOPC_E_BOUND),
        ([_job(P, (4, 4), mode=3)], 0, lopc.LOPC_E_ARG),
        ([_job(P, (4, 4), d_in=(1 << 20) + 4)], 0, lopc.LOPC_E_ARG),   # field not 16-aligned
        ([_job(P, (4, 4), d_out=(1 << 21) + 2)], 0, lopc.LOPC_E_ARG),  # stream not 4-aligned
        ([_job(P, (4, 4), d_in=0)], 0, lopc.LOPC_E_ARG),
        ([_job(P, (4, 4), in_bytes=67)], 1, lopc.LOPC_E_FORMAT),       # < header + table
        ([_job(P, (4, 4), in_bytes=68, out_cap=63)], 1, lopc.LOPC_E_CAPACITY),
        ([_job(P, (4, 4), dtype=1, in_bytes=68, d_out=(1 << 21) + 4)], 1, lopc.LOPC_E_ARG),
    ]
    ok_d = [_job(P, (4, 4), in_bytes=68, out_cap=64)]
    for jobs, op, want in cases:
        st, _ = _batch_ws(P, op, (ok if op == 0 else ok_d) + jobs)
        assert st == want, (op, want, st)
    st, _ = _batch_ws(P, 1, [_job(P, (4, 4), in_bytes=68, out_cap=64)])
    assert st == 0
    arr = (P.Job * 1)()
    n = ctypes.c_size_t()
    assert lopc.load().lopc_batch_workspace_size(None, 0, 0, arr, ctypes.byref(n)) == lopc.LOPC_E_ARG
    assert lopc.load().lopc_batch_workspace_size(None, 2, 1, arr, ctypes.byref(n)) == lopc.LOPC_E_ARG
