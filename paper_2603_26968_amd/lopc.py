"""ctypes binding of liblopc.so (include/lopc.h).

Argument marshalling only: every step of compression and decompression runs
in the library's HIP kernels.  torch supplies device memory (the caching
allocator) and the current stream.  If the shared library is missing this
module raises at import time; there is no fallback path.

Low-level names mirror the C ABI (``lopc_compress`` ...); ``compress`` and
``decompress`` wrap them for torch tensors.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblopc.so")

LOPC_OK = 0
LOPC_E_ARG, LOPC_E_NONFINITE, LOPC_E_BOUND, LOPC_E_RANGE = -1, -2, -3, -4
LOPC_E_CAPACITY, LOPC_E_FORMAT, LOPC_E_HIP, LOPC_E_NOMEM, LOPC_E_INTERNAL = -5, -6, -7, -8, -9
LOPC_F32, LOPC_F64 = 0, 1
LOPC_EB_ABS, LOPC_EB_NOA = 0, 1
HEADER_BYTES = 64

EXPORTS = ("lopc_ctx_create", "lopc_ctx_destroy", "lopc_compress_bound",
           "lopc_workspace_size", "lopc_compress", "lopc_stream_info",
           "lopc_decompress", "lopc_strerror", "lopc_ctx_set_timing",
           "lopc_ctx_last_timings", "lopc_ctx_last_hip_error", "lopc_decompress_h",
           "lopc_ctx_last_header")
PHASES = ("range", "quant", "repair", "encode", "offsets", "decode")


class LopcError(RuntimeError):
    def __init__(self, code: int, what: str = "", ctx: int | None = None):
        msg = load().lopc_strerror(code).decode()
        if code == LOPC_E_HIP and ctx:
            msg += ": " + load().lopc_ctx_last_hip_error(ctx, None).decode()
        super().__init__(f"{what}: {msg} (status {code})" if what else msg)
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("repair_sweeps", ctypes.c_uint64),
                ("active_tiles_total", ctypes.c_uint64), ("bins_bytes", ctypes.c_uint64),
                ("subbins_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_lock = threading.Lock()


def load() -> ctypes.CDLL:
    """Load liblopc.so (built by paper_2603_26968_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2603_26968_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, ci, cd = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    i64p = ctypes.POINTER(ctypes.c_int64)
    szp = ctypes.POINTER(ctypes.c_size_t)
    L.lopc_ctx_create.argtypes = [ci, ctypes.POINTER(vp)]
    L.lopc_ctx_create.restype = ci
    L.lopc_ctx_destroy.argtypes = [vp]
    L.lopc_ctx_destroy.restype = None
    L.lopc_compress_bound.argtypes = [ci, ci, i64p, szp]
    L.lopc_compress_bound.restype = ci
    L.lopc_workspace_size.argtypes = [vp, ci, ci, i64p, ci, szp]
    L.lopc_workspace_size.restype = ci
    L.lopc_compress.argtypes = [vp, vp, ci, ci, i64p, cd, ci, vp, sz, szp, vp, sz, vp,
                                ctypes.POINTER(Stats)]
    L.lopc_compress.restype = ci
    L.lopc_stream_info.argtypes = [vp, sz, ctypes.POINTER(ci), ctypes.POINTER(ci), i64p,
                                   ctypes.POINTER(cd), szp]
    L.lopc_stream_info.restype = ci
    L.lopc_decompress.argtypes = [vp, vp, sz, vp, sz, vp, sz, vp]
    L.lopc_decompress.restype = ci
    L.lopc_strerror.argtypes = [ci]
    L.lopc_strerror.restype = ctypes.c_char_p
    L.lopc_ctx_set_timing.argtypes = [vp, ci]
    L.lopc_ctx_set_timing.restype = ci
    L.lopc_ctx_last_timings.argtypes = [vp, ctypes.POINTER(cd), ci]
    L.lopc_ctx_last_timings.restype = ci
    L.lopc_decompress_h.argtypes = [vp, vp, vp, sz, vp, sz, vp, sz, vp]
    L.lopc_decompress_h.restype = ci
    L.lopc_ctx_last_header.argtypes = [vp, vp]
    L.lopc_ctx_last_header.restype = ci
    L.lopc_ctx_last_hip_error.argtypes = [vp, ctypes.POINTER(ci)]
    L.lopc_ctx_last_hip_error.restype = ctypes.c_char_p
    _lib = L
    return L


# ------------------------------------------------------------------ C ABI names
def lopc_ctx_create(device: int) -> int:
    h = ctypes.c_void_p()
    st = load().lopc_ctx_create(device, ctypes.byref(h))
    if st:
        raise LopcError(st, "lopc_ctx_create")
    return h.value


def lopc_ctx_destroy(ctx: int) -> None:
    load().lopc_ctx_destroy(ctx)


def lopc_ctx_set_timing(ctx: int, enable: bool) -> None:
    st = load().lopc_ctx_set_timing(ctx, 1 if enable else 0)
    if st:
        raise LopcError(st, "lopc_ctx_set_timing")


def lopc_ctx_last_timings(ctx: int) -> dict:
    """Milliseconds of each phase of the last compress / decompress call."""
    buf = (ctypes.c_double * len(PHASES))()
    st = load().lopc_ctx_last_timings(ctx, buf, len(PHASES))
    if st:
        raise LopcError(st, "lopc_ctx_last_timings")
    return {name: buf[i] for i, name in enumerate(PHASES)}


def _dims(shape):
    d = (ctypes.c_int64 * 3)(1, 1, 1)
    for i, s in enumerate(shape):
        d[i] = int(s)
    return d


def _dtype_code(dtype) -> int:
    if dtype == torch.float32:
        return LOPC_F32
    if dtype == torch.float64:
        return LOPC_F64
    raise TypeError("LOPC compresses float32 and float64 fields")


def lopc_compress_bound(shape, dtype) -> int:
    n = ctypes.c_size_t()
    st = load().lopc_compress_bound(_dtype_code(dtype), len(shape), _dims(shape), ctypes.byref(n))
    if st:
        raise LopcError(st, "lopc_compress_bound")
    return n.value


def lopc_workspace_size(ctx: int, shape, dtype, op: int) -> int:
    n = ctypes.c_size_t()
    st = load().lopc_workspace_size(ctx, _dtype_code(dtype), len(shape), _dims(shape), op,
                                    ctypes.byref(n))
    if st:
        raise LopcError(st, "lopc_workspace_size")
    return n.value


def lopc_stream_info(header: bytes) -> dict:
    h = bytes(header)[:HEADER_BYTES]
    buf = ctypes.create_string_buffer(h, len(h))
    dt, nd = ctypes.c_int(), ctypes.c_int()
    dims = (ctypes.c_int64 * 3)()
    eps = ctypes.c_double()
    fb = ctypes.c_size_t()
    st = load().lopc_stream_info(buf, len(h), ctypes.byref(dt), ctypes.byref(nd), dims,
                                 ctypes.byref(eps), ctypes.byref(fb))
    if st:
        raise LopcError(st, "lopc_stream_info")
    return {"dtype": torch.float32 if dt.value == 0 else torch.float64,
            "shape": tuple(int(dims[i]) for i in range(nd.value)),
            "eps": eps.value, "field_bytes": fb.value}


def lopc_compress(ctx, d_field, dtype_code, shape, error_bound, mode, d_stream, cap,
                  d_ws, ws_bytes, stream):
    """Raw call: returns (status, stream size, Stats)."""
    size = ctypes.c_size_t()
    stats = Stats()
    st = load().lopc_compress(ctx, d_field, dtype_code, len(shape), _dims(shape),
                              float(error_bound), mode, d_stream, cap, ctypes.byref(size),
                              d_ws, ws_bytes, stream, ctypes.byref(stats))
    return st, size.value, stats


def lopc_decompress(ctx, d_stream, size, d_field, cap, d_ws, ws_bytes, stream) -> int:
    return load().lopc_decompress(ctx, d_stream, size, d_field, cap, d_ws, ws_bytes, stream)


def lopc_decompress_h(ctx, header: bytes, d_stream, size, d_field, cap, d_ws, ws_bytes,
                      stream) -> int:
    buf = ctypes.create_string_buffer(bytes(header)[:HEADER_BYTES], HEADER_BYTES)
    return load().lopc_decompress_h(ctx, buf, d_stream, size, d_field, cap, d_ws, ws_bytes,
                                    stream)


def lopc_ctx_last_header(ctx) -> bytes:
    buf = ctypes.create_string_buffer(HEADER_BYTES)
    st = load().lopc_ctx_last_header(ctx, buf)
    if st:
        raise LopcError(st, "lopc_ctx_last_header")
    return buf.raw


# ------------------------------------------------------------------ torch API
_ctx = {}


def context(device=None) -> int:
    dev = torch.cuda.current_device() if device is None else int(device)
    with _lock:
        if dev not in _ctx:
            _ctx[dev] = lopc_ctx_create(dev)
        return _ctx[dev]


def _mode(mode) -> int:
    if isinstance(mode, str):
        m = mode.lower()
        if m not in ("abs", "noa"):
            raise ValueError("mode is 'abs' or 'noa'")
        return LOPC_EB_ABS if m == "abs" else LOPC_EB_NOA
    return int(mode)


def _check_field(x: torch.Tensor):
    if not x.is_cuda:
        raise ValueError("field must be a device tensor")
    if x.dim() not in (2, 3):
        raise ValueError("field must be 2D or 3D")
    if not x.is_contiguous():
        raise ValueError("field must be contiguous (C order)")
    return _dtype_code(x.dtype)


_sizes = {}


def _sizes_for(ctx, shape, dtype):
    """(compress bound, compress workspace, decompress workspace), cached."""
    key = (tuple(shape), dtype)
    v = _sizes.get(key)
    if v is None:
        v = (lopc_compress_bound(shape, dtype), lopc_workspace_size(ctx, shape, dtype, 0),
             lopc_workspace_size(ctx, shape, dtype, 1))
        _sizes[key] = v
    return v


def compress(x: torch.Tensor, error_bound: float, mode="noa", stats: bool = False,
             out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
             header: bool = False):
    """Compress a 2D/3D float32/float64 device tensor.  Returns a uint8 device
    tensor holding the stream (a view of ``out`` if given), then a stats dict
    when ``stats`` is true, then the 64-byte header (host bytes) when
    ``header`` is true."""
    code = _check_field(x)
    dev = x.device
    ctx = context(dev.index)
    cap, wsz, _ = _sizes_for(ctx, x.shape, x.dtype)
    if out is None or out.numel() < cap:
        out = torch.empty(cap, dtype=torch.uint8, device=dev)
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(wsz, dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream(dev).cuda_stream
    st, size, stt = lopc_compress(ctx, x.data_ptr(), code, tuple(x.shape), error_bound,
                                  _mode(mode), out.data_ptr(), out.numel(),
                                  workspace.data_ptr(), workspace.numel(), s)
    if st:
        raise LopcError(st, "lopc_compress", ctx)
    res = [out[:size]]
    if stats:
        res.append(stt.as_dict())
    if header:
        res.append(lopc_ctx_last_header(ctx))
    return res[0] if len(res) == 1 else tuple(res)


def decompress(stream: torch.Tensor, out: torch.Tensor | None = None,
               workspace: torch.Tensor | None = None,
               header: bytes | None = None) -> torch.Tensor:
    """Decompress a uint8 device tensor holding exactly one stream.  If the
    caller holds the stream's 64-byte header on the host (``header``, e.g.
    from ``compress(..., header=True)``) no device-to-host read is needed."""
    if not stream.is_cuda or stream.dtype != torch.uint8 or not stream.is_contiguous():
        raise ValueError("stream must be a contiguous uint8 device tensor")
    if stream.numel() < HEADER_BYTES:
        raise LopcError(LOPC_E_FORMAT, "lopc_decompress")
    hdr = bytes(header) if header is not None else \
        stream[:HEADER_BYTES].cpu().numpy().tobytes()
    info = lopc_stream_info(hdr)
    dev = stream.device
    ctx = context(dev.index)
    if out is None:
        out = torch.empty(info["shape"], dtype=info["dtype"], device=dev)
    wsz = _sizes_for(ctx, info["shape"], info["dtype"])[2]
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(wsz, dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream(dev).cuda_stream
    st = lopc_decompress_h(ctx, hdr, stream.data_ptr(), stream.numel(), out.data_ptr(),
                           out.numel() * out.element_size(), workspace.data_ptr(),
                           workspace.numel(), s)
    if st:
        raise LopcError(st, "lopc_decompress", ctx)
    return out


# load eagerly: a missing library is an import error, never a silent fallback
load()
