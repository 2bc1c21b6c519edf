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
           "lopc_ctx_last_header", "lopc_batch_workspace_size", "lopc_compress_batch",
           "lopc_decompress_batch", "lopc_ctx_last_batch", "lopc_ctx_set_option", "lopc_ctx_get_option",
           "lopc_ctx_last_batch_headers", "lopc_batch_autotune", "lopc_verify",
           "lopc_verify_workspace_size", "lopc_decompress_static")
LOPC_OPT_BATCH_GRAPH, LOPC_OPT_GRAPH_SWEEPS, LOPC_OPT_PERSIST_PCT, LOPC_OPT_REPAIR = 1, 2, 3, 4
LOPC_OPT_TILE_3D, LOPC_OPT_TILE_2D, LOPC_OPT_SWEEP_ORDER = 5, 6, 7
# the repair tile shapes behind LOPC_OPT_TILE_2D / _3D values (z x y x x)
kTile2Names = ("1x32x64", "1x16x128")
kTile3Names = ("4x8x32", "8x8x32", "8x16x16")
LOPC_REPAIR_AUTO, LOPC_REPAIR_HYBRID, LOPC_REPAIR_QUEUE, LOPC_REPAIR_SWEEPS = 0, 1, 2, 3
LOPC_REPAIR_POINTS = 4
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
                ("subbins_bytes", ctypes.c_uint64), ("relax_iterations", ctypes.c_uint64),
                ("queue_runs", ctypes.c_uint64), ("queue_parks", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Job(ctypes.Structure):
    """lopc_job: one field of a batch."""
    _fields_ = [("d_in", ctypes.c_void_p), ("in_bytes", ctypes.c_size_t),
                ("d_out", ctypes.c_void_p), ("out_cap", ctypes.c_size_t),
                ("dtype", ctypes.c_int), ("ndim", ctypes.c_int),
                ("dims", ctypes.c_int64 * 3), ("error_bound", ctypes.c_double),
                ("mode", ctypes.c_int), ("d_out_size", ctypes.c_void_p),
                ("d_status", ctypes.c_void_p)]


class BatchStats(ctypes.Structure):
    _fields_ = [("repair_sweeps", ctypes.c_uint64), ("active_tiles_total", ctypes.c_uint64),
                ("graph", ctypes.c_int), ("continued", ctypes.c_int),
                ("relax_iterations", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class VerifyReport(ctypes.Structure):
    _fields_ = [("points", ctypes.c_uint64), ("bound_violations", ctypes.c_uint64),
                ("max_abs_error", ctypes.c_double), ("edges", ctypes.c_uint64),
                ("order_violations", ctypes.c_uint64), ("types_orig", ctypes.c_uint64 * 4),
                ("types_recon", ctypes.c_uint64 * 4), ("type_mismatches", ctypes.c_uint64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["types_orig"] = list(self.types_orig)
        d["types_recon"] = list(self.types_recon)
        return d


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
    L.lopc_compress.argtypes = [vp, vp, ci, ci, i64p, cd, ci, vp, sz, szp, vp, vp, vp, sz, vp,
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
    L.lopc_decompress_static.argtypes = [vp, vp, vp, sz, vp, sz, vp]
    L.lopc_decompress_static.restype = ci
    L.lopc_decompress_h.restype = ci
    L.lopc_ctx_last_header.argtypes = [vp, vp]
    L.lopc_ctx_last_header.restype = ci
    L.lopc_ctx_last_hip_error.argtypes = [vp, ctypes.POINTER(ci)]
    L.lopc_ctx_last_hip_error.restype = ctypes.c_char_p
    jp = ctypes.POINTER(Job)
    L.lopc_batch_workspace_size.argtypes = [vp, ci, ci, jp, szp]
    L.lopc_batch_workspace_size.restype = ci
    L.lopc_compress_batch.argtypes = [vp, ci, jp, vp, sz, vp, ctypes.POINTER(BatchStats)]
    L.lopc_compress_batch.restype = ci
    L.lopc_decompress_batch.argtypes = [vp, ci, jp, vp, sz, vp]
    L.lopc_decompress_batch.restype = ci
    L.lopc_ctx_last_batch.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_int32)]
    L.lopc_ctx_last_batch.restype = ci
    L.lopc_batch_autotune.argtypes = [vp, ci, ci, jp, vp, sz, vp, ci, ctypes.POINTER(ci)]
    L.lopc_batch_autotune.restype = ci
    L.lopc_verify_workspace_size.argtypes = []
    L.lopc_verify_workspace_size.restype = sz
    L.lopc_verify.argtypes = [vp, vp, vp, ci, ci, i64p, cd, vp, sz, vp,
                              ctypes.POINTER(VerifyReport)]
    L.lopc_verify.restype = ci
    L.lopc_ctx_last_batch_headers.argtypes = [vp, ci, vp]
    L.lopc_ctx_last_batch_headers.restype = ci
    L.lopc_ctx_set_option.argtypes = [vp, ci, ctypes.c_int64]
    L.lopc_ctx_set_option.restype = ci
    L.lopc_ctx_get_option.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_int64)]
    L.lopc_ctx_get_option.restype = ci
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


def lopc_ctx_set_timing(ctx: int, phases=True) -> None:
    """Time the phases named in ``phases`` (names from PHASES) in the calls
    that follow; True: every phase, False / empty: none."""
    if phases is True:
        mask = (1 << len(PHASES)) - 1
    elif not phases:
        mask = 0
    else:
        mask = 0
        for p in phases:
            mask |= 1 << PHASES.index(p)
    st = load().lopc_ctx_set_timing(ctx, mask)
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
                  d_ws, ws_bytes, stream, want_stats: bool = True, d_size=None, d_status=None,
                  enqueue_only: bool = False):
    """Raw call: returns (status, stream size, Stats or None).  enqueue_only:
    h_stream_size NULL (d_size required); the size is then None."""
    size = ctypes.c_size_t()
    stats = Stats() if want_stats and not enqueue_only else None
    st = load().lopc_compress(ctx, d_field, dtype_code, len(shape), _dims(shape),
                              float(error_bound), mode, d_stream, cap,
                              None if enqueue_only else ctypes.byref(size), d_size, d_status,
                              d_ws, ws_bytes, stream,
                              ctypes.byref(stats) if stats is not None else None)
    return st, (None if enqueue_only else size.value), stats


def lopc_decompress(ctx, d_stream, size, d_field, cap, d_ws, ws_bytes, stream) -> int:
    return load().lopc_decompress(ctx, d_stream, size, d_field, cap, d_ws, ws_bytes, stream)


def lopc_decompress_h(ctx, header: bytes, d_stream, size, d_field, cap, d_ws, ws_bytes,
                      stream) -> int:
    h = header if type(header) is bytes and len(header) == HEADER_BYTES else \
        ctypes.create_string_buffer(bytes(header)[:HEADER_BYTES], HEADER_BYTES)
    return load().lopc_decompress_h(ctx, h, d_stream, size, d_field, cap, d_ws, ws_bytes,
                                    stream)


def lopc_decompress_static(ctx, header: bytes, d_stream, size, d_field, cap, stream) -> int:
    """Raw call of the allocation-free decompression (library-held scratch)."""
    return load().lopc_decompress_static(ctx, header, d_stream, size, d_field, cap, stream)


def lopc_ctx_last_header(ctx) -> bytes:
    buf = ctypes.create_string_buffer(HEADER_BYTES)
    st = load().lopc_ctx_last_header(ctx, buf)
    if st:
        raise LopcError(st, "lopc_ctx_last_header")
    return buf.raw


def lopc_ctx_set_option(ctx: int, option: int, value: int) -> None:
    st = load().lopc_ctx_set_option(ctx, option, int(value))
    if st:
        raise LopcError(st, "lopc_ctx_set_option")


def lopc_ctx_get_option(ctx: int, option: int) -> int:
    v = ctypes.c_int64()
    st = load().lopc_ctx_get_option(ctx, option, ctypes.byref(v))
    if st:
        raise LopcError(st, "lopc_ctx_get_option")
    return v.value


def lopc_batch_workspace_size(ctx: int, op: int, jobs) -> int:
    n = ctypes.c_size_t()
    st = load().lopc_batch_workspace_size(ctx, op, len(jobs), jobs, ctypes.byref(n))
    if st:
        raise LopcError(st, "lopc_batch_workspace_size")
    return n.value


def lopc_compress_batch(ctx, jobs, d_ws, ws_bytes, stream):
    """Raw call: returns (status, BatchStats)."""
    stats = BatchStats()
    st = load().lopc_compress_batch(ctx, len(jobs), jobs, d_ws, ws_bytes, stream,
                                    ctypes.byref(stats))
    return st, stats


def lopc_decompress_batch(ctx, jobs, d_ws, ws_bytes, stream) -> int:
    return load().lopc_decompress_batch(ctx, len(jobs), jobs, d_ws, ws_bytes, stream)


def lopc_ctx_last_batch(ctx, n: int):
    """(sizes, statuses) of the most recent batch call, in job order."""
    sizes = (ctypes.c_uint64 * n)()
    sts = (ctypes.c_int32 * n)()
    st = load().lopc_ctx_last_batch(ctx, n, sizes, sts)
    if st:
        raise LopcError(st, "lopc_ctx_last_batch")
    return list(sizes), list(sts)


def lopc_batch_autotune(ctx, op, jobs, d_ws, ws_bytes, stream, reps: int = 2) -> int:
    """Pick the persistent grid size for this batch; returns it (percent)."""
    pct = ctypes.c_int()
    st = load().lopc_batch_autotune(ctx, op, len(jobs), jobs, d_ws, ws_bytes, stream, reps,
                                    ctypes.byref(pct))
    if st:
        raise LopcError(st, "lopc_batch_autotune", ctx)
    return pct.value


def lopc_ctx_last_batch_headers(ctx, n: int):
    """64-byte stream headers of the most recent compress batch, in job order."""
    buf = ctypes.create_string_buffer(n * HEADER_BYTES)
    st = load().lopc_ctx_last_batch_headers(ctx, n, buf)
    if st:
        raise LopcError(st, "lopc_ctx_last_batch_headers")
    raw = buf.raw
    return [raw[i * HEADER_BYTES:(i + 1) * HEADER_BYTES] for i in range(n)]


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


def _stream_handle(dev: torch.device) -> int:
    """The current HIP stream of device `dev` as an integer handle."""
    return torch._C._cuda_getCurrentRawStream(dev.index)


_infos = {}


def _stream_info_cached(hdr: bytes) -> dict:
    """lopc_stream_info of a header, remembered per header (headers repeat
    when the same fields are decompressed again)."""
    v = _infos.get(hdr)
    if v is None:
        v = lopc_stream_info(hdr)
        if len(_infos) > 4096:
            _infos.clear()
        _infos[hdr] = v
    return v


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
    """(compress bound, compress workspace, decompress workspace), cached
    (the compress workspace also depends on whether the context's repair
    scheduler is the point worklists)."""
    key = (tuple(shape), dtype,
           lopc_ctx_get_option(ctx, LOPC_OPT_REPAIR) == LOPC_REPAIR_POINTS)
    v = _sizes.get(key)
    if v is None:
        v = (lopc_compress_bound(shape, dtype), lopc_workspace_size(ctx, shape, dtype, 0),
             lopc_workspace_size(ctx, shape, dtype, 1))
        _sizes[key] = v
    return v


def compress(x: torch.Tensor, error_bound: float, mode="noa", stats: bool = False,
             out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
             header: bool = False, ctx: int | None = None):
    """Compress a 2D/3D float32/float64 device tensor.  Returns a uint8 device
    tensor holding the stream (a view of ``out`` if given), then a stats dict
    when ``stats`` is true, then the 64-byte header (host bytes) when
    ``header`` is true.  ``ctx``: a library context of the caller's thread
    (default: the shared one of the device)."""
    code = _check_field(x)
    dev = x.device
    ctx = context(dev.index) if ctx is None else ctx
    cap, wsz, _ = _sizes_for(ctx, x.shape, x.dtype)
    if out is None or out.numel() < cap:
        out = torch.empty(cap, dtype=torch.uint8, device=dev)
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(wsz, dtype=torch.uint8, device=dev)
    s = _stream_handle(dev)
    st, size, stt = lopc_compress(ctx, x.data_ptr(), code, tuple(x.shape), error_bound,
                                  _mode(mode), out.data_ptr(), out.numel(),
                                  workspace.data_ptr(), workspace.numel(), s, stats)
    if st:
        raise LopcError(st, "lopc_compress", ctx)
    res = [out[:size]]
    if stats:
        res.append(stt.as_dict())
    if header:
        res.append(lopc_ctx_last_header(ctx))
    return res[0] if len(res) == 1 else tuple(res)


def compress_enqueue(x: torch.Tensor, error_bound: float, mode="noa",
                     out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                     size: torch.Tensor | None = None, status: torch.Tensor | None = None,
                     ctx: int | None = None):
    """Enqueue a compression on the current stream without waiting for it
    (lopc_compress with h_stream_size NULL).  Returns (out, size, status):
    the stream buffer (capacity: the compress bound), a one-element int64
    device tensor that receives the stream size and a one-element int32
    device tensor that receives the status.  The call touches no host memory
    after it returns, so it can be captured into a CUDA/HIP graph (pass
    preallocated ``out``, ``workspace``, ``size`` and ``status`` then)."""
    code = _check_field(x)
    dev = x.device
    ctx = context(dev.index) if ctx is None else ctx
    cap, wsz, _ = _sizes_for(ctx, x.shape, x.dtype)
    if out is None or out.numel() < cap:
        out = torch.empty(cap, dtype=torch.uint8, device=dev)
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(wsz, dtype=torch.uint8, device=dev)
    if size is None:
        size = torch.empty(1, dtype=torch.int64, device=dev)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
    s = _stream_handle(dev)
    st, _, _ = lopc_compress(ctx, x.data_ptr(), code, tuple(x.shape), error_bound, _mode(mode),
                             out.data_ptr(), out.numel(), workspace.data_ptr(),
                             workspace.numel(), s, False, size.data_ptr(), status.data_ptr(),
                             enqueue_only=True)
    if st:
        raise LopcError(st, "lopc_compress", ctx)
    return out, size, status


def decompress(stream: torch.Tensor, out: torch.Tensor | None = None,
               workspace: torch.Tensor | None = None,
               header: bytes | None = None, ctx: int | None = None) -> torch.Tensor:
    """Decompress a uint8 device tensor holding exactly one stream.  If the
    caller holds the stream's 64-byte header on the host (``header``, e.g.
    from ``compress(..., header=True)``) no device-to-host read is needed."""
    if not stream.is_cuda or stream.dtype != torch.uint8 or not stream.is_contiguous():
        raise ValueError("stream must be a contiguous uint8 device tensor")
    if stream.numel() < HEADER_BYTES:
        raise LopcError(LOPC_E_FORMAT, "lopc_decompress")
    hdr = (header if type(header) is bytes else bytes(header)) if header is not None else \
        stream[:HEADER_BYTES].cpu().numpy().tobytes()
    info = _stream_info_cached(hdr)
    dev = stream.device
    ctx = context(dev.index) if ctx is None else ctx
    if out is None:
        out = torch.empty(info["shape"], dtype=info["dtype"], device=dev)
    wsz = _sizes_for(ctx, info["shape"], info["dtype"])[2]
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(wsz, dtype=torch.uint8, device=dev)
    s = _stream_handle(dev)
    st = lopc_decompress_h(ctx, hdr, stream.data_ptr(), stream.numel(), out.data_ptr(),
                           out.numel() * out.element_size(), workspace.data_ptr(),
                           workspace.numel(), s)
    if st:
        raise LopcError(st, "lopc_decompress", ctx)
    return out


def verify(x: torch.Tensor, y: torch.Tensor, eps: float, ctx=None) -> dict:
    """Check a reconstruction y of x on the device: error bound, order of
    every edge, critical types (lopc_verify).  Returns the report as a dict
    (types in the order regular, minima, maxima, saddles)."""
    code = _check_field(x)
    if y.shape != x.shape or y.dtype != x.dtype or not y.is_contiguous() or y.device != x.device:
        raise ValueError("y must be a contiguous tensor of x's shape, dtype and device")
    ctx = context(x.device.index) if ctx is None else ctx
    ws = torch.empty(load().lopc_verify_workspace_size(), dtype=torch.uint8, device=x.device)
    rep = VerifyReport()
    st = load().lopc_verify(ctx, x.data_ptr(), y.data_ptr(), code, x.dim(), _dims(x.shape),
                            float(eps), ws.data_ptr(), ws.numel(),
                            torch.cuda.current_stream(x.device).cuda_stream, ctypes.byref(rep))
    if st:
        raise LopcError(st, "lopc_verify", ctx)
    return rep.as_dict()


# ------------------------------------------------------------------ batches
_ws_cache = {}


def _workspace(ctx, nbytes, dev, workspace=None):
    """Caller's workspace, else a per-context one grown as needed (a stable
    address lets the library replay its captured launch sequence)."""
    if workspace is not None:
        if workspace.numel() < nbytes:
            raise ValueError(f"workspace holds {workspace.numel()} bytes, {nbytes} needed")
        return workspace
    w = _ws_cache.get(ctx)
    if w is None or w.numel() < nbytes:
        w = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
        _ws_cache[ctx] = w
    return w


def _align(v, a=256):
    return (v + a - 1) // a * a


def _compress_jobs(fields, error_bounds, modes, out, ctx):
    n = len(fields)
    ebs = list(error_bounds) if hasattr(error_bounds, "__len__") else [error_bounds] * n
    mds = list(modes) if isinstance(modes, (list, tuple)) else [modes] * n
    if len(ebs) != n or len(mds) != n:
        raise ValueError("one error bound and one mode per field")
    dev = fields[0].device
    ctx = context(dev.index) if ctx is None else ctx
    caps = []
    for x in fields:
        _check_field(x)
        if x.device != dev:
            raise ValueError("all fields of a batch live on one device")
        caps.append(_sizes_for(ctx, x.shape, x.dtype)[0])
    offs, total = [], 0
    for c in caps:
        offs.append(total)
        total += _align(c)
    if out is None or out.numel() < total:
        out = torch.empty(total, dtype=torch.uint8, device=dev)
    jobs = (Job * n)()
    base = out.data_ptr()
    for i, x in enumerate(fields):
        j = jobs[i]
        j.d_in = x.data_ptr()
        j.d_out = base + offs[i]
        j.out_cap = caps[i]
        j.dtype = _dtype_code(x.dtype)
        j.ndim = x.dim()
        for d in range(x.dim()):
            j.dims[d] = int(x.shape[d])
        j.error_bound = float(ebs[i])
        j.mode = _mode(mds[i])
    return jobs, out, offs, ctx, dev


def compress_batch(fields, error_bounds, modes="noa", out: torch.Tensor | None = None,
                   workspace: torch.Tensor | None = None, stats: bool = False, ctx=None,
                   raise_on_error: bool = True, headers: bool = False):
    """Compress many independent 2D/3D float32/float64 device tensors in one
    batch call.  ``error_bounds`` and ``modes`` are scalars or one per field.
    Streams are packed into ``out`` (allocated if None) at 256-byte aligned
    offsets; returns the list of stream views (None for a failed field when
    ``raise_on_error`` is false), then the batch stats dict if ``stats``,
    then the list of 64-byte headers (host bytes) if ``headers``."""
    n = len(fields)
    if n == 0:
        return ([], {}) if stats else []
    jobs, out, offs, ctx, dev = _compress_jobs(fields, error_bounds, modes, out, ctx)
    wsz = lopc_batch_workspace_size(ctx, 0, jobs)
    ws = _workspace(ctx, wsz, dev, workspace)
    s = torch.cuda.current_stream(dev).cuda_stream
    st, bst = lopc_compress_batch(ctx, jobs, ws.data_ptr(), ws.numel(), s)
    if st and (raise_on_error or st in (LOPC_E_ARG, LOPC_E_HIP, LOPC_E_INTERNAL)):
        raise LopcError(st, "lopc_compress_batch", ctx)
    sizes, sts = lopc_ctx_last_batch(ctx, n)
    res = [out[offs[i]:offs[i] + sizes[i]] if sts[i] == 0 else None for i in range(n)]
    ret = [res]
    if stats:
        d = bst.as_dict()
        d["status"] = sts
        ret.append(d)
    if headers:
        ret.append(lopc_ctx_last_batch_headers(ctx, n))
    return ret[0] if len(ret) == 1 else tuple(ret)


def autotune_compress_batch(fields, error_bounds, modes="noa", out=None, workspace=None,
                            ctx=None, reps: int = 2) -> int:
    """Tune the persistent grid size and the repair tile shapes of the batch
    path on this batch (kept in the context); returns the chosen grid
    percentage."""
    jobs, out, offs, ctx, dev = _compress_jobs(fields, error_bounds, modes, out, ctx)
    wsz = lopc_batch_workspace_size(ctx, 0, jobs)
    ws = _workspace(ctx, wsz, dev, workspace)
    return lopc_batch_autotune(ctx, 0, jobs, ws.data_ptr(), ws.numel(),
                               torch.cuda.current_stream(dev).cuda_stream, reps)


def decompress_batch(streams, outs=None, workspace: torch.Tensor | None = None,
                     headers=None, ctx=None, raise_on_error: bool = True):
    """Decompress many streams (contiguous uint8 device tensors) in one batch
    call.  Shapes and dtypes come from ``headers`` (host bytes, one per
    stream) or from each stream's first 64 bytes.  Returns the list of
    fields (None for a failed stream when ``raise_on_error`` is false)."""
    n = len(streams)
    if n == 0:
        return []
    dev = streams[0].device
    ctx = context(dev.index) if ctx is None else ctx
    if headers is None:
        heads = torch.stack([s[:HEADER_BYTES] for s in streams]).cpu().numpy()
        headers = [heads[i].tobytes() for i in range(n)]
    infos = [lopc_stream_info(h) for h in headers]
    if outs is None:
        outs = [torch.empty(inf["shape"], dtype=inf["dtype"], device=dev) for inf in infos]
    jobs = (Job * n)()
    for i, (s, inf, y) in enumerate(zip(streams, infos, outs)):
        if not s.is_cuda or s.dtype != torch.uint8 or not s.is_contiguous():
            raise ValueError("streams must be contiguous uint8 device tensors")
        j = jobs[i]
        j.d_in = s.data_ptr()
        j.in_bytes = s.numel()
        j.d_out = y.data_ptr()
        j.out_cap = y.numel() * y.element_size()
        j.dtype = _dtype_code(inf["dtype"])
        j.ndim = len(inf["shape"])
        for d, v in enumerate(inf["shape"]):
            j.dims[d] = v
    wsz = lopc_batch_workspace_size(ctx, 1, jobs)
    ws = _workspace(ctx, wsz, dev, workspace)
    st = lopc_decompress_batch(ctx, jobs, ws.data_ptr(), ws.numel(),
                               torch.cuda.current_stream(dev).cuda_stream)
    if st and (raise_on_error or st in (LOPC_E_ARG, LOPC_E_HIP, LOPC_E_INTERNAL)):
        raise LopcError(st, "lopc_decompress_batch", ctx)
    _, sts = lopc_ctx_last_batch(ctx, n)
    return [outs[i] if sts[i] == 0 else None for i in range(n)]


# load eagerly: a missing library is an import error, never a silent fallback
load()
