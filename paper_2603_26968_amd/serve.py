"""Serving loop for LOPC requests on one GPU.

A request compresses a device-resident field or decompresses a
device-resident stream.  Requests arrive over time; each one is admitted
when its HBM footprint fits the budget beside the requests in flight (first
come, first served: a large request at the head is not overtaken), then runs
on a free slot.  A slot is a worker thread with its own library context, its
own HIP stream (default priority) and its own workspace, grown on demand and
kept between requests up to a per-slot limit; the library calls release the
interpreter lock while they wait, so requests on different slots overlap on
the GPU.  A request's latency runs from its arrival to the moment its result
is ready.

Memory: the workspaces the slots keep are a standing reservation taken out
of the budget up front (slots x keep limit), so the bytes of the requests in
flight plus the kept workspaces never exceed the budget.

Stream order: submit() records an event on the caller's current stream; the
slot's stream waits for it before the request runs, so a field or stream
written by a kernel the caller has not synchronised is read only after that
kernel.  The result is marked as used by the caller's stream, so the
allocator does not hand its memory to the slot's stream while the caller's
work on it may still be pending.

Nothing here computes: every byte of every result comes from the library's
kernels (``lopc.compress`` / ``lopc.decompress`` with the slot's context).
"""
from __future__ import annotations

import collections
import math
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Optional

import numpy as np


@dataclass
class Request:
    op: str                      # "compress" or "decompress"
    data: Any                    # device field (compress) or stream (decompress)
    eb: float = 1e-3             # compress: error bound
    mode: str = "noa"            # compress: "noa" or "abs"
    header: Optional[bytes] = None  # decompress: the stream's header, if known
    tag: Any = None              # caller's label (e.g. a template index)
    keep: bool = True            # False: drop the result once done (timing runs)
    arrival: float = 0.0         # time.perf_counter() at arrival
    # filled in by the server
    ready: Any = None            # event on the caller's stream at submit (device data)
    caller_stream: Any = None    # the caller's stream at submit (device data)
    footprint: int = 0
    start: float = 0.0
    end: float = 0.0
    result: Any = None
    error: Optional[BaseException] = None
    done: threading.Event = field(default_factory=threading.Event, repr=False)

    @property
    def latency(self) -> float:
        return self.end - self.arrival

    def wait(self, timeout=None):
        if not self.done.wait(timeout):
            raise TimeoutError("request not finished")
        if self.error is not None:
            raise self.error
        return self.result


class Admission:
    """First-come-first-served admission against a byte budget.  acquire()
    blocks until the request is at the head of the line and fits; a request
    larger than the whole budget is refused at once."""

    def __init__(self, budget: int):
        if budget <= 0:
            raise ValueError("budget must be positive")
        self.budget = int(budget)
        self.in_use = 0
        self.peak = 0
        self._cv = threading.Condition()
        self._line = collections.deque()

    def acquire(self, nbytes: int, timeout: float | None = None) -> bool:
        if nbytes > self.budget:
            raise MemoryError(f"request needs {nbytes} B, budget is {self.budget} B")
        me = object()
        deadline = None if timeout is None else time.perf_counter() + timeout
        with self._cv:
            self._line.append(me)
            try:
                while self._line[0] is not me or self.in_use + nbytes > self.budget:
                    left = None if deadline is None else deadline - time.perf_counter()
                    if left is not None and left <= 0:
                        return False
                    self._cv.wait(left)
                self.in_use += nbytes
                self.peak = max(self.peak, self.in_use)
                return True
            finally:
                self._line.remove(me)
                self._cv.notify_all()

    def release(self, nbytes: int) -> None:
        with self._cv:
            self.in_use -= nbytes
            assert self.in_use >= 0
            self._cv.notify_all()


class Server:
    """``slots`` workers behind an admission queue.  ``execute(slot, req)``
    runs a request on a slot and returns its result; ``footprint(req)`` gives
    its HBM bytes.  Both default to the GPU executor (``GpuSlots``); tests on
    the CPU pass their own."""

    def __init__(self, budget: int, slots: int = 4, execute: Callable | None = None,
                 footprint: Callable | None = None, device: int = 0,
                 keep_limit: int | None = None, kept: Callable | None = None):
        if slots < 1:
            raise ValueError("at least one slot")
        # workspaces kept between requests: at most keep_limit bytes per
        # slot (default: a quarter of the budget over all slots for the GPU
        # executor; none for a caller's executor unless given), reserved from
        # the budget up front
        gpu = execute is None or footprint is None
        if keep_limit is None:
            keep_limit = budget // (4 * slots) if gpu else 0
        self.keep_limit = int(keep_limit)
        if slots * self.keep_limit >= budget:
            raise ValueError("the kept workspaces would take the whole budget")
        self._gpu = None
        if gpu:
            self._gpu = GpuSlots(slots, device, self.keep_limit)
            execute = execute or self._gpu.execute
            footprint = footprint or self._gpu.footprint
            kept = kept or self._gpu.kept_bytes
        self.execute, self.footprint = execute, footprint
        self.kept = kept or (lambda: 0)
        self.budget = int(budget)
        self.admission = Admission(budget - slots * self.keep_limit)
        self.peak_total = 0  # largest in-flight + kept bytes seen at a release
        self._pending = queue.Queue()
        self._free = queue.Queue()
        for s in range(slots):
            self._free.put(s)
        self._work = [queue.Queue() for _ in range(slots)]
        self._closed = False
        self._threads = [threading.Thread(target=self._worker, args=(s,), daemon=True)
                         for s in range(slots)]
        self._threads.append(threading.Thread(target=self._scheduler, daemon=True))
        for t in self._threads:
            t.start()

    def submit(self, req: Request) -> Request:
        if self._closed:
            raise RuntimeError("server closed")
        if not req.arrival:
            req.arrival = time.perf_counter()
        if self._gpu is not None:
            self._gpu.mark_ready(req)
        self._pending.put(req)
        return req

    def _finish(self, req, result=None, error=None):
        req.result, req.error = result, error
        req.end = time.perf_counter()
        req.done.set()

    def _scheduler(self):
        while True:
            req = self._pending.get()
            if req is None:
                break
            try:
                req.footprint = int(self.footprint(req))
                self.admission.acquire(req.footprint)
            except BaseException as e:  # refused: the request fails, the line moves on
                self._finish(req, error=e)
                continue
            slot = self._free.get()
            self._work[slot].put(req)
        for w in self._work:
            w.put(None)

    def _worker(self, slot):
        while True:
            req = self._work[slot].get()
            if req is None:
                break
            req.start = time.perf_counter()
            try:
                res = self.execute(slot, req)
                err = None
            except BaseException as e:
                res, err = None, e
            if not req.keep:
                res = None
            with self.admission._cv:
                self.peak_total = max(self.peak_total, self.admission.in_use + self.kept())
            self.admission.release(req.footprint)
            self._free.put(slot)
            self._finish(req, res, err)

    def close(self):
        """Finish what was submitted, then stop the threads."""
        if not self._closed:
            self._closed = True
            self._pending.put(None)
            for t in self._threads:
                t.join()
            if self._gpu is not None:
                self._gpu.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class GpuSlots:
    """The GPU executor: per slot a library context, a HIP stream and a
    workspace tensor kept between requests while it is at most keep_limit
    bytes."""

    def __init__(self, slots: int, device: int = 0, keep_limit: int = 0):
        import torch

        from . import lopc
        self.torch, self.lopc = torch, lopc
        self.dev = torch.device("cuda", device)
        self.ctx = [lopc.lopc_ctx_create(device) for _ in range(slots)]
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.ws = [None] * slots
        self.keep_limit = keep_limit

    def kept_bytes(self) -> int:
        return sum(w.numel() for w in self.ws if w is not None)

    def mark_ready(self, req):
        """On the caller's thread at submit: an event after the caller's work
        so far on its current stream (which produced the request's data)."""
        torch = self.torch
        if isinstance(req.data, torch.Tensor) and req.data.is_cuda:
            req.caller_stream = torch.cuda.current_stream(req.data.device)
            req.ready = torch.cuda.Event()
            req.ready.record(req.caller_stream)

    def _info(self, req):
        if req.header is None:
            req.header = req.data[:self.lopc.HEADER_BYTES].cpu().numpy().tobytes()
        return self.lopc.lopc_stream_info(req.header)

    def footprint(self, req) -> int:
        L = self.lopc
        if req.op == "compress":
            x = req.data
            cap, wsz, _ = L._sizes_for(self.ctx[0], x.shape, x.dtype)
            return wsz + cap
        info = self._info(req)
        _, _, wsz = L._sizes_for(self.ctx[0], info["shape"], info["dtype"])
        return wsz + info["field_bytes"]

    def _workspace(self, slot, nbytes):
        w = self.ws[slot]
        if w is None or w.numel() < nbytes:
            self.ws[slot] = None
            w = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.dev)
            self.ws[slot] = w
        return w

    def execute(self, slot, req):
        torch, L = self.torch, self.lopc
        ctx = self.ctx[slot]
        st = self.streams[slot]
        try:
            with torch.cuda.stream(st):
                if req.ready is not None:
                    st.wait_event(req.ready)
                    req.data.record_stream(st)
                if req.op == "compress":
                    x = req.data
                    _, wsz, _ = L._sizes_for(ctx, x.shape, x.dtype)
                    out = L.compress(x, req.eb, req.mode, ctx=ctx,
                                     workspace=self._workspace(slot, wsz))
                elif req.op == "decompress":
                    info = self._info(req)
                    _, _, wsz = L._sizes_for(ctx, info["shape"], info["dtype"])
                    out = L.decompress(req.data, header=req.header, ctx=ctx,
                                       workspace=self._workspace(slot, wsz))
                else:
                    raise ValueError(f"unknown op {req.op!r}")
            if req.caller_stream is not None:
                out.record_stream(req.caller_stream)
            return out
        finally:
            # a workspace above the keep limit is not kept
            w = self.ws[slot]
            if w is not None and w.numel() > self.keep_limit:
                self.ws[slot] = None

    def close(self):
        for c in self.ctx:
            self.lopc.lopc_ctx_destroy(c)
        self.ctx = []


def poisson_arrivals(n: int, rate: float, seed: int = 7) -> np.ndarray:
    """Arrival offsets (seconds) of n requests of a Poisson process."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def run_arrivals(server: Server, make: Callable[[int], Request], offsets) -> list:
    """Submit request i = make(i) at time offsets[i] after the start; wait
    for all of them; return the requests."""
    reqs = []
    t0 = time.perf_counter()
    for i, off in enumerate(offsets):
        r = make(i)
        now = time.perf_counter()
        if t0 + off > now:
            time.sleep(t0 + off - now)
        r.arrival = time.perf_counter()
        reqs.append(server.submit(r))
    for r in reqs:
        r.done.wait()
    return reqs


def latency_stats(reqs, bytes_of: Callable[[Request], int]) -> dict:
    ok = [r for r in reqs if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.end for r in reqs) - min(r.arrival for r in reqs) if reqs else 0.0
    total = sum(bytes_of(r) for r in ok)
    return {"requests": len(reqs), "failed": len(reqs) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "mean_ms": float(lat.mean()) if len(lat) else math.nan,
            "GBps": total / span / 1e9 if span > 0 else 0.0}
