#!/usr/bin/env python
"""Benchmark of the LOPC hot path on one MI355X.

Default workload (the headline line): one step = compress + decompress
(every step of the path: NOA range, quantize, order flags, repair to the
fixed point, chunk encoders and stream assembly, record offsets, chunk
decoders and reconstruction) of the 3D float64 512^3 lognormal field (1 GiB:
exp(2 g), g a GRF with P(k) ~ k^-2.5, floored at its 10th percentile), the
largest single-GPU workload, at a NOA bound of 1e-3, bit-exact.  The field
is resident in HBM before the timed region starts.  value = uncompressed
bytes / median round-trip time, GB/s (1e9 B/s); the timing block gives the
median, min and p90 of the timed steps for the round trip, compress and
decompress.  roofline: the dominant kernel (the longest of the first tile
pass, the encode phase and the decoder; the repair sweeps move only
intermediate arrays, so they have no algorithmic bytes and appear in
phase_ms) per launch against the 8 TB/s HBM peak, counting only algorithmic
bytes (the field and the stream); roofline_path: the same for whole
compress, decompress and round trip.
The CPU oracle runs beside it in child processes: on a bounded sample (the
cpu_baseline) and on the whole field (parity of the stream and the
reconstruction, compared through SHA-256).

Other workloads (--workload), one JSON line each:
  turb3d       3D float32 256^3 power-law GRF (P(k) ~ k^-3) + 1% noise, NOA 1e-3
  smooth2d     2D float32 512^2 Gaussian bumps, NOA 1e-3
  fronts2d     2D float32 1800 x 3600 periodic fronts, NOA 1e-3
  batch        256 uneven float32 fields (2D side 64..1024, 3D side 32..192,
               NOA bounds 1e-4..1e-2): one batch compress + one batch
               decompress per step
  serve        Poisson request streams (compress or decompress, 1 MiB to
               512 MiB, float32/float64, 2D/3D) at 0.25 .. 1.1 times the
               single-slot service rate, served on 4 slots under a 64 GiB
               HBM budget: p50 / p99 latency and GB/s per rate
  copy         device-to-device copy of 256 MiB (the achievable HBM rate)
  repair-study the single-field repair schedulers side by side on the fields
               above and on long falling chains (repair time, sweeps, tile runs)

Prints one JSON line per run.  Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lognormal3d]
                  [--eb 1e-3] [--no-cpu-baseline] [--no-parity] [--eb-sweep]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, public spec


def _log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)
# the headline metric; value = uncompressed bytes / median round-trip time
METRIC = "compress/decompress GB/s per MI355X at fixed eb (bit-exact), %HBM peak; p99 latency"

SINGLE = {
    # name: (generator, shape, description)
    "turb3d": ("turbulence_field", (256, 256, 256),
               "3D float32 256^3 GRF P(k)~k^-3 + 1% noise, [0,1]"),
    "smooth2d": ("smooth_field", (512, 512), "2D float32 512^2 32 Gaussian bumps + N(0,1e-3)"),
    "fronts2d": ("fronts_field", (1800, 3600), "2D float32 1800x3600 periodic sinusoids + fronts"),
    "lognormal3d": ("lognormal_field", (512, 512, 512),
                    "3D float64 512^3 exp(2g), g GRF P(k)~k^-2.5, floored at 10th pct"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal3d",
                    choices=list(SINGLE) + ["batch", "serve", "copy", "repair-study"])
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the whole-field oracle run (parity) of a large field")
    ap.add_argument("--oracle-job", help=argparse.SUPPRESS)
    ap.add_argument("--oracle-out", help=argparse.SUPPRESS)
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests per rate")
    ap.add_argument("--sweep-whole", action="store_true",
                    help="eb sweep of a field above 16M points: oracle parity on the whole "
                         "field at every bound (one oracle process per bound, beside the GPU)")
    ap.add_argument("--eb-sweep", action="store_true",
                    help="single-field workloads: also run NOA bounds 1e0 .. 1e-6 (CR, "
                         "throughput, sweeps, bins/subbins byte split)")
    return ap.parse_args()


# ------------------------------------------------------------------ single field
def _pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def measured_traffic(workload, phase):
    """HBM bytes per launch of the kernels of `phase` ("quant", "encode" or
    "decode") on `workload`, from the committed counter summary
    profiles/<workload>_traffic.md (FETCH_SIZE + WRITE_SIZE scaled by a copy
    kernel), or None if there is none or it was taken on other kernel
    sources than the current ones."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("lopc_codec.hip", "lopc_kernels.hip", "lopc_device.h", "lopc_internal.h",
              "lopc_numeric.h"):
        h.update(open(os.path.join(ROOT, "paper_2603_26968_amd", "csrc", f), "rb").read())
    src = h.hexdigest()[:16]
    for line in open(path):
        if line.startswith("traffic ") and f" {phase} " in line and f"sources={src}" in line:
            fields = dict(kv.split("=") for kv in line.split() if "=" in kv)
            return int(fields["fetch_bytes"]) + int(fields["write_bytes"])
    return None


# the error-bound sweep: NOA bounds 10^-e
SWEEP_EXPONENTS = range(0, 7)


def oracle_job(path, eb, out):
    """The CPU baseline leg, run as a child process: the oracle compresses and
    decompresses the field stored at `path` (single thread) and writes the
    times and the SHA-256 of its stream and reconstruction to `out`."""
    import hashlib
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liblopc_ref.so")):
        oracle.build()
    x = np.load(path, allow_pickle=False)
    t0 = time.perf_counter()
    s = oracle.compress(x, eb, oracle.NOA)
    t1 = time.perf_counter()
    _log(f"oracle: compressed {x.nbytes / 1e6:.0f} MB in {t1 - t0:.1f} s")
    y = oracle.decompress(s)
    t2 = time.perf_counter()
    _log(f"oracle: decompressed in {t2 - t1:.1f} s")
    res = {"bytes": int(x.nbytes), "shape": list(x.shape), "compress_s": t1 - t0,
           "decompress_s": t2 - t1, "stream_bytes": len(s),
           "stream_sha256": hashlib.sha256(s).hexdigest(),
           "recon_sha256": hashlib.sha256(y.view(np.uint8).tobytes()).hexdigest()}
    with open(out, "w") as f:
        json.dump(res, f)


def _start_oracle(xh, eb, tmp, tag, path=None):
    """Start one oracle job on `xh` at bound `eb` (a child process); `path`:
    the field already saved there."""
    import subprocess
    if path is None:
        path = os.path.join(tmp, f"{tag}.npy")
        np.save(path, xh, allow_pickle=False)
    out = os.path.join(tmp, f"{tag}.json")
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-job", path, "--eb", repr(eb),
           "--oracle-out", out]
    return subprocess.Popen(cmd), out


def _finish_oracle(job):
    proc, out = job
    rc = proc.wait()
    if rc != 0:
        raise RuntimeError(f"oracle job failed with status {rc}")
    with open(out) as f:
        return json.load(f)


def run_steps(P, lopc, ctx, x, eb, steps, bufs, timing):
    """`steps` round trips, each compress and decompress timed on the host
    clock around the synchronous calls; `timing`: the phases the library
    times from its own dispatches (True: all).  Returns (per-step compress
    and decompress seconds, mean ms per timed phase, stats of the last
    compress, its stream)."""
    import torch
    stream_buf, ws_c, ws_d, y = bufs
    lopc.lopc_ctx_set_timing(ctx, timing)
    phase = {k: 0.0 for k in lopc.PHASES}
    tc, td = [], []
    s = stats = None
    torch.cuda.synchronize()
    for i in range(steps):
        # the statistics (sweeps, stream part sizes: one more small kernel)
        # are taken from the last step only
        last = i == steps - 1
        t0 = time.perf_counter()
        r = P.compress(x, eb, "noa", stats=last, header=True, out=stream_buf, workspace=ws_c)
        if last:
            s, stats, hdr = r
        else:
            s, hdr = r
        t1 = time.perf_counter()
        if timing:
            ph = lopc.lopc_ctx_last_timings(ctx)
        P.decompress(s, out=y, workspace=ws_d, header=hdr)
        t2 = time.perf_counter()
        tc.append(t1 - t0)
        td.append(t2 - t1)
        if timing:
            ph2 = lopc.lopc_ctx_last_timings(ctx)
            for k in ("range", "quant", "repair", "encode"):
                phase[k] += ph[k]
            for k in ("offsets", "decode"):
                phase[k] += ph2[k]
    torch.cuda.synchronize()
    lopc.lopc_ctx_set_timing(ctx, False)
    return tc, td, {k: v / max(steps, 1) for k, v in phase.items()}, stats, s


def _sweep_parity(P, xh, eb, gpu_stream):
    """Stream identity with the oracle at one bound of the error-bound sweep:
    the whole field when it is at most 16M points (gpu_stream: its stream),
    else the leading slab of about 16M points, compressed by both."""
    import oracle
    import torch
    if not os.path.exists(os.path.join(ROOT, "oracle", "liblopc_ref.so")):
        oracle.build()
    if gpu_stream is not None:
        sl, got = xh, gpu_stream.cpu().numpy().tobytes()
    else:
        rows = max(1, (1 << 24) // (xh.size // xh.shape[0]))
        sl = np.ascontiguousarray(xh[:rows])
        got = P.compress(torch.from_numpy(sl).cuda(), eb, "noa").cpu().numpy().tobytes()
    try:
        want = oracle.compress(sl, eb, oracle.NOA)
    except oracle.OracleError as e:
        return {"scope": "whole field" if sl is xh else f"leading slab {list(sl.shape)}",
                "oracle_error": e.code}
    return {"scope": "whole field" if sl is xh else f"leading slab {list(sl.shape)}",
            "stream_identical": got == want}


def bench_single(args, name):
    import hashlib
    import tempfile
    gen, shape, desc = SINGLE[name]
    _log("generating", name)
    from paper_2603_26968_amd import synth
    xh = getattr(synth, gen)(shape, seed=args.seed)
    _log("generated")
    n, k = xh.size, xh.itemsize

    # the CPU baseline leg, started before the GPU is touched and run beside
    # it: the oracle on a bounded sample (the whole field up to 16M points,
    # else its leading slab of about 16M points), and on the whole field for
    # the parity check when the sample is smaller
    tmp = tempfile.mkdtemp(prefix="lopc_bench_")
    jobs = {}
    sample = xh
    if not args.no_cpu_baseline:
        if xh.size > (1 << 24):
            rows = max(1, (1 << 24) // (xh.size // xh.shape[0]))
            sample = np.ascontiguousarray(xh[:rows])
        jobs["sample"] = _start_oracle(sample, args.eb, tmp, "sample")
        if sample is not xh and not args.no_parity:
            jobs["full"] = _start_oracle(xh, args.eb, tmp, "full")
        if args.eb_sweep and args.sweep_whole and sample is not xh:
            # whole-field parity at every bound of the sweep: one oracle
            # process per bound, all beside the GPU run
            fpath = os.path.join(tmp, "field.npy")
            np.save(fpath, xh, allow_pickle=False)
            for e in SWEEP_EXPONENTS:
                jobs[f"sweep{e}"] = _start_oracle(xh, 10.0 ** (-e), tmp, f"sweep{e}", fpath)

    import torch

    import paper_2603_26968_amd as P
    from paper_2603_26968_amd import lopc
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xh).to(dev)
    ctx = lopc.context(0)
    cap = lopc.lopc_compress_bound(x.shape, x.dtype)
    bufs = (torch.empty(cap, dtype=torch.uint8, device=dev),
            torch.empty(lopc.lopc_workspace_size(ctx, x.shape, x.dtype, 0), dtype=torch.uint8,
                        device=dev),
            torch.empty(lopc.lopc_workspace_size(ctx, x.shape, x.dtype, 1), dtype=torch.uint8,
                        device=dev),
            torch.empty_like(x))

    run_steps(P, lopc, ctx, x, args.eb, args.warmup, bufs, False)
    # phase breakdown and statistics: a few steps before the timed region,
    # every phase timed (a timed dispatch delays the next launch a little)
    _, _, phase, stats, _ = run_steps(P, lopc, ctx, x, args.eb, 5, bufs, True)
    # the dominant kernel: the longest single launch among the first tile
    # pass (k_tile0, phase "quant"), the decoder and the encode phase
    dom = max(("quant", "encode", "decode"), key=lambda q: phase[q])
    _log("breakdown", {q: round(v, 3) for q, v in phase.items()}, "dominant", dom)
    # timed region: K steps; the dominant kernel is timed by HIP events the
    # library takes from its own dispatches on their stream
    tc, td, phase_k, _, s = run_steps(P, lopc, ctx, x, args.eb, args.steps, bufs, (dom,))
    _log("timed", args.steps, "steps")
    S = int(s.numel())
    trip = [a + b for a, b in zip(tc, td)]
    med_c, med_d, med_t = _pct(tc, 50), _pct(td, 50), _pct(trip, 50)
    value = n * k / med_t / 1e9

    # algorithmic bytes (what the method itself moves, not intermediate
    # arrays): compress reads the field and writes the stream, decompress
    # reads the stream and writes the field.  Per kernel: the first tile
    # pass reads the field (its outputs are intermediates), the encode phase
    # writes the stream (it reads intermediates), the decoder reads the
    # stream and writes the field.
    alg = {"quant": n * k, "encode": S, "decode": S + n * k}
    kname = {"quant": "k_tile0", "decode": "k_decode",
             "encode": "k_encode+k_record_offsets+k_place"}[dom]
    # the first pass of a field of at least 32768 repair tiles (default 3D
    # tile 4 x 8 x 32) runs as two launches, one per checkerboard colour of
    # tiles, each over half the field
    ntiles = -(-xh.shape[0] // 4) * -(-xh.shape[1] // 8) * -(-xh.shape[2] // 32) \
        if xh.ndim == 3 and xh.shape[0] > 1 else 0
    nl = 2 if dom == "quant" and ntiles >= 32768 else 1
    t_dom = phase_k[dom] / nl
    achieved = alg[dom] / nl / (t_dom * 1e-3) / 1e9
    wl = {"turb3d": "turb3d_256_f32", "lognormal3d": "lognormal3d_512_f64",
          "fronts2d": "fronts2d_1800x3600_f32"}.get(name)
    traffic = measured_traffic(f"{wl}_eb{args.eb:.0e}".replace("e-0", "e-"), dom) if wl else None
    if traffic:
        traffic //= nl
    roof = {"bound": "hbm", "kernel": kname, "launches_per_step": nl,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic, "algorithmic_bytes_per_launch": alg[dom] // nl,
            "launch_ms": round(t_dom, 4),
            "traffic_over_algorithmic": round(traffic / (alg[dom] // nl), 3) if traffic else None}
    path_roof = {}
    for what, nbytes, t in (("compress", n * k + S, med_c), ("decompress", S + n * k, med_d),
                            ("round_trip", 2 * (n * k + S), med_t)):
        path_roof[what] = {"algorithmic_bytes": nbytes, "median_ms": round(t * 1e3, 4),
                           "GBps": round(nbytes / t / 1e9, 1),
                           "frac": round(nbytes / t / 1e9 / HBM_PEAK_GBPS, 4)}

    # the reconstruction's invariants, checked on the device (error bound,
    # order of every edge, critical types)
    torch.cuda.synchronize()
    tv = time.perf_counter()
    rep = P.verify(x, bufs[3], stats["eps"])
    tv = time.perf_counter() - tv
    check = {q: rep[q] for q in ("bound_violations", "order_violations", "type_mismatches",
                                 "max_abs_error", "edges")}
    check["critical_points"] = dict(zip(("regular", "minima", "maxima", "saddles"),
                                         rep["types_orig"]))
    check["ms"] = round(tv * 1e3, 3)
    gpu_stream_sha = hashlib.sha256(s.cpu().numpy().tobytes()).hexdigest()
    gpu_recon_sha = hashlib.sha256(bufs[3].cpu().numpy().view(np.uint8).tobytes()).hexdigest()

    extra_sweep = None
    sweep_sha = {}
    if args.eb_sweep:
        extra_sweep = {}
        for e in SWEEP_EXPONENTS:
            eb = 10.0 ** (-e)
            _log("eb sweep", eb)
            try:
                tce, tde, ph, st, se = run_steps(P, lopc, ctx, x, eb, 3, bufs, True)
            except lopc.LopcError as err:  # e.g. a bin range beyond the integer type
                extra_sweep[f"1e-{e}"] = {"error": str(err)}
                continue
            Se = int(se.numel())
            par = None
            if f"sweep{e}" in jobs:
                # compared with the whole-field oracle job when it ends
                ye = P.decompress(se)
                sweep_sha[e] = (hashlib.sha256(se.cpu().numpy().tobytes()).hexdigest(), Se,
                                hashlib.sha256(ye.cpu().numpy().view(np.uint8).tobytes())
                                .hexdigest())
                del ye
            elif not args.no_cpu_baseline:
                par = _sweep_parity(P, xh, eb, se if sample is xh else None)
            extra_sweep[f"1e-{e}"] = {
                "CR": round(n * k / Se, 3),
                "GBps_roundtrip": round(n * k / _pct([a + b for a, b in zip(tce, tde)], 50) / 1e9, 2),
                "compress_GBps": round(n * k / _pct(tce, 50) / 1e9, 2),
                "decompress_GBps": round(n * k / _pct(tde, 50) / 1e9, 2),
                "repair_ms": round(ph["repair"], 4), "repair_sweeps": int(st["repair_sweeps"]),
                "active_tiles_total": int(st["active_tiles_total"]),
                "relax_iterations": int(st["relax_iterations"]),
                "bins_share": round(st["bins_bytes"] / Se, 4),
                "subbins_share": round(st["subbins_bytes"] / Se, 4),
                "parity": par}

    dtname = "f32" if k == 4 else "f64"
    out = {
        "metric": METRIC,
        "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(med_t * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtname, "data": "synthetic",
        "config": {"workload": f"{name}: {desc}; NOA eb {args.eb:g}; compress + decompress",
                   "shape": list(xh.shape), "field_dtype": dtname, "eb": args.eb, "mode": "NOA",
                   "arithmetic": "binary64 quantizer/decoder, 32-bit integer repair and codecs"},
        "timing": {"statistic": "median of the timed steps (host clock around each "
                                "synchronous call; field resident in HBM)",
                   "round_trip_ms": {"median": round(med_t * 1e3, 4),
                                     "min": round(min(trip) * 1e3, 4),
                                     "p90": round(_pct(trip, 90) * 1e3, 4)},
                   "compress_ms": {"median": round(med_c * 1e3, 4), "min": round(min(tc) * 1e3, 4),
                                   "p90": round(_pct(tc, 90) * 1e3, 4)},
                   "decompress_ms": {"median": round(med_d * 1e3, 4),
                                     "min": round(min(td) * 1e3, 4),
                                     "p90": round(_pct(td, 90) * 1e3, 4)}},
        "compress_GBps": round(n * k / med_c / 1e9, 2),
        "decompress_GBps": round(n * k / med_d / 1e9, 2),
        "phase_ms": {q: round(v, 4) for q, v in phase.items()},
        "CR": round(n * k / S, 3), "stream_bytes": S,
        "repair_sweeps": int(stats["repair_sweeps"]),
        "active_tiles_total": int(stats["active_tiles_total"]),
        "relax_iterations": int(stats["relax_iterations"]),
        "bins_bytes": int(stats["bins_bytes"]), "subbins_bytes": int(stats["subbins_bytes"]),
        "roofline": roof,
        "roofline_path": path_roof,
        "invariants": check,
    }
    if extra_sweep:
        out["eb_sweep"] = extra_sweep

    if jobs:
        _log("waiting for the oracle")
        smp = _finish_oracle(jobs["sample"])
        t_cpu = smp["compress_s"] + smp["decompress_s"]
        what = "the whole field" if sample is xh else f"its leading slab {smp['shape']}"
        out["cpu_baseline"] = {"value": round(smp["bytes"] / t_cpu / 1e9, 5), "unit": "GB/s",
                               "cores": 1, "host_cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"one compress + decompress of {what} "
                                         f"({smp['bytes'] / 1e6:.0f} MB), single-threaded C "
                                         f"oracle, {t_cpu:.1f} s"}
        full = _finish_oracle(jobs["full"]) if "full" in jobs else (smp if sample is xh else None)
        if full is not None:
            out["parity"] = {"scope": "whole field",
                             "stream_identical": full["stream_sha256"] == gpu_stream_sha
                             and full["stream_bytes"] == S,
                             "reconstruction_identical": full["recon_sha256"] == gpu_recon_sha}
            if "full" in jobs:
                out["cpu_baseline"]["whole_field_s"] = round(full["compress_s"] +
                                                             full["decompress_s"], 1)
        for e in SWEEP_EXPONENTS:
            if f"sweep{e}" not in jobs:
                continue
            res = _finish_oracle(jobs[f"sweep{e}"])
            if e not in sweep_sha:  # the GPU refused this bound
                continue
            sha, Se, rsha = sweep_sha[e]
            out["eb_sweep"][f"1e-{e}"]["parity"] = {
                "scope": "whole field",
                "stream_identical": res["stream_sha256"] == sha and res["stream_bytes"] == Se,
                "reconstruction_identical": res["recon_sha256"] == rsha}
    import shutil
    shutil.rmtree(tmp, ignore_errors=True)
    return out


# ------------------------------------------------------------------ repair study
def bench_repair_study(args):
    """The single-field repair schedulers side by side (LOPC_OPT_REPAIR):
    for each field and scheduler, the median repair-phase time (library
    dispatch events), the compress time, sweeps, tile runs, queue runs and
    parks (for the point worklists: iterations and listed points); the
    streams of all schedulers of a field must be identical."""
    import torch

    import paper_2603_26968_amd as P
    from paper_2603_26968_amd import lopc, synth
    modes = {"sweeps": lopc.LOPC_REPAIR_SWEEPS, "hybrid": lopc.LOPC_REPAIR_HYBRID,
             "queue": lopc.LOPC_REPAIR_QUEUE, "auto": lopc.LOPC_REPAIR_AUTO,
             "points": lopc.LOPC_REPAIR_POINTS}

    def chain(n):
        return (np.arange(n, 0, -1, dtype=np.float64) / n).astype(np.float32).reshape(1, n)

    cases = [
        ("turb3d 256^3 f32 NOA 1e-3", lambda: synth.turbulence_field(), 1e-3, "noa", 5,
         ("sweeps", "hybrid", "queue", "points", "auto")),
        ("turb3d 256^3 f32 NOA 1e-2", lambda: synth.turbulence_field(), 1e-2, "noa", 5,
         ("sweeps", "hybrid", "queue", "points", "auto")),
        ("turb3d 256^3 f32 NOA 1e0", lambda: synth.turbulence_field(), 1.0, "noa", 3,
         ("sweeps", "hybrid", "queue", "points", "auto")),
        ("fronts2d 1800x3600 f32 NOA 1e-3", lambda: synth.fronts_field(), 1e-3, "noa", 5,
         ("sweeps", "hybrid", "queue", "points", "auto")),
        ("smooth2d 512^2 f32 NOA 1e-3", lambda: synth.smooth_field(), 1e-3, "noa", 5,
         ("sweeps", "hybrid", "queue", "points", "auto")),
        ("lognormal3d 512^3 f64 NOA 1e-3", lambda: synth.lognormal_field(), 1e-3, "noa", 3,
         ("sweeps", "hybrid", "queue", "points", "auto")),
        ("falling chain (1, 2^16) f32 ABS 10", lambda: chain(1 << 16), 10.0, "abs", 2,
         ("sweeps", "queue", "points", "auto")),
        ("falling chain (1, 2^20) f32 ABS 10", lambda: chain(1 << 20), 10.0, "abs", 1,
         ("queue", "auto")),
    ]
    rows = []
    for name, gen, eb, mode, reps, which in cases:
        _log("repair study:", name)
        t = torch.from_numpy(gen()).cuda()
        streams = {}
        for mn in which:
            ctx = lopc.lopc_ctx_create(0)
            try:
                lopc.lopc_ctx_set_option(ctx, lopc.LOPC_OPT_REPAIR, modes[mn])
                lopc.lopc_ctx_set_timing(ctx, ("repair",))
                P.compress(t, eb, mode, ctx=ctx)  # learns its sweep count
                rep_ms, tot_ms = [], []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s, st = P.compress(t, eb, mode, stats=True, ctx=ctx)
                    tot_ms.append((time.perf_counter() - t0) * 1e3)
                    rep_ms.append(lopc.lopc_ctx_last_timings(ctx)["repair"])
                streams[mn] = s.cpu().numpy().tobytes()
                rows.append({"field": name, "scheduler": mn,
                             "repair_ms": round(_pct(rep_ms, 50), 4),
                             "compress_ms": round(_pct(tot_ms, 50), 4),
                             "sweeps": int(st["repair_sweeps"]),
                             "tile_runs": int(st["active_tiles_total"]),
                             "queue_runs": int(st["queue_runs"]),
                             "queue_parks": int(st["queue_parks"])})
                _log(json.dumps(rows[-1]))
            finally:
                lopc.lopc_ctx_destroy(ctx)
        same = len(set(streams.values())) == 1
        for r in rows:
            if r["field"] == name:
                r["streams_identical_across_schedulers"] = same
        del t
    return {"metric": "repair-phase time of each scheduler (ms, lower is better)",
            "value": None, "unit": "ms", "n_gpus": 1, "steps": None, "warmup": 1,
            "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "repair-study: schedulers x fields"}, "rows": rows}


# ------------------------------------------------------------------ batch
def _oracle_field(args_tuple):
    x, eb = args_tuple
    import oracle
    t0 = time.perf_counter()
    s = oracle.compress(x, eb, oracle.NOA)
    oracle.decompress(s)
    return time.perf_counter() - t0, len(s)


def bench_batch(args):
    import torch

    import paper_2603_26968_amd as P
    from paper_2603_26968_amd import lopc, synth

    _log("generating 256 fields")
    fields = synth.batch_fields(256, seed=args.seed)
    _log("generated", sum(x.nbytes for x, _ in fields) / 1e6, "MB")
    xs = [torch.from_numpy(x).cuda() for x, _ in fields]
    ebs = [eb for _, eb in fields]
    nbytes = sum(x.nbytes for x, _ in fields)
    ctx = lopc.context(0)
    caps = [lopc.lopc_compress_bound(x.shape, x.dtype) for x in xs]
    out = torch.empty(sum((c + 255) // 256 * 256 for c in caps), dtype=torch.uint8, device="cuda")
    ys = [torch.empty_like(x) for x in xs]

    def step():
        streams, st, hdrs = P.compress_batch(xs, ebs, "noa", out=out, stats=True, headers=True)
        P.decompress_batch(streams, outs=ys, headers=hdrs)
        return streams, st

    # the autotuner picks the grid mode and the repair tile shapes of this
    # batch (kept in the context for the timed steps)
    t0 = time.perf_counter()
    pct = P.autotune_compress_batch(xs, ebs, "noa", out=out, ctx=ctx, reps=1)
    tuned = {"persist_pct": pct,
             "tile_2d": lopc.kTile2Names[lopc.lopc_ctx_get_option(ctx, lopc.LOPC_OPT_TILE_2D)],
             "tile_3d": lopc.kTile3Names[lopc.lopc_ctx_get_option(ctx, lopc.LOPC_OPT_TILE_3D)],
             "tuning_s": round(time.perf_counter() - t0, 2)}
    _log("autotuned", tuned)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tc = td = 0.0
    for _ in range(args.steps):
        t0 = time.perf_counter()
        streams, st, hdrs = P.compress_batch(xs, ebs, "noa", out=out, stats=True, headers=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.decompress_batch(streams, outs=ys, headers=hdrs)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tc += t1 - t0
        td += t2 - t1
    tc /= args.steps
    td /= args.steps
    _log("timed", tc, td)
    S = sum(int(s.numel()) for s in streams)
    # identity: every batch stream equals its single-field stream, every
    # decoded field the single-field decode; the same loop times one call
    # per field for comparison
    ident = True
    t_single = 0.0
    for x, eb, s, y in zip(xs, ebs, streams, ys):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s1, h1 = P.compress(x, eb, "noa", header=True)
        y1 = P.decompress(s1, header=h1)
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t0
        if not torch.equal(s1, s) or not torch.equal(y1.view(torch.uint8), y.view(torch.uint8)):
            ident = False
    res = {
        "metric": METRIC, "value": round(nbytes / (tc + td) / 1e9, 3), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round((tc + td) * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch: 256 float32 fields, 2D side log-U[64,1024] or 3D side "
                               "log-U[32,192], NOA eb log-U[1e-4,1e-2]; one batch compress + "
                               "one batch decompress",
                   "fields": len(xs), "total_bytes": nbytes},
        "compress_GBps": round(nbytes / tc / 1e9, 2), "decompress_GBps": round(nbytes / td / 1e9, 2),
        "CR": round(nbytes / S, 3), "repair_sweeps": int(st["repair_sweeps"]),
        "graph": int(st["graph"]), "sweeps_continued": int(st["continued"]),
        "relax_iterations": int(st["relax_iterations"]),
        "one_call_per_field_GBps": round(nbytes / t_single / 1e9, 2),
        "hbm_frac_algorithmic": round(2 * (nbytes + S) / (tc + td) / 1e9 / HBM_PEAK_GBPS, 4),
        "identity_batch_vs_single": ident,
        "autotuned": tuned,
    }
    if not args.no_cpu_baseline:
        from concurrent.futures import ProcessPoolExecutor
        import oracle
        if not os.path.exists(os.path.join(ROOT, "oracle", "liblopc_ref.so")):
            oracle.build()
        sample = fields[::16]
        sb = sum(x.nbytes for x, _ in sample)
        workers = min(16, os.cpu_count() or 1, len(sample))
        t0 = time.perf_counter()
        with ProcessPoolExecutor(workers) as ex:
            list(ex.map(_oracle_field, sample))
        tw = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(sb / tw / 1e9, 5), "unit": "GB/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"every 16th field ({len(sample)} fields, {sb / 1e6:.0f} MB), "
                                         f"one process per field, {tw:.1f} s"}
    return res


# ------------------------------------------------------------------ serving
def bench_serve(args):
    import torch

    import paper_2603_26968_amd as P
    from paper_2603_26968_amd import serve, synth

    n_templates = 64
    _log("building serving templates")
    base2 = torch.from_numpy(synth.smooth_field()).cuda()
    base3 = torch.from_numpy(synth.turbulence_field((256, 256, 256))).cuda()
    T = []
    for spec in synth.serving_requests(n_templates, seed=7):
        base = base2 if len(spec["shape"]) == 2 else base3
        x = synth.reflect_tile(base, spec["shape"])
        x = x.to(torch.float32 if spec["dtype"] == np.float32 else torch.float64).contiguous()
        s, hdr = P.compress(x, spec["eb"], "noa", header=True)
        s = s.clone()
        if spec["op"] == "compress":
            T.append(dict(op="compress", data=x, eb=spec["eb"], want=s, bytes=x.nbytes))
        else:
            y = P.decompress(s, header=hdr)
            T.append(dict(op="decompress", data=s, header=hdr, want=y, bytes=y.nbytes))
            del x
    torch.cuda.synchronize()
    budget = 64 << 30
    slots = 4

    def make(i, keep):
        t = T[i % n_templates]
        return serve.Request(t["op"], t["data"], eb=t.get("eb", 0.0), header=t.get("header"),
                             tag=i % n_templates, keep=keep)

    def same(r):
        got, want = r.result, T[r.tag]["want"]
        return got.shape == want.shape and torch.equal(
            got.view(torch.uint8) if got.dtype != torch.uint8 else got,
            want.view(torch.uint8) if want.dtype != torch.uint8 else want)

    # service rate of one slot, requests back to back
    with serve.Server(budget, slots=1) as one:
        reqs = [one.submit(make(i, False)) for i in range(n_templates)]
        for r in reqs:
            r.done.wait()
        t0 = time.perf_counter()
        reqs = [one.submit(make(i, False)) for i in range(n_templates)]
        for r in reqs:
            r.done.wait()
        mu = n_templates / (time.perf_counter() - t0)
    rates = {}
    ident = True
    with serve.Server(budget, slots=slots) as srv:
        for f in (0.25, 0.5, 0.75, 0.9, 1.1):
            offs = serve.poisson_arrivals(args.requests, rate=f * mu, seed=7)
            reqs = serve.run_arrivals(srv, lambda i: make(i, i % 50 == 0), offs)
            st = serve.latency_stats(reqs, lambda r: T[r.tag]["bytes"])
            kept = [r for r in reqs if r.keep and r.error is None]
            st["identity_checked"] = len(kept)
            st["identity_alone_vs_mix"] = all(same(r) for r in kept)
            ident = ident and st["identity_alone_vs_mix"] and st["failed"] == 0
            st["rate_per_s"] = round(f * mu, 2)
            rates[str(f)] = {q: (round(v, 3) if isinstance(v, float) else v) for q, v in st.items()}
            del reqs, kept
            print(json.dumps({"serve_rate_done": f, **rates[str(f)]}), file=sys.stderr, flush=True)
        peak = srv.admission.peak
    top = rates["0.9"]
    return {
        "metric": METRIC, "value": top["GBps"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.requests, "warmup": n_templates, "ms_per_step": top["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "serve: Poisson requests (compress or decompress, 1-512 MiB, "
                               "f32/f64, 2D/3D, NOA eb log-U[1e-4,1e-2]) on 4 slots, 64 GiB budget; "
                               "value = GB/s served at 0.9 x the single-slot service rate",
                   "templates": n_templates, "requests_per_rate": args.requests, "slots": slots},
        "service_rate_one_slot_per_s": round(mu, 2),
        "rates": rates, "identity_alone_vs_mix": ident, "admission_peak_bytes": peak,
    }


# ------------------------------------------------------------------ copy roof
def bench_copy(args):
    """A plain device-to-device copy of 256 MiB, as a DMA-engine blit and as
    an element-wise kernel (torch.neg on float32): the achievable HBM rate,
    and the kernel whose counters calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    nb = 256 << 20
    a = torch.empty(nb // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    res = {}
    for name, f in (("blit", lambda: b.copy_(a)), ("elementwise", lambda: torch.neg(a, out=b))):
        for _ in range(args.warmup):
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            f()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = {"GBps": round(2 * nb / dt / 1e9, 1), "ms": round(dt * 1e3, 4)}
    best = max(v["GBps"] for v in res.values())
    return {"metric": "device-to-device copy GB/s (bytes read + written / time)",
            "value": best, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": min(v["ms"] for v in res.values()),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": {"workload": "copy: 256 MiB device to device",
                                            "bytes_each_way": nb},
            "variants": res, "frac_of_peak": round(best / HBM_PEAK_GBPS, 4)}


def main():
    args = parse()
    if args.oracle_job:
        oracle_job(args.oracle_job, args.eb, args.oracle_out)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is "
                          "described in DESIGN.md and not built", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "batch":
        out = bench_batch(args)
    elif args.workload == "serve":
        out = bench_serve(args)
    elif args.workload == "copy":
        out = bench_copy(args)
    elif args.workload == "repair-study":
        out = bench_repair_study(args)
    else:
        out = bench_single(args, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
