// lopc_api.cpp -- host runtime of liblopc.so: argument validation, workspace
// layout, launch sequence, status reporting.  The public contract is in
// include/lopc.h.
#include <new>

#include "lopc_host.h"

using namespace lopc;

using namespace lopc_host;

extern "C" {

const char* lopc_strerror(int status) {
  switch (status) {
    case LOPC_OK: return "ok";
    case LOPC_E_ARG: return "invalid argument";
    case LOPC_E_NONFINITE: return "field holds NaN or Inf";
    case LOPC_E_BOUND: return "error bound must be finite and > 0 (NOA: field range > 0)";
    case LOPC_E_RANGE: return "a bin number does not fit its integer type";
    case LOPC_E_CAPACITY: return "output buffer too small";
    case LOPC_E_FORMAT: return "malformed or corrupt stream";
    case LOPC_E_HIP: return "HIP runtime error";
    case LOPC_E_NOMEM: return "out of host memory";
    case LOPC_E_INTERNAL: return "internal limit exceeded";
    default: return "unknown status";
  }
}

int lopc_ctx_create(int hip_device, lopc_ctx** out) {
  if (!out) return LOPC_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 ||
      hip_device >= count)
    return LOPC_E_HIP;
  HIP_TRY(hipSetDevice(hip_device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
  lopc_ctx* c = new (std::nothrow) lopc_ctx();
  if (!c) return LOPC_E_NOMEM;
  c->device = hip_device;
  c->num_cu = prop.multiProcessorCount;
  void* p = nullptr;
  // pinned host slots: the compress report (Params, counters, queue: under
  // 4 KiB) and, from 4 KiB on, the verify report
  if (hipHostMalloc(&p, 8192, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return LOPC_E_HIP;
  }
  c->h_prm = (Params*)p;
  c->h_cnt = (uint32_t*)((uint8_t*)p + 4096);
  // the device address of this device's copy of the library-held scratch
  // (lopc_decompress_static), looked up with the device current
  if (static_scratch_address(&c->scratch) != hipSuccess || !c->scratch) {
    (void)hipHostFree(p);
    delete c;
    return LOPC_E_HIP;
  }
  c->timing = 0;
  c->have_header = 0;
  c->hip_error = 0;
  c->hip_where[0] = 0;
  {
    const char* v = std::getenv("LOPC_SYNC_CHECK");
    c->sync_check = v && v[0] == '1';
  }
  for (hipEvent_t& e : c->ev) e = nullptr;
  for (int i = 0; i < LOPC_PHASES; ++i) c->ms[i] = 0.0;
  c->use_graph = 1;
  c->graph_sweeps = 0;
  c->sweeps_hint = 16;
  c->persist_pct = 0;
  c->sweep_hint = 4;
  c->repair_mode = LOPC_REPAIR_AUTO;
  c->sweep_order = 0;
  for (int i = 0; i < kTileShapes; ++i) c->rq_per_cu[i] = c->sl_per_cu[i] = 0;
  c->tile2 = 0;
  c->tile3 = 0;
  *out = c;
  return LOPC_OK;
}

void lopc_ctx_destroy(lopc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (BatchGraph& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->h_plan) (void)hipHostFree(ctx->h_plan);
  if (ctx->h_back) (void)hipHostFree(ctx->h_back);
  if (ctx->h_prm) (void)hipHostFree(ctx->h_prm);
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

int lopc_ctx_set_timing(lopc_ctx* ctx, int phases) {
  if (!ctx || (phases & ~LOPC_TIMING_ALL)) return LOPC_E_ARG;
  if (phases && !ctx->ev[0]) {
    HIP_TRY(hipSetDevice(ctx->device));
    for (hipEvent_t& e : ctx->ev) HIP_TRY(hipEventCreate(&e));
  }
  ctx->timing = phases;
  return LOPC_OK;
}

const char* lopc_ctx_last_hip_error(lopc_ctx* ctx, int* code) {
  if (!ctx) return "";
  if (code) *code = ctx->hip_error;
  static thread_local char buf[160];
  std::snprintf(buf, sizeof(buf), "%s (%s)",
                ctx->hip_error ? hipGetErrorString((hipError_t)ctx->hip_error) : "no error",
                ctx->hip_where);
  return buf;
}

int lopc_ctx_last_timings(lopc_ctx* ctx, double* h_ms, int n) {
  if (!ctx || !h_ms || n < 0) return LOPC_E_ARG;
  for (int i = 0; i < n && i < LOPC_PHASES; ++i) h_ms[i] = ctx->ms[i];
  return LOPC_OK;
}

int lopc_compress_bound(int dtype, int ndim, const int64_t* dims,
                        size_t* bytes) {
  if ((dtype != 0 && dtype != 1) || !bytes) return LOPC_E_ARG;
  Shape s;
  int st = make_shape(ndim, dims, &s);
  if (st) return st;
  const uint64_t k = dtype == 0 ? 4 : 8, W = kChunkBytes / k;
  const uint64_t nch = (s.n + W - 1) / W;
  const uint64_t full = s.n / W, last = s.n - full * W;
  uint64_t total = kHeaderBytes + 4 * nch +
                   full * (kRecordHeaderBytes + 2 * W * k);
  if (last) total += kRecordHeaderBytes + 2 * ((last + 63) / 64 * 64) * k;
  *bytes = (size_t)total;
  return LOPC_OK;
}

int lopc_workspace_size(lopc_ctx* ctx, int dtype, int ndim,
                        const int64_t* dims, int op, size_t* bytes) {
  if ((dtype != 0 && dtype != 1) || !bytes || (op != 0 && op != 1))
    return LOPC_E_ARG;
  Shape s;
  int st = make_shape(ndim, dims, &s);
  if (st) return st;
  // the largest over every tile shape, so that a workspace stays valid when
  // the context's tile options change; the point worklists when selected
  const bool points = ctx && ctx->repair_mode == LOPC_REPAIR_POINTS;
  size_t b = 0;
  if (op == 0)
    for (int t2 = 0; t2 < kTiles2; ++t2)
      for (int t3 = 0; t3 < kTiles3; ++t3)
        b = std::max(b, compress_layout(s, dtype, t2, t3, points).total);
  else
    b = decompress_ws(s, dtype);
  *bytes = b;
  return LOPC_OK;
}

// Repair sweeps driven from the host (LOPC_REPAIR_SWEEPS): the first
// group of K sweeps (K from the previous call on this context) is enqueued
// with the encoder, which runs only if no tile is marked for sweep K + 1;
// one read of the status, the counters and Params then ends a typical call.
// Otherwise sweeps continue in groups (4, 8, 16), one read per group, and
// the encoder runs after them.  A sweep with no marked tile costs one empty
// launch.  Every sweep that runs raises a subbin, and a dependency chain
// crosses at most n tiles, so n + 1 sweeps always reach the fixed point.
// Past `limit` sweeps, once the tile runs exceed kChainRuns per tile, it
// returns kRestartOnQueue (the encoder has not run).
constexpr int kRestartOnQueue = 1;
constexpr uint64_t kChainRuns = 16;
static int repair_by_sweeps(lopc_ctx* ctx, const Shape& s, const CompressLayout& L, int dtype,
                            uint8_t* ws, void* d_stream, size_t stream_cap, const Tiling& tl,
                            bool want_parts, hipStream_t hs, uint64_t limit,
                            uint64_t* sweeps_out, uint64_t* active_out) {
  uint32_t* sub = (uint32_t*)(ws + L.sub);
  uint32_t* stamp = (uint32_t*)(ws + L.stamp);
  uint32_t* counters = (uint32_t*)(ws + L.counters);
  uint64_t* offs = (uint64_t*)(ws + L.offs);
  Params* prm = (Params*)(ws + L.prm);
  const uint64_t k = dtype == 0 ? 4 : 8, W = kChunkBytes / k;
  const uint32_t nch = (uint32_t)((s.n + W - 1) / W);
  uint64_t sweeps = 1, active = tl.ntiles;
  const uint32_t K = (uint32_t)ctx->sweep_hint;
  const size_t report = L.queue + sizeof(RepairQueue);
  for (uint32_t t = 1; t <= K; ++t) {
    Ev e = t == 1 ? ev_first(ctx, LOPC_PHASE_REPAIR) : Ev{};
    if (t == K) e.b = ev_last(ctx, LOPC_PHASE_REPAIR).b;
    HIP_CTX(ctx, launch_repair(s.box, tl, (const uint16_t*)(ws + L.mask), sub, stamp,
                               counters, t, hs, e));
  }
  HIP_CTX(ctx, launch_encode(dtype, (uint32_t)s.n, ws + L.bins, sub, (uint16_t*)(ws + L.mask),
                             ws + L.tail, offs, (uint32_t*)(ws + L.parts), prm,
                             (uint8_t*)d_stream, stream_cap, counters + 1 + ((K + 1) & 63), hs,
                             ev_only(ctx, LOPC_PHASE_ENCODE)));
  if (want_parts)
    HIP_CTX(ctx, launch_sum_parts((const uint32_t*)(ws + L.parts), nch, prm, hs));
  HIP_CTX(ctx, hipMemcpyAsync(ctx->h_prm, ws, report, hipMemcpyDeviceToHost, hs));
  HIP_CTX(ctx, hipStreamSynchronize(hs));
  uint32_t next = 1, batch = K;
  for (;;) {
    const uint32_t* hc = (const uint32_t*)((const uint8_t*)ctx->h_prm + L.counters);
    if (hc[0]) return LOPC_E_INTERNAL;
    const int code = status_code(ctx->h_prm->status);
    if (code != LOPC_OK && code != LOPC_E_CAPACITY) return code;
    // marks for sweep t are hc[1 + t % 64]; sweep t ran iff they are nonzero
    bool done = false;
    for (uint32_t t = next; t <= next + batch; ++t) {
      const uint32_t m = hc[1 + (t & 63)];
      if (m == 0) {
        done = true;
        break;
      }
      if (t < next + batch) {
        ++sweeps;
        active += m;
      }
    }
    if (done) break;
    // clear the ring slots consumed by this group (marks for sweep
    // next + batch stay: the next group starts with it)
    for (uint32_t t = next; t < next + batch; ++t)
      HIP_CTX(ctx, launch_zero_n(counters + 1 + (t & 63), 1, hs));
    next += batch;
    batch = next == K + 1 ? 4 : std::min<uint32_t>(batch * 2, 16);
    // a limit below n + 2 (the default's) holds only while the tile runs so
    // far exceed kChainRuns per tile: a chain across T tiles reruns nearly
    // every tile it has not settled yet in each sweep, so it passes that mark
    // within the limit and goes to the queue, while a field that merely needs
    // many sweeps keeps sweeping
    const uint64_t cap =
        limit < s.n + 2 && active <= kChainRuns * (uint64_t)tl.ntiles ? s.n + 2 : limit;
    if (next > cap) {
      *sweeps_out = sweeps;
      *active_out = active;
      return cap >= s.n + 2 ? LOPC_E_INTERNAL : kRestartOnQueue;  // the former unreachable
    }
    batch = (uint32_t)std::min<uint64_t>(batch, cap + 1 - next);  // the last group ends at cap
    for (uint32_t b = 0; b < batch; ++b)
      HIP_CTX(ctx, launch_repair(s.box, tl, (const uint16_t*)(ws + L.mask), sub, stamp,
                                 counters, next + b, hs,
                                 b + 1 == batch ? ev_last(ctx, LOPC_PHASE_REPAIR) : Ev{}));
    HIP_CTX(ctx, hipMemcpyAsync(ctx->h_prm, ws, report, hipMemcpyDeviceToHost, hs));
    HIP_CTX(ctx, hipStreamSynchronize(hs));
  }
  // the next call starts with as many sweeps as this one needed, plus one
  ctx->sweep_hint = (int)std::min<uint64_t>(16, std::max<uint64_t>(2, sweeps));
  if (next > 1) {
    // the gated encoder did not run: encode now
    HIP_CTX(ctx, launch_encode(dtype, (uint32_t)s.n, ws + L.bins, sub,
                               (uint16_t*)(ws + L.mask), ws + L.tail, offs,
                               (uint32_t*)(ws + L.parts), prm, (uint8_t*)d_stream, stream_cap,
                               nullptr, hs, ev_only(ctx, LOPC_PHASE_ENCODE)));
    if (want_parts)
      HIP_CTX(ctx, launch_sum_parts((const uint32_t*)(ws + L.parts), nch, prm, hs));
    HIP_CTX(ctx, hipMemcpyAsync(ctx->h_prm, prm, sizeof(Params), hipMemcpyDeviceToHost, hs));
    HIP_CTX(ctx, hipStreamSynchronize(hs));
  }
  *sweeps_out = sweeps;
  *active_out = active;
  return LOPC_OK;
}

// The paper's point worklists (LOPC_REPAIR_POINTS), driven from the host:
// after the first tile pass every point with flags is listed; iterations are
// enqueued in groups (4, 8, 16), each reading its list length on the
// device, with one read of the length ring per group; the repair ends with
// the first empty list.  Every iteration that runs raises a subbin, so
// n + 1 iterations always reach the fixed point (past that: an error).
static int repair_by_points(lopc_ctx* ctx, const Shape& s, const CompressLayout& L, int dtype,
                            uint8_t* ws, void* d_stream, size_t stream_cap, bool want_parts,
                            hipStream_t hs, uint64_t* iters_out, uint64_t* listed_out) {
  uint32_t* sub = (uint32_t*)(ws + L.sub);
  uint32_t* counters = (uint32_t*)(ws + L.counters);
  uint32_t* ring = counters + kCursorWord;  // the work-list cursors are unused here
  uint32_t* wl[2] = {(uint32_t*)(ws + L.pw0), (uint32_t*)(ws + L.pw1)};
  uint32_t* pstamp = (uint32_t*)(ws + L.pstamp);
  const uint16_t* mask = (const uint16_t*)(ws + L.mask);
  Params* prm = (Params*)(ws + L.prm);
  const uint64_t k = dtype == 0 ? 4 : 8, W = kChunkBytes / k;
  const uint32_t nch = (uint32_t)((s.n + W - 1) / W);
  // grid-stride kernels of 256-thread workgroups, 8 per CU at most
  const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((s.n + 255) / 256,
                                                                  (uint64_t)ctx->num_cu * 8));
  const size_t report = L.queue + sizeof(RepairQueue);
  HIP_CTX(ctx, launch_zero_n(pstamp, s.n, hs, ev_first(ctx, LOPC_PHASE_REPAIR)));
  HIP_CTX(ctx, launch_point_seed(mask, (uint32_t)s.n, wl[0], ring, grid, hs));
  uint32_t it = 0, batch = 4;
  uint64_t listed = 0;
  for (;;) {
    for (uint32_t b = 0; b < batch; ++b, ++it)
      HIP_CTX(ctx, launch_point_iter(s.box, mask, sub, wl[it & 1], wl[(it + 1) & 1], ring, pstamp,
                                     it, grid, hs,
                                     b + 1 == batch ? ev_last(ctx, LOPC_PHASE_REPAIR) : Ev{}));
    HIP_CTX(ctx, hipMemcpyAsync(ctx->h_prm, ws, report, hipMemcpyDeviceToHost, hs));
    HIP_CTX(ctx, hipStreamSynchronize(hs));
    const uint32_t* hc = (const uint32_t*)((const uint8_t*)ctx->h_prm + L.counters) + kCursorWord;
    const int code = status_code(ctx->h_prm->status);
    if (code != LOPC_OK && code != LOPC_E_CAPACITY) return code;
    // lists it - batch .. it ran; the list of iteration it is still to run
    bool done = false;
    for (uint32_t t = it - batch; t <= it; ++t) {
      const uint32_t m = hc[t & 63];
      if (m == 0) {
        done = true;
        *iters_out = t + 1;  // the first pass counts as one
        break;
      }
      if (t < it) listed += m;
    }
    if (done) break;
    if ((uint64_t)it > s.n + 2) return LOPC_E_INTERNAL;  // unreachable
    // clear the slots of the lists consumed by this group (the list of
    // iteration it stays: the next group starts with it)
    for (uint32_t t = it - batch; t < it; ++t) HIP_CTX(ctx, launch_zero_n(ring + (t & 63), 1, hs));
    batch = std::min<uint32_t>(batch * 2, 16);
  }
  *listed_out = listed;
  HIP_CTX(ctx, launch_encode(dtype, (uint32_t)s.n, ws + L.bins, sub, (uint16_t*)(ws + L.mask),
                             ws + L.tail, (uint64_t*)(ws + L.offs), (uint32_t*)(ws + L.parts), prm,
                             (uint8_t*)d_stream, stream_cap, nullptr, hs,
                             ev_only(ctx, LOPC_PHASE_ENCODE)));
  if (want_parts)
    HIP_CTX(ctx, launch_sum_parts((const uint32_t*)(ws + L.parts), nch, prm, hs));
  HIP_CTX(ctx, hipMemcpyAsync(ctx->h_prm, prm, sizeof(Params), hipMemcpyDeviceToHost, hs));
  HIP_CTX(ctx, hipStreamSynchronize(hs));
  return LOPC_OK;
}

int lopc_compress(lopc_ctx* ctx, const void* d_field, int dtype, int ndim,
                  const int64_t* dims, double error_bound, int mode,
                  void* d_stream, size_t stream_cap, size_t* h_stream_size,
                  uint64_t* d_stream_size, int32_t* d_status,
                  void* d_ws, size_t ws_bytes, void* stream,
                  lopc_stats* h_stats) {
  if (!ctx || !d_field || !d_stream || !d_ws) return LOPC_E_ARG;
  const bool enqueue_only = h_stream_size == nullptr;
  // enqueued calls report on the device only, through a device-driven repair
  if (enqueue_only && (!d_stream_size || h_stats || ctx->repair_mode == LOPC_REPAIR_SWEEPS ||
                       ctx->repair_mode == LOPC_REPAIR_POINTS))
    return LOPC_E_ARG;
  if ((dtype != 0 && dtype != 1) || (mode != 0 && mode != 1)) return LOPC_E_ARG;
  Shape s;
  int st = make_shape(ndim, dims, &s);
  if (st) return st;
  if (!std::isfinite(error_bound) || !(error_bound > 0)) return LOPC_E_BOUND;
  if (((uintptr_t)d_field & 15) || ((uintptr_t)d_stream & 3)) return LOPC_E_ARG;
  if (((uintptr_t)d_stream_size & 7) || ((uintptr_t)d_status & 3)) return LOPC_E_ARG;
  CompressLayout L = compress_layout(s, dtype, ctx->tile2, ctx->tile3,
                                     ctx->repair_mode == LOPC_REPAIR_POINTS);
  if (ws_bytes < L.total || ((uintptr_t)d_ws & 255)) return LOPC_E_ARG;
  hipStream_t hs = (hipStream_t)stream;
  HIP_CTX(ctx, hipSetDevice(ctx->device));

  uint8_t* ws = (uint8_t*)d_ws;
  Params* prm = (Params*)(ws + L.prm);
  uint32_t* sub = (uint32_t*)(ws + L.sub);
  uint32_t* stamp = (uint32_t*)(ws + L.stamp);
  uint32_t* counters = (uint32_t*)(ws + L.counters);
  uint64_t* offs = (uint64_t*)(ws + L.offs);
  const uint64_t k = dtype == 0 ? 4 : 8, W = kChunkBytes / k;
  const uint64_t nch = (s.n + W - 1) / W;
  Tiling tl = make_tiling(s.box, ctx->tile2, ctx->tile3);
  if (s.box.nz == 1) tl.lev = ws + L.lev;
  tl.coloured = ctx->sweep_order == 1 || (ctx->sweep_order == 0 && tl.ntiles >= kColourMinTiles);
  const int rmode = ctx->repair_mode;
  QueueRef Q{};
  {
    Q.q = (RepairQueue*)(ws + L.queue);
    Q.ring = (unsigned long long*)(ws + L.ring);
    Q.st = (uint32_t*)(ws + L.qstate);
    Q.parked = (uint32_t*)(ws + L.parked);
    Q.blockers = (uint32_t*)(ws + L.blockers);
    Q.depth = (uint32_t*)(ws + L.depth);
    Q.cap_log2 = L.cap_log2;
  }

  int nblocks = (int)std::min<uint64_t>(kMinmaxBlocks, (s.n + 2047) / 2048);
  if (nblocks < 1) nblocks = 1;
  // the zeroed prefix of the workspace is cleared by the range pass (NOA),
  // else by a fill kernel
  if (mode == LOPC_EB_NOA)
    HIP_CTX(ctx, launch_minmax(dtype, d_field, (uint32_t)s.n, (double*)(ws + L.part),
                               nblocks, ws, L.zero_end, hs, ev_first(ctx, LOPC_PHASE_RANGE)));
  else
    HIP_CTX(ctx, launch_zero_n((uint32_t*)ws, L.zero_end / 4, hs,
                               ev_first(ctx, LOPC_PHASE_RANGE)));
  HIP_CTX(ctx, launch_params(dtype, mode, error_bound, (const double*)(ws + L.part),
                             nblocks, prm, (uint8_t*)d_stream, stream_cap, ndim,
                             s.d, hs, ev_last(ctx, LOPC_PHASE_RANGE)));
  uint64_t sweeps = 1, active = tl.ntiles, qruns = 0, qparks = 0;
  const int sid = tl.sid;
  // Device-driven repair (Alg. 1 loop at tile granularity, no host read):
  // the first pass (quantize, order flags, first relaxation, fused per
  // tile), K sweeps over work lists, the repair queue for whatever is still
  // listed (nothing, when K sweeps were enough; with K = 0 the first pass
  // lists its tiles in the queue itself), then the encoder and the report.
  auto device_repair = [&](uint32_t K) -> int {
    if (!ctx->rq_per_cu[sid]) ctx->rq_per_cu[sid] = repair_q_blocks_per_cu(sid);
    if (!ctx->sl_per_cu[sid]) ctx->sl_per_cu[sid] = sweep_list_blocks_per_cu(sid);
    uint32_t* lists = K ? (uint32_t*)(ws + L.lists) : nullptr;
    HIP_CTX(ctx, launch_tile0(dtype, d_field, s.box, tl, prm, ws + L.bins,
                              (uint16_t*)(ws + L.mask), sub, stamp, counters, lists,
                              K ? QueueRef{} : Q, hs, ev_only(ctx, LOPC_PHASE_QUANT)));
    const int sgrid = (int)std::max<uint64_t>(
        1, std::min<uint64_t>(tl.ntiles, (uint64_t)ctx->sl_per_cu[sid] * ctx->num_cu));
    for (uint32_t t = 1; t <= K; ++t)
      HIP_CTX(ctx, launch_sweep_list(s.box, tl, (const uint16_t*)(ws + L.mask), sub, stamp,
                                     counters, lists, t, sgrid, hs,
                                     t == 1 ? ev_first(ctx, LOPC_PHASE_REPAIR) : Ev{}));
    if (K) HIP_CTX(ctx, launch_seed_queue(counters, lists, tl.ntiles, K + 1, Q, hs));
    const int grid = (int)std::max<uint64_t>(
        1, std::min<uint64_t>(tl.ntiles, (uint64_t)ctx->rq_per_cu[sid] * ctx->num_cu));
    HIP_CTX(ctx, launch_repair_q(s.box, tl, (const uint16_t*)(ws + L.mask), sub, counters, Q,
                                 grid, hs,
                                 K ? ev_last(ctx, LOPC_PHASE_REPAIR)
                                   : ev_only(ctx, LOPC_PHASE_REPAIR)));
    HIP_CTX(ctx, launch_encode(dtype, (uint32_t)s.n, ws + L.bins, sub, (uint16_t*)(ws + L.mask),
                               ws + L.tail, offs, (uint32_t*)(ws + L.parts), prm,
                               (uint8_t*)d_stream, stream_cap, nullptr, hs,
                               ev_only(ctx, LOPC_PHASE_ENCODE)));
    if (h_stats)
      HIP_CTX(ctx, launch_sum_parts((const uint32_t*)(ws + L.parts), (uint32_t)nch, prm, hs));
    if (d_stream_size || d_status)
      HIP_CTX(ctx, launch_report(prm, Q.q, d_stream_size, d_status, hs));
    if (enqueue_only) return LOPC_OK;
    HIP_CTX(ctx, hipMemcpyAsync(ctx->h_prm, ws, L.queue + sizeof(RepairQueue),
                                hipMemcpyDeviceToHost, hs));
    HIP_CTX(ctx, hipStreamSynchronize(hs));
    const uint32_t* hc = (const uint32_t*)((const uint8_t*)ctx->h_prm + L.counters);
    const RepairQueue* hq = (const RepairQueue*)((const uint8_t*)ctx->h_prm + L.queue);
    if (hc[0] || hq->err) return LOPC_E_INTERNAL;
    for (uint32_t t = 1; t <= K; ++t) {
      const uint32_t m = hc[1 + (t & 63)];
      if (!m) break;
      ++sweeps;
      active += m;
    }
    if (hq->runs) sweeps = std::max<uint64_t>(sweeps, 1 + hq->max_depth);
    active += hq->runs;
    qruns = hq->runs;
    qparks = hq->parks;
    // the next call sweeps as often as this one needed, plus one
    if (K)
      ctx->sweep_hint = (int)std::min<uint64_t>(kMaxListSweeps, std::max<uint64_t>(2, sweeps));
    return LOPC_OK;
  };

  int rc;
  if (rmode == LOPC_REPAIR_QUEUE) {
    rc = device_repair(0);
  } else if (rmode == LOPC_REPAIR_POINTS) {
    HIP_CTX(ctx, launch_tile0(dtype, d_field, s.box, tl, prm, ws + L.bins,
                              (uint16_t*)(ws + L.mask), sub, stamp, counters, nullptr,
                              QueueRef{}, hs, ev_only(ctx, LOPC_PHASE_QUANT)));
    rc = repair_by_points(ctx, s, L, dtype, ws, d_stream, stream_cap, h_stats != nullptr, hs,
                          &sweeps, &active);
    if (rc == LOPC_OK && (d_stream_size || d_status))
      HIP_CTX(ctx, launch_report(prm, nullptr, d_stream_size, d_status, hs));
  } else if (rmode == LOPC_REPAIR_HYBRID || (rmode == LOPC_REPAIR_AUTO && enqueue_only)) {
    rc = device_repair((uint32_t)std::min<int>(std::max(ctx->sweep_hint, 1), (int)kMaxListSweeps));
  } else {
    // host-driven sweeps (the fastest schedule when dependencies cross few
    // tiles); the default gives up after kAutoSweeps sweeps if by then the
    // sweeps have run more than kChainRuns tiles per tile of the field, and
    // restarts the repair from the first pass on the queue, which runs a
    // chain across many tiles a few times per tile instead of once per sweep
    HIP_CTX(ctx, launch_tile0(dtype, d_field, s.box, tl, prm, ws + L.bins,
                              (uint16_t*)(ws + L.mask), sub, stamp, counters, nullptr,
                              QueueRef{}, hs, ev_only(ctx, LOPC_PHASE_QUANT),
                              tl.coloured != 0));
    const uint64_t limit = rmode == LOPC_REPAIR_AUTO ? kAutoSweeps : s.n + 2;
    rc = repair_by_sweeps(ctx, s, L, dtype, ws, d_stream, stream_cap, tl, h_stats != nullptr,
                          hs, limit, &sweeps, &active);
    if (rc == kRestartOnQueue) {
      const uint64_t swept = sweeps, runs = active;
      sweeps = 1;
      active = tl.ntiles;
      rc = device_repair(0);
      sweeps = std::max(sweeps, swept);
      active += runs;
    } else if (rc == LOPC_OK && (d_stream_size || d_status)) {
      HIP_CTX(ctx, launch_report(prm, nullptr, d_stream_size, d_status, hs));
    }
  }
  if (rc == LOPC_E_HIP || rc == LOPC_E_INTERNAL) return rc;
  if (rc != LOPC_OK) {
    *h_stream_size = 0;
    return rc;
  }
  if (enqueue_only) return LOPC_OK;
  if (ctx->timing) {
    for (int p = LOPC_PHASE_RANGE; p <= LOPC_PHASE_ENCODE; ++p) ctx->ms[p] = phase_ms(ctx, p);
  }
  const Params& hp = *ctx->h_prm;
  const int code = status_code(hp.status);
  if (code != LOPC_OK && code != LOPC_E_CAPACITY) {
    *h_stream_size = 0;
    return code;
  }
  *h_stream_size = (size_t)hp.stream_size;
  std::memcpy(ctx->last_header, hp.header, kHeaderBytes);
  ctx->have_header = code == LOPC_OK;
  if (h_stats) {
    const uint32_t* hc = (const uint32_t*)((const uint8_t*)ctx->h_prm + L.counters);
    uint64_t relax_iters = 0;
    for (int q = 0; q < 64; ++q) {
      uint64_t v;
      std::memcpy(&v, hc + kRelaxWord + 2 * q, 8);
      relax_iters += v;
    }
    h_stats->eps = hp.eps;
    h_stats->repair_sweeps = sweeps;
    h_stats->active_tiles_total = active;
    h_stats->relax_iterations = relax_iters;
    h_stats->bins_bytes = hp.bins_bytes;
    h_stats->subbins_bytes = hp.sub_bytes;
    h_stats->queue_runs = qruns;
    h_stats->queue_parks = qparks;
  }
  return code;
}

int lopc_stream_info(const void* h_header, size_t n, int* dtype, int* ndim,
                     int64_t* dims, double* eps, size_t* field_bytes) {
  const uint8_t* h = (const uint8_t*)h_header;
  if (!h || n < kHeaderBytes) return LOPC_E_FORMAT;
  if (rd_u32(h) != kMagic || (h[4] | (h[5] << 8)) != (int)kVersion)
    return LOPC_E_FORMAT;
  const int dt = h[6], nd = h[7];
  if ((dt != 0 && dt != 1) || (nd != 2 && nd != 3)) return LOPC_E_FORMAT;
  if (h[32] > 1 || rd_u32(h + 36) != kChunkBytes) return LOPC_E_FORMAT;
  int64_t d[3];
  uint64_t pts = 1;
  for (int i = 0; i < 3; ++i) {
    uint64_t v = rd_u64(h + 8 + 8 * i);
    if (v < 1 || v > ((uint64_t)1 << 40)) return LOPC_E_FORMAT;
    d[i] = (int64_t)v;
    if (pts > ((uint64_t)1 << 48) / v) return LOPC_E_FORMAT;
    pts *= v;
  }
  if (nd == 2 && d[2] != 1) return LOPC_E_FORMAT;
  const double e = rd_f64(h + 48), v = rd_f64(h + 56);
  if (!std::isfinite(e) || !(e > 0) || !std::isfinite(v) || !(v > 0))
    return LOPC_E_FORMAT;
  // inv must be the smallest binary64 with inv * eps >= 1
  if (std::fma(v, e, -1.0) < 0 || std::fma(std::nextafter(v, 0.0), e, -1.0) >= 0)
    return LOPC_E_FORMAT;
  if (dtype) *dtype = dt;
  if (ndim) *ndim = nd;
  if (dims)
    for (int i = 0; i < 3; ++i) dims[i] = d[i];
  if (eps) *eps = e;
  if (field_bytes) *field_bytes = (size_t)(pts * (dt == 0 ? 4 : 8));
  return LOPC_OK;
}

static int decompress_core(lopc_ctx* ctx, const uint8_t* hdr, const void* d_stream,
                           size_t stream_size, void* d_field, size_t field_cap,
                           void* d_ws, size_t ws_bytes, hipStream_t hs) {
  int dtype, ndim;
  int64_t dims[3];
  size_t fbytes;
  int st = lopc_stream_info(hdr, kHeaderBytes, &dtype, &ndim, dims, nullptr, &fbytes);
  if (st) return st;
  Shape s;
  if (make_shape(ndim, dims, &s) != LOPC_OK) return LOPC_E_ARG;  // > 2^32 points
  const uint64_t k = dtype == 0 ? 4 : 8, W = kChunkBytes / k;
  const uint64_t nch = (s.n + W - 1) / W;
  if (stream_size < kHeaderBytes + 4 * nch) return LOPC_E_FORMAT;
  if (field_cap < fbytes) return LOPC_E_CAPACITY;
  if (((uintptr_t)d_stream & 3) || ((uintptr_t)d_field & (k - 1))) return LOPC_E_ARG;
  if (ws_bytes < decompress_ws(s, dtype) || ((uintptr_t)d_ws & 255)) return LOPC_E_ARG;
  uint8_t* ws = (uint8_t*)d_ws;
  Params* prm = (Params*)ws;
  uint64_t* offsets = (uint64_t*)(ws + align256(sizeof(Params)));
  HIP_CTX(ctx, launch_offsets((const uint8_t*)d_stream, (uint32_t)nch,
                              stream_size - kHeaderBytes - 4 * nch, offsets, prm, hs,
                              ev_only(ctx, LOPC_PHASE_OFFSETS)));
  HIP_CTX(ctx, launch_decode(dtype, (const uint8_t*)d_stream, (uint32_t)s.n, offsets,
                             prm, d_field, hs, ev_only(ctx, LOPC_PHASE_DECODE)));
  HIP_CTX(ctx, hipMemcpyAsync(&ctx->h_prm->status, &prm->status, 4, hipMemcpyDeviceToHost, hs));
  HIP_CTX(ctx, hipStreamSynchronize(hs));
  if (ctx->timing) {
    for (int p = LOPC_PHASE_OFFSETS; p <= LOPC_PHASE_DECODE; ++p) ctx->ms[p] = phase_ms(ctx, p);
  }
  return status_code(ctx->h_prm->status);
}

int lopc_decompress(lopc_ctx* ctx, const void* d_stream, size_t stream_size,
                    void* d_field, size_t field_cap, void* d_ws,
                    size_t ws_bytes, void* stream) {
  if (!ctx || !d_stream || !d_field || !d_ws) return LOPC_E_ARG;
  if (stream_size < kHeaderBytes) return LOPC_E_FORMAT;
  hipStream_t hs = (hipStream_t)stream;
  HIP_CTX(ctx, hipSetDevice(ctx->device));
  uint8_t* hh = (uint8_t*)ctx->h_prm;  // pinned staging for the header
  HIP_CTX(ctx, hipMemcpyAsync(hh, d_stream, kHeaderBytes, hipMemcpyDeviceToHost, hs));
  HIP_CTX(ctx, hipStreamSynchronize(hs));
  uint8_t hdr[kHeaderBytes];
  std::memcpy(hdr, hh, kHeaderBytes);
  return decompress_core(ctx, hdr, d_stream, stream_size, d_field, field_cap, d_ws, ws_bytes, hs);
}

int lopc_decompress_static(lopc_ctx* ctx, const void* h_header, const void* d_stream,
                           size_t stream_size, void* d_field, size_t field_cap, void* stream) {
  if (!ctx || !h_header || !d_stream || !d_field) return LOPC_E_ARG;
  if (stream_size < kHeaderBytes) return LOPC_E_FORMAT;
  int dtype, ndim;
  int64_t dims[3];
  if (int st = lopc_stream_info(h_header, kHeaderBytes, &dtype, &ndim, dims, nullptr, nullptr))
    return st;
  Shape s;
  if (make_shape(ndim, dims, &s) != LOPC_OK) return LOPC_E_ARG;
  // the scratch holds Params and one offset per chunk: larger streams are
  // refused before any device work
  if (decompress_ws(s, dtype) > kStaticScratchBytes) return LOPC_E_CAPACITY;
  HIP_CTX(ctx, hipSetDevice(ctx->device));
  return decompress_core(ctx, (const uint8_t*)h_header, d_stream, stream_size, d_field,
                         field_cap, ctx->scratch, kStaticScratchBytes, (hipStream_t)stream);
}

int lopc_decompress_h(lopc_ctx* ctx, const void* h_header, const void* d_stream,
                      size_t stream_size, void* d_field, size_t field_cap, void* d_ws,
                      size_t ws_bytes, void* stream) {
  if (!ctx || !h_header || !d_stream || !d_field || !d_ws) return LOPC_E_ARG;
  if (stream_size < kHeaderBytes) return LOPC_E_FORMAT;
  HIP_CTX(ctx, hipSetDevice(ctx->device));
  return decompress_core(ctx, (const uint8_t*)h_header, d_stream, stream_size, d_field,
                         field_cap, d_ws, ws_bytes, (hipStream_t)stream);
}

size_t lopc_verify_workspace_size(void) { return 256; }

int lopc_verify(lopc_ctx* ctx, const void* d_orig, const void* d_recon, int dtype, int ndim,
                const int64_t* dims, double eps, void* d_ws, size_t ws_bytes, void* stream,
                lopc_verify_report* h_report) {
  if (!ctx || !d_orig || !d_recon || !d_ws || !h_report || (dtype != 0 && dtype != 1))
    return LOPC_E_ARG;
  Shape s;
  if (int st = make_shape(ndim, dims, &s)) return st;
  if (ws_bytes < 256 || ((uintptr_t)d_ws & 255)) return LOPC_E_ARG;
  const uint64_t k = dtype == 0 ? 4 : 8;
  if (((uintptr_t)d_orig & (k - 1)) || ((uintptr_t)d_recon & (k - 1))) return LOPC_E_ARG;
  if (!std::isfinite(eps) || !(eps >= 0)) return LOPC_E_BOUND;
  hipStream_t hs = (hipStream_t)stream;
  HIP_CTX(ctx, hipSetDevice(ctx->device));
  unsigned long long* out = (unsigned long long*)d_ws;
  HIP_CTX(ctx, hipMemsetAsync(out, 0, 256, hs));
  const int blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ctx->num_cu * 8,
                                                                   (s.n + 255) / 256));
  HIP_CTX(ctx, launch_verify(dtype, d_orig, d_recon, s.box, eps, out, blocks, hs));
  unsigned long long* h = (unsigned long long*)ctx->h_cnt;
  HIP_CTX(ctx, hipMemcpyAsync(h, out, 14 * 8, hipMemcpyDeviceToHost, hs));
  HIP_CTX(ctx, hipStreamSynchronize(hs));
  h_report->points = h[0];
  h_report->bound_violations = h[1];
  std::memcpy(&h_report->max_abs_error, &h[2], 8);
  h_report->edges = h[3];
  h_report->order_violations = h[4];
  for (int i = 0; i < 4; ++i) {
    h_report->types_orig[i] = h[5 + i];
    h_report->types_recon[i] = h[9 + i];
  }
  h_report->type_mismatches = h[13];
  return LOPC_OK;
}

int lopc_ctx_last_header(lopc_ctx* ctx, void* h_header) {
  if (!ctx || !h_header) return LOPC_E_ARG;
  if (!ctx->have_header) return LOPC_E_ARG;
  std::memcpy(h_header, ctx->last_header, kHeaderBytes);
  return LOPC_OK;
}

}  // extern "C"
