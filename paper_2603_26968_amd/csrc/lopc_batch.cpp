// lopc_batch.cpp -- host runtime of the batch calls of liblopc.so: job
// validation, the batch plan and workspace layout, the persistent launch
// sequence, its capture as a HIP graph, and the eager continuation of repair
// sweeps beyond the captured ones.  The public contract is in include/lopc.h.
//
// Workspace of a batch (every region 256-byte aligned):
//   plan      BatchDesc, then the job table            (uploaded per call)
//   cleared   BatchCounters, Params per job, and for compress the tile stamps,
//             look-back words and part sizes of every field
//   results   BatchResult per job
//   compress: min/max partials, two tile work lists, then per field its
//             bins, order flags and subbins
//   decompress: record offsets of every field
#include <chrono>
#include <new>

#include "lopc_host.h"

using namespace lopc;
using namespace lopc_host;

namespace {

constexpr int kMaxGraphs = 8;
constexpr int kMaxGraphSweeps = (int)kRing - 2;

// group: dtype and tile shape (a 3D field one point thick uses plane tiles,
// as in the single-field path)
int group_of(const lopc_job& j) {
  return 2 * j.dtype + (j.ndim == 3 && j.dims[0] > 1 ? 1 : 0);
}

struct Plan {
  std::vector<int> order;  // plan position -> job index
  std::vector<Job> jobs;
  BatchDesc desc;
  uint32_t gmask = 0;
  size_t plan_bytes = 0;   // BatchDesc + jobs
  size_t zero_off = 0, zero_end = 0;
  size_t total = 0;
  uint64_t tiles = 0;
};

// Validate the jobs and lay the batch out on workspace base `ws` (0 to size
// it).  On a bad job returns its status and sets *bad to its index.
int make_plan(int op, int n, const lopc_job* in, uintptr_t ws, int t2, int t3, Plan& P,
              int* bad) {
  *bad = -1;
  if (n < 1 || !in) return LOPC_E_ARG;
  P.order.resize(n);
  std::vector<Shape> shp(n);
  for (int i = 0; i < n; ++i) {
    const lopc_job& j = in[i];
    *bad = i;
    if (!j.d_in || !j.d_out || (j.dtype != 0 && j.dtype != 1)) return LOPC_E_ARG;
    if (make_shape(j.ndim, j.dims, &shp[i]) != LOPC_OK) return LOPC_E_ARG;
    const uint64_t k = j.dtype == 0 ? 4 : 8, W = kChunkBytes / k;
    const uint64_t nch = (shp[i].n + W - 1) / W;
    if (op == 0) {
      if (j.mode != 0 && j.mode != 1) return LOPC_E_ARG;
      if (((uintptr_t)j.d_in & 15) || ((uintptr_t)j.d_out & 3)) return LOPC_E_ARG;
      if (!std::isfinite(j.error_bound) || !(j.error_bound > 0)) return LOPC_E_BOUND;
    } else {
      if (((uintptr_t)j.d_in & 3) || ((uintptr_t)j.d_out & (k - 1))) return LOPC_E_ARG;
      if (j.in_bytes < kHeaderBytes + 4 * nch) return LOPC_E_FORMAT;
      if (j.out_cap < shp[i].n * k) return LOPC_E_CAPACITY;
    }
    P.order[i] = i;
  }
  *bad = -1;
  std::stable_sort(P.order.begin(), P.order.end(),
                   [&](int a, int b) { return group_of(in[a]) < group_of(in[b]); });

  // items of every phase, batch-wide
  P.jobs.assign(n, Job{});
  BatchDesc& D = P.desc;
  std::memset(&D, 0, sizeof(D));
  uint64_t it[PH_N] = {0, 0, 0};
  int g_prev = -1;
  for (int q = 0; q < n; ++q) {
    const int i = P.order[q];
    const lopc_job& j = in[i];
    const int g = group_of(j);
    while (g_prev < g) {
      ++g_prev;
      D.job0[g_prev] = (uint32_t)q;
      for (int ph = 0; ph < PH_N; ++ph) D.item0[ph][g_prev] = (uint32_t)it[ph];
    }
    P.gmask |= 1u << g;
    const Shape& s = shp[i];
    Job& J = P.jobs[q];
    const uint64_t k = j.dtype == 0 ? 4 : 8, W = kChunkBytes / k;
    J.box = s.box;
    J.tl = make_tiling(s.box, t2, t3);
    J.nch = (uint32_t)((s.n + W - 1) / W);
    J.dtype = j.dtype;
    J.mode = op == 0 ? j.mode : 0;
    J.ndim = j.ndim;
    for (int d = 0; d < 3; ++d) J.dims[d] = s.d[d];
    J.eb = j.error_bound;
    J.out_size = j.d_out_size;
    J.out_status = j.d_status;
    if (op == 0) {
      J.x = j.d_in;
      J.stream = (uint8_t*)j.d_out;
      J.cap = j.out_cap;
      J.mm_blocks = j.mode == LOPC_EB_NOA ? (int32_t)((s.n + kMinmaxSpan - 1) / kMinmaxSpan) : 0;
    } else {
      J.y = j.d_out;
      J.stream = (uint8_t*)j.d_in;
      J.stream_size = j.in_bytes;
    }
    J.mm0 = (uint32_t)it[PH_MM];
    J.t0 = (uint32_t)it[PH_T];
    J.c0 = (uint32_t)it[PH_C];
    it[PH_MM] += (uint64_t)J.mm_blocks;
    it[PH_T] += J.tl.ntiles;
    it[PH_C] += J.nch;
  }
  while (g_prev < kGroups) {
    ++g_prev;
    D.job0[g_prev] = (uint32_t)n;
    for (int ph = 0; ph < PH_N; ++ph) D.item0[ph][g_prev] = (uint32_t)it[ph];
  }
  for (int ph = 0; ph < PH_N; ++ph)
    if (it[ph] >= (1ull << 31)) return LOPC_E_ARG;  // batch-wide items fit 31 bits
  P.tiles = it[PH_T];

  // layout
  size_t o = 0;
  P.plan_bytes = sizeof(BatchDesc) + (size_t)n * sizeof(Job);
  o += align256(P.plan_bytes);
  P.zero_off = o;
  const size_t bc_off = o;
  o += align256(sizeof(BatchCounters));
  const size_t prm_off = o;
  o += (size_t)n * sizeof(Params);
  size_t stamp_off = 0, lookback_off = 0, parts_off = 0;
  if (op == 0) {
    stamp_off = o;
    o += align256(P.tiles * 4);
    uint64_t nch = it[PH_C];
    lookback_off = o;
    o += align256(nch * 8);
    parts_off = o;
    o += align256(nch * 8);
  }
  P.zero_end = o;
  const size_t res_off = o;
  o += align256((size_t)n * sizeof(BatchResult));
  size_t part_off = 0, lists_off = 0, off_off = 0;
  if (op == 0) {
    part_off = o;
    o += align256(it[PH_MM] * 16);
    lists_off = o;
    o += align256(2 * P.tiles * 4);
  } else {
    off_off = o;
    o += align256(it[PH_C] * 8);
  }
  for (int q = 0; q < n; ++q) {
    Job& J = P.jobs[q];
    J.prm = (Params*)(ws + prm_off + (size_t)q * sizeof(Params));
    if (op == 0) {
      const uint64_t k = J.dtype == 0 ? 4 : 8;
      J.stamp = (uint32_t*)(ws + stamp_off) + J.t0;
      J.lookback = (uint64_t*)(ws + lookback_off) + J.c0;
      J.parts = (uint32_t*)(ws + parts_off) + 2ull * J.c0;
      J.part = (int64_t*)(ws + part_off) + 2ull * J.mm0;
      J.bins = (void*)(ws + o);
      o += align256((size_t)J.box.n * k);
      J.mask = (uint16_t*)(ws + o);
      o += align256((size_t)J.box.n * 2);
      J.sub = (uint32_t*)(ws + o);
      o += align256((size_t)J.box.n * 4);
    } else {
      J.offsets = (uint64_t*)(ws + off_off) + J.c0;
    }
  }
  P.total = o;
  // a field whose repair falls back to its own compression runs it inside
  // this workspace
  if (op == 0)
    for (int i = 0; i < n; ++i) P.total = std::max(P.total, compress_layout(shp[i], in[i].dtype, t2, t3).total);
  D.tiles = (uint32_t)P.tiles;
  D.zero_words = (P.zero_end - P.zero_off) / 4;
  D.zero_base = (uint32_t*)(ws + P.zero_off);
  D.bc = (BatchCounters*)(ws + bc_off);
  D.lists = (uint32_t*)(ws + lists_off);
  D.res = (BatchResult*)(ws + res_off);
  return LOPC_OK;
}

// persistent grid of kernel pk
int grid_of(lopc_ctx* c, int pk) {
  if (!c->per_cu[pk])
    c->per_cu[pk] = pk >= PK_ENCODE ? codec_blocks_per_cu(pk) : batch_blocks_per_cu(pk);
  const long g = (long)c->per_cu[pk] * c->num_cu * c->persist_pct / 100;
  return (int)std::max(1L, g);
}

int grow_pinned(void** p, size_t* cap, size_t need) {
  if (*cap >= need) return LOPC_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  size_t sz = std::max<size_t>(need, 4096);
  if (hipHostMalloc(p, sz, hipHostMallocDefault) != hipSuccess) {
    *p = nullptr;
    return LOPC_E_HIP;
  }
  *cap = sz;
  return LOPC_OK;
}

// Item counts of the groups [g0, g1) in phase ph.
uint32_t items(const BatchDesc& D, int ph, int g0, int g1) {
  return D.item0[ph][g1] - D.item0[ph][g0];
}

// The launch sequence of a batch, everything addressed from the workspace.
// Persistent mode (persist_pct > 0): fixed grids drain the queues, so the
// sequence does not depend on the batch's sizes.  Direct mode: one
// workgroup per item, grids from the plan D.
hipError_t enqueue(lopc_ctx* c, int op, uint8_t* ws, const BatchDesc& D, uint32_t gmask,
                   int sweeps, hipStream_t s) {
  const BatchDesc* bd = (const BatchDesc*)ws;
  const Job* jobs = (const Job*)(ws + sizeof(BatchDesc));
  const bool pers = c->persist_pct > 0;
  hipError_t e;
#define Q(x)                            \
  do {                                  \
    if ((e = (x)) != hipSuccess) return e; \
  } while (0)
  Q(launch_zero_p(bd, grid_of(c, PK_ZERO), s));
  const bool has[2] = {(gmask & 3u) != 0, (gmask & 12u) != 0};
  if (op == 0) {
    for (int d = 0; d < 2; ++d) {
      if (!has[d]) continue;
      const int g0 = 2 * d, g1 = 2 * d + 2;
      if (pers) {
        Q(launch_minmax_p(d, bd, jobs, grid_of(c, PK_MINMAX), s));
        Q(launch_params_p(d, bd, jobs, grid_of(c, PK_PARAMS), s));
      } else {
        Q(launch_minmax_d(d, bd, jobs, items(D, PH_MM, g0, g1), s));
        Q(launch_params_d(d, bd, jobs, D.job0[g1] - D.job0[g0], s));
      }
    }
    for (int g = 0; g < kGroups; ++g) {
      if (!(gmask & (1u << g))) continue;
      if (pers) Q(launch_tile0_p(g, c->tile2, c->tile3, bd, jobs, grid_of(c, PK_TILE0), s));
      else Q(launch_tile0_d(g, c->tile2, c->tile3, bd, jobs, items(D, PH_T, g, g + 1), s));
    }
    for (int t = 1; t <= sweeps; ++t) {
      if (pers)
        Q(launch_repair_p(c->tile2, c->tile3, bd, jobs, (uint32_t)t, grid_of(c, PK_REPAIR), s));
      else
        Q(launch_repair_d(c->tile2, c->tile3, bd, jobs, (uint32_t)t, D.tiles, s));
    }
    for (int d = 0; d < 2; ++d) {
      if (!has[d]) continue;
      if (pers) Q(launch_encode_p(d, bd, jobs, sweeps + 1, grid_of(c, PK_ENCODE), s));
      else Q(launch_encode_d(d, bd, jobs, sweeps + 1, items(D, PH_C, 2 * d, 2 * d + 2), s));
    }
    Q(launch_finalize_c(bd, jobs, sweeps + 1, s));
  } else {
    Q(launch_dhead_p(bd, jobs, pers ? grid_of(c, PK_DHEAD) : (int)D.job0[kGroups], s));
    for (int d = 0; d < 2; ++d) {
      if (!has[d]) continue;
      if (pers) Q(launch_decode_p(d, bd, jobs, grid_of(c, PK_DECODE), s));
      else Q(launch_decode_d(d, bd, jobs, items(D, PH_C, 2 * d, 2 * d + 2), s));
    }
    Q(launch_finalize_d(bd, jobs, s));
  }
#undef Q
  return hipSuccess;
}

// a captured sequence fits this batch
bool graph_fits(const BatchGraph& g, lopc_ctx* c, int op, const void* ws, uint32_t gmask,
                int sweeps, const BatchDesc& D) {
  if (g.op != op || g.ws != ws || g.gmask != gmask || g.sweeps != sweeps ||
      g.grid_pct != c->persist_pct || g.tile2 != c->tile2 || g.tile3 != c->tile3)
    return false;
  if (c->persist_pct > 0) return true;
  // direct grids: the batch's shape must match
  return std::memcmp(g.job0, D.job0, sizeof(D.job0)) == 0 &&
         std::memcmp(g.item0, D.item0, sizeof(D.item0)) == 0 && g.tiles == D.tiles;
}

// Run the sequence: replay a cached graph (capturing it first if needed) or
// launch directly.  *graph = 1 when a graph ran.
int run_sequence(lopc_ctx* c, int op, uint8_t* ws, const BatchDesc& D, uint32_t gmask,
                 int sweeps, hipStream_t s, int* graph) {
  *graph = 0;
  if (!c->use_graph) {
    HIP_CTX(c, enqueue(c, op, ws, D, gmask, sweeps, s));
    return LOPC_OK;
  }
  BatchGraph* hit = nullptr;
  for (BatchGraph& g : c->graphs)
    if (graph_fits(g, c, op, ws, gmask, sweeps, D)) hit = &g;
  if (!hit) {
    if (!c->cap_stream) HIP_CTX(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_CTX(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    hipError_t e = enqueue(c, op, ws, D, gmask, sweeps, c->cap_stream);
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    HIP_CTX(c, e);
    if ((int)c->graphs.size() >= kMaxGraphs) {
      auto old = std::min_element(c->graphs.begin(), c->graphs.end(),
                                  [](const BatchGraph& a, const BatchGraph& b) { return a.used < b.used; });
      (void)hipGraphExecDestroy(old->exec);
      c->graphs.erase(old);
    }
    BatchGraph g{};
    g.op = op;
    g.ws = ws;
    g.gmask = gmask;
    g.sweeps = sweeps;
    g.grid_pct = c->persist_pct;
    g.tile2 = c->tile2;
    g.tile3 = c->tile3;
    std::memcpy(g.job0, D.job0, sizeof(D.job0));
    std::memcpy(g.item0, D.item0, sizeof(D.item0));
    g.tiles = D.tiles;
    g.exec = exec;
    c->graphs.push_back(g);
    hit = &c->graphs.back();
  }
  hit->used = ++c->use_clock;
  HIP_CTX(c, hipGraphLaunch(hit->exec, s));
  *graph = 1;
  return LOPC_OK;
}

// Read back the counters and the results; returns the batch status.
int read_back(lopc_ctx* c, const Plan& P, uint8_t* ws, int n, hipStream_t s) {
  const size_t rb = align256(sizeof(BatchCounters)) + (size_t)n * sizeof(BatchResult);
  if (int st = grow_pinned(&c->h_back, &c->h_back_cap, rb)) return st;
  uint8_t* hb = (uint8_t*)c->h_back;
  HIP_CTX(c, hipMemcpyAsync(hb, P.desc.bc, sizeof(BatchCounters), hipMemcpyDeviceToHost, s));
  HIP_CTX(c, hipMemcpyAsync(hb + align256(sizeof(BatchCounters)), P.desc.res,
                            (size_t)n * sizeof(BatchResult), hipMemcpyDeviceToHost, s));
  HIP_CTX(c, hipStreamSynchronize(s));
  (void)ws;
  return LOPC_OK;
}

const BatchCounters* host_counters(lopc_ctx* c) { return (const BatchCounters*)c->h_back; }
const BatchResult* host_results(lopc_ctx* c) {
  return (const BatchResult*)((const uint8_t*)c->h_back + align256(sizeof(BatchCounters)));
}

// Copy the results into the context in job order; return the first failure.
int collect(lopc_ctx* c, const Plan& P, int n) {
  const BatchResult* r = host_results(c);
  c->last_sizes.assign(n, 0);
  c->last_status.assign(n, 0);
  c->last_headers.assign((size_t)n * kHeaderBytes, 0);
  for (int q = 0; q < n; ++q) {
    const int i = P.order[q];
    c->last_sizes[i] = r[q].size;
    c->last_status[i] = r[q].status;
    std::memcpy(&c->last_headers[(size_t)i * kHeaderBytes], r[q].header, kHeaderBytes);
  }
  for (int i = 0; i < n; ++i)
    if (c->last_status[i]) return c->last_status[i];
  return LOPC_OK;
}

void reject(lopc_ctx* c, int n, int bad, int st) {
  c->last_sizes.assign(n > 0 ? n : 0, 0);
  c->last_status.assign(n > 0 ? n : 0, 0);
  c->last_headers.assign((size_t)(n > 0 ? n : 0) * kHeaderBytes, 0);
  if (bad >= 0 && bad < n) c->last_status[bad] = st;
}

int upload_plan(lopc_ctx* c, const Plan& P, uint8_t* ws, hipStream_t s) {
  if (int st = grow_pinned(&c->h_plan, &c->h_plan_cap, P.plan_bytes)) return st;
  std::memcpy(c->h_plan, &P.desc, sizeof(BatchDesc));
  std::memcpy((uint8_t*)c->h_plan + sizeof(BatchDesc), P.jobs.data(), P.jobs.size() * sizeof(Job));
  HIP_CTX(c, hipMemcpyAsync(ws, c->h_plan, P.plan_bytes, hipMemcpyHostToDevice, s));
  return LOPC_OK;
}

int batch_common(lopc_ctx* c, int op, int n, const lopc_job* jobs, void* d_ws,
                 size_t ws_bytes, hipStream_t s, Plan& P) {
  if (!c) return LOPC_E_ARG;
  if (!d_ws || ((uintptr_t)d_ws & 255)) {
    reject(c, n, -1, 0);
    return LOPC_E_ARG;
  }
  int bad;
  int st = make_plan(op, n, jobs, (uintptr_t)d_ws, c->tile2, c->tile3, P, &bad);
  if (st) {
    reject(c, n, bad, st);
    return st;
  }
  if (ws_bytes < P.total) {
    reject(c, n, -1, 0);
    return LOPC_E_ARG;
  }
  HIP_CTX(c, hipSetDevice(c->device));
  return upload_plan(c, P, (uint8_t*)d_ws, s);
}

}  // namespace

extern "C" {

int lopc_batch_workspace_size(lopc_ctx* ctx, int op, int n, const lopc_job* jobs,
                              size_t* bytes) {
  if (!bytes || (op != 0 && op != 1)) return LOPC_E_ARG;
  (void)ctx;
  // the largest over every tile shape, as lopc_workspace_size
  size_t b = 0;
  for (int t2 = 0; t2 < (op == 0 ? kTiles2 : 1); ++t2)
    for (int t3 = 0; t3 < (op == 0 ? kTiles3 : 1); ++t3) {
      Plan P;
      int bad;
      int st = make_plan(op, n, jobs, 0, t2, t3, P, &bad);
      if (st) return st;
      b = std::max(b, (size_t)P.total);
    }
  *bytes = b;
  return LOPC_OK;
}

int lopc_compress_batch(lopc_ctx* ctx, int n, const lopc_job* jobs, void* d_ws,
                        size_t ws_bytes, void* stream, lopc_batch_stats* h_stats) {
  hipStream_t hs = (hipStream_t)stream;
  Plan P;
  if (int st = batch_common(ctx, 0, n, jobs, d_ws, ws_bytes, hs, P)) return st;
  uint8_t* ws = (uint8_t*)d_ws;
  const int K = ctx->graph_sweeps ? ctx->graph_sweeps : ctx->sweeps_hint;
  int graph = 0;
  if (int st = run_sequence(ctx, 0, ws, P.desc, P.gmask, K, hs, &graph)) return st;
  if (int st = read_back(ctx, P, ws, n, hs)) return st;
  const BatchCounters* hc = host_counters(ctx);
  if (hc->err) return LOPC_E_INTERNAL;
  uint64_t sweeps = 1, active = P.tiles;
  for (int t = 1; t <= K; ++t) {
    const uint32_t m = hc->lens[t % kRing];
    if (!m) break;
    ++sweeps;
    active += m;
  }
  bool continued = false;
  std::vector<char> redo(P.jobs.size(), 0);  // plan positions to compress on their own
  if (hc->lens[(K + 1) % kRing]) {
    // the captured sweeps did not reach the fixed point: keep sweeping with
    // direct launches (reading the ring once per group of sweeps), then
    // encode again
    continued = true;
    BatchCounters* bc = P.desc.bc;
    const BatchDesc* bd = (const BatchDesc*)ws;
    const Job* dj = (const Job*)(ws + sizeof(BatchDesc));
    uint32_t next = (uint32_t)K + 1, batch = 2;
    for (;;) {
      // slots of sweeps past the ring length hold counts read long ago
      for (uint32_t t = next; t <= next + batch; ++t) {
        if (t >= kRing && t > next) HIP_CTX(ctx, hipMemsetAsync(&bc->lens[t % kRing], 0, 4, hs));
        if (t >= kRing && t < next + batch)
          HIP_CTX(ctx, hipMemsetAsync(&bc->cursors[t % kRing], 0, 4, hs));
      }
      for (uint32_t b = 0; b < batch; ++b) {
        if (ctx->persist_pct > 0)
          HIP_CTX(ctx, launch_repair_p(ctx->tile2, ctx->tile3, bd, dj, next + b,
                                       grid_of(ctx, PK_REPAIR), hs));
        else
          HIP_CTX(ctx, launch_repair_d(ctx->tile2, ctx->tile3, bd, dj, next + b, P.desc.tiles,
                                       hs));
      }
      if (int st = read_back(ctx, P, ws, n, hs)) return st;
      hc = host_counters(ctx);
      if (hc->err) return LOPC_E_INTERNAL;
      bool done = false;
      for (uint32_t t = next; t <= next + batch; ++t) {
        const uint32_t m = hc->lens[t % kRing];
        if (!m) {
          done = true;
          break;
        }
        if (t < next + batch) {
          ++sweeps;
          active += m;
        }
      }
      if (done) break;
      next += batch;
      batch = std::min<uint32_t>(batch * 2, 16);
      if (next + batch > kAutoSweeps) {
        // a dependency chain across many tiles (every sweep reruns nearly
        // every tile of its field): the fields that still have tiles listed
        // for sweep `next` are compressed again on their own below, where
        // the repair restarts on the device queue
        std::vector<uint32_t> items(hc->lens[next % kRing]);
        if (!items.empty()) {
          HIP_CTX(ctx, hipMemcpyAsync(items.data(), P.desc.lists + (next & 1) * P.desc.tiles,
                                      items.size() * 4, hipMemcpyDeviceToHost, hs));
          HIP_CTX(ctx, hipStreamSynchronize(hs));
        }
        for (uint32_t it : items) {
          int lo = 0, hi = (int)P.jobs.size() - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (P.jobs[mid].t0 <= it) lo = mid;
            else hi = mid - 1;
          }
          redo[lo] = 1;
        }
        break;
      }
    }
    // encoder state is still clear (the gated encoders did not run)
    for (int d = 0; d < 2; ++d) {
      if (!(P.gmask & (d ? 12u : 3u))) continue;
      if (ctx->persist_pct > 0)
        HIP_CTX(ctx, launch_encode_p(d, bd, dj, 0, grid_of(ctx, PK_ENCODE), hs));
      else
        HIP_CTX(ctx, launch_encode_d(d, bd, dj, 0, items(P.desc, PH_C, 2 * d, 2 * d + 2), hs));
    }
    HIP_CTX(ctx, launch_finalize_c(bd, dj, 0, hs));
    if (int st = read_back(ctx, P, ws, n, hs)) return st;
    if (!ctx->graph_sweeps) {
      int h = 16;
      while (h < (int)sweeps + 1 && h < kMaxGraphSweeps) h *= 2;
      ctx->sweeps_hint = std::min(h, kMaxGraphSweeps);
    }
  }
  // fields left to compress on their own: the batch workspace (no longer
  // needed, and at least as large as any field's own workspace) serves the
  // single-field call, which writes the field's stream, size and status
  // words; its results replace the batch's
  BatchResult* hr = (BatchResult*)host_results(ctx);
  for (size_t q = 0; q < redo.size(); ++q) {
    if (!redo[q]) continue;
    const lopc_job& j = jobs[P.order[q]];
    const int saved = ctx->repair_mode;
    ctx->repair_mode = LOPC_REPAIR_AUTO;
    size_t size = 0;
    lopc_stats st1;
    const int rc = lopc_compress(ctx, j.d_in, j.dtype, j.ndim, j.dims, j.error_bound, j.mode,
                                 j.d_out, j.out_cap, &size, j.d_out_size, j.d_status, d_ws,
                                 ws_bytes, stream, &st1);
    ctx->repair_mode = saved;
    if (rc == LOPC_E_HIP || rc == LOPC_E_ARG) return rc;
    hr[q].size = size;
    hr[q].status = rc;
    std::memset(hr[q].header, 0, kHeaderBytes);
    if (rc == LOPC_OK) std::memcpy(hr[q].header, ctx->last_header, kHeaderBytes);
    sweeps = std::max<uint64_t>(sweeps, st1.repair_sweeps);
    active += st1.active_tiles_total;
  }
  if (h_stats) {
    h_stats->repair_sweeps = sweeps;
    h_stats->active_tiles_total = active;
    uint64_t it = 0;
    for (int q = 0; q < 64; ++q) it += host_counters(ctx)->relax_iters[q];
    h_stats->relax_iterations = it;
    h_stats->graph = graph;
    h_stats->continued = continued ? 1 : 0;
  }
  return collect(ctx, P, n);
}

int lopc_decompress_batch(lopc_ctx* ctx, int n, const lopc_job* jobs, void* d_ws,
                          size_t ws_bytes, void* stream) {
  hipStream_t hs = (hipStream_t)stream;
  Plan P;
  if (int st = batch_common(ctx, 1, n, jobs, d_ws, ws_bytes, hs, P)) return st;
  uint8_t* ws = (uint8_t*)d_ws;
  int graph = 0;
  if (int st = run_sequence(ctx, 1, ws, P.desc, P.gmask, 0, hs, &graph)) return st;
  if (int st = read_back(ctx, P, ws, n, hs)) return st;
  return collect(ctx, P, n);
}

int lopc_ctx_last_batch(lopc_ctx* ctx, int n, uint64_t* h_sizes, int32_t* h_status) {
  if (!ctx || n < 0 || (size_t)n != ctx->last_sizes.size()) return LOPC_E_ARG;
  for (int i = 0; i < n; ++i) {
    if (h_sizes) h_sizes[i] = ctx->last_sizes[i];
    if (h_status) h_status[i] = ctx->last_status[i];
  }
  return LOPC_OK;
}

int lopc_batch_autotune(lopc_ctx* ctx, int op, int n, const lopc_job* jobs, void* d_ws,
                        size_t ws_bytes, void* stream, int reps, int* h_pct) {
  if (!ctx || (op != 0 && op != 1) || reps < 1 || n < 1 || !jobs) return LOPC_E_ARG;
  static const int kCand[] = {0, 50, 100, 200};
  // tile shapes matter to compression only, and only for the kinds of field
  // present; a shape whose workspace exceeds ws_bytes is skipped
  bool has2 = false, has3 = false;
  for (int i = 0; i < n; ++i) (group_of(jobs[i]) & 1 ? has3 : has2) = true;
  const int n2 = op == 0 && has2 ? kTiles2 : 1, n3 = op == 0 && has3 ? kTiles3 : 1;
  const int keep_pct = ctx->persist_pct, keep2 = ctx->tile2, keep3 = ctx->tile3;
  int best_pct = keep_pct, best2 = keep2, best3 = keep3;
  double best_t = 1e300;
  for (int i2 = 0; i2 < n2; ++i2) {
    for (int i3 = 0; i3 < n3; ++i3) {
      const int t2 = n2 > 1 ? i2 : keep2, t3 = n3 > 1 ? i3 : keep3;
      if (op == 0) {
        Plan P;
        int bad;
        if (make_plan(op, n, jobs, 0, t2, t3, P, &bad) != LOPC_OK || P.total > ws_bytes)
          continue;
      }
      ctx->tile2 = t2;
      ctx->tile3 = t3;
      for (int pct : kCand) {
        ctx->persist_pct = pct;
        // one call to capture (or warm) this configuration, then the timed ones
        double t = 0.0;
        for (int r = 0; r <= reps; ++r) {
          auto t0 = std::chrono::steady_clock::now();
          int st = op == 0 ? lopc_compress_batch(ctx, n, jobs, d_ws, ws_bytes, stream, nullptr)
                           : lopc_decompress_batch(ctx, n, jobs, d_ws, ws_bytes, stream);
          auto t1 = std::chrono::steady_clock::now();
          if (st == LOPC_E_ARG || st == LOPC_E_HIP || st == LOPC_E_INTERNAL) {
            ctx->persist_pct = keep_pct;
            ctx->tile2 = keep2;
            ctx->tile3 = keep3;
            return st;
          }
          if (r) t += std::chrono::duration<double>(t1 - t0).count();
        }
        if (t < best_t) {
          best_t = t;
          best_pct = pct;
          best2 = t2;
          best3 = t3;
        }
      }
    }
  }
  ctx->persist_pct = best_pct;
  ctx->tile2 = best2;
  ctx->tile3 = best3;
  if (h_pct) *h_pct = best_pct;
  return LOPC_OK;
}

int lopc_ctx_last_batch_headers(lopc_ctx* ctx, int n, void* h_headers) {
  if (!ctx || !h_headers || n < 0 || (size_t)n != ctx->last_sizes.size()) return LOPC_E_ARG;
  std::memcpy(h_headers, ctx->last_headers.data(), (size_t)n * kHeaderBytes);
  return LOPC_OK;
}

int lopc_ctx_set_option(lopc_ctx* ctx, int option, int64_t value) {
  if (!ctx) return LOPC_E_ARG;
  switch (option) {
    case LOPC_OPT_BATCH_GRAPH:
      if (value != 0 && value != 1) return LOPC_E_ARG;
      ctx->use_graph = (int)value;
      return LOPC_OK;
    case LOPC_OPT_GRAPH_SWEEPS:
      if (value < 0 || value > kMaxGraphSweeps) return LOPC_E_ARG;
      ctx->graph_sweeps = (int)value;
      return LOPC_OK;
    case LOPC_OPT_PERSIST_PCT:
      if (value < 0 || value > 400) return LOPC_E_ARG;
      ctx->persist_pct = (int)value;
      return LOPC_OK;
    case LOPC_OPT_TILE_2D:
      if (value < 0 || value >= kTiles2) return LOPC_E_ARG;
      ctx->tile2 = (int)value;
      return LOPC_OK;
    case LOPC_OPT_TILE_3D:
      if (value < 0 || value >= kTiles3) return LOPC_E_ARG;
      ctx->tile3 = (int)value;
      return LOPC_OK;
    case LOPC_OPT_REPAIR:
      if (value < LOPC_REPAIR_AUTO || value > LOPC_REPAIR_POINTS) return LOPC_E_ARG;
      ctx->repair_mode = (int)value;
      return LOPC_OK;
    case LOPC_OPT_SWEEP_ORDER:
      if (value < 0 || value > 2) return LOPC_E_ARG;
      ctx->sweep_order = (int)value;
      return LOPC_OK;
    default:
      return LOPC_E_ARG;
  }
}

int lopc_ctx_get_option(lopc_ctx* ctx, int option, int64_t* h_value) {
  if (!ctx || !h_value) return LOPC_E_ARG;
  switch (option) {
    case LOPC_OPT_BATCH_GRAPH: *h_value = ctx->use_graph; return LOPC_OK;
    case LOPC_OPT_GRAPH_SWEEPS: *h_value = ctx->graph_sweeps; return LOPC_OK;
    case LOPC_OPT_PERSIST_PCT: *h_value = ctx->persist_pct; return LOPC_OK;
    case LOPC_OPT_TILE_2D: *h_value = ctx->tile2; return LOPC_OK;
    case LOPC_OPT_TILE_3D: *h_value = ctx->tile3; return LOPC_OK;
    case LOPC_OPT_REPAIR: *h_value = ctx->repair_mode; return LOPC_OK;
    case LOPC_OPT_SWEEP_ORDER: *h_value = ctx->sweep_order; return LOPC_OK;
    default: return LOPC_E_ARG;
  }
}

}  // extern "C"
