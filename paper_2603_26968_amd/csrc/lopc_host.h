// lopc_host.h -- host-side internals of liblopc.so shared by the single-field
// calls (lopc_api.cpp) and the batch calls (lopc_batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/lopc.h"
#include "lopc_internal.h"

// A captured batch launch sequence.
struct BatchGraph {
  int op;              // 0 compress, 1 decompress
  const void* ws;      // workspace it was captured on
  uint32_t gmask;      // groups present
  int sweeps;          // repair sweeps captured (compress)
  int grid_pct;        // persistent grid size it was captured with (0: direct)
  int tile2, tile3;    // tile shapes it was captured with
  uint32_t job0[lopc::kGroups + 1];             // direct grids: the batch shape
  uint32_t item0[lopc::PH_N][lopc::kGroups + 1];
  uint32_t tiles;
  uint64_t used;       // last use (for eviction)
  hipGraphExec_t exec;
};

struct lopc_ctx {
  int device;
  int num_cu;
  // pinned host slots for small device-to-host reads
  lopc::Params* h_prm;
  uint32_t* h_cnt;
  // header of the most recent successful compression
  uint8_t last_header[64];
  int have_header;
  // last HIP failure (for diagnostics)
  int hip_error;
  char hip_where[64];
  int sync_check;  // LOPC_SYNC_CHECK=1: synchronise after every launch
  // phase timing
  int timing;
  hipEvent_t ev[2 * LOPC_PHASES];  // per phase: first kernel's start, last kernel's end
  double ms[LOPC_PHASES];
  int sweep_hint;      // single field: repair sweeps enqueued before the first read
  int repair_mode;     // single field: LOPC_REPAIR_HYBRID, _QUEUE or _SWEEPS
  int sweep_order;     // single field, host-driven sweeps: LOPC_OPT_SWEEP_ORDER
  int rq_per_cu[lopc::kTileShapes];  // resident repair-queue workgroups per CU, per tile shape
  int sl_per_cu[lopc::kTileShapes];  // resident list-sweep workgroups per CU, per tile shape
  int tile2, tile3;    // tile shape indices (kTile2 / kTile3)
  void* scratch;       // device address of the library-held scratch on this device
  // batches
  int use_graph;       // capture batch sequences as graphs
  int graph_sweeps;    // sweeps per graph (0 = adaptive)
  int sweeps_hint;     // adaptive capture size
  int persist_pct;     // persistent grid size, % of resident capacity; 0: direct grids
  int per_cu[lopc::PK_COUNT];  // resident blocks per CU (0 = not queried)
  hipStream_t cap_stream;      // stream used for captures
  void* h_plan;        // pinned staging of the plan + job table
  size_t h_plan_cap;
  void* h_back;        // pinned read-back of counters + results
  size_t h_back_cap;
  uint64_t use_clock;
  std::vector<BatchGraph> graphs;
  std::vector<uint64_t> last_sizes;
  std::vector<int32_t> last_status;
  std::vector<uint8_t> last_headers;  // 64 bytes per job (compress batches)
};

namespace lopc_host {
using namespace lopc;

constexpr int kMinmaxBlocks = 1024;

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Shape {
  int ndim;
  int64_t d[3];  // as given (2D: d[2] = 1)
  uint64_t n;
  Box box;
};

inline int make_shape(int ndim, const int64_t* dims, Shape* s) {
  if ((ndim != 2 && ndim != 3) || !dims) return LOPC_E_ARG;
  s->ndim = ndim;
  uint64_t n = 1;
  for (int i = 0; i < 3; ++i) {
    int64_t v = i < ndim ? dims[i] : 1;
    if (v < 1 || v > (int64_t)kMaxPoints) return LOPC_E_ARG;
    s->d[i] = v;
    n *= (uint64_t)v;
    if (n > kMaxPoints) return LOPC_E_ARG;
  }
  s->n = n;
  if (ndim == 2) {
    s->box.nz = 1;
    s->box.ny = (int32_t)s->d[0];
    s->box.nx = (int32_t)s->d[1];
  } else {
    s->box.nz = (int32_t)s->d[0];
    s->box.ny = (int32_t)s->d[1];
    s->box.nx = (int32_t)s->d[2];
  }
  s->box.n = (uint32_t)n;
  return LOPC_OK;
}

// t2 / t3: the 2D and 3D tile shape indices (kTile2 / kTile3)
inline Tiling make_tiling(const Box& b, int t2, int t3) {
  Tiling t;
  const int* e = b.nz == 1 ? kTile2[t2] : kTile3[t3];
  t.tz = e[0]; t.ty = e[1]; t.tx = e[2];
  t.sid = b.nz == 1 ? t2 : kTiles2 + t3;
  t.ntz = (b.nz + t.tz - 1) / t.tz;
  t.nty = (b.ny + t.ty - 1) / t.ty;
  t.ntx = (b.nx + t.tx - 1) / t.tx;
  t.ntiles = (uint32_t)t.ntz * t.nty * t.ntx;
  t.lev = nullptr;
  t.coloured = 0;
  return t;
}

struct CompressLayout {
  size_t prm, counters, queue, stamp, qstate, parked, depth, ring, zero_end;  // zeroed prefix
  size_t blockers, lists, offs, parts, part, bins, mask, sub, lev, tail, total;
  size_t pw0, pw1, pstamp;  // point worklists and stamps (LOPC_REPAIR_POINTS; else 0)
  uint32_t cap_log2;  // repair queue ring: 2^cap_log2 slots
};

// repair counters (kCounterWords words): [0] internal error flag,
// [1 + s % 64] tiles marked for sweep s (a ring the host clears after
// reading), [kRelaxWord] 64-bit relaxation iteration total

inline CompressLayout compress_layout(const Shape& s, int dtype, int t2, int t3,
                                      bool points = false) {
  const size_t k = dtype == 0 ? 4 : 8;
  const uint64_t W = kChunkBytes / k;
  const uint64_t nch = (s.n + W - 1) / W;
  Tiling t = make_tiling(s.box, t2, t3);
  CompressLayout L;
  size_t o = 0;
  L.cap_log2 = queue_cap_log2(t.ntiles);
  L.prm = o; o += align256(sizeof(Params));
  L.counters = o; o += align256(kCounterWords * 4);
  L.queue = o; o += align256(sizeof(RepairQueue));
  L.stamp = o; o += align256((size_t)t.ntiles * 4);
  L.qstate = o; o += align256((size_t)t.ntiles * 4);
  L.parked = o; o += align256((size_t)t.ntiles * 4);
  L.depth = o; o += align256((size_t)t.ntiles * 4);
  L.ring = o; o += align256((size_t)8 << L.cap_log2);
  static_assert(align256(sizeof(Params)) + align256(kCounterWords * 4) + sizeof(RepairQueue) <= 4096,
                "the compress report fits its pinned host slot");
  L.zero_end = o;
  L.blockers = o; o += align256((size_t)t.ntiles * 4);
  L.lists = o; o += align256((size_t)t.ntiles * 8);
  L.offs = o; o += align256(nch * 8);
  L.parts = o; o += align256(nch * 8);
  L.part = o; o += align256(16 * kMinmaxBlocks);
  L.bins = o; o += align256(s.n * k);
  L.mask = o; o += align256(s.n * 2);
  L.sub = o; o += align256(s.n * 4);
  L.lev = o; o += align256(s.box.nz == 1 ? s.n : 0);
  L.tail = o; o += align256(kRecordTailBytes);
  L.pw0 = L.pw1 = L.pstamp = 0;
  if (points) {
    L.pw0 = o; o += align256(s.n * 4);
    L.pw1 = o; o += align256(s.n * 4);
    L.pstamp = o; o += align256(s.n * 4);
  }
  L.total = o;
  return L;
}

inline size_t decompress_ws(const Shape& s, int dtype) {
  const size_t k = dtype == 0 ? 4 : 8;
  const uint64_t W = kChunkBytes / k;
  const uint64_t nch = (s.n + W - 1) / W;
  return align256(sizeof(Params)) + align256(nch * 8);
}

inline int status_code(uint32_t st) {
  if (st & ST_NONFINITE) return LOPC_E_NONFINITE;
  if (st & ST_BOUND) return LOPC_E_BOUND;
  if (st & ST_RANGE) return LOPC_E_RANGE;
  if (st & ST_FORMAT) return LOPC_E_FORMAT;
  if (st & ST_INTERNAL) return LOPC_E_INTERNAL;
  if (st & ST_CAPACITY) return LOPC_E_CAPACITY;
  return LOPC_OK;
}

#define HIP_TRY(expr)                         \
  do {                                        \
    if ((expr) != hipSuccess) return LOPC_E_HIP; \
  } while (0)

// like HIP_TRY, but records the error and the call site in the context
#define HIP_CTX(c, expr)                                              \
  do {                                                                \
    hipError_t e_ = (expr);                                           \
    if (e_ == hipSuccess && (c)->sync_check) e_ = hipDeviceSynchronize(); \
    if (e_ != hipSuccess) {                                           \
      (c)->hip_error = (int)e_;                                       \
      std::strncpy((c)->hip_where, #expr, sizeof((c)->hip_where) - 1); \
      return LOPC_E_HIP;                                              \
    }                                                                 \
  } while (0)

// timing events for the kernels of phase p (none unless timing is on):
// the first kernel of the phase records its start, the last its end
inline bool timed(const lopc_ctx* c, int p) { return (c->timing >> p) & 1; }
inline Ev ev_first(lopc_ctx* c, int p) { return timed(c, p) ? Ev{c->ev[2 * p], nullptr} : Ev{}; }
inline Ev ev_last(lopc_ctx* c, int p) { return timed(c, p) ? Ev{nullptr, c->ev[2 * p + 1]} : Ev{}; }
inline Ev ev_only(lopc_ctx* c, int p) {
  return timed(c, p) ? Ev{c->ev[2 * p], c->ev[2 * p + 1]} : Ev{};
}
// ms of phase p (after the stream has drained; 0 unless timed)
inline double phase_ms(lopc_ctx* c, int p) {
  float ms = 0.f;
  if (!timed(c, p)) return 0.0;
  if (hipEventElapsedTime(&ms, c->ev[2 * p], c->ev[2 * p + 1]) != hipSuccess) return 0.0;
  return (double)ms;
}

inline uint64_t rd_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i);
  return v;
}
inline uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
         ((uint32_t)p[3] << 24);
}
inline double rd_f64(const uint8_t* p) {
  uint64_t u = rd_u64(p);
  double d;
  std::memcpy(&d, &u, 8);
  return d;
}

}  // namespace lopc_host
