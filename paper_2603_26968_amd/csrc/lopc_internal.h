// Internal declarations shared by the kernels and the host runtime of
// liblopc.so.  Not part of the public ABI (include/lopc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lopc {

constexpr uint32_t kChunkBytes = 16384;  // 16 kB chunks (Sec. III-B / IV-C)
constexpr uint32_t kHeaderBytes = 64;
constexpr uint32_t kRecordHeaderBytes = 16;
// room for the largest record of a chunk: header + two parts of at most the
// chunk's bytes each
constexpr uint32_t kRecordTailBytes = kRecordHeaderBytes + 2 * kChunkBytes;
constexpr uint32_t kMagic = 0x43504F4Cu;  // "LOPC"
constexpr uint32_t kVersion = 1;
constexpr uint64_t kMaxPoints = 0xFFFFFFFFull;  // subbins kept in 32 bits

// Device status bits, OR-ed into Params::status by any kernel.
enum : uint32_t {
  ST_NONFINITE = 1u,
  ST_BOUND = 2u,
  ST_RANGE = 4u,
  ST_FORMAT = 8u,
  ST_CAPACITY = 16u,
  ST_INTERNAL = 32u,
};

// Per-call parameters and results, at the start of the workspace.
struct alignas(256) Params {
  double eb;          // bound as given
  double eps;         // absolute bound applied
  double inv;         // smallest binary64 with inv * eps >= 1
  double winv;        // 1 / inv rounded (only a starting point for walks)
  uint32_t status;    // ST_* bits
  uint32_t ticket;    // chunk ticket counter of the encoder
  uint64_t stream_size;
  uint64_t bins_bytes;
  uint64_t sub_bytes;
  int64_t kmin, kmax;  // order keys of the smallest / largest value
  uint32_t mode;
  uint32_t dtype;
  uint8_t header[64];  // copy of the stream header (read back with Params)
};

// A field as a 3D box (a 2D field d0 x d1 is the box 1 x d0 x d1: the same
// neighbours and the same linear indices).
struct Box {
  int32_t nz, ny, nx;
  uint32_t n;  // points
};

// Tile shapes of the repair compiled into the library, chosen per context
// (LOPC_OPT_TILE_2D / LOPC_OPT_TILE_3D): index 0 of each is the default.
// A shape id numbers all of them: 2D shapes 0..1, 3D shapes 2..4.
constexpr int kTiles2 = 2, kTiles3 = 3, kTileShapes = kTiles2 + kTiles3;
constexpr int kTile2[kTiles2][3] = {{1, 32, 64}, {1, 16, 128}};
constexpr int kTile3[kTiles3][3] = {{4, 8, 32}, {8, 8, 32}, {8, 16, 16}};

// Repair tiling.
struct Tiling {
  int32_t tz, ty, tx;     // tile extent
  int32_t ntz, nty, ntx;  // tiles per axis
  uint32_t ntiles;
  int32_t sid;            // shape id (see kTile2 / kTile3)
  uint8_t* lev;           // per point of a 2D field: its level inside its
                          // tile (255: unknown), kept by the first pass;
                          // null: not kept
  int32_t coloured;       // host-driven sweeps in checkerboard order
};

// Run the statements after t with TZ, TY, TX the compile-time extents of
// tiling t's shape.
#define LOPC_WITH_TILE(t, ...)                                                  \
  do {                                                                          \
    switch ((t).sid) {                                                          \
      case 0: { constexpr int TZ = 1, TY = 32, TX = 64; __VA_ARGS__; } break;   \
      case 1: { constexpr int TZ = 1, TY = 16, TX = 128; __VA_ARGS__; } break;  \
      case 2: { constexpr int TZ = 4, TY = 8, TX = 32; __VA_ARGS__; } break;    \
      case 3: { constexpr int TZ = 8, TY = 8, TX = 32; __VA_ARGS__; } break;    \
      default: { constexpr int TZ = 8, TY = 16, TX = 16; __VA_ARGS__; } break;  \
    }                                                                           \
  } while (0)

// ------------------------------------------------------------------ batches
// A batch runs every phase as one persistent launch per (dtype, tile shape)
// group over a batch-wide work-queue of (field, block), (field, tile) or
// (field, chunk) items.  Everything a launch needs is read from device
// memory (the plan below and the job table), so one captured launch sequence
// serves every batch of the same composition and workspace.

// Points per item of the batched min/max pass.
constexpr uint32_t kMinmaxSpan = 16384;
// Work-list ring: slot s % 64 holds sweep s.
constexpr uint32_t kRing = 64;
// Single-field repair counters: [0] error flag, [1 + s % 64] tiles marked for
// sweep s (the length of its work list), from [kRelaxWord] 64 64-bit slots of
// relaxation-pass counts, from [kCursorWord] the work-list cursor of sweep s
// at [kCursorWord + s % 64].
constexpr uint32_t kRelaxWord = 66;
constexpr uint32_t kCursorWord = kRelaxWord + 128;
constexpr uint32_t kCounterWords = kCursorWord + 64;
// Sweeps that the hybrid repair runs over work lists before the queue takes
// over (the ring of list lengths must not wrap).
constexpr uint32_t kMaxListSweeps = 48;
// Host-driven sweeps of the default scheduler before it restarts the repair
// on the queue (a dependency chain across this many tiles reruns nearly
// every tile on every sweep).
constexpr uint32_t kAutoSweeps = 64;

// ------------------------------------------------------------- repair queue
// Device-driven repair: tiles whose halo changed are listed in a work queue
// that a persistent grid drains until no tile is listed or running, so the
// fixed point is reached inside one launch, whatever the number of tiles a
// dependency chain crosses.  The ring holds 64-bit slots: high word 2L + 1
// while it holds the item of lap L (low word), 2L when it is free for lap L
// (so zeroed memory is an empty queue); head and tail are tickets.  A tile
// is listed at most once at a time (its state word), so a ring of at least
// as many slots as tiles never overruns.
//
// A tile that already ran in this repair and is taken again while a
// neighbour tile of higher index that it depends on is listed or running
// would only see values about to change: it parks on that tile instead (bit
// of its direction in the neighbour's parked word) and is listed again when
// the neighbour's run ends.  Parking follows strictly increasing tile index,
// so it never forms a cycle; a chain that crosses T tiles then costs about
// 2T tile runs instead of up to T^2 / 2.
// (the words that waiting workers poll sit on cache lines of their own)
struct alignas(256) RepairQueue {
  unsigned long long head;  // tickets taken by workers
  uint8_t pad0[248];
  unsigned long long tail;  // tickets taken by producers
  uint8_t pad1[248];
  int32_t pending;          // tiles listed (queued or parked) or running
  uint8_t pad2[252];
  uint32_t err;             // a wait saw no progress of the queue for kQueueStall
  uint32_t max_depth;       // longest chain of tile runs (first pass = 0)
  unsigned long long runs;  // tile runs of the repair kernel
  unsigned long long parks; // times a taken tile parked
};
// A wait in the repair queue that sees neither tail nor pending move for
// this many wall-clock ticks (100 MHz: 20 s) gives up and flags `err`
// (never expected: it turns a scheduling bug into LOPC_E_INTERNAL instead
// of a kernel that does not end).
constexpr unsigned long long kQueueStall = 2000000000ull;
enum : uint32_t { TS_LISTED = 1u, TS_RUNNING = 2u, TS_RAN = 4u };
struct QueueRef {
  RepairQueue* q;
  unsigned long long* ring;
  uint32_t* st;        // per tile item: TS_* bits (zeroed)
  uint32_t* parked;    // per tile item: directions of the tiles parked on it (zeroed)
  uint32_t* blockers;  // per tile item: higher-index directions it depends on
                       // (bits 14..26 of the 27-direction set; written by the first pass)
  uint32_t* depth;     // per tile item: chain depth it was listed at (max; zeroed)
  uint32_t cap_log2;
};
constexpr uint32_t kNoTile = 0xffffffffu;
// ring slots for `tiles` tile items: the next power of two, at least 64
inline uint32_t queue_cap_log2(uint64_t tiles) {
  uint32_t l = 6;
  while ((1ull << l) < tiles) ++l;
  return l;
}

// group of a field: 2 * dtype + (3D)
constexpr int kGroups = 4;
enum { PH_MM = 0, PH_T = 1, PH_C = 2, PH_N = 3 };

// Counters at the start of a batch workspace (cleared with the rest of the
// zeroed prefix at the start of every batch).
struct alignas(256) BatchCounters {
  uint32_t err;           // relaxation limit hit (never expected)
  uint32_t zero;          // stays 0: the gate of launches that must run
  uint32_t enc_cursor[2];  // encoder tickets per dtype
  uint32_t dec_cursor[2];  // decoder tickets per dtype
  uint32_t pad[2];
  uint32_t lens[kRing];     // tiles listed for sweep s (slot s % 64)
  uint32_t cursors[kRing];  // work-queue cursor of sweep s
  unsigned long long relax_iters[64];  // relaxation passes (slot = tile % 64)
};

// Per-field descriptor.  Items of every phase are numbered batch-wide (jobs
// sorted by group); a field owns [mm0, mm0 + mm_blocks) etc.
struct Job {
  const void* x;         // field to compress
  void* y;               // field to decode into
  uint8_t* stream;       // stream (compress output / decompress input)
  uint64_t cap;          // stream capacity (compress)
  uint64_t stream_size;  // stream size (decompress input)
  uint64_t* out_size;    // caller's result words (may be null)
  int32_t* out_status;
  Box box;
  Tiling tl;
  uint32_t nch;
  int32_t dtype, mode, ndim, mm_blocks;
  int64_t dims[3];
  double eb;
  Params* prm;
  void* bins;
  uint16_t* mask;
  uint32_t* sub;
  uint32_t* stamp;
  uint64_t* lookback;
  uint32_t* parts;
  int64_t* part;      // min/max partials
  uint64_t* offsets;  // record offsets (decompress)
  uint32_t mm0, t0, c0;
};

// Result of one field, read back by the host after the batch.
struct BatchResult {
  uint64_t size;   // stream bytes (compress) / field bytes (decompress)
  int32_t status;  // lopc_status
  uint32_t pad;
  uint8_t header[64];  // compress: the stream header
};

// Batch plan: jobs of group g are [job0[g], job0[g + 1]); items of group g in
// phase ph are [item0[ph][g], item0[ph][g + 1]).
// The job table follows the plan in memory.
struct alignas(256) BatchDesc {
  uint32_t job0[kGroups + 1];
  uint32_t item0[PH_N][kGroups + 1];
  uint32_t tiles;        // capacity of each work list
  uint32_t pad;
  uint64_t zero_words;   // 32-bit words cleared at the start of a batch
  uint32_t* zero_base;   // start of the cleared region (bc is its head)
  BatchCounters* bc;
  uint32_t* lists;       // two work lists of `tiles` items (sweep parity)
  BatchResult* res;      // one result per job
};

// index of the job owning batch-wide item `item` of the phase whose
// prefixes start at member `first`, among jobs [lo, hi) (sorted by it; the
// largest index whose prefix is <= item, which skips fields with no items)
template <uint32_t Job::*first>
__device__ __forceinline__ int find_job(const Job* jobs, int lo, int hi, uint32_t item) {
  hi -= 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (jobs[mid].*first <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Timing events of one launch: a receives the kernel's start, b its end,
// both taken from the dispatch itself (hipExtLaunchKernel), so timing adds
// no packet between kernels; null = not recorded.
struct Ev {
  hipEvent_t a = nullptr, b = nullptr;
};

// Launchers (lopc_kernels.hip).  All enqueue on `s` and return the HIP
// status of the last launch.  launch_minmax also clears zero_bytes (a
// multiple of 16) at zero.
hipError_t launch_minmax(int dtype, const void* x, uint32_t n, double* part,
                         int nblocks, void* zero, size_t zero_bytes, hipStream_t s, Ev ev = {});
hipError_t launch_params(int dtype, int mode, double eb, const double* part,
                         int nblocks, Params* prm, uint8_t* stream,
                         size_t cap, int ndim, const int64_t* dims,
                         hipStream_t s, Ev ev = {});
// Q.q null: marks tiles for host-driven sweeps (launch_repair); else lists
// them in the repair queue drained by launch_repair_q.
// lists (may be null): the marked tiles are also appended to the work list
// of sweep 1.  coloured (host-driven sweeps only): two launches, the tiles
// of the second checkerboard colour taking the results of the first as
// their halo.
hipError_t launch_tile0(int dtype, const void* x, Box box, Tiling t, Params* prm, void* bins,
                        uint16_t* mask, uint32_t* sub, uint32_t* stamp,
                        uint32_t* counters, uint32_t* lists, const QueueRef& Q, hipStream_t s,
                        Ev ev = {}, bool coloured = false);
// One sweep over the work list of sweep `sweep` (lists: two arrays of
// t.ntiles items, sweep parity), appending the tiles it marks to the list
// of the next sweep; a persistent grid of `grid` workgroups drains the list.
hipError_t launch_sweep_list(Box box, Tiling t, const uint16_t* mask, uint32_t* sub,
                             uint32_t* stamp, uint32_t* counters, uint32_t* lists,
                             uint32_t sweep, int grid, hipStream_t s, Ev ev = {});
int sweep_list_blocks_per_cu(int sid);
// Lists the tiles of the work list of sweep `sweep` in the repair queue.
hipError_t launch_seed_queue(const uint32_t* counters, const uint32_t* lists, uint32_t ntiles,
                             uint32_t sweep, const QueueRef& Q, hipStream_t s);
// Device-driven repair over the queue filled by launch_tile0 (grid: the
// resident capacity, repair_q_blocks_per_cu per CU).
hipError_t launch_repair_q(Box box, Tiling t, const uint16_t* mask, uint32_t* sub,
                           uint32_t* counters, const QueueRef& Q, int grid, hipStream_t s,
                           Ev ev = {});
int repair_q_blocks_per_cu(int sid);
// Writes the stream size (0 after a failure other than capacity) and the
// lopc_status code of a compression to the caller's device words (either
// may be null); q (may be null): its repair queue.
hipError_t launch_report(const Params* prm, const RepairQueue* q, uint64_t* d_size,
                         int32_t* d_status, hipStream_t s);
// Host-driven sweeps of a field with many tiles run in checkerboard order
// by default (two launches per sweep and for the first pass: fewer sweeps
// and tile runs); on smaller fields the second launch costs more than it
// saves.
constexpr uint32_t kColourMinTiles = 32768;

// One host-driven sweep: the tiles marked for `sweep`; with t.coloured,
// in two launches by tile colour (checkerboard), so that a tile of the
// second colour sees the changes of its face and corner neighbours in the
// same sweep.  Ev: start of the first launch, end of the last.
hipError_t launch_repair(Box box, Tiling t, const uint16_t* mask,
                         uint32_t* sub, uint32_t* stamp, uint32_t* counters,
                         uint32_t sweep, hipStream_t s, Ev ev = {});
// Point worklists (LOPC_REPAIR_POINTS): list every point with flags for
// iteration 0 (its length in ring[0]); one iteration `it` over the list win
// (length ring[it % 64]) appending to wout (length ring[(it + 1) % 64]).
// Grid-stride kernels of `grid` workgroups.
hipError_t launch_point_seed(const uint16_t* mask, uint32_t n, uint32_t* wl, uint32_t* ring,
                             int grid, hipStream_t s, Ev ev = {});
hipError_t launch_point_iter(Box box, const uint16_t* mask, uint32_t* sub, const uint32_t* win,
                             uint32_t* wout, uint32_t* ring, uint32_t* pstamp, uint32_t it,
                             int grid, hipStream_t s, Ev ev = {});
// Encoder of a single field: encodes every chunk, parking its record in the
// chunk's rows of bins / sub / mask (which it overwrites) or, for the last
// chunk, in tail (kRecordTailBytes); then the record offsets (into offs, one
// per chunk) and the placement into the stream.  Ev: start of the first
// kernel, end of the last.
hipError_t launch_encode(int dtype, uint32_t n, const void* bins, uint32_t* sub,
                         uint16_t* mask, uint8_t* tail, uint64_t* offs, uint32_t* parts,
                         Params* prm, uint8_t* stream, size_t cap, const uint32_t* gate,
                         hipStream_t s, Ev ev = {});
hipError_t launch_sum_parts(const uint32_t* parts, uint32_t nch, Params* prm,
                            hipStream_t s);
hipError_t launch_offsets(const uint8_t* stream, uint32_t nch,
                          uint64_t body_bytes, uint64_t* offsets,
                          Params* prm, hipStream_t s, Ev ev = {});
hipError_t launch_decode(int dtype, const uint8_t* stream, uint32_t n,
                         const uint64_t* offsets, Params* prm, void* field,
                         hipStream_t s, Ev ev = {});

// Batch launchers (persistent grids; `grid` blocks drain the queue).  Every
// launch reads the plan `bd` and the job table `jobs` that follows it.
// `gate_sweep` > 0: skip unless no tile was listed for that sweep.
hipError_t launch_zero_p(const BatchDesc* bd, int grid, hipStream_t s);
hipError_t launch_zero_n(uint32_t* words, uint64_t nwords, hipStream_t s, Ev ev = {});
hipError_t launch_minmax_p(int dtype, const BatchDesc* bd, const Job* jobs, int grid,
                           hipStream_t s);
hipError_t launch_params_p(int dtype, const BatchDesc* bd, const Job* jobs, int grid,
                           hipStream_t s);
// t2 / t3: the batch's 2D and 3D tile shape indices (kTile2 / kTile3)
hipError_t launch_tile0_p(int group, int t2, int t3, const BatchDesc* bd, const Job* jobs,
                          int grid, hipStream_t s);
hipError_t launch_repair_p(int t2, int t3, const BatchDesc* bd, const Job* jobs, uint32_t sweep,
                           int grid, hipStream_t s);
hipError_t launch_encode_p(int dtype, const BatchDesc* bd, const Job* jobs, int gate_sweep,
                           int grid, hipStream_t s);
hipError_t launch_finalize_c(const BatchDesc* bd, const Job* jobs, int gate_sweep,
                             hipStream_t s);
hipError_t launch_dhead_p(const BatchDesc* bd, const Job* jobs, int grid, hipStream_t s);
hipError_t launch_decode_p(int dtype, const BatchDesc* bd, const Job* jobs, int grid,
                           hipStream_t s);
hipError_t launch_finalize_d(const BatchDesc* bd, const Job* jobs, hipStream_t s);

// Direct-grid variants: one workgroup per item; `items` is the phase's item
// count of the launch's groups (the repair: the work-list capacity).
hipError_t launch_minmax_d(int dtype, const BatchDesc* bd, const Job* jobs, uint32_t items,
                           hipStream_t s);
hipError_t launch_params_d(int dtype, const BatchDesc* bd, const Job* jobs, uint32_t njobs,
                           hipStream_t s);
hipError_t launch_tile0_d(int group, int t2, int t3, const BatchDesc* bd, const Job* jobs,
                          uint32_t items, hipStream_t s);
hipError_t launch_repair_d(int t2, int t3, const BatchDesc* bd, const Job* jobs, uint32_t sweep,
                           uint32_t tiles, hipStream_t s);
hipError_t launch_encode_d(int dtype, const BatchDesc* bd, const Job* jobs, int gate_sweep,
                           uint32_t items, hipStream_t s);
hipError_t launch_decode_d(int dtype, const BatchDesc* bd, const Job* jobs, uint32_t items,
                           hipStream_t s);

// Library-held scratch of lopc_decompress_static (lopc_static.hip): Params
// and the record offsets of up to kStaticMaxChunks chunks.  Its address on
// the current device (the host-side name of the array is not a device
// address and must never be passed to a kernel).
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
hipError_t static_scratch_address(void** ptr);

// Invariant checker (lopc_verify.hip): adds 14 report words to out.
hipError_t launch_verify(int dtype, const void* x, const void* y, Box box, double eps,
                         unsigned long long* out, int blocks, hipStream_t s);

// Resident blocks per CU of each persistent batch kernel (occupancy query).
enum { PK_ZERO, PK_MINMAX, PK_PARAMS, PK_TILE0, PK_REPAIR, PK_ENCODE, PK_DHEAD,
       PK_DECODE, PK_COUNT };
int batch_blocks_per_cu(int kernel);
int codec_blocks_per_cu(int kernel);

}  // namespace lopc
