/*
 * lopc.h -- C ABI of liblopc.so, a GPU (AMD MI355X, gfx950) implementation of
 * the compress and decompress path of LOPC, the Local-Order-Preserving
 * Compressor (Fallin et al., arXiv 2603.26968).
 *
 * What a stream holds (paper sections in brackets):
 *   - every value x is mapped to an integer bin, the nearest integer to
 *     x / eps with eps the absolute error bound (ABS) or eb * (max - min)
 *     (NOA) [Sec. IV-A];
 *   - every point gets a subbin, the least integer solution of
 *       s(p) = max(0, max over same-bin neighbours n below p of
 *                     s(n) + [index(n) > index(p)])
 *     so that decoding preserves the order of every pair of neighbours, ties
 *     broken by index [Sec. IV-B, Alg. 1, Alg. 2, Sec. IV-E];
 *   - bins are stored as DIFFNB_k BIT_k RZE_1 and subbins as BIT_k RZE_k RZE_1
 *     in independent 16 kB chunks [Sec. III-B, Sec. IV-C];
 *   - decompression maps (bin, subbin) to the subbin-th representable value
 *     above the lowest value of the bin [Sec. IV-E].
 * The byte layout of the container is this library's own (the paper gives
 * none); it is identical to the CPU oracle's, byte for byte.
 *
 * Conventions for every call:
 *   - fields are C-order arrays (last axis fastest) of float32 or float64 with
 *     ndim = 2 or 3 and fewer than 2^32 points; the index that breaks ties is
 *     the linear offset;
 *   - pointers prefixed d_ are device memory, h_ host memory; every buffer is
 *     owned by the caller; the library never allocates device memory in the
 *     compress/decompress calls (scratch lives in the caller's workspace);
 *   - `stream` is a hipStream_t (NULL = default stream); all device work is
 *     ordered on it; the calls below block until their own work on that
 *     stream is done (they return sizes and status codes to the host),
 *     except lopc_compress called with h_stream_size = NULL, which only
 *     enqueues its work and reports on the device;
 *   - return value: LOPC_OK (0) or a negative lopc_status; arguments are
 *     validated before any launch; on error the output buffers hold
 *     unspecified bytes but nothing outside them is written;
 *   - alignment: a field to compress must start on a 16-byte boundary, a
 *     stream on a 4-byte boundary, a field to decode into on its element
 *     size, a workspace on a 256-byte boundary (torch allocations are);
 *   - a context may be used by one host thread at a time.
 */
#ifndef LOPC_H
#define LOPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { LOPC_F32 = 0, LOPC_F64 = 1 } lopc_dtype;

/* Error-bound mode [Sec. IV-A]: ABS bounds |x - x'| by error_bound; NOA by
 * error_bound * (max(x) - min(x)). */
typedef enum { LOPC_EB_ABS = 0, LOPC_EB_NOA = 1 } lopc_eb_mode;

typedef enum {
  LOPC_OK = 0,
  LOPC_E_ARG = -1,       /* bad pointer, shape, dtype, mode or workspace     */
  LOPC_E_NONFINITE = -2, /* NaN or Inf in the field                          */
  LOPC_E_BOUND = -3,     /* bound not finite and > 0, or NOA on zero range   */
  LOPC_E_RANGE = -4,     /* a bin does not fit (|b| > 2^31-2 f32, 2^62 f64)  */
  LOPC_E_CAPACITY = -5,  /* output buffer too small (required size returned) */
  LOPC_E_FORMAT = -6,    /* malformed or corrupt stream                      */
  LOPC_E_HIP = -7,       /* a HIP runtime call failed                        */
  LOPC_E_NOMEM = -8,     /* host allocation failed                           */
  LOPC_E_INTERNAL = -9   /* an internal consistency check failed (a bug)     */
} lopc_status;

typedef struct lopc_ctx lopc_ctx;

/* Optional per-call figures of a compression.  repair_sweeps counts the
 * first pass and every sweep that ran; when the repair queue ran, it is at
 * least 1 + the longest chain of tile runs that listed one another. */
typedef struct {
  double eps;                  /* absolute bound actually applied           */
  uint64_t repair_sweeps;      /* global sweeps of the repair to fixed point */
  uint64_t active_tiles_total; /* tile runs, the first pass included        */
  uint64_t bins_bytes;         /* bytes of all bins parts                   */
  uint64_t subbins_bytes;      /* bytes of all subbin parts                 */
  uint64_t relax_iterations;   /* in-tile relaxation passes, all tiles/sweeps */
  uint64_t queue_runs;         /* tile runs taken from the repair queue      */
  uint64_t queue_parks;        /* times a taken tile parked on another one   */
} lopc_stats;

/* Context for one HIP device: device properties, pinned host slots for the
 * status words.  Returns LOPC_E_HIP if the device cannot be used. */
int lopc_ctx_create(int hip_device, lopc_ctx** out);
void lopc_ctx_destroy(lopc_ctx* ctx);

/* Largest stream compress can produce for this shape (every stage stored
 * verbatim): 64 + 4*chunks + sum over chunks (16 + 2*m*k), m = points of the
 * chunk rounded up to 64, k = 4 (f32) or 8 (f64). */
int lopc_compress_bound(int dtype, int ndim, const int64_t* dims,
                        size_t* bytes);

/* Device workspace (bytes, 256-byte aligned pointer expected) that
 * lopc_compress (op = 0) or lopc_decompress (op = 1) needs for this shape. */
int lopc_workspace_size(lopc_ctx* ctx, int dtype, int ndim,
                        const int64_t* dims, int op, size_t* bytes);

/* Compress d_field (dtype, ndim, dims) with error_bound under mode into
 * d_stream (capacity stream_cap bytes) [Sec. IV-A to IV-C: quantize, order
 * flags, repair to the least fixed point, lossless stages].
 * d_ws/ws_bytes: workspace of at least lopc_workspace_size(op = 0).
 *
 * Synchronous (h_stream_size != NULL): returns when the stream is complete;
 * *h_stream_size receives the stream size -- also when LOPC_E_CAPACITY is
 * returned, so the caller can retry; h_stats may be NULL.
 *
 * Enqueued (h_stream_size == NULL, d_stream_size required, h_stats NULL):
 * every launch is enqueued on `stream` and the call returns LOPC_OK without
 * waiting (argument errors are still returned at once).  No host memory is
 * touched after the call returns, so the sequence can be captured into a HIP
 * graph; the repair reaches its fixed point on the device (LOPC_E_ARG under
 * LOPC_REPAIR_SWEEPS).
 *
 * In both modes, when given, the device words *d_stream_size (8-byte
 * aligned) and *d_status (4-byte aligned) receive, in stream order, the
 * stream size (also on LOPC_E_CAPACITY; 0 after any other failure) and the
 * call's lopc_status. */
int lopc_compress(lopc_ctx* ctx, const void* d_field, int dtype, int ndim,
                  const int64_t* dims, double error_bound, int mode,
                  void* d_stream, size_t stream_cap, size_t* h_stream_size,
                  uint64_t* d_stream_size, int32_t* d_status,
                  void* d_ws, size_t ws_bytes, void* stream,
                  lopc_stats* h_stats);

/* Parse the 64-byte header of a stream held in host memory (n >= 64).
 * Any output pointer may be NULL.  dims receives 3 values (unused = 1). */
int lopc_stream_info(const void* h_header, size_t n, int* dtype, int* ndim,
                     int64_t* dims, double* eps, size_t* field_bytes);

/* Decompress the stream d_stream (exactly stream_size bytes) into d_field
 * (capacity field_cap bytes).  d_ws/ws_bytes: workspace of at least
 * lopc_workspace_size(op = 1) for the stream's shape. */
int lopc_decompress(lopc_ctx* ctx, const void* d_stream, size_t stream_size,
                    void* d_field, size_t field_cap, void* d_ws,
                    size_t ws_bytes, void* stream);

/* lopc_decompress with the stream's 64-byte header also given in host memory
 * (for a caller that already holds it, e.g. from lopc_ctx_last_header); this
 * saves a device-to-host read.  h_header must equal the first 64 bytes of
 * d_stream: shapes come from h_header, the error-bound parameters from the
 * device copy, so a mismatch gives wrong values (or LOPC_E_FORMAT) but never
 * an access outside the given buffers. */
int lopc_decompress_h(lopc_ctx* ctx, const void* h_header, const void* d_stream,
                      size_t stream_size, void* d_field, size_t field_cap,
                      void* d_ws, size_t ws_bytes, void* stream);

/* lopc_decompress_h for callers that cannot allocate (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): no
 * workspace argument and no allocation of any kind.  Its scratch (the
 * decoder's parameter block and one 8-byte record offset per chunk) is a
 * 4 MiB array held by the library on each GPU until the process ends, so
 * streams of at most 524,256 chunks are accepted (a float32 field of up to
 * about 2.1e9 points, float64 1.07e9); a larger stream returns
 * LOPC_E_CAPACITY before any device work.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other host threads, or
 * other streams) race and must be serialised by the caller.  The array
 * keeps the last call's contents; each call clears what must start at zero.
 * Otherwise as lopc_decompress_h (the same kernels, stream order, checks
 * and status codes). */
int lopc_decompress_static(lopc_ctx* ctx, const void* h_header, const void* d_stream,
                           size_t stream_size, void* d_field, size_t field_cap, void* stream);

/* Copy the 64-byte header of the most recent successful lopc_compress on this
 * context into h_header.  LOPC_E_ARG if there is none. */
int lopc_ctx_last_header(lopc_ctx* ctx, void* h_header);

/* ------------------------------------------------------------------ batches
 * Many independent fields in one call.  Each phase (range, quantize, order
 * flags + first relaxation, each repair sweep, chunk encoder; header check,
 * chunk decoder) is one launch per group of fields with the same dtype and
 * tile shape over a batch-wide work-queue of (field, block), (field, tile)
 * or (field, chunk) items; repair sweeps run over a device work list of the
 * tiles marked by the previous sweep.  Launches are either direct grids (one
 * workgroup per item; the default) or persistent grids that drain the queue
 * (LOPC_OPT_PERSIST_PCT).  The launch sequence reads everything from the
 * workspace; it is captured as a HIP graph once per context, workspace,
 * composition (groups present) and -- for direct grids -- batch shape, and
 * replayed; a batch whose repair needs more sweeps than the graph holds
 * continues with direct launches (and the next capture holds more).
 * Fields never interact: every field's stream equals its lopc_compress
 * stream byte for byte, and every decoded field its lopc_decompress output.
 */
typedef struct {
  const void* d_in;      /* compress: field; decompress: stream              */
  size_t in_bytes;       /* decompress: stream size (compress: ignored)      */
  void* d_out;           /* compress: stream; decompress: field              */
  size_t out_cap;        /* bytes available at d_out                         */
  int dtype;             /* lopc_dtype (decompress: must match the header)   */
  int ndim;              /* 2 or 3 (decompress: must match the header)       */
  int64_t dims[3];       /* unused trailing dims ignored                     */
  double error_bound;    /* compress only                                    */
  int mode;              /* compress only: lopc_eb_mode                      */
  uint64_t* d_out_size;  /* optional device word: stream / field bytes       */
  int32_t* d_status;     /* optional device word: this field's lopc_status   */
} lopc_job;

/* Optional figures of a batch compression. */
typedef struct {
  uint64_t repair_sweeps;      /* sweeps over all fields, first pass included */
  uint64_t active_tiles_total; /* tiles processed over all sweeps             */
  int graph;                   /* 1: the launch sequence was a graph replay   */
  int continued;               /* 1: sweeps beyond the captured ones ran      */
  uint64_t relax_iterations;   /* in-tile relaxation passes, all tiles/sweeps */
} lopc_batch_stats;

/* Workspace bytes a batch of n jobs needs (op 0 = compress, 1 = decompress). */
int lopc_batch_workspace_size(lopc_ctx* ctx, int op, int n, const lopc_job* jobs,
                              size_t* bytes);

/* Compress / decompress n jobs (n >= 1) with workspace d_ws (ws_bytes >=
 * lopc_batch_workspace_size).  Every job is validated before any launch: a
 * bad pointer, shape, dtype, mode or alignment returns LOPC_E_ARG, a bad
 * bound LOPC_E_BOUND, a decompress stream shorter than its table
 * LOPC_E_FORMAT, a decompress field capacity below the field size
 * LOPC_E_CAPACITY, and nothing runs.  Otherwise every field is processed
 * and its size and status are written to d_out_size / d_status (when given)
 * and kept for lopc_ctx_last_batch; the call returns LOPC_OK if every field
 * succeeded, else the status of the first failing job.  Buffers of different
 * jobs must not overlap.  The first batch of a composition on a workspace
 * allocates its graph (owned by the context until it is destroyed). */
int lopc_compress_batch(lopc_ctx* ctx, int n, const lopc_job* jobs, void* d_ws,
                        size_t ws_bytes, void* stream, lopc_batch_stats* h_stats);
int lopc_decompress_batch(lopc_ctx* ctx, int n, const lopc_job* jobs, void* d_ws,
                          size_t ws_bytes, void* stream);

/* Per-job results of the most recent batch call, in job order (n must equal
 * that batch's n; either array may be NULL).  After a call rejected before
 * launch, *h_status of the offending job holds the error and the rest 0. */
int lopc_ctx_last_batch(lopc_ctx* ctx, int n, uint64_t* h_sizes, int32_t* h_status);

/* The 64-byte stream headers of the most recent lopc_compress_batch, in job
 * order (n * 64 bytes into h_headers; zeros for a failed job), e.g. to pass
 * to lopc_decompress_h without reading them back from the streams. */
int lopc_ctx_last_batch_headers(lopc_ctx* ctx, int n, void* h_headers);

/* Autotuner of the batch path: runs the batch (op 0 = compress, 1 =
 * decompress) with direct grids and with persistent grids of 50, 100 and
 * 200 % of the resident capacity and, for compression, with every repair
 * tile shape (LOPC_OPT_TILE_2D / _3D) of the kinds of field in the batch,
 * once untimed and `reps` times timed
 * (host clock around the synchronous call).  It keeps the fastest in the
 * context (LOPC_OPT_PERSIST_PCT, 0 = direct, and the tile options; read them
 * back with lopc_ctx_get_option) and returns the grid percentage in *h_pct
 * (may be NULL).  The outputs are those of an ordinary call.  Errors as
 * lopc_compress_batch; a per-field failure does not stop the tuning. */
int lopc_batch_autotune(lopc_ctx* ctx, int op, int n, const lopc_job* jobs, void* d_ws,
                        size_t ws_bytes, void* stream, int reps, int* h_pct);

/* Context options.
 *   LOPC_OPT_BATCH_GRAPH   1 (default): capture and replay batch launch
 *                          sequences as HIP graphs; 0: direct launches.
 *   LOPC_OPT_GRAPH_SWEEPS  repair sweeps captured in a batch graph (1..62);
 *                          0 (default): adaptive, starting at 16.
 *   LOPC_OPT_PERSIST_PCT   0 (default): direct grids, one workgroup per
 *                          item; 1..400: persistent grids of that percentage
 *                          of the resident capacity, draining the queues (one
 *                          captured graph then serves every batch shape).
 *   LOPC_OPT_REPAIR        scheduler of the single-field repair [Alg. 1
 *                          loop, Sec. IV-B]; every one reaches the same
 *                          least fixed point:
 *                          LOPC_REPAIR_AUTO (default): synchronous calls
 *                          as LOPC_REPAIR_SWEEPS up to 64 sweeps, then the
 *                          repair restarts from its first pass on the queue
 *                          (a dependency chain across that many tiles);
 *                          enqueued calls as LOPC_REPAIR_HYBRID;
 *                          LOPC_REPAIR_HYBRID: K sweeps over device work
 *                          lists of the tiles whose halo changed (K learned
 *                          from the previous call on the context, at most
 *                          48), then a device work queue drained by one
 *                          persistent launch for whatever is still listed;
 *                          LOPC_REPAIR_QUEUE: the work queue alone, from the
 *                          first pass on;
 *                          LOPC_REPAIR_SWEEPS: global sweeps over the marked
 *                          tiles, launched by the host in groups, until no
 *                          tile is marked (not available to enqueued calls);
 *                          LOPC_REPAIR_POINTS: the paper's point worklists
 *                          [Sec. IV-D]: after the first tile pass, every
 *                          point with a same-bin lower neighbour is listed;
 *                          each iteration recomputes the listed points and
 *                          lists, once per iteration (a per-point stamp of
 *                          the last iteration it was listed for), the upper
 *                          neighbours of those that rose, in the other of
 *                          two lists; host-driven like the sweeps (not
 *                          available to enqueued calls).  It needs 12 more
 *                          workspace bytes per point: query
 *                          lopc_workspace_size after setting it.
 *   LOPC_OPT_TILE_3D       tile of the repair of 3D fields (each workgroup
 *                          holds one tile and a one-point halo in LDS):
 *                          0 (default) 4 x 8 x 32, 1: 8 x 8 x 32,
 *                          2: 8 x 16 x 16 points (z, y, x);
 *   LOPC_OPT_TILE_2D       tile of 2D fields: 0 (default) 32 x 64,
 *                          1: 16 x 128.
 *                          Neither the result nor the workspace size
 *                          (the largest over the shapes) depends on them.
 *   LOPC_OPT_SWEEP_ORDER   order of the tiles in the host-driven sweeps of
 *                          the single-field repair: 0 (default) as 1 for a
 *                          field of at least 32768 tiles, else as 2;
 *                          1: checkerboard (the first pass and every sweep
 *                          run the tiles of one colour, then the other, so
 *                          that the second sees the first's changes);
 *                          2: all tiles in one launch.  The result does not
 *                          depend on it. */
enum { LOPC_OPT_BATCH_GRAPH = 1, LOPC_OPT_GRAPH_SWEEPS = 2, LOPC_OPT_PERSIST_PCT = 3,
       LOPC_OPT_REPAIR = 4, LOPC_OPT_TILE_3D = 5, LOPC_OPT_TILE_2D = 6,
       LOPC_OPT_SWEEP_ORDER = 7 };
enum { LOPC_REPAIR_AUTO = 0, LOPC_REPAIR_HYBRID = 1, LOPC_REPAIR_QUEUE = 2,
       LOPC_REPAIR_SWEEPS = 3, LOPC_REPAIR_POINTS = 4 };
int lopc_ctx_set_option(lopc_ctx* ctx, int option, int64_t value);
/* The current value of a context option into *h_value; LOPC_E_ARG for an
 * unknown option or a NULL argument. */
int lopc_ctx_get_option(lopc_ctx* ctx, int option, int64_t* h_value);

/* ------------------------------------------------------------------ checks
 * What LOPC guarantees of a reconstruction d_recon of d_orig (same dtype and
 * shape), measured on the device: the error bound |x - x'| <= eps, checked
 * exactly [Sec. IV-A]; the (value, index) order of the two ends of every
 * edge of the triangulation, ties broken by the lower index [Sec. II,
 * Sec. IV-E]; and the critical type of every vertex (minimum: no lower link
 * vertex; maximum: no upper one; regular: one connected component each;
 * saddle otherwise; boundary vertices use the in-grid part of the link)
 * [Sec. II].  d_ws: lopc_verify_workspace_size() bytes. */
typedef struct {
  uint64_t points;
  uint64_t bound_violations;   /* points with |x - x'| > eps               */
  double max_abs_error;        /* largest |x - x'| (rounded to binary64)   */
  uint64_t edges;              /* edges with both ends in the grid         */
  uint64_t order_violations;   /* edges whose end points swapped order     */
  uint64_t types_orig[4];      /* regular, minima, maxima, saddles         */
  uint64_t types_recon[4];
  uint64_t type_mismatches;    /* vertices whose critical type changed     */
} lopc_verify_report;

size_t lopc_verify_workspace_size(void);
int lopc_verify(lopc_ctx* ctx, const void* d_orig, const void* d_recon, int dtype, int ndim,
                const int64_t* dims, double eps, void* d_ws, size_t ws_bytes, void* stream,
                lopc_verify_report* h_report);

/* Static text for a status code. */
const char* lopc_strerror(int status);

/* After LOPC_E_HIP: the HIP error string and the failing call of the most
 * recent failure on this context (*code receives the hipError_t value; may be
 * NULL).  The text stays valid until the next call on this thread.  Setting
 * the environment variable LOPC_SYNC_CHECK=1 before lopc_ctx_create makes
 * every call synchronise after each launch so that a failure names its kernel. */
const char* lopc_ctx_last_hip_error(lopc_ctx* ctx, int* code);

/* Phase timing (for benchmarks).  `phases` is a bit mask over the phases
 * below (1 << LOPC_PHASE_x; LOPC_TIMING_ALL: every phase; 0: off).  In each
 * compress/decompress call the first kernel of a timed phase records its
 * start and the last its end in HIP events, taken from the dispatches
 * themselves; a timed kernel still delays the next launch by a few
 * microseconds, so time only the phases needed.  After its final
 * synchronisation the call stores the elapsed milliseconds of each timed
 * phase (0 for the others):
 *   LOPC_PHASE_RANGE    compress: NOA min/max (with the workspace clear) +
 *                       error parameters
 *   LOPC_PHASE_QUANT    compress: quantize + order flags + first relaxation
 *   LOPC_PHASE_REPAIR   compress: all repair sweeps (host waits included)
 *   LOPC_PHASE_ENCODE   compress: chunk encoder + stream assembly
 *   LOPC_PHASE_OFFSETS  decompress: record offsets
 *   LOPC_PHASE_DECODE   decompress: chunk decoder + reconstruction
 * lopc_ctx_last_timings copies min(n, LOPC_PHASES) values of the most recent
 * call of each kind and returns LOPC_OK.  A mask with other bits set is
 * LOPC_E_ARG. */
enum {
  LOPC_PHASE_RANGE = 0,
  LOPC_PHASE_QUANT = 1,
  LOPC_PHASE_REPAIR = 2,
  LOPC_PHASE_ENCODE = 3,
  LOPC_PHASE_OFFSETS = 4,
  LOPC_PHASE_DECODE = 5,
  LOPC_PHASES = 6,
  LOPC_TIMING_ALL = (1 << LOPC_PHASES) - 1
};
int lopc_ctx_set_timing(lopc_ctx* ctx, int phases);
int lopc_ctx_last_timings(lopc_ctx* ctx, double* h_ms, int n);

#ifdef __cplusplus
}
#endif
#endif
