// lopc_kernels.hip -- gfx950 kernels of liblopc.so (LOPC, arXiv 2603.26968).
//
// Wave64 throughout: bit planes and zero bitmaps are built with __ballot,
// compaction offsets with mbcnt and block scans, chunk offsets of the
// compressed stream with a decoupled look-back over a ticket-ordered chunk
// queue.  No MFMA: nothing here is a dense contraction.
//
// Paper map: error bound and quantizer Sec. IV-A; neighbour order flags and
// subbin raising Alg. 1 / Alg. 2 / Sec. IV-B; lossless stages Sec. III-B and
// Sec. IV-C; decoding rule Sec. IV-E.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lopc_internal.h"
#include "lopc_numeric.h"

namespace lopc {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ int lane() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave() { return threadIdx.x >> 6; }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t lane_prefix(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void set_status(Params* prm, uint32_t bits) {
  atomicOr(&prm->status, bits);
}

template <int K> struct Traits;
template <> struct Traits<4> {
  using Raw = uint32_t;   // bits of a value
  using Bin = int32_t;
  using Word = uint32_t;  // stage word
  static constexpr int64_t kBinLimit = 2147483646ll;
  static constexpr int64_t kMaxKey = 0x7f7fffffll;
  __device__ static int64_t key(Raw u) { return key32(u); }
  __device__ static Raw unkey(int64_t k) { return unkey32(k); }
  __device__ static bool finite(Raw u) { return finite32(u); }
  __device__ static double to_double(Raw u) { return (double)__uint_as_float(u); }
};
template <> struct Traits<8> {
  using Raw = uint64_t;
  using Bin = int64_t;
  using Word = uint64_t;
  static constexpr int64_t kBinLimit = 4611686018427387904ll;
  static constexpr int64_t kMaxKey = 0x7fefffffffffffffll;
  __device__ static int64_t key(Raw u) { return key64(u); }
  __device__ static Raw unkey(int64_t k) { return unkey64(k); }
  __device__ static bool finite(Raw u) { return finite64(u); }
  __device__ static double to_double(Raw u) { return __longlong_as_double((long long)u); }
};

// ------------------------------------------------------------------ stencil
// Edges of the Freudenthal triangulation: +-d for nonzero d in {0,1}^3,
// listed as (dz, dy, dx); bit j of a point's mask refers to offset j.  Even
// entries point to a higher linear index (raising weight 1), odd ones lower.
__constant__ int8_t c_off[14][3] = {
    {0, 0, 1},  {0, 0, -1},  {0, 1, 0},  {0, -1, 0}, {0, 1, 1},
    {0, -1, -1}, {1, 0, 0},  {-1, 0, 0}, {1, 0, 1},  {-1, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, 1, 1},  {-1, -1, -1}};

// ------------------------------------------------------------------ scans
template <typename V>
__device__ V block_excl_scan(V v, V* sh, V& total) {
  V x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    V y = __shfl_up(x, d, 64);
    if (lane() >= d) x += y;
  }
  if (lane() == 63) sh[wave()] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    V acc = 0;
    for (int w = 0; w < kWaves; ++w) {
      V t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[kWaves] = acc;
  }
  __syncthreads();
  V res = x - v + sh[wave()];
  total = sh[kWaves];
  __syncthreads();
  return res;
}

// ------------------------------------------------------------------ a0
template <int K>
__global__ __launch_bounds__(kThreads) void k_minmax(
    const typename Traits<K>::Raw* x, uint32_t n, int64_t* part, Params* prm) {
  using Tr = Traits<K>;
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  bool bad = false;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n;
       i += gridDim.x * kThreads) {
    typename Tr::Raw u = x[i];
    bad |= !Tr::finite(u);
    int64_t k = Tr::key(u);
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
  if (bad) set_status(prm, ST_NONFINITE);
  __shared__ int64_t slo[kThreads], shi[kThreads];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = slo[0];
    part[2 * blockIdx.x + 1] = shi[0];
  }
}

__device__ void put_bytes(uint8_t* dst, uint64_t v, int nbytes) {
  for (int i = 0; i < nbytes; ++i) dst[i] = (uint8_t)(v >> (8 * i));
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_params(
    int mode, double eb, const int64_t* part, int nblocks, Params* prm,
    uint8_t* stream, uint64_t cap, int ndim, int64_t d0, int64_t d1,
    int64_t d2) {
  using Tr = Traits<K>;
  __shared__ int64_t slo[kThreads], shi[kThreads];
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  if (mode == 1)
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
      lo = min(lo, part[2 * b]);
      hi = max(hi, part[2 * b + 1]);
    }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double e = eb;
  if (mode == 1) {
    // NOA: eps = eb * (max - min), all in binary64 (Sec. IV-A)
    double vlo = Tr::to_double(Tr::unkey(slo[0]));
    double vhi = Tr::to_double(Tr::unkey(shi[0]));
    double range = vhi - vlo;
    e = eb * range;
    prm->kmin = slo[0];
    prm->kmax = shi[0];
  }
  double v = 1.0 / e;
  bool ok = (e > 0.0) && finite64((uint64_t)__double_as_longlong(e)) &&
            finite64((uint64_t)__double_as_longlong(v));
  if (ok && fma(v, e, -1.0) < 0.0)
    v = __longlong_as_double(__double_as_longlong(v) + 1);  // next up
  ok = ok && finite64((uint64_t)__double_as_longlong(v));
  if (!ok) {
    set_status(prm, ST_BOUND);
    e = 1.0;
    v = 1.0;
  }
  prm->eb = eb;
  prm->eps = e;
  prm->inv = v;
  prm->winv = 1.0 / v;
  if (cap >= kHeaderBytes) {
    uint8_t* h = stream;
    put_bytes(h + 0, kMagic, 4);
    put_bytes(h + 4, kVersion, 2);
    h[6] = (uint8_t)(K == 4 ? 0 : 1);
    h[7] = (uint8_t)ndim;
    put_bytes(h + 8, (uint64_t)d0, 8);
    put_bytes(h + 16, (uint64_t)d1, 8);
    put_bytes(h + 24, (uint64_t)d2, 8);
    h[32] = (uint8_t)mode;
    h[33] = h[34] = h[35] = 0;
    put_bytes(h + 36, kChunkBytes, 4);
    put_bytes(h + 40, (uint64_t)__double_as_longlong(eb), 8);
    put_bytes(h + 48, (uint64_t)__double_as_longlong(e), 8);
    put_bytes(h + 56, (uint64_t)__double_as_longlong(v), 8);
  }
}

// ------------------------------------------------------------------ a1, a2
template <int K>
__global__ __launch_bounds__(kThreads) void k_quant(
    const typename Traits<K>::Raw* x, uint32_t n, Params* prm,
    typename Traits<K>::Bin* bins) {
  using Tr = Traits<K>;
  const double inv = prm->inv;
  bool bad_v = false, bad_r = false;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n;
       i += gridDim.x * kThreads) {
    typename Tr::Raw u = x[i];
    bad_v |= !Tr::finite(u);
    int64_t b = q_bin(Tr::to_double(u), inv);
    bad_r |= (b > Tr::kBinLimit || b < -Tr::kBinLimit);
    bins[i] = (typename Tr::Bin)b;
  }
  if (bad_v) set_status(prm, ST_NONFINITE);
  if (bad_r) set_status(prm, ST_RANGE);
}

// One thread per point: bit j of mask[p] is set when neighbour p + off[j]
// is in the grid, has the same bin, and comes before p in the order
// (value, index) -- the flags of Alg. 1.
template <int K>
__global__ __launch_bounds__(kThreads) void k_mask(
    const typename Traits<K>::Raw* x, Box box,
    const typename Traits<K>::Bin* bins, uint16_t* mask) {
  using Tr = Traits<K>;
  const int ix = blockIdx.x * kThreads + threadIdx.x;
  if (ix >= box.nx) return;
  for (int64_t row = blockIdx.y; row < (int64_t)box.nz * box.ny;
       row += gridDim.y) {
    const int iz = (int)(row / box.ny), iy = (int)(row % box.ny);
    const uint32_t p = (uint32_t)(row * box.nx + ix);
    const int64_t kp = Tr::key(x[p]);
    const typename Tr::Bin bp = bins[p];
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 14; ++j) {
      int z = iz + c_off[j][0], y = iy + c_off[j][1], xx = ix + c_off[j][2];
      if (z < 0 || z >= box.nz || y < 0 || y >= box.ny || xx < 0 || xx >= box.nx)
        continue;
      uint32_t q = (uint32_t)(((int64_t)z * box.ny + y) * box.nx + xx);
      if (bins[q] != bp) continue;
      int64_t kq = Tr::key(x[q]);
      bool below = kq < kp || (kq == kp && (j & 1));  // odd j: lower index
      if (below) m |= 1u << j;
    }
    mask[p] = (uint16_t)m;
  }
}

// ------------------------------------------------------------------ a3
// One workgroup per tile: subbins of the tile plus a one-point halo in LDS,
// relaxed in place (monotone, so concurrent reads of stale values are
// harmless) until nothing changes; halo values come from the global array
// and are treated as fixed.  A tile whose boundary changed marks its 26
// neighbour tiles for the next sweep; the host sweeps until no tile is
// marked.  Every subbin only grows and stays below the least fixed point,
// so the result is that fixed point, whatever the order of tiles.
template <int TZ, int TY, int TX>
__global__ __launch_bounds__(kThreads) void k_repair(
    Box box, Tiling tl, const uint16_t* __restrict__ mask,
    uint32_t* __restrict__ sub, uint32_t* stamp, uint32_t* counters,
    uint32_t sweep) {
  constexpr int ZO = TZ == 1 ? 0 : 1;  // 2D tiles carry no z halo
  constexpr int HZ = TZ + 2 * ZO, HY = TY + 2, HX = TX + 2;
  constexpr int NPT = TZ * TY * TX;
  constexpr int PER = NPT / kThreads;
  static_assert(NPT % kThreads == 0, "tile must be a multiple of the block");
  __shared__ uint32_t S[HZ * HY * HX];
  __shared__ uint16_t Mk[NPT];

  const uint32_t t = blockIdx.x;
  if (stamp[t] < sweep) return;
  const int tz = (int)(t / (uint32_t)(tl.nty * tl.ntx));
  const int ty = (int)((t / (uint32_t)tl.ntx) % (uint32_t)tl.nty);
  const int tx = (int)(t % (uint32_t)tl.ntx);
  const int z0 = tz * TZ, y0 = ty * TY, x0 = tx * TX;

  for (int i = threadIdx.x; i < HZ * HY * HX; i += kThreads) {
    int hz = i / (HY * HX), hy = (i / HX) % HY, hx = i % HX;
    int z = z0 + hz - ZO, y = y0 + hy - 1, x = x0 + hx - 1;
    uint32_t v = 0;
    if (z >= 0 && z < box.nz && y >= 0 && y < box.ny && x >= 0 && x < box.nx)
      v = sub[((int64_t)z * box.ny + y) * box.nx + x];
    S[i] = v;
  }
  for (int i = threadIdx.x; i < NPT; i += kThreads) {
    int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
    int z = z0 + iz, y = y0 + iy, x = x0 + ix;
    uint16_t m = 0;
    if (z < box.nz && y < box.ny && x < box.nx)
      m = mask[((int64_t)z * box.ny + y) * box.nx + x];
    Mk[i] = m;
  }
  int doff[14];
#pragma unroll
  for (int j = 0; j < 14; ++j)
    doff[j] = c_off[j][0] * (HY * HX) + c_off[j][1] * HX + c_off[j][2];
  __syncthreads();

  uint32_t old[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int i = threadIdx.x + k * kThreads;
    int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
    old[k] = S[((iz + ZO) * HY + iy + 1) * HX + ix + 1];
  }
  int iters = 0;
  for (;;) {
    int changed = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      int i = threadIdx.x + k * kThreads;
      uint32_t m = Mk[i];
      if (!m) continue;
      int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
      int li = ((iz + ZO) * HY + iy + 1) * HX + ix + 1;
      uint32_t cur = S[li], best = cur;
      while (m) {
        int j = __builtin_ctz(m);
        m &= m - 1;
        uint32_t v = S[li + doff[j]] + ((j & 1) ? 0u : 1u);
        best = v > best ? v : best;
      }
      if (best > cur) {
        S[li] = best;
        changed = 1;
      }
    }
    if (!__syncthreads_or(changed)) break;
    if (++iters > NPT + 2) {  // unreachable: the order inside a tile is acyclic
      if (threadIdx.x == 0) atomicOr(&counters[0], 1u);
      break;
    }
  }
  int edge = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int i = threadIdx.x + k * kThreads;
    int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
    uint32_t v = S[((iz + ZO) * HY + iy + 1) * HX + ix + 1];
    if (v != old[k]) {
      int z = z0 + iz, y = y0 + iy, x = x0 + ix;
      sub[((int64_t)z * box.ny + y) * box.nx + x] = v;
      if ((TZ > 1 && (iz == 0 || iz == TZ - 1)) || iy == 0 || iy == TY - 1 ||
          ix == 0 || ix == TX - 1)
        edge = 1;
    }
  }
  edge = __syncthreads_or(edge);
  if (edge && threadIdx.x < 27) {
    int dz = (int)threadIdx.x / 9 - 1, dy = ((int)threadIdx.x / 3) % 3 - 1,
        dx = (int)threadIdx.x % 3 - 1;
    int nz = tz + dz, ny = ty + dy, nx = tx + dx;
    if ((dz | dy | dx) != 0 && nz >= 0 && nz < tl.ntz && ny >= 0 &&
        ny < tl.nty && nx >= 0 && nx < tl.ntx) {
      uint32_t u = ((uint32_t)nz * tl.nty + ny) * tl.ntx + nx;
      uint32_t prev = atomicMax(&stamp[u], sweep + 1);
      if (prev < sweep + 1) atomicAdd(&counters[sweep + 2], 1u);
    }
  }
}

// ------------------------------------------------------------------ stages
// Scratch of the RZE encoder / decoder (bitmap levels, ranks).
struct RzeScratch {
  uint64_t bm[2048 / 8];      // level-1 bitmap (up to 16384 items)
  uint8_t lv1[256 + 8];       // level-2 bitmap
  uint8_t lv2[32 + 8];        // level-3 bitmap
  uint8_t lv3[8 + 8];         // level-4 bitmap
  uint8_t kept0[2048];        // kept bytes of level 1
  uint8_t kept1[256];         // kept bytes of level 2
  uint8_t kept2[32];          // kept bytes of level 3
  uint32_t gpos[kThreads];    // per-group exclusive counts
  uint32_t scan[kWaves + 1];
  uint64_t scan64[kWaves + 1];
  uint32_t nkept[4];
};

__device__ __forceinline__ uint8_t* level_buf(RzeScratch& sc, int l) {
  return l == 0 ? (uint8_t*)sc.bm : (l == 1 ? sc.lv1 : (l == 2 ? sc.lv2 : sc.lv3));
}
__device__ __forceinline__ uint8_t* kept_buf(RzeScratch& sc, int l) {
  return l == 0 ? sc.kept0 : (l == 1 ? sc.kept1 : sc.kept2);
}

__device__ __forceinline__ int rze_levels(uint32_t items, uint32_t* sz) {
  int top = 0;
  sz[0] = (items + 7) / 8;
  while (sz[top] > 8) {
    sz[top + 1] = (sz[top] + 7) / 8;
    ++top;
  }
  return top;
}

template <int W>
__device__ __forceinline__ bool word_nonzero(const uint8_t* in, uint32_t i) {
  if (W == 1) return in[i] != 0;
  if (W == 4) return *(const uint32_t*)(in + 4 * i) != 0;
  return *(const uint64_t*)(in + 8 * i) != 0;
}

// RZE_W of len bytes (LDS, W-aligned for W > 1) into out (LDS).  Returns the
// output length; pt = stored verbatim.  len <= 16384, len % W == 0.
template <int W>
__device__ uint32_t rze_encode(const uint8_t* in, uint32_t len, uint8_t* out,
                               RzeScratch& sc, int& pt) {
  const uint32_t items = len / W;
  const uint32_t groups = (items + 63) / 64;
  for (uint32_t g = wave(); g < groups; g += kWaves) {
    uint32_t it = g * 64 + lane();
    bool nz = it < items && word_nonzero<W>(in, it);
    uint64_t m = __ballot(nz);
    if (lane() == 0) sc.bm[g] = m;
  }
  __syncthreads();
  uint32_t total;
  {
    uint32_t c = threadIdx.x < groups ? (uint32_t)__popcll(sc.bm[threadIdx.x]) : 0u;
    uint32_t e = block_excl_scan<uint32_t>(c, sc.scan, total);
    if (threadIdx.x < groups) sc.gpos[threadIdx.x] = e;
  }
  const uint32_t npay = total;
  uint32_t sz[8];
  const int top = rze_levels(items, sz);
  // zero the tail of the level-1 bitmap beyond its byte length
  // (already zero: bits beyond items are never set by the ballot)
  for (int l = 0; l < top; ++l) {
    const uint8_t* cur = level_buf(sc, l);
    uint8_t* nxt = level_buf(sc, l + 1);
    uint8_t* kept = kept_buf(sc, l);
    const uint32_t n = sz[l];
    const uint32_t g2 = (n + 63) / 64;
    // bitmap of bytes that differ from their predecessor
    for (uint32_t g = wave(); g < g2; g += kWaves) {
      uint32_t i = g * 64 + lane();
      bool diff = i < n && cur[i] != (i ? cur[i - 1] : (uint8_t)0);
      uint64_t m = __ballot(diff);
      if (lane() == 0) {
        for (int b = 0; b < 8; ++b) nxt[g * 8 + b] = (uint8_t)(m >> (8 * b));
      }
    }
    __syncthreads();
    uint32_t cnt = 0;
    if (threadIdx.x < g2) {
      uint64_t m = 0;
      for (int b = 0; b < 8; ++b) m |= (uint64_t)nxt[threadIdx.x * 8 + b] << (8 * b);
      cnt = (uint32_t)__popcll(m);
    }
    uint32_t kt;
    uint32_t e = block_excl_scan<uint32_t>(cnt, sc.scan, kt);
    if (threadIdx.x < g2) sc.gpos[threadIdx.x] = e;
    __syncthreads();
    for (uint32_t g = wave(); g < g2; g += kWaves) {
      uint32_t i = g * 64 + lane();
      uint64_t m = 0;
      for (int b = 0; b < 8; ++b) m |= (uint64_t)nxt[g * 8 + b] << (8 * b);
      if ((m >> lane()) & 1) kept[sc.gpos[g] + lane_prefix(m)] = cur[i];
    }
    if (threadIdx.x == 0) sc.nkept[l] = kt;
    __syncthreads();
    // restore level-1 group offsets for the payload (gpos was reused)
  }
  uint32_t out_len = sz[top] + npay * W;
  for (int l = 0; l < top; ++l) out_len += sc.nkept[l];
  if (out_len >= len) {
    for (uint32_t i = threadIdx.x; i < len; i += kThreads) out[i] = in[i];
    pt = 1;
    __syncthreads();
    return len;
  }
  pt = 0;
  // top bitmap, kept bytes from the top level down, then the nonzero words
  uint32_t pos = 0;
  {
    const uint8_t* tb = level_buf(sc, top);
    for (uint32_t i = threadIdx.x; i < sz[top]; i += kThreads) out[i] = tb[i];
    pos = sz[top];
  }
  for (int l = top - 1; l >= 0; --l) {
    const uint8_t* kept = kept_buf(sc, l);
    for (uint32_t i = threadIdx.x; i < sc.nkept[l]; i += kThreads) out[pos + i] = kept[i];
    pos += sc.nkept[l];
  }
  // payload positions: recompute the level-1 group offsets
  {
    uint32_t c = threadIdx.x < groups ? (uint32_t)__popcll(sc.bm[threadIdx.x]) : 0u;
    uint32_t tt;
    uint32_t e = block_excl_scan<uint32_t>(c, sc.scan, tt);
    if (threadIdx.x < groups) sc.gpos[threadIdx.x] = e;
  }
  __syncthreads();
  for (uint32_t g = wave(); g < groups; g += kWaves) {
    uint32_t it = g * 64 + lane();
    uint64_t m = sc.bm[g];
    if (it < items && ((m >> lane()) & 1)) {
      uint32_t d = pos + (sc.gpos[g] + lane_prefix(m)) * W;
#pragma unroll
      for (int b = 0; b < W; ++b) out[d + b] = in[it * W + b];
    }
  }
  __syncthreads();
  return out_len;
}

// Inverse of rze_encode.  in: in_len bytes (global or LDS); out: len bytes in
// LDS (W-aligned).  Returns false on a malformed input (reads stay inside
// [in, in + in_len)).
template <int W>
__device__ bool rze_decode(const uint8_t* in, uint32_t in_len, uint32_t len,
                           uint8_t* out, RzeScratch& sc) {
  const uint32_t items = len / W;
  uint32_t sz[8];
  const int top = rze_levels(items, sz);
  if (sz[top] > in_len) return false;
  {
    uint8_t* tb = level_buf(sc, top);
    for (uint32_t i = threadIdx.x; i < 16; i += kThreads) tb[i] = i < sz[top] ? in[i] : 0;
  }
  __syncthreads();
  uint32_t pos = sz[top];
  for (int l = top - 1; l >= -1; --l) {
    // parent bitmap = level l+1, describing `cn` child entries
    const uint8_t* par = level_buf(sc, l + 1);
    const uint32_t cn = l >= 0 ? sz[l] : items;
    const uint32_t pw = (cn + 63) / 64;  // parent u64 words (<= 256)
    uint64_t pm = 0;
    if (threadIdx.x < pw) {
      for (int b = 0; b < 8; ++b) pm |= (uint64_t)par[threadIdx.x * 8 + b] << (8 * b);
      uint32_t valid = cn - threadIdx.x * 64;
      if (valid < 64) pm &= (1ull << valid) - 1;
    }
    uint32_t cnt = threadIdx.x < pw ? (uint32_t)__popcll(pm) : 0u;
    uint32_t total;
    uint32_t e = block_excl_scan<uint32_t>(cnt, sc.scan, total);
    if (threadIdx.x < pw) sc.gpos[threadIdx.x] = e;
    __syncthreads();
    if (l >= 0) {
      if (pos + total > in_len) return false;
      uint8_t* child = level_buf(sc, l);
      for (uint32_t i = threadIdx.x; i < ((cn + 7) / 8) * 8 + 8 && i < 2048 + 8; i += kThreads) {
        uint8_t v = 0;
        if (i < cn) {
          uint32_t w = i / 64, b = i % 64;
          uint64_t m = 0;
          for (int q = 0; q < 8; ++q) m |= (uint64_t)par[w * 8 + q] << (8 * q);
          uint32_t valid = cn - w * 64;
          if (valid < 64) m &= (1ull << valid) - 1;
          uint32_t c = sc.gpos[w] + (uint32_t)__popcll(m & ((2ull << b) - 1));
          v = c ? in[pos + c - 1] : (uint8_t)0;
        }
        if (l > 0 || i < 2048) child[i] = v;
      }
      pos += total;
      __syncthreads();
    } else {
      if (pos + total * W != in_len) return false;
      for (uint32_t i = threadIdx.x; i < items; i += kThreads) {
        uint32_t w = i / 64, b = i % 64;
        uint64_t m = 0;
        for (int q = 0; q < 8; ++q) m |= (uint64_t)par[w * 8 + q] << (8 * q);
        uint32_t valid = cn - w * 64;
        if (valid < 64) m &= (1ull << valid) - 1;
        bool set = (m >> b) & 1;
        uint32_t r = sc.gpos[w] + (uint32_t)__popcll(m & ((1ull << b) - 1));
#pragma unroll
        for (int q = 0; q < W; ++q) out[i * W + q] = set ? in[pos + r * W + q] : (uint8_t)0;
      }
      __syncthreads();
    }
  }
  return true;
}

// BIT_K: plane j (8K planes, lowest bit first) = bit j of every word.
template <int K>
__device__ void bit_encode(const uint8_t* words, uint32_t m, uint8_t* planes) {
  using Word = typename Traits<K>::Word;
  const uint32_t groups = m / 64, pb = m / 8;
  for (uint32_t g = wave(); g < groups; g += kWaves) {
    Word v = ((const Word*)words)[g * 64 + lane()];
    uint64_t mine = 0;
#pragma unroll
    for (int j = 0; j < 8 * K; ++j) {
      uint64_t b = __ballot((v >> j) & 1);
      if (lane() == j) mine = b;
    }
    if (lane() < 8 * K) *(uint64_t*)(planes + lane() * pb + g * 8) = mine;
  }
}

template <int K>
__device__ void bit_decode(const uint8_t* planes, uint32_t m, uint8_t* words) {
  using Word = typename Traits<K>::Word;
  const uint32_t groups = m / 64, pb = m / 8;
  for (uint32_t g = wave(); g < groups; g += kWaves) {
    Word v = 0;
#pragma unroll 8
    for (int j = 0; j < 8 * K; ++j) {
      uint64_t p = *(const uint64_t*)(planes + j * pb + g * 8);
      v |= (Word)((p >> lane()) & 1) << j;
    }
    ((Word*)words)[g * 64 + lane()] = v;
  }
}

// ------------------------------------------------------------------ a4-a6
// One workgroup per 16 kB chunk; chunk ids come from a ticket counter so a
// workgroup only ever waits for chunks that started before it (decoupled
// look-back: every chunk publishes its record size at once and its
// inclusive offset as soon as its predecessor's is known).
constexpr uint64_t kLbAgg = 1ull << 62, kLbInc = 2ull << 62,
                   kLbVal = (1ull << 62) - 1;

template <int K>
__global__ __launch_bounds__(kThreads) void k_encode(
    uint32_t n, const typename Traits<K>::Bin* __restrict__ bins,
    const uint32_t* __restrict__ sub, uint64_t* lookback, Params* prm,
    uint8_t* stream, uint64_t cap, uint32_t nch) {
  using Tr = Traits<K>;
  using Word = typename Tr::Word;
  constexpr uint32_t W = kChunkBytes / K;
  __shared__ __attribute__((aligned(16))) uint8_t bufA[kChunkBytes];
  __shared__ __attribute__((aligned(16))) uint8_t bufB[kChunkBytes];
  __shared__ __attribute__((aligned(16))) uint8_t rec[kRecordHeaderBytes + 2 * kChunkBytes];
  __shared__ RzeScratch sc;
  __shared__ uint32_t s_chunk;
  __shared__ uint64_t s_excl;

  if (threadIdx.x == 0) s_chunk = atomicAdd(&prm->ticket, 1u);
  __syncthreads();
  const uint32_t c = s_chunk;
  if (c >= nch) return;
  const uint32_t p0 = c * W;
  const uint32_t nc = min(W, n - p0);
  const uint32_t m = (nc + 63) / 64 * 64;
  const uint32_t L = m * K;
  const Word M = (Word)0xAAAAAAAAAAAAAAAAull;

  // bins: DIFFNB_K (delta from the previous bin, 0 before the chunk, then
  // negabinary), zero words up to m, BIT_K, RZE_1
  for (uint32_t i = threadIdx.x; i < m; i += kThreads) {
    Word v = 0;
    if (i < nc) {
      Word cur = (Word)bins[p0 + i];
      Word prev = i ? (Word)bins[p0 + i - 1] : (Word)0;
      Word d = cur - prev;
      v = (d + M) ^ M;
    }
    ((Word*)bufA)[i] = v;
  }
  __syncthreads();
  bit_encode<K>(bufA, m, bufB);
  __syncthreads();
  int pt_b = 0, pt_s1 = 0, pt_s2 = 0;
  const uint32_t blen = rze_encode<1>(bufB, L, rec + kRecordHeaderBytes, sc, pt_b);

  // subbins: zero words up to m, BIT_K, RZE_K, RZE_1
  for (uint32_t i = threadIdx.x; i < m; i += kThreads)
    ((Word*)bufA)[i] = i < nc ? (Word)sub[p0 + i] : (Word)0;
  __syncthreads();
  bit_encode<K>(bufA, m, bufB);
  __syncthreads();
  const uint32_t smid = rze_encode<K>(bufB, L, bufA, sc, pt_s1);
  const uint32_t slen =
      rze_encode<1>(bufA, smid, rec + kRecordHeaderBytes + blen, sc, pt_s2);

  uint32_t size = kRecordHeaderBytes + blen + slen;
  const uint32_t padded = (size + 3) & ~3u;
  if (threadIdx.x == 0) {
    rec[0] = (uint8_t)pt_b;
    rec[1] = (uint8_t)(pt_s1 | (pt_s2 << 1));
    rec[2] = (uint8_t)nc;
    rec[3] = (uint8_t)(nc >> 8);
    put_bytes(rec + 4, blen, 4);
    put_bytes(rec + 8, smid, 4);
    put_bytes(rec + 12, slen, 4);
    for (uint32_t i = size; i < padded; ++i) rec[i] = 0;
  }
  size = padded;

  // look-back for this chunk's offset in the stream body
  if (threadIdx.x == 0) {
    uint64_t excl = 0;
    if (c == 0) {
      __hip_atomic_store(&lookback[0], kLbInc | size, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&lookback[c], kLbAgg | size, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
      int64_t j = (int64_t)c - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        uint64_t v = __hip_atomic_load(&lookback[j], __ATOMIC_ACQUIRE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        uint64_t st = v & ~kLbVal;
        if (st == 0) {
          if (++spins > (1u << 26)) {  // never reached when every chunk runs
            set_status(prm, ST_INTERNAL);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += v & kLbVal;
        if (st == kLbInc) break;
        --j;
      }
      __hip_atomic_store(&lookback[c], kLbInc | (excl + size), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    s_excl = excl;
    atomicAdd((unsigned long long*)&prm->bins_bytes, (unsigned long long)blen);
    atomicAdd((unsigned long long*)&prm->sub_bytes, (unsigned long long)slen);
  }
  __syncthreads();
  const uint64_t body = kHeaderBytes + 4ull * nch;
  const uint64_t dst = body + s_excl;
  if (threadIdx.x == 0) {
    if (kHeaderBytes + 4ull * c + 4 <= cap)
      *(uint32_t*)(stream + kHeaderBytes + 4ull * c) = size;
    if (c == nch - 1) prm->stream_size = dst + size;
  }
  if (dst + size <= cap) {
    for (uint32_t i = threadIdx.x; i < size / 4; i += kThreads)
      ((uint32_t*)(stream + dst))[i] = ((const uint32_t*)rec)[i];
  } else if (threadIdx.x == 0) {
    set_status(prm, ST_CAPACITY);
  }
}

// ------------------------------------------------------------------ a7, a8
// Exclusive offsets of the records from the size table; the sizes must add
// up to the stream body exactly.
__global__ __launch_bounds__(kThreads) void k_offsets(
    const uint8_t* stream, uint32_t nch, uint64_t body_bytes,
    uint64_t* offsets, Params* prm) {
  __shared__ uint64_t sh[kWaves + 1];
  const uint32_t per = (nch + kThreads - 1) / kThreads;
  const uint32_t b = threadIdx.x * per, e = min(nch, b + per);
  const uint32_t* tab = (const uint32_t*)(stream + kHeaderBytes);
  uint64_t sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += tab[i];
  uint64_t total;
  uint64_t off = block_excl_scan<uint64_t>(sum, sh, total);
  for (uint32_t i = b; i < e; ++i) {
    offsets[i] = off;
    off += tab[i];
  }
  if (threadIdx.x == 0 && total != body_bytes) set_status(prm, ST_FORMAT);
}

// Lowest representable value of bin b (as an order key): start next to the
// real lower edge (b - 1/2) / inv and step to the first value whose bin is b.
template <int K>
__device__ __forceinline__ bool bin_floor_key(int64_t b, double inv,
                                              double winv, int64_t& out) {
  using Tr = Traits<K>;
  if (b > Tr::kBinLimit || b < -Tr::kBinLimit) return false;
  double c = ((double)b - 0.5) * winv;
  int64_t k;
  if (K == 4) {
    float f = (float)c;
    uint32_t u = __float_as_uint(f);
    if (!finite32(u)) return false;
    k = key32(u);
  } else {
    uint64_t u = (uint64_t)__double_as_longlong(c);
    if (!finite64(u)) return false;
    k = key64(u);
  }
  int steps = 0;
  while (k > -Tr::kMaxKey && q_bin(Tr::to_double(Tr::unkey(k - 1)), inv) >= b) {
    --k;
    if (++steps > 8) return false;
  }
  while (q_bin(Tr::to_double(Tr::unkey(k)), inv) < b) {
    if (k >= Tr::kMaxKey || ++steps > 8) return false;
    ++k;
  }
  if (q_bin(Tr::to_double(Tr::unkey(k)), inv) != b) return false;
  out = k;
  return true;
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_decode(
    const uint8_t* __restrict__ stream, uint32_t n,
    const uint64_t* __restrict__ offsets, Params* prm,
    typename Traits<K>::Raw* __restrict__ out) {
  using Tr = Traits<K>;
  using Word = typename Tr::Word;
  constexpr uint32_t W = kChunkBytes / K;
  __shared__ __attribute__((aligned(16))) uint8_t P[kChunkBytes];
  __shared__ __attribute__((aligned(16))) uint8_t Wb[kChunkBytes];
  __shared__ __attribute__((aligned(16))) uint8_t Mb[kChunkBytes];
  __shared__ RzeScratch sc;
  __shared__ uint64_t sh64[kWaves + 1];
  __shared__ int s_bad;

  const uint32_t nch = gridDim.x, c = blockIdx.x;
  const uint32_t p0 = c * W, nc = min(W, n - p0);
  const uint32_t m = (nc + 63) / 64 * 64, L = m * K;
  const uint64_t body = kHeaderBytes + 4ull * nch;
  const uint32_t rsize = ((const uint32_t*)(stream + kHeaderBytes))[c];
  const uint8_t* rec = stream + body + offsets[c];
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if (rsize < kRecordHeaderBytes || (rsize & 3) || (prm->status & ST_FORMAT)) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }
  double inv = __longlong_as_double(*(const long long*)(stream + 56));
  double winv = 1.0 / inv;
  const uint32_t bfl = rec[0], sfl = rec[1];
  const uint32_t npts = rec[2] | (rec[3] << 8);
  const uint32_t blen = *(const uint32_t*)(rec + 4);
  const uint32_t smid = *(const uint32_t*)(rec + 8);
  const uint32_t slen = *(const uint32_t*)(rec + 12);
  bool ok = !(bfl & ~1u) && !(sfl & ~3u) && npts == nc && blen <= L &&
            smid <= L && slen <= L;
  const uint32_t used = kRecordHeaderBytes + blen + slen;
  ok = ok && ((used + 3) & ~3u) == rsize;
  if (ok && threadIdx.x < rsize - used && rec[used + threadIdx.x] != 0) s_bad = 1;
  __syncthreads();
  ok = ok && !s_bad;
  if (!ok) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }
  const uint8_t* bp = rec + kRecordHeaderBytes;
  const uint8_t* sp = bp + blen;

  // bins: RZE_1 -> BIT_K -> negabinary -> prefix sum
  if (bfl & 1) {
    if (blen != L) ok = false;
    else
      for (uint32_t i = threadIdx.x; i < L; i += kThreads) P[i] = bp[i];
  } else {
    ok = rze_decode<1>(bp, blen, L, P, sc);
  }
  __syncthreads();
  if (!ok) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }
  bit_decode<K>(P, m, Wb);
  __syncthreads();
  {
    // each thread owns a run of consecutive words; prefix sums modulo 2^(8K)
    const Word M = (Word)0xAAAAAAAAAAAAAAAAull;
    constexpr uint32_t per = W / kThreads;
    const uint32_t b0 = threadIdx.x * per;
    Word loc = 0;
    for (uint32_t q = 0; q < per; ++q) {
      uint32_t i = b0 + q;
      if (i < nc) loc += (((Word*)Wb)[i] ^ M) - M;
    }
    uint64_t tot;
    uint64_t run = block_excl_scan<uint64_t>((uint64_t)loc, sh64, tot);
    Word acc = (Word)run;
    for (uint32_t q = 0; q < per; ++q) {
      uint32_t i = b0 + q;
      if (i < nc) {
        acc += (((Word*)Wb)[i] ^ M) - M;
        ((Word*)Wb)[i] = acc;
      }
    }
  }
  __syncthreads();

  // subbins: RZE_1 -> RZE_K -> BIT_K
  if (sfl & 2) {
    if (slen != smid) ok = false;
    else
      for (uint32_t i = threadIdx.x; i < smid; i += kThreads) Mb[i] = sp[i];
  } else {
    ok = rze_decode<1>(sp, slen, smid, Mb, sc);
  }
  __syncthreads();
  if (ok) {
    if (sfl & 1) {
      if (smid != L) ok = false;
      else
        for (uint32_t i = threadIdx.x; i < L; i += kThreads) P[i] = Mb[i];
    } else {
      ok = rze_decode<K>(Mb, smid, L, P, sc);
    }
  }
  __syncthreads();
  if (!ok) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }
  bit_decode<K>(P, m, Mb);
  __syncthreads();

  // reconstruct (Sec. IV-E)
  bool bad = false;
  for (uint32_t i = threadIdx.x; i < nc; i += kThreads) {
    int64_t b;
    if (K == 4) b = (int64_t)(int32_t)((const uint32_t*)Wb)[i];
    else b = (int64_t)((const uint64_t*)Wb)[i];
    uint64_t s = (uint64_t)((const Word*)Mb)[i];
    int64_t klo;
    typename Tr::Raw v = 0;
    if (!bin_floor_key<K>(b, inv, winv, klo) ||
        s > (uint64_t)(Tr::kMaxKey - klo)) {
      bad = true;
    } else {
      v = Tr::unkey(klo + (int64_t)s);
      if (q_bin(Tr::to_double(v), inv) != b) bad = true;
    }
    out[p0 + i] = v;
  }
  if (bad) set_status(prm, ST_FORMAT);
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_minmax(int dtype, const void* x, uint32_t n, double* part,
                         int nblocks, Params* prm, hipStream_t s) {
  if (dtype == 0)
    k_minmax<4><<<nblocks, kThreads, 0, s>>>((const uint32_t*)x, n, (int64_t*)part, prm);
  else
    k_minmax<8><<<nblocks, kThreads, 0, s>>>((const uint64_t*)x, n, (int64_t*)part, prm);
  return hipGetLastError();
}

hipError_t launch_params(int dtype, int mode, double eb, const double* part,
                         int nblocks, Params* prm, uint8_t* stream, size_t cap,
                         int ndim, const int64_t* dims, hipStream_t s) {
  int64_t d2 = ndim == 3 ? dims[2] : 1;
  if (dtype == 0)
    k_params<4><<<1, kThreads, 0, s>>>(mode, eb, (const int64_t*)part, nblocks, prm,
                                       stream, cap, ndim, dims[0], dims[1], d2);
  else
    k_params<8><<<1, kThreads, 0, s>>>(mode, eb, (const int64_t*)part, nblocks, prm,
                                       stream, cap, ndim, dims[0], dims[1], d2);
  return hipGetLastError();
}

hipError_t launch_quant_mask(int dtype, const void* x, Box box, Params* prm,
                             void* bins, uint16_t* mask, hipStream_t s) {
  int qb = (int)std::min<uint64_t>(8192, ((uint64_t)box.n + kThreads - 1) / kThreads);
  dim3 mg((box.nx + kThreads - 1) / kThreads,
          (unsigned)std::min<int64_t>((int64_t)box.nz * box.ny, 65535), 1);
  if (dtype == 0) {
    k_quant<4><<<qb, kThreads, 0, s>>>((const uint32_t*)x, box.n, prm, (int32_t*)bins);
    k_mask<4><<<mg, kThreads, 0, s>>>((const uint32_t*)x, box, (const int32_t*)bins, mask);
  } else {
    k_quant<8><<<qb, kThreads, 0, s>>>((const uint64_t*)x, box.n, prm, (int64_t*)bins);
    k_mask<8><<<mg, kThreads, 0, s>>>((const uint64_t*)x, box, (const int64_t*)bins, mask);
  }
  return hipGetLastError();
}

hipError_t launch_repair(Box box, Tiling t, const uint16_t* mask, uint32_t* sub,
                         uint32_t* stamp, uint32_t* counters, uint32_t sweep,
                         hipStream_t s) {
  if (t.tz == 1)
    k_repair<1, 32, 64><<<t.ntiles, kThreads, 0, s>>>(box, t, mask, sub, stamp, counters, sweep);
  else
    k_repair<8, 8, 32><<<t.ntiles, kThreads, 0, s>>>(box, t, mask, sub, stamp, counters, sweep);
  return hipGetLastError();
}

hipError_t launch_encode(int dtype, uint32_t n, const void* bins,
                         const uint32_t* sub, uint64_t* lookback, Params* prm,
                         uint8_t* stream, size_t cap, hipStream_t s) {
  uint32_t W = kChunkBytes / (dtype == 0 ? 4 : 8);
  uint32_t nch = (n + W - 1) / W;
  if (dtype == 0)
    k_encode<4><<<nch, kThreads, 0, s>>>(n, (const int32_t*)bins, sub, lookback, prm,
                                         stream, cap, nch);
  else
    k_encode<8><<<nch, kThreads, 0, s>>>(n, (const int64_t*)bins, sub, lookback, prm,
                                         stream, cap, nch);
  return hipGetLastError();
}

hipError_t launch_offsets(const uint8_t* stream, uint32_t nch,
                          uint64_t body_bytes, uint64_t* offsets, Params* prm,
                          hipStream_t s) {
  k_offsets<<<1, kThreads, 0, s>>>(stream, nch, body_bytes, offsets, prm);
  return hipGetLastError();
}

hipError_t launch_decode(int dtype, const uint8_t* stream, uint32_t n,
                         const uint64_t* offsets, Params* prm, void* field,
                         hipStream_t s) {
  uint32_t W = kChunkBytes / (dtype == 0 ? 4 : 8);
  uint32_t nch = (n + W - 1) / W;
  if (dtype == 0)
    k_decode<4><<<nch, kThreads, 0, s>>>(stream, n, offsets, prm, (uint32_t*)field);
  else
    k_decode<8><<<nch, kThreads, 0, s>>>(stream, n, offsets, prm, (uint64_t*)field);
  return hipGetLastError();
}

}  // namespace lopc
