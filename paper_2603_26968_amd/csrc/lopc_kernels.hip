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
#include <hip/hip_ext.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "lopc_device.h"

namespace lopc {
namespace {

// ------------------------------------------------------------------ a0
template <int K>
__device__ __forceinline__ void minmax_body(const typename Traits<K>::Raw* x, uint32_t n,
                                            int64_t* part, uint32_t blk, uint32_t nblk) {
  using Tr = Traits<K>;
  using Raw = typename Tr::Raw;
  constexpr int V = 16 / K;  // values per 16-byte vector
  constexpr int U = 4;       // vectors in flight per thread
  // non-finite values are flagged by the tile pass, which sees every point
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  auto take = [&](Raw u) {
    const int64_t k = Tr::key(u);
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  };
  const uint32_t nv = n / V, stride = nblk * kThreads;
  uint32_t i = blk * kThreads + threadIdx.x;
  for (; i + (U - 1) * stride < nv; i += U * stride) {
    Raw u[U][V];
#pragma unroll
    for (int q = 0; q < U; ++q) *(uint4*)u[q] = ((const uint4*)x)[i + q * stride];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int k = 0; k < V; ++k) take(u[q][k]);
  }
  for (; i < nv; i += stride) {
    Raw u[V];
    *(uint4*)u = ((const uint4*)x)[i];
#pragma unroll
    for (int k = 0; k < V; ++k) take(u[k]);
  }
  for (uint32_t t = nv * V + blk * kThreads + threadIdx.x; t < n; t += stride) take(x[t]);
  lo = wave_reduce(lo, OpMin{});
  hi = wave_reduce(hi, OpMax{});
  __shared__ int64_t slo[kWaves], shi[kWaves];
  if (lane() == 0) {
    slo[wave()] = lo;
    shi[wave()] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; ++w) {
      lo = slo[w] < lo ? slo[w] : lo;
      hi = shi[w] > hi ? shi[w] : hi;
    }
    part[2 * blk] = lo;
    part[2 * blk + 1] = hi;
  }
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_minmax(
    const typename Traits<K>::Raw* x, uint32_t n, int64_t* part, uint4* zero, uint32_t nzero) {
  // the zeroed prefix of the workspace (Params, counters, stamps, look-back
  // words), which no earlier work of the call touches, is cleared here
  // rather than by a separate fill
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < nzero; i += gridDim.x * kThreads)
    zero[i] = make_uint4(0, 0, 0, 0);
  minmax_body<K>(x, n, part, blockIdx.x, gridDim.x);
}


template <int K>
__device__ __forceinline__ void params_body(int mode, double eb, const int64_t* part, int nblocks,
                            Params* prm, uint8_t* stream, uint64_t cap, int ndim,
                            int64_t d0, int64_t d1, int64_t d2) {
  using Tr = Traits<K>;
  __shared__ int64_t slo[kWaves], shi[kWaves];
  __shared__ uint32_t hw[kHeaderBytes / 4];
  int64_t lo = INT64_MAX, hi = INT64_MIN;
  if (mode == 1)
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
      const longlong2 p = ((const longlong2*)part)[b];
      lo = min(lo, (int64_t)p.x);
      hi = max(hi, (int64_t)p.y);
    }
  lo = wave_reduce(lo, OpMin{});
  hi = wave_reduce(hi, OpMax{});
  if (lane() == 0) {
    slo[wave()] = lo;
    shi[wave()] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; ++w) {
      lo = min(lo, slo[w]);
      hi = max(hi, shi[w]);
    }
    double e = eb;
    if (mode == 1) {
      // NOA: eps = eb * (max - min), all in binary64 (Sec. IV-A)
      double vlo = Tr::to_double(Tr::unkey(lo));
      double vhi = Tr::to_double(Tr::unkey(hi));
      double range = vhi - vlo;
      e = eb * range;
      prm->kmin = lo;
      prm->kmax = hi;
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
    // the stream header as 16 little-endian words
    const uint64_t q[8] = {(uint64_t)kMagic | (uint64_t)(kVersion | (K == 4 ? 0u : 1u) << 16 |
                                                           (uint32_t)ndim << 24) << 32,
                           (uint64_t)d0, (uint64_t)d1, (uint64_t)d2,
                           (uint64_t)(uint32_t)mode | (uint64_t)kChunkBytes << 32,
                           (uint64_t)__double_as_longlong(eb), (uint64_t)__double_as_longlong(e),
                           (uint64_t)__double_as_longlong(v)};
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      hw[2 * w] = (uint32_t)q[w];
      hw[2 * w + 1] = (uint32_t)(q[w] >> 32);
    }
  }
  __syncthreads();
  if (threadIdx.x < kHeaderBytes / 4) {
    ((uint32_t*)prm->header)[threadIdx.x] = hw[threadIdx.x];
    if (cap >= kHeaderBytes) ((uint32_t*)stream)[threadIdx.x] = hw[threadIdx.x];
  }
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_params(
    int mode, double eb, const int64_t* part, int nblocks, Params* prm,
    uint8_t* stream, uint64_t cap, int ndim, int64_t d0, int64_t d1,
    int64_t d2) {
  params_body<K>(mode, eb, part, nblocks, prm, stream, cap, ndim, d0, d1, d2);
}


// ------------------------------------------------------------------ a3
// Tiles of the subbin repair.  A workgroup owns a TZ x TY x TX tile and keeps
// the subbins of the tile plus a one-point halo in LDS.  It relaxes them in
// place until nothing changes (the raising rule of Alg. 2 with the halo held
// fixed; every value only grows and stays below the least fixed point, so
// concurrent reads of stale values are harmless), writes back what changed,
// and, if a boundary value changed, marks the 26 neighbour tiles for the next
// sweep.  Sweeps repeat until no tile is marked; the result is the least
// fixed point whatever the order in which tiles run.
template <int TZ, int TY, int TX>
struct TileGeom {
  static constexpr int ZO = TZ == 1 ? 0 : 1;  // 2D tiles carry no z halo
  static constexpr int HZ = TZ + 2 * ZO, HY = TY + 2, HX = TX + 2;
  static constexpr int H = HZ * HY * HX;
  static constexpr int NPT = TZ * TY * TX;
  static constexpr int PER = NPT / kThreads;
  static_assert(NPT % kThreads == 0, "tile must be a multiple of the block");
  // owned point tid + k * kThreads (slot k of thread tid) lies kSlot LDS
  // words after slot 0: the block covers whole planes of a 3D tile, or whole
  // rows of a 2D one
  static_assert((TZ > 1 && TY * TX == kThreads) || (TZ == 1 && kThreads % TX == 0),
                "slots of a thread are evenly spaced in LDS");
  static constexpr int kSlot = TZ > 1 ? HY * HX : (kThreads / TX) * HX;
  // halo-local index of interior point i
  __device__ static int local(int i) {
    int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
    return ((iz + ZO) * HY + iy + 1) * HX + ix + 1;
  }
  __device__ static bool on_edge(int i) {
    int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
    return (TZ > 1 && (iz == 0 || iz == TZ - 1)) || iy == 0 || iy == TY - 1 ||
           ix == 0 || ix == TX - 1;
  }
};

// Neighbour tiles reached from owned point i along the stencil offsets in
// `bits` (a subset of the point's 14 / 6 offsets), as a 27-bit set: bit
// (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) for tile offset (dz, dy, dx).
// Offsets that stay inside the tile add nothing.
template <int TZ, int TY, int TX>
__device__ __forceinline__ uint32_t out_dirs(int i, uint32_t bits) {
  const int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
  uint32_t d = 0;
  while (bits) {
    const int j = __builtin_ctz(bits);
    bits &= bits - 1;
    const int z = iz + off_z(j), y = iy + off_y(j), x = ix + off_x(j);
    const int dz = z < 0 ? -1 : (z >= TZ ? 1 : 0), dy = y < 0 ? -1 : (y >= TY ? 1 : 0),
              dx = x < 0 ? -1 : (x >= TX ? 1 : 0);
    if (dz | dy | dx) d |= 1u << ((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1));
  }
  return d;
}

// OR of v over the workgroup (every thread gets it)
__device__ __forceinline__ uint32_t block_or32(uint32_t v) {
  __shared__ uint32_t w[kWaves];
  v = wave_reduce(v, OpOr{});
  if (lane() == 0) w[wave()] = v;
  __syncthreads();
  uint32_t r = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) r |= w[q];
  __syncthreads();
  return r;
}

// OR of v over the workgroup (every thread gets it)
__device__ __forceinline__ uint64_t block_or64(uint64_t v) {
  __shared__ uint64_t w[kWaves];
  v = wave_reduce(v, OpOr{});
  if (lane() == 0) w[wave()] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) r |= w[q];
  __syncthreads();
  return r;
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// index.  Give each XCD a contiguous range of tiles instead, so that tiles
// that share halo data share an L2: workgroup b (of n) takes tile
// start(b % 8) + b / 8.  A bijection of [0, n); only locality depends on
// the dealing order.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t x = b & 7u, per = n >> 3, rem = n & 7u;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

// Colour of a tile: the parity of the sum of its tile coordinates (a
// checkerboard: face and corner neighbours have the other colour, edge
// neighbours the same).
__device__ __forceinline__ uint32_t tile_colour(int tz, int ty, int tx) {
  return (uint32_t)((tz + ty + tx) & 1);
}

// neighbour directions (27-direction set, bit (dz+1)*9 + (dy+1)*3 + dx+1)
// towards a tile of the same colour: two nonzero offsets
constexpr uint32_t same_colour_dirs() {
  uint32_t m = 0;
  for (int d = 0; d < 27; ++d) {
    const int nz = (d / 9 != 1) + ((d / 3) % 3 != 1) + (d % 3 != 1);
    if (nz == 2) m |= 1u << d;
  }
  return m;
}

// Tile of block b in a launch over the tiles of one colour: the (b mod hx)-th
// tile of that colour in tile row b / hx (hx: half a row, rounded up); none
// (ntiles) for the last block of a row that has one tile fewer.
__device__ __forceinline__ uint32_t colour_tile(uint32_t b, uint32_t colour, const Tiling& tl) {
  const uint32_t hx = (uint32_t)(tl.ntx + 1) / 2;
  const uint32_t row = b / hx, tz = row / (uint32_t)tl.nty, ty = row % (uint32_t)tl.nty;
  const uint32_t tx = ((colour + tz + ty) & 1u) + 2 * (b % hx);
  return tx < (uint32_t)tl.ntx ? (tz * tl.nty + ty) * tl.ntx + tx : tl.ntiles;
}

struct TileCoord {
  int tz, ty, tx, z0, y0, x0;
};

template <int TZ, int TY, int TX>
__device__ __forceinline__ TileCoord tile_coord(uint32_t t, const Tiling& tl) {
  TileCoord c;
  c.tz = (int)(t / (uint32_t)(tl.nty * tl.ntx));
  c.ty = (int)((t / (uint32_t)tl.ntx) % (uint32_t)tl.nty);
  c.tx = (int)(t % (uint32_t)tl.ntx);
  c.z0 = c.tz * TZ;
  c.y0 = c.ty * TY;
  c.x0 = c.tx * TX;
  return c;
}

// local fixed point of the tile (masks of the owned points in registers)
// the relaxation-iteration slots of the single-field counters block
__device__ __forceinline__ unsigned long long* relax_total(uint32_t* counters) {
  return (unsigned long long*)(counters + kRelaxWord);
}

// Lower neighbours of a point as LDS offsets for the relaxation: up to three
// 10-bit fields (offset + 512; an unused field holds 512, the point itself),
// the count in bits 30-31; more than three: kDense (the full mask is used).
constexpr uint32_t kDense = 0xffffffffu;
template <int TZ, int TY, int TX>
__device__ __forceinline__ uint32_t walk_code(uint32_t m) {
  using G = TileGeom<TZ, TY, TX>;
  const uint32_t n = (uint32_t)__popc(m);
  if (n > 3) return kDense;
  uint32_t code = n << 30 | 512u | 512u << 10 | 512u << 20;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    if (m) {
      const int j = __builtin_ctz(m);
      m &= m - 1;
      code += (uint32_t)off_lin(j, G::HX, G::HY * G::HX) << (10 * f);
    }
  }
  return code;
}

// The best raise of the point at LDS index li from all its stencil
// neighbours, selected by its lower-neighbour mask m without branches or
// compares: bit j of m widened to an all-ones / zero word masks the
// neighbour's subbin, and for an even j (a neighbour of higher index, weight
// 1) subtracting the widened bit adds the weight only where the bit is set.
// The maxima fold three at a time.
template <int NJ, int HX, int HXY>
__device__ __forceinline__ uint32_t dense_best(const uint32_t* S, int li, uint32_t m,
                                               uint32_t cur) {
  uint32_t c[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const uint32_t v = S[li + kOff[j][0] * HXY + kOff[j][1] * HX + kOff[j][2]];
    const uint32_t w = (uint32_t)((int32_t)(m << (31 - j)) >> 31);
    // one AND (kept as written: the compiler would otherwise turn the masked
    // maximum back into a compare and a select)
    uint32_t vw;
    asm("v_and_b32 %0, %1, %2" : "=v"(vw) : "v"(v), "v"(w));
    c[j] = (j & 1) ? vw : vw - w;
  }
  uint32_t a = max(max(cur, c[0]), c[1]);
  uint32_t b = max(max(c[2], c[3]), c[4]);
  uint32_t r = max(max(a, b), c[5]);
  if constexpr (NJ > 6) {
    const uint32_t d = max(max(c[6], c[7]), c[8]);
    const uint32_t e = max(max(c[9], c[10]), c[11]);
    const uint32_t f = max(max(c[12], c[13]), d);
    r = max(max(r, e), f);
  }
  return r;
}

// Mask bits j of a point's flags spread over bytes: byte b of word r is
// 0xff when bit 4r + b is set, so that an SDWA operand sign-extends byte b
// to the all-ones / zero word dense_best builds with one instruction per
// neighbour.
template <int NW>
__device__ __forceinline__ void spread_mask(uint32_t m, uint32_t (&pk)[NW]) {
#pragma unroll
  for (int r = 0; r < NW; ++r) {
    const uint32_t x = (m >> (4 * r)) & 0xfu;
    const uint32_t y = (x * 0x00204081u) & 0x01010101u;  // bit b of x to bit 8b
    pk[r] = (y << 8) - y;                                  // 0x01 -> 0xff
  }
}
// v & sext(byte B of p), and (v & sext(byte B of p)) - sext(byte B of p)
template <int B>
__device__ __forceinline__ uint32_t and_sext(uint32_t v, uint32_t p) {
  uint32_t r;
  if constexpr (B == 0)
    asm("v_and_b32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0" : "=v"(r) : "v"(v), "v"(p));
  else if constexpr (B == 1)
    asm("v_and_b32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1" : "=v"(r) : "v"(v), "v"(p));
  else if constexpr (B == 2)
    asm("v_and_b32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2" : "=v"(r) : "v"(v), "v"(p));
  else
    asm("v_and_b32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3" : "=v"(r) : "v"(v), "v"(p));
  return r;
}
template <int B>
__device__ __forceinline__ uint32_t sub_sext(uint32_t v, uint32_t p) {
  uint32_t r;
  if constexpr (B == 0)
    asm("v_sub_u32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0" : "=v"(r) : "v"(v), "v"(p));
  else if constexpr (B == 1)
    asm("v_sub_u32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1" : "=v"(r) : "v"(v), "v"(p));
  else if constexpr (B == 2)
    asm("v_sub_u32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2" : "=v"(r) : "v"(v), "v"(p));
  else
    asm("v_sub_u32_sdwa %0, %1, sext(%2) dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3" : "=v"(r) : "v"(v), "v"(p));
  return r;
}
// the masked candidates of neighbours J.. (J a compile-time constant)
template <int J, int NJ, int HX, int HXY, int NW>
__device__ __forceinline__ void pk_cands(const uint32_t* S, int li, const uint32_t (&pk)[NW],
                                         uint32_t* c) {
  if constexpr (J < NJ) {
    const uint32_t v = S[li + kOff[J][0] * HXY + kOff[J][1] * HX + kOff[J][2]];
    const uint32_t vw = and_sext<J & 3>(v, pk[J >> 2]);
    if constexpr (J & 1) c[J] = vw;
    else c[J] = sub_sext<J & 3>(vw, pk[J >> 2]);
    pk_cands<J + 1, NJ, HX, HXY, NW>(S, li, pk, c);
  }
}
// dense_best with the mask spread over bytes (spread_mask)
template <int NJ, int HX, int HXY, int NW>
__device__ __forceinline__ uint32_t dense_best_pk(const uint32_t* S, int li, const uint32_t (&pk)[NW],
                                                  uint32_t cur) {
  uint32_t c[NJ];
  pk_cands<0, NJ, HX, HXY, NW>(S, li, pk, c);
  uint32_t a = max(max(cur, c[0]), c[1]);
  uint32_t b = max(max(c[2], c[3]), c[4]);
  uint32_t r = max(max(a, b), c[5]);
  if constexpr (NJ > 6) {
    const uint32_t d = max(max(c[6], c[7]), c[8]);
    const uint32_t e = max(max(c[9], c[10]), c[11]);
    const uint32_t f = max(max(c[12], c[13]), d);
    r = max(max(r, e), f);
  }
  return r;
}

// Local fixed point of the tile (masks of the owned points in registers):
// Gauss-Seidel passes over the owned points until none rises; the halo is
// fixed.  Only points with a same-bin lower neighbour can rise; in a 3D
// tile whose wave holds at most 64 of them over its slots, the wave first
// gathers them into one lane each (a per-wave list in LDS), so that a pass
// costs one step per wave instead of one per slot, and each listed point
// with at most three lower neighbours reads them at precomputed offsets
// (walk_code: three loads issued back to back).  Otherwise a pass visits the
// slots and walks the mask bits.  When some lane of the wave has more than
// three lower neighbours, the wave loads all stencil neighbours and selects
// under the mask.  Adds the pass count to one of 64 statistics slots
// itot[t % 64].  PK (3D tiles): the slots' masks are spread over bytes once
// (spread_mask) and the dense visit masks with one SDWA instruction per
// neighbour: fewer vector instructions, 16 more registers (used by the
// float64 first pass and the repair of four-slot tiles; the float32 first
// pass loses more occupancy than it saves).
template <int TZ, int TY, int TX, bool PK = false>
__device__ void relax(uint32_t* S, const uint16_t* mk, uint32_t* counters,
                      unsigned long long* itot, uint32_t t) {
  using G = TileGeom<TZ, TY, TX>;
  constexpr int NJ = TZ == 1 ? 6 : 14;  // 2D tiles: the in-plane offsets only
  static_assert(G::H < 4096, "halo index in 12 bits");
  __shared__ uint32_t wl_pt[kThreads], wl_cd[kThreads];  // wave w: entries [64w, 64w + 64)
  // a listed point: rise to the best of its lower neighbours (a positive
  // offset, even j, reaches a higher index and adds one)
  auto step = [&](int li, uint32_t m, uint32_t cd) -> bool {
    const uint32_t cur = S[li];
    uint32_t best = cur;
    if (__ballot(cd == kDense)) {
      best = dense_best<NJ, G::HX, G::HY * G::HX>(S, li, m, cur);
    } else {
      const int o0 = (int)(cd & 1023u) - 512, o1 = (int)((cd >> 10) & 1023u) - 512,
                o2 = (int)((cd >> 20) & 1023u) - 512;
      const uint32_t c0 = S[li + o0] + (o0 > 0), c1 = S[li + o1] + (o1 > 0),
                     c2 = S[li + o2] + (o2 > 0);
      best = max(max(best, c0), max(c1, c2));
    }
    if (best > cur) {
      S[li] = best;
      return true;
    }
    return false;
  };
  // gather this wave's candidate points (3D tiles; in 2D fields same-bin
  // neighbours are common and the lists rarely fit)
  constexpr bool kList = TZ > 1;
  constexpr int LP = kList ? G::PER : 1;
  uint64_t act[LP];  // wave-uniform
  uint32_t n = kList ? 0u : 65u;
#pragma unroll
  for (int k = 0; k < (kList ? G::PER : 0); ++k) {
    act[k] = __ballot(mk[k] != 0);
    n += (uint32_t)__popcll(act[k]);
  }
  const bool listed = n <= 64;
  if (kList && listed) {
    uint32_t base = 0;
#pragma unroll
    for (int k = 0; k < LP; ++k) {
      if (mk[k]) {
        const uint32_t pos = base + (uint32_t)__popcll(act[k] & ((1ull << lane()) - 1ull));
        wl_pt[wave() * 64 + pos] =
            (uint32_t)G::local(threadIdx.x + k * kThreads) | (uint32_t)mk[k] << 12;
        wl_cd[wave() * 64 + pos] = walk_code<TZ, TY, TX>(mk[k]);
      }
      base += (uint32_t)__popcll(act[k]);
    }
  }
  uint32_t my_pt = 0, my_cd = 0;
  __builtin_amdgcn_wave_barrier();
  if (listed && (uint32_t)lane() < n) {
    my_pt = wl_pt[wave() * 64 + lane()];
    my_cd = wl_cd[wave() * 64 + lane()];
  }
  // slot k of this thread lies kSlot LDS words after slot 0
  const int li0 = G::local(threadIdx.x);
  // whether any point rose in pass p: flag[p % 3], set by the waves that
  // raised one, read by all after the pass's barrier; thread 0 clears
  // flag[(p + 1) % 3] during pass p (last read after the barrier of pass
  // p - 2, next set in pass p + 1), so one barrier per pass suffices
  __shared__ uint32_t flag[3];
  if (threadIdx.x < 3) flag[threadIdx.x] = 0;
  __syncthreads();
  constexpr int NW = (NJ + 3) / 4;
  uint32_t pk[PK && TZ > 1 ? G::PER : 1][NW];
  if constexpr (PK && TZ > 1) {
#pragma unroll
    for (int k = 0; k < G::PER; ++k) spread_mask<NW>(mk[k], pk[k]);
  }
  int iters = 0;
  for (;;) {
    int changed = 0;
    if (threadIdx.x == 0) flag[(iters + 1) % 3] = 0;
    if (listed) {
      if (my_pt && step((int)(my_pt & 4095u), my_pt >> 12, my_cd)) changed = 1;
    } else {
      // Gauss-Seidel along the thread's slots (one column of points along
      // z in a 3D tile, one row in four in a 2D tile), in alternating
      // directions from pass to pass, so a chain along that axis crosses
      // the tile in a pass or two whichever way it runs
      if constexpr (PK && TZ > 1) {
        // the slots' masks spread over bytes once per run (below), slot
        // order fixed at compile time in both directions
        auto visit = [&](int k) {
          if (!mk[k]) return;
          const int li = li0 + k * G::kSlot;
          const uint32_t cur = S[li];
          const uint32_t best = dense_best_pk<NJ, G::HX, G::HY * G::HX>(S, li, pk[k], cur);
          if (best > cur) {
            S[li] = best;
            changed = 1;
          }
        };
        if (iters & 1) {
#pragma unroll
          for (int kk = 0; kk < G::PER; ++kk) visit(G::PER - 1 - kk);
        } else {
#pragma unroll
          for (int kk = 0; kk < G::PER; ++kk) visit(kk);
        }
      } else {
      const bool rev = iters & 1;
#pragma unroll 2
      for (int kk = 0; kk < G::PER; ++kk) {
        const int k = rev ? G::PER - 1 - kk : kk;
        const uint32_t m = mk[k];
        if (!m) continue;
        const int li = li0 + k * G::kSlot;
        const uint32_t cur = S[li];
        // every stencil neighbour at once (one LDS round trip), masked
        const uint32_t best = dense_best<NJ, G::HX, G::HY * G::HX>(S, li, m, cur);
        if (best > cur) {
          S[li] = best;
          changed = 1;
        }
      }
      }
    }
    if (__ballot(changed) && lane() == 0) flag[iters % 3] = 1;
    __syncthreads();
    if (!flag[iters % 3]) break;
    if (++iters > G::NPT + 2) {  // unreachable: the order inside a tile is acyclic
      if (threadIdx.x == 0) atomicOr(&counters[0], 1u);
      break;
    }
  }
  if (threadIdx.x == 0) atomicAdd(&itot[t % 64], (unsigned long long)(iters + 1));
}

// ------------------------------------------------------------------ levels
// 2D tiles.  The level of an owned point is the length of the longest path
// of same-bin lower neighbours inside the tile that ends at it (0: no lower
// neighbour inside).  Taking the points level by level, each after every
// level below it, visits every point once with all its lower neighbours
// already final: one pass in a topological order of the tile's part of the
// order graph reaches the tile's fixed point for a fixed halo (the raising
// rule of Alg. 2).  The first pass finds the levels by peeling (Kahn's
// order: a point is ready once all its lower neighbours inside the tile are
// done) and keeps them, one byte per point, saturating at 255; later runs
// of the tile sort their points by the kept levels.  A 2D tile holds eight
// slots per thread, so a relaxation pass costs eight visits per wave, while
// a level costs one visit of the waves its points fall to: levels pay off
// there.  3D tiles (four slots per thread, and more levels per tile) keep
// the relaxation passes.

// stencil offsets j of owned point i whose neighbour lies inside the tile
template <int TZ, int TY, int TX>
__device__ __forceinline__ uint32_t inside_bits(int i) {
  constexpr int NJ = TZ == 1 ? 6 : 14;
  const int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
  uint32_t b = 0;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int z = iz + kOff[j][0], y = iy + kOff[j][1], x = ix + kOff[j][2];
    if (z >= 0 && z < TZ && y >= 0 && y < TY && x >= 0 && x < TX) b |= 1u << j;
  }
  return b;
}

// owned-index offset of stencil offset j (known only at run time)
template <int TZ, int TY, int TX>
__device__ __forceinline__ int own_off(int j) {
  return off_z(j) * (TY * TX) + off_y(j) * TX + off_x(j);
}

// the best raise of the point at LDS index li (lower-neighbour mask m)
template <int TZ, int TY, int TX>
__device__ __forceinline__ uint32_t raise_of(const uint32_t* S, int li, uint32_t m, uint32_t cur) {
  using G = TileGeom<TZ, TY, TX>;
  constexpr int NJ = TZ == 1 ? 6 : 14;
  if (__ballot(__popc(m) > 3)) return dense_best<NJ, G::HX, G::HY * G::HX>(S, li, m, cur);
  uint32_t best = cur;
  while (m) {
    const int j = __builtin_ctz(m);
    m &= m - 1;
    const uint32_t c = S[li + off_lin(j, G::HX, G::HY * G::HX)] + ((j & 1) ? 0u : 1u);
    best = c > best ? c : best;
  }
  return best;
}

// LDS of the peeling pass: per owned point its masks (lower | inside upper
// << 16), its count of unfinished lower neighbours inside the tile (bytes),
// its level (bytes) and the ready list; three list counters.
template <int TZ, int TY, int TX>
struct KahnLds {
  static constexpr int NPT = TZ * TY * TX;
  static constexpr int kBytes = NPT * 4 + NPT + NPT + NPT * 2 + 16;
};

// First pass of a tile with the halo subbins at 0: peel the tile's points
// level by level (a point joins the ready list when its last lower
// neighbour inside the tile is done) and raise each as it is taken.  Leaves
// the levels in lvb.  Every thread must call it; returns the number of
// levels (block-uniform).
template <int TZ, int TY, int TX>
__device__ int kahn_relax(uint32_t* S, uint8_t* lds, const uint16_t* mk, const uint16_t* up,
                          uint8_t*& lvb_out) {
  using G = TileGeom<TZ, TY, TX>;
  constexpr int NPT = G::NPT;
  uint32_t* W = (uint32_t*)lds;
  uint32_t* cnt4 = (uint32_t*)(lds + NPT * 4);
  uint8_t* cnt = (uint8_t*)cnt4;
  uint8_t* lvb = lds + NPT * 4 + NPT;
  uint16_t* list = (uint16_t*)(lds + NPT * 6);
  uint32_t* kc = (uint32_t*)(lds + NPT * 8);
  lvb_out = lvb;
  if (threadIdx.x < 3) kc[threadIdx.x] = 0;
  uint32_t deg[G::PER], wk[G::PER];
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    const int i = threadIdx.x + k * kThreads;
    const uint32_t inb = inside_bits<TZ, TY, TX>(i);
    wk[k] = (uint32_t)mk[k] | (uint32_t)(up[k] & inb) << 16;
    deg[k] = (uint32_t)__popc(mk[k] & inb);
    W[i] = wk[k];
    cnt[i] = (uint8_t)deg[k];
    lvb[i] = 0;
  }
  __syncthreads();
  // level 0: nothing below inside the tile, and something to do (a lower
  // neighbour in the halo to raise from, or upper neighbours to release)
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    const bool go = deg[k] == 0 && wk[k] != 0;
    const uint64_t rb = __ballot(go);
    if (rb) {
      uint32_t base = 0;
      if (lane() == 0) base = atomicAdd(&kc[0], (uint32_t)__popcll(rb));
      base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
      if (go) list[base + lane_prefix(rb)] = (uint16_t)(threadIdx.x + k * kThreads);
    }
  }
  __syncthreads();
  int beg = 0, end = (int)kc[0], level = 0;
  while (beg < end) {
    const int nxt = (level + 1) % 3;
    if (threadIdx.x == 0) kc[(level + 2) % 3] = 0;  // read two levels ago, appended next level
    for (int e = beg + (int)threadIdx.x; e < end; e += kThreads) {
      const int i = list[e];
      const uint32_t w = W[i];
      const uint32_t m = w & 0xffffu;
      if (m) {
        const int li = G::local(i);
        const uint32_t cur = S[li];
        const uint32_t b = raise_of<TZ, TY, TX>(S, li, m, cur);
        if (b > cur) S[li] = b;
      }
      lvb[i] = (uint8_t)(level < 255 ? level : 255);
      uint32_t u = w >> 16;
      while (u) {
        const int j = __builtin_ctz(u);
        u &= u - 1;
        const int q = i + own_off<TZ, TY, TX>(j);
        const uint32_t sh = 8u * (uint32_t)(q & 3);
        const uint32_t old = atomicSub(&cnt4[q >> 2], 1u << sh);
        const bool ready = ((old >> sh) & 0xffu) == 1u;
        const uint64_t rb = __ballot(ready);
        if (rb) {
          const int leader = __builtin_ctzll(rb);
          uint32_t base = 0;
          if (lane() == leader) base = atomicAdd(&kc[nxt], (uint32_t)__popcll(rb));
          base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
          if (ready) list[end + base + lane_prefix(rb)] = (uint16_t)q;
        }
      }
    }
    __syncthreads();
    beg = end;
    end += (int)kc[nxt];
    ++level;
  }
  return level;
}

// A later run of a tile: its points sorted by their kept levels (lv, 255 =
// unknown), then raised level by level.  Levels of at most 64 points run on
// wave 0 alone, with no block barrier between consecutive ones (a wave's
// LDS accesses are ordered); a block barrier separates the rest.  Returns
// the number of levels, or -1 (block-uniform) when some point's level is
// unknown, before touching S.
template <int TZ, int TY, int TX>
__device__ int level_relax(uint32_t* S, const uint16_t* mk, const uint8_t* lv) {
  using G = TileGeom<TZ, TY, TX>;
  __shared__ uint32_t hist[257];
  __shared__ uint32_t list[G::NPT];
  for (int h = threadIdx.x; h < 257; h += kThreads) hist[h] = 0;
  __syncthreads();
  bool unknown = false;
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    if (mk[k]) {
      if (lv[k] == 255) unknown = true;
      else atomicAdd(&hist[lv[k]], 1u);
    }
  }
  if (__syncthreads_or(unknown)) return -1;
  if (threadIdx.x < 64) {
    // exclusive scan of the 255 counts, four per lane; hist[256] = levels
    uint32_t v[4], t = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = hist[4 * lane() + q];
      t += v[q];
    }
    const uint32_t incl = wave_scan_u32(t);
    uint32_t run = incl - t;
    int top = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      hist[4 * lane() + q] = run;
      run += v[q];
      if (v[q]) top = 4 * lane() + q;
    }
    top = wave_reduce(top, OpMax{});
    if (lane() == 0) hist[256] = (uint32_t)(top + 1);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    if (mk[k]) {
      const uint32_t pos = atomicAdd(&hist[lv[k]], 1u);
      list[pos] = (uint32_t)(threadIdx.x + k * kThreads) | (uint32_t)mk[k] << 12;
    }
  }
  __syncthreads();
  // hist[l] is now the end of level l
  const int nlev = (int)hist[256];
  int beg = 0;
  bool wide = false;
  for (int l = 0; l < nlev; ++l) {
    const int end = (int)hist[l];
    const bool w = end - beg > 64;
    if (w || wide) {
      __syncthreads();
      wide = false;
    }
    for (int e = beg + (int)threadIdx.x; e < end; e += kThreads) {
      const uint32_t ent = list[e];
      const int li = G::local((int)(ent & 4095u));
      const uint32_t cur = S[li];
      const uint32_t b = raise_of<TZ, TY, TX>(S, li, ent >> 12, cur);
      if (b > cur) S[li] = b;
    }
    wide = wide || w;
    beg = end;
  }
  __syncthreads();
  return nlev;
}

// mark the neighbour tiles in `dirs` (27-bit set, see out_dirs) for sweep
// `next`; one atomic per block adds the number of newly marked tiles to
// counters[1 + next % 64]
__device__ void mark_neighbours(uint32_t dirs, const TileCoord& c, const Tiling& tl,
                                uint32_t* stamp, uint32_t* counters,
                                uint32_t next) {
  bool newly = false;
  if (threadIdx.x < 27 && ((dirs >> threadIdx.x) & 1u)) {
    int dz = (int)threadIdx.x / 9 - 1, dy = ((int)threadIdx.x / 3) % 3 - 1,
        dx = (int)threadIdx.x % 3 - 1;
    int nz = c.tz + dz, ny = c.ty + dy, nx = c.tx + dx;
    if ((dz | dy | dx) != 0 && nz >= 0 && nz < tl.ntz && ny >= 0 &&
        ny < tl.nty && nx >= 0 && nx < tl.ntx) {
      uint32_t u = ((uint32_t)nz * tl.nty + ny) * tl.ntx + nx;
      uint32_t prev = atomicMax(&stamp[u], next);
      newly = prev < next;
    }
  }
  if (threadIdx.x < 64) {
    uint64_t m = __ballot(newly);
    if (threadIdx.x == 0 && m)
      atomicAdd(&counters[1 + (next & 63)], (uint32_t)__popcll(m));
  }
}

// mark_neighbours, and also append the newly marked tiles to the work list
// of sweep `next` (lists: two arrays of tl.ntiles items, sweep parity; each
// tile is listed at most once per sweep, so a list never overflows)
__device__ void mark_list1(uint32_t dirs, const TileCoord& c, const Tiling& tl, uint32_t* stamp,
                           uint32_t* counters, uint32_t* lists, uint32_t next) {
  if (threadIdx.x >= 64) return;
  bool newly = false;
  uint32_t u = 0;
  if (threadIdx.x < 27 && ((dirs >> threadIdx.x) & 1u)) {
    const int dz = (int)threadIdx.x / 9 - 1, dy = ((int)threadIdx.x / 3) % 3 - 1,
              dx = (int)threadIdx.x % 3 - 1;
    const int nz = c.tz + dz, ny = c.ty + dy, nx = c.tx + dx;
    if ((dz | dy | dx) != 0 && nz >= 0 && nz < tl.ntz && ny >= 0 && ny < tl.nty && nx >= 0 &&
        nx < tl.ntx) {
      u = ((uint32_t)nz * tl.nty + ny) * tl.ntx + nx;
      newly = atomicMax(&stamp[u], next) < next;
    }
  }
  const uint64_t m = __ballot(newly);
  if (!m) return;
  uint32_t pos = 0;
  if (threadIdx.x == 0) pos = atomicAdd(&counters[1 + (next & 63)], (uint32_t)__popcll(m));
  pos = __shfl(pos, 0, 64);
  if (newly) lists[(next & 1) * tl.ntiles + pos + lane_prefix(m)] = u;
}

// ------------------------------------------------------------- repair queue
// Tile item of the neighbour in direction bit `d` (27-direction set) of the
// tile at c, in a field whose tile items start at t0.
__device__ __forceinline__ uint32_t dir_tile(int d, const TileCoord& c, const Tiling& tl,
                                             uint32_t t0) {
  const int nz = c.tz + d / 9 - 1, ny = c.ty + (d / 3) % 3 - 1, nx = c.tx + d % 3 - 1;
  return t0 + ((uint32_t)nz * tl.nty + ny) * tl.ntx + nx;
}
__device__ __forceinline__ bool dir_inside(int d, const TileCoord& c, const Tiling& tl) {
  const int nz = c.tz + d / 9 - 1, ny = c.ty + (d / 3) % 3 - 1, nx = c.tx + d % 3 - 1;
  return d != 13 && nz >= 0 && nz < tl.ntz && ny >= 0 && ny < tl.nty && nx >= 0 &&
         nx < tl.ntx;
}

// Publish a listed tile item in the ring (any lane): a tail ticket, then
// wait until the slot's previous item has been taken (never long: at most
// as many items as tiles are in the ring at once).  Release: what the
// caller did before (counting the item as pending) is visible to the worker
// that takes it.
// Watchdog of a queue wait: true once the queue has shown no progress (tail
// and pending unchanged) for kQueueStall ticks, or another wait gave up.
struct QueueWatch {
  unsigned long long tail = ~0ull, since = 0;
  int32_t pending = -1;
  __device__ bool stalled(const QueueRef& Q) {
    if (__hip_atomic_load(&Q.q->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
    const unsigned long long tl =
        __hip_atomic_load(&Q.q->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t pd = __hip_atomic_load(&Q.q->pending, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long now = wall_clock64();
    if (tl != tail || pd != pending) {
      tail = tl;
      pending = pd;
      since = now;
      return false;
    }
    if (now - since < kQueueStall) return false;
    atomicOr(&Q.q->err, 1u);
    return true;
  }
};

__device__ void q_publish(const QueueRef& Q, uint32_t item) {
  const unsigned long long pos = atomicAdd(&Q.q->tail, 1ull);
  unsigned long long* slot = Q.ring + (pos & ((1ull << Q.cap_log2) - 1ull));
  const uint32_t lap2 = (uint32_t)(pos >> Q.cap_log2) * 2u;
  QueueWatch w;
  for (uint32_t k = 0;
       (uint32_t)(__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) !=
       lap2;
       ++k) {
    if ((k & 63u) == 63u && w.stalled(Q)) return;
    __builtin_amdgcn_s_sleep(2);
  }
  __hip_atomic_store(slot, (unsigned long long)(lap2 + 1u) << 32 | item, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// List tile item `item` (any lane): nothing if it is listed already, else
// count it as pending and publish it.  The caller has released the subbins
// it wrote (a fence at agent scope) before listing; the worker that runs the
// item acquires them through its state word.
__device__ void q_push(const QueueRef& Q, uint32_t item, uint32_t depth) {
  atomicMax(&Q.depth[item], depth);
  if (__hip_atomic_fetch_or(&Q.st[item], TS_LISTED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
      TS_LISTED)
    return;
  atomicAdd(&Q.q->pending, 1);
  q_publish(Q, item);
}

// Take the next item from the ring (one thread of a workgroup): a head
// ticket, then wait for its slot to be filled; kNoTile once nothing is
// listed or running (nothing can be listed after that: only running tiles
// list others).
__device__ uint32_t q_pop(const QueueRef& Q) {
  const unsigned long long pos = atomicAdd(&Q.q->head, 1ull);
  unsigned long long* slot = Q.ring + (pos & ((1ull << Q.cap_log2) - 1ull));
  const uint32_t full = (uint32_t)(pos >> Q.cap_log2) * 2u + 1u;
  unsigned long long v;
  QueueWatch w;
  // back off while waiting: a thousand idle workers polling at full rate
  // would crowd the memory channel of the words they poll
  uint32_t nap = 1;
  for (uint32_t k = 0;; ++k) {
    v = __hip_atomic_load(slot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(v >> 32) == full) break;
    if ((k & 3u) == 3u &&
        __hip_atomic_load(&Q.q->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      return kNoTile;
    if ((k & 255u) == 255u && w.stalled(Q)) return kNoTile;
    for (uint32_t z = 0; z < nap; ++z) __builtin_amdgcn_s_sleep(8);
    nap = nap < 16u ? nap * 2u : 16u;
  }
  __hip_atomic_store(slot, (unsigned long long)(full + 1u) << 32, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  return (uint32_t)v;
}

// Decide what to do with a taken item t (one thread): true = run it now.
// * t is running on another worker (it was listed again during that run):
//   it parks on itself (direction 13) and is published again when that run
//   ends, so two runs of one tile never overlap (a slower run could
//   otherwise store smaller values over a faster one's).
// * t ran before in this repair: it parks on the first listed or running
//   neighbour of higher index that it depends on (its blockers, stored by
//   its first run), and is published again when that neighbour's run ends.
// * otherwise it runs (`first`: its first run in this repair): it clears
//   its listed bit, acquiring the subbins released by every worker that
//   listed it; a change after that lists it again.
// The parking handshakes (parked bit, then the other tile's state; the
// other tile at the end of its run: its state, then its parked word) are
// sequentially consistent, so no wake-up is lost; a parker that finds the
// other tile idle takes its bit back and publishes itself.
__device__ bool q_park(const QueueRef& Q, uint32_t t, uint32_t v, uint32_t bit) {
  __hip_atomic_fetch_or(&Q.parked[v], bit, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
  if (!(__hip_atomic_fetch_or(&Q.st[v], 0u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT) &
        (v == t ? TS_RUNNING : (TS_LISTED | TS_RUNNING)))) {
    if (__hip_atomic_fetch_and(&Q.parked[v], ~bit, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT) &
        bit)
      q_publish(Q, t);
  }
  return false;
}

__device__ bool q_claim(const QueueRef& Q, uint32_t t, const TileCoord& c, const Tiling& tl,
                        uint32_t t0, unsigned long long& parks, bool& first) {
  const uint32_t old =
      __hip_atomic_fetch_or(&Q.st[t], TS_RUNNING, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
  if (old & TS_RUNNING) {
    ++parks;
    return q_park(Q, t, t, 1u << 13);
  }
  if (old & TS_RAN) {
    uint32_t bl = __hip_atomic_load(&Q.blockers[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (bl) {
      const int d = 31 - __builtin_clz(bl);  // the farthest in index first
      bl &= ~(1u << d);
      const uint32_t v = dir_tile(d, c, tl, t0);
      if (!(__hip_atomic_load(&Q.st[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
            (TS_LISTED | TS_RUNNING)))
        continue;
      __hip_atomic_fetch_and(&Q.st[t], ~TS_RUNNING, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
      ++parks;
      return q_park(Q, t, v, 1u << (26 - d));
    }
  }
  first = !(old & TS_RAN);
  __hip_atomic_fetch_and(&Q.st[t], ~TS_LISTED, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  if (first)
    __hip_atomic_fetch_or(&Q.st[t], TS_RAN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// End of a run of tile t (wave 0 of its block): list the neighbour tiles in
// `dirs` (27-bit set, see out_dirs) after releasing the block's subbin
// stores, stop running, publish the tiles parked on t, and stop counting
// the run as pending.
__device__ void q_finish(uint32_t dirs, uint32_t t, const TileCoord& c, const Tiling& tl,
                         const QueueRef& Q, uint32_t t0, uint32_t depth) {
  if (dirs) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (threadIdx.x < 27 && ((dirs >> threadIdx.x) & 1u) && dir_inside((int)threadIdx.x, c, tl))
    q_push(Q, dir_tile((int)threadIdx.x, c, tl, t0), depth);
  uint32_t woke = 0;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_and(&Q.st[t], ~TS_RUNNING, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
    woke = __hip_atomic_exchange(&Q.parked[t], 0u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
  }
  woke = __shfl(woke, 0, 64);
  if (threadIdx.x < 27 && ((woke >> threadIdx.x) & 1u))
    q_publish(Q, dir_tile((int)threadIdx.x, c, tl, t0));
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(&Q.q->pending, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Same-bin flags of an owned point of a float64 tile whose halo bins span
// 2^31 or more: every neighbour in the grid re-quantized from its key (one
// at a time; a rare path).
template <int K, int TZ, int TY, int TX>
__device__ __forceinline__ uint32_t wide_same(const int64_t* Pk, int li, int64_t b, double inv,
                                              int z, int y, int x, const Box& box) {
  using G = TileGeom<TZ, TY, TX>;
  constexpr int NJ = TZ == 1 ? 6 : 14;
  uint32_t sm = 0;
#pragma unroll 1
  for (int j = 0; j < NJ; ++j) {
    const int zz = z + off_z(j), yy = y + off_y(j), xx = x + off_x(j);
    if (zz < 0 || zz >= box.nz || yy < 0 || yy >= box.ny || xx < 0 || xx >= box.nx) continue;
    const int64_t kq = Pk[li + off_lin(j, G::HX, G::HY * G::HX)];
    sm |= (uint32_t)(Traits<8>::q(Traits<8>::to_double(Traits<8>::unkey(kq)), inv) == b) << j;
  }
  return sm;
}

// First pass, fused: build the order flags of the owned points (a2, the
// flags of Alg. 1) from the bins and values of the tile and its halo, write
// them, then relax with halo subbins 0 (the first sweep of a3).
// Returns (block-uniform) the neighbour tiles to sweep next: those holding a
// point that has a nonzero boundary point of this tile as a same-bin lower
// neighbour (only their relaxation depends on it).
template <int K, int TZ, int TY, int TX>
__device__ __forceinline__ uint32_t tile0_body(const typename Traits<K>::Raw* __restrict__ x, Box box,
                           Tiling tl, Params* prm, typename Traits<K>::Bin* __restrict__ bins,
                           uint16_t* __restrict__ mask, uint32_t* __restrict__ sub,
                           uint32_t* counters, unsigned long long* itot, uint32_t t,
                           TileCoord& c, int hc = -1) {
  using Tr = Traits<K>;
  using G = TileGeom<TZ, TY, TX>;
  using Key = typename Tr::Bin;  // keys fit the signed type of the bins
  using Bin = typename Tr::Bin;
  // float32: key and bin of a halo point side by side, one 8-byte LDS read
  // per neighbour.  float64: the 8-byte key, and the low 32 bits of the bin
  // (12 instead of 16 bytes per point), which decide equality of two bins
  // exactly whenever the halo's bins span less than 2^31; a tile whose bins
  // span more ("wide") re-quantizes a neighbour's value to compare bins.
  using KB = uint2;
  constexpr int NJ = TZ == 1 ? 6 : 14;  // 2D: only the in-plane offsets
  constexpr int kKB = G::H * (K == 4 ? 8 : 12);
  // the subbins of the halo, then (2D) the peeling state, reuse the buffer
  constexpr int kS = G::H * 4 + (TZ == 1 ? KahnLds<TZ, TY, TX>::kBytes : 0);
  constexpr int kBytes = kKB > kS ? kKB : kS;
  constexpr int HL = (G::H + kThreads - 1) / kThreads;  // halo loads per thread
  __shared__ __attribute__((aligned(16))) uint8_t buf[kBytes];
  KB* P = (KB*)buf;                                  // float32
  int64_t* Pk = (int64_t*)buf;                       // float64: keys
  int32_t* Pb = (int32_t*)(buf + (K == 8 ? G::H * 8 : 0));  // float64: bin offsets
  uint32_t* S = (uint32_t*)buf;  // reused once the flags are built
  __shared__ int64_t s_rng[2][kWaves];  // float64: per-wave least / greatest bin
  int64_t bref = 0;   // float64: the halo's lowest bin
  bool wide = false;  // float64: the halo's bins span 2^31 or more

  c = tile_coord<TZ, TY, TX>(t, tl);
  {
    // the values of the halo (every load issued first); their bins are
    // computed here (Sec. IV-A), not read back from a separate pass
    typename Tr::Raw u[HL];
    // a halo inside the grid (most tiles): 32-bit offsets from the halo's
    // first point, every load unconditional, no bounds checks
    const bool hin = c.z0 - G::ZO >= 0 && c.z0 + TZ - 1 + G::ZO < box.nz && c.y0 >= 1 &&
                     c.y0 + TY < box.ny && c.x0 >= 1 && c.x0 + TX < box.nx &&
                     (uint64_t)box.ny * (uint64_t)box.nx * G::HZ < (1ull << 31);
    if (hin) {
      const int64_t g0 = ((int64_t)(c.z0 - G::ZO) * box.ny + (c.y0 - 1)) * box.nx + (c.x0 - 1);
      const uint32_t nyx = (uint32_t)box.ny * (uint32_t)box.nx;
#pragma unroll
      for (int q = 0; q < HL; ++q) {
        const int i = threadIdx.x + q * kThreads;
        const uint32_t hz = (uint32_t)i / (G::HY * G::HX), hy = ((uint32_t)i / G::HX) % G::HY,
                       hx = (uint32_t)i % G::HX;
        const bool in = i < G::H;
        const typename Tr::Raw v =
            x[in ? g0 + (int64_t)(hz * nyx + hy * (uint32_t)box.nx + hx) : 0];
        u[q] = in ? v : (typename Tr::Raw)0;
      }
    } else {
#pragma unroll
      for (int q = 0; q < HL; ++q) {
        const int i = threadIdx.x + q * kThreads;
        u[q] = 0;
        if (i < G::H) {
          int hz = i / (G::HY * G::HX), hy = (i / G::HX) % G::HY, hx = i % G::HX;
          int z = c.z0 + hz - G::ZO, y = c.y0 + hy - 1, xx = c.x0 + hx - 1;
          if (z >= 0 && z < box.nz && y >= 0 && y < box.ny && xx >= 0 && xx < box.nx)
            u[q] = x[((int64_t)z * box.ny + y) * box.nx + xx];
        }
      }
    }
    const double inv = prm->inv;
    bool bad_v = false, bad_r = false;
    if constexpr (K == 4) {
#pragma unroll
      for (int q = 0; q < HL; ++q) {
        const int i = threadIdx.x + q * kThreads;
        if (i < G::H) {
          bad_v |= !Tr::finite(u[q]);
          const int64_t bq = Tr::q(Tr::to_double(u[q]), inv);
          bad_r |= bq > Tr::kBinLimit || bq < -Tr::kBinLimit;
          KB e;
          e.x = (uint32_t)(Key)Tr::key(u[q]);
          e.y = (uint32_t)(Bin)bq;
          P[i] = e;
        }
      }
    } else {
      // bins of the halo points in the grid (others are never compared),
      // their least and greatest over the block, then keys and offsets
      int64_t lo = INT64_MAX, hi = INT64_MIN;
#pragma unroll
      for (int q = 0; q < HL; ++q) {
        const int i = threadIdx.x + q * kThreads;
        if (i < G::H) {
          bad_v |= !Tr::finite(u[q]);
          const int64_t bq = Tr::q(Tr::to_double(u[q]), inv);
          bad_r |= bq > Tr::kBinLimit || bq < -Tr::kBinLimit;
          Pk[i] = Tr::key(u[q]);
          Pb[i] = (int32_t)(uint32_t)(uint64_t)bq;
          const int hz = i / (G::HY * G::HX), hy = (i / G::HX) % G::HY, hx = i % G::HX;
          const int z = c.z0 + hz - G::ZO, y = c.y0 + hy - 1, xx = c.x0 + hx - 1;
          if (z >= 0 && z < box.nz && y >= 0 && y < box.ny && xx >= 0 && xx < box.nx) {
            lo = bq < lo ? bq : lo;
            hi = bq > hi ? bq : hi;
          }
        }
      }
      lo = wave_reduce(lo, OpMin{});
      hi = wave_reduce(hi, OpMax{});
      if (lane() == 0) {
        s_rng[0][wave()] = lo;
        s_rng[1][wave()] = hi;
      }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        lo = s_rng[0][w] < lo ? s_rng[0][w] : lo;
        hi = s_rng[1][w] > hi ? s_rng[1][w] : hi;
      }
      // hi >= lo: the tile's owned points lie in the grid
      bref = lo;
      wide = (uint64_t)hi - (uint64_t)lo >= (1ull << 31);
    }
    if (bad_v) set_status(prm, ST_NONFINITE);
    if (bad_r) set_status(prm, ST_RANGE);
  }
  __syncthreads();
  // key and bin of the halo point at LDS index l (the bin compared with
  // another point's only for equality, so float64 uses its offset)
  auto key_at = [&](int l) -> Key {
    if constexpr (K == 4) return (Key)(int32_t)P[l].x;
    else return (Key)Pk[l];
  };
  auto bin_at = [&](int l) -> int64_t {
    if constexpr (K == 4) return (int64_t)(int32_t)P[l].y;
    else return (int64_t)Pb[l];  // low 32 bits: equality only (not wide)
  };

  // the halo lies inside the grid: no neighbour needs a bounds check
  const bool inner = c.z0 - G::ZO >= 0 && c.z0 + TZ - 1 + G::ZO < box.nz && c.y0 >= 1 &&
                     c.y0 + TY < box.ny && c.x0 >= 1 && c.x0 + TX < box.nx;
  // per owned point: mk = same bin and lower (the flags), up = same bin and
  // higher (the neighbours whose relaxation depends on this point)
  uint16_t mk[G::PER], up[G::PER];
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    const int i = threadIdx.x + k * kThreads;
    const int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
    const int z = c.z0 + iz, y = c.y0 + iy, xx = c.x0 + ix;
    uint32_t sm = 0, lm = 0;
    const int li = G::local(i);
    const Key kp = key_at(li);
    const int64_t bp = bin_at(li);  // float64: low 32 bits
    // float64: the whole bin (from its low bits and the halo's lowest bin,
    // or re-quantized when the halo is wide)
    int64_t bfull = bp;
    if constexpr (K == 8)
      bfull = wide ? Tr::q(Tr::to_double(Tr::unkey(kp)), prm->inv)
                   : bref + (int64_t)(uint32_t)((uint32_t)bp - (uint32_t)bref);
    if (z < box.nz && y < box.ny && xx < box.nx)  // for the encoder
      bins[((int64_t)z * box.ny + y) * box.nx + xx] = (Bin)bfull;
    if (inner) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int ln = li + kOff[j][0] * (G::HY * G::HX) + kOff[j][1] * G::HX + kOff[j][2];
        const Key kq = key_at(ln);
        // branch-free: same bin, and lower in (value, index) order
        const bool lower = (kq < kp) | ((kq == kp) & ((j & 1) != 0));
        sm |= (uint32_t)(bin_at(ln) == bp) << j;
        lm |= (uint32_t)lower << j;
      }
      if (K == 8 && wide) sm = wide_same<K, TZ, TY, TX>(Pk, li, bfull, prm->inv, z, y, xx, box);
      mask[((int64_t)z * box.ny + y) * box.nx + xx] = (uint16_t)(sm & lm);
    } else if (z < box.nz && y < box.ny && xx < box.nx) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        int zz = z + kOff[j][0], yy = y + kOff[j][1], xq = xx + kOff[j][2];
        if (zz < 0 || zz >= box.nz || yy < 0 || yy >= box.ny || xq < 0 || xq >= box.nx)
          continue;
        const int ln = li + kOff[j][0] * (G::HY * G::HX) + kOff[j][1] * G::HX + kOff[j][2];
        const Key kq = key_at(ln);
        // odd j: the neighbour has the lower index
        const bool lower = (kq < kp) | ((kq == kp) & ((j & 1) != 0));
        sm |= (uint32_t)(bin_at(ln) == bp) << j;
        lm |= (uint32_t)lower << j;
      }
      if (K == 8 && wide) sm = wide_same<K, TZ, TY, TX>(Pk, li, bfull, prm->inv, z, y, xx, box);
      mask[((int64_t)z * box.ny + y) * box.nx + xx] = (uint16_t)(sm & lm);
    }
    mk[k] = (uint16_t)(sm & lm);
    up[k] = (uint16_t)(sm & ~lm);
  }
  __syncthreads();
  // halo subbins: 0, or (hc >= 0) those of the neighbour tiles of colour hc,
  // final from an earlier launch
  if (TZ > 1 && hc >= 0) {
    // loads in flight four at a time (points not taken read point 0)
#pragma unroll
    for (int q0 = 0; q0 < HL; q0 += 4) {
    uint32_t hv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = q0 + r;
      const int i = threadIdx.x + q * kThreads;
      const int hz = i / (G::HY * G::HX), hy = (i / G::HX) % G::HY, hx = i % G::HX;
      const int z = c.z0 + hz - G::ZO, y = c.y0 + hy - 1, xx = c.x0 + hx - 1;
      const bool own = hz >= G::ZO && hz < G::ZO + TZ && hy >= 1 && hy <= TY && hx >= 1 &&
                       hx <= TX;
      const bool take = i < G::H && !own && z >= 0 && z < box.nz && y >= 0 && y < box.ny &&
                        xx >= 0 && xx < box.nx &&
                        tile_colour(z / TZ, y / TY, xx / TX) == (uint32_t)hc;
      const uint32_t v = sub[take ? ((int64_t)z * box.ny + y) * box.nx + xx : 0];
      hv[r] = take ? v : 0u;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = threadIdx.x + (q0 + r) * kThreads;
      if (i < G::H) S[i] = hv[r];
    }
    }
  } else {
    for (int i = threadIdx.x; i < G::H; i += kThreads) {
      uint32_t v = 0;
      if (hc >= 0) {  // 2D tiles: one load at a time (fewer registers)
        const int hy = i / G::HX, hx = i % G::HX;
        const int y = c.y0 + hy - 1, xx = c.x0 + hx - 1;
        const bool own = hy >= 1 && hy <= TY && hx >= 1 && hx <= TX;
        if (!own && y >= 0 && y < box.ny && xx >= 0 && xx < box.nx &&
            tile_colour(c.z0, y / TY, xx / TX) == (uint32_t)hc)
          v = sub[((int64_t)c.z0 * box.ny + y) * box.nx + xx];
      }
      S[i] = v;
    }
  }
  __syncthreads();
  uint8_t* lvb = nullptr;
  if constexpr (TZ == 1) {
    const int nlev = kahn_relax<TZ, TY, TX>(S, buf + G::H * 4, mk, up, lvb);
    if (threadIdx.x == 0) atomicAdd(&itot[t % 64], (unsigned long long)(nlev + 1));
  } else {
    relax<TZ, TY, TX, K == 8>(S, mk, counters, itot, t);
  }
  uint32_t dirs = 0;
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    const int i = threadIdx.x + k * kThreads;
    const int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
    const int z = c.z0 + iz, y = c.y0 + iy, xx = c.x0 + ix;
    if (z < box.nz && y < box.ny && xx < box.nx) {
      const uint32_t v = S[G::local(i)];
      const int64_t g = ((int64_t)z * box.ny + y) * box.nx + xx;
      sub[g] = v;
      if (TZ == 1 && tl.lev) tl.lev[g] = lvb[i];
      if (v && up[k]) dirs |= out_dirs<TZ, TY, TX>(i, up[k]);
    }
  }
  return block_or32(dirs);
}

// Q.q null: mark the tiles to sweep next (and append them to the work list
// of sweep 1 when lists is given); else list them in the repair queue (the
// kernel boundary publishes the subbins).
template <int K, int TZ, int TY, int TX>
__global__ __launch_bounds__(kThreads) void k_tile0(
    const typename Traits<K>::Raw* __restrict__ x, Box box, Tiling tl, Params* prm,
    typename Traits<K>::Bin* __restrict__ bins,
    uint16_t* __restrict__ mask, uint32_t* __restrict__ sub, uint32_t* stamp,
    uint32_t* counters, uint32_t* lists, QueueRef Q, uint32_t colour) {
  TileCoord c;
  // colour 2: every tile; 0 / 1: the tiles of that colour, those of colour 1
  // taking the subbins of their neighbours of colour 0 as halo
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t t = colour < 2 ? colour_tile(b, colour, tl) : b;
  if (t >= tl.ntiles) return;
  uint32_t dirs = tile0_body<K, TZ, TY, TX>(x, box, tl, prm, bins, mask, sub, counters,
                                            relax_total(counters), t, c, colour == 1 ? 0 : -1);
  // tiles of colour 1 read the results of colour 0 in the next launch
  if (colour == 0) dirs &= same_colour_dirs();
  if (Q.q) {
    if (threadIdx.x < 27 && ((dirs >> threadIdx.x) & 1u) && dir_inside((int)threadIdx.x, c, tl))
      q_push(Q, dir_tile((int)threadIdx.x, c, tl, 0), 1);
  } else if (lists) {
    mark_list1(dirs, c, tl, stamp, counters, lists, 1);
  } else {
    mark_neighbours(dirs, c, tl, stamp, counters, 1);
  }
}


// Later sweeps: tiles marked for this sweep reload their halo and relax.
// One sweep of tile t if it is marked for it.  Returns (block-uniform) the
// neighbour tiles holding a point whose flags name a changed boundary point
// of this tile as a lower neighbour (0 if the tile did not run).
// QM (queue mode): the tile was taken from the repair queue, and other
// workgroups change subbins while it runs, so subbins are read and written
// as relaxed atomics at agent scope (coherent across the XCDs' L2 caches).
// With `blockers` given, thread 0 stores there the higher-index
// neighbour tiles holding a same-bin lower neighbour of one of the tile's
// points (the tiles its run depends on; bits 14..26 of the 27-direction set).
// LV: a 2D tile relaxes in the order of the levels kept by the first pass
// (tl.lev), if any and all known; otherwise relaxation passes.
template <int TZ, int TY, int TX, bool QM = false, bool LV = false>
__device__ __forceinline__ uint32_t repair_body(Box box, Tiling tl, const uint16_t* __restrict__ mask,
                            uint32_t* __restrict__ sub, const uint32_t* stamp,
                            uint32_t* counters, unsigned long long* itot, uint32_t sweep,
                            uint32_t t, TileCoord& c, uint32_t* blockers = nullptr) {
  using G = TileGeom<TZ, TY, TX>;
  constexpr int NJ = TZ == 1 ? 6 : 14;
  __shared__ uint32_t S[G::H];
  __shared__ uint16_t M[G::H];  // flags of the halo and the owned points
  // one read decides for the whole block (a neighbour may raise the stamp
  // concurrently)
  if constexpr (!QM) {
    __shared__ uint32_t go;
    if (threadIdx.x == 0) go = stamp[t] >= sweep;
    __syncthreads();
    if (!go) return 0;
  }
  c = tile_coord<TZ, TY, TX>(t, tl);
  constexpr int HL = (G::H + kThreads - 1) / kThreads;
  {
    uint32_t hv[HL];
    uint16_t hm[HL];
    // every load issued unconditionally (points outside the grid or the
    // halo read point 0 and are zeroed afterwards), so that all of them are
    // in flight together instead of one wait per halo point
    auto take = [&](int q, int64_t g, bool in) {
      const uint32_t v =
          QM ? __hip_atomic_load(sub + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : sub[g];
      const uint16_t m = mask[g];
      hv[q] = in ? v : 0u;
      hm[q] = in ? m : (uint16_t)0;
    };
    // a halo inside the grid (most tiles): 32-bit offsets from the halo's
    // first point, no bounds checks
    const bool inner = c.z0 - G::ZO >= 0 && c.z0 + TZ - 1 + G::ZO < box.nz && c.y0 >= 1 &&
                       c.y0 + TY < box.ny && c.x0 >= 1 && c.x0 + TX < box.nx &&
                       (uint64_t)box.ny * (uint64_t)box.nx * G::HZ < (1ull << 31);
    if (inner) {
      const int64_t g0 = ((int64_t)(c.z0 - G::ZO) * box.ny + (c.y0 - 1)) * box.nx + (c.x0 - 1);
      const uint32_t nyx = (uint32_t)box.ny * (uint32_t)box.nx;
#pragma unroll
      for (int q = 0; q < HL; ++q) {
        const int i = threadIdx.x + q * kThreads;
        const uint32_t hz = (uint32_t)i / (G::HY * G::HX), hy = ((uint32_t)i / G::HX) % G::HY,
                       hx = (uint32_t)i % G::HX;
        const bool in = i < G::H;
        take(q, in ? g0 + (int64_t)(hz * nyx + hy * (uint32_t)box.nx + hx) : 0, in);
      }
    } else {
#pragma unroll
      for (int q = 0; q < HL; ++q) {
        const int i = threadIdx.x + q * kThreads;
        const int hz = i / (G::HY * G::HX), hy = (i / G::HX) % G::HY, hx = i % G::HX;
        const int z = c.z0 + hz - G::ZO, y = c.y0 + hy - 1, x = c.x0 + hx - 1;
        const bool in = i < G::H && z >= 0 && z < box.nz && y >= 0 && y < box.ny && x >= 0 &&
                        x < box.nx;
        take(q, in ? ((int64_t)z * box.ny + y) * box.nx + x : 0, in);
      }
    }
#pragma unroll
    for (int q = 0; q < HL; ++q) {
      const int i = threadIdx.x + q * kThreads;
      if (i < G::H) {
        S[i] = hv[q];
        M[i] = hm[q];
      }
    }
  }
  __syncthreads();
  uint16_t mk[G::PER];
  uint32_t old[G::PER];
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    const int li = G::local(threadIdx.x + k * kThreads);
    mk[k] = M[li];
    old[k] = S[li];
  }
  int nlev = -1;
  if constexpr (LV && TZ == 1) {
    if (tl.lev) {
      uint8_t lv[G::PER];
#pragma unroll
      for (int k = 0; k < G::PER; ++k) {
        // a point with flags lies in the grid
        const int i = threadIdx.x + k * kThreads;
        lv[k] = mk[k] ? tl.lev[((int64_t)(c.y0 + i / TX)) * box.nx + c.x0 + i % TX] : 0;
      }
      nlev = level_relax<TZ, TY, TX>(S, mk, lv);
    }
  }
  // four-slot 3D tiles relax with the masks spread over bytes (k_repair is
  // held to six workgroups per CU for the registers that takes)
  if (nlev < 0) relax<TZ, TY, TX, (TZ > 1 && G::PER <= 4)>(S, mk, counters, itot, t);
  else if (threadIdx.x == 0) atomicAdd(&itot[t % 64], (unsigned long long)(nlev + 1));
  uint32_t dirs = 0;
#pragma unroll
  for (int k = 0; k < G::PER; ++k) {
    const int i = threadIdx.x + k * kThreads;
    const int li = G::local(i);
    const uint32_t v = S[li];
    if (v != old[k]) {
      const int iz = i / (TY * TX), iy = (i / TX) % TY, ix = i % TX;
      uint32_t* dst = sub + ((int64_t)(c.z0 + iz) * box.ny + c.y0 + iy) * box.nx + c.x0 + ix;
      if (QM) __hip_atomic_store(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else *dst = v;
      if (G::on_edge(i)) {
        // halo neighbours whose flags name this point (offset j from here is
        // offset j ^ 1 from there)
        uint32_t dep = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int z = iz + kOff[j][0], y = iy + kOff[j][1], x = ix + kOff[j][2];
          if (z < 0 || z >= TZ || y < 0 || y >= TY || x < 0 || x >= TX) {
            const int ln = li + kOff[j][0] * (G::HY * G::HX) + kOff[j][1] * G::HX + kOff[j][2];
            dep |= (uint32_t)((M[ln] >> (j ^ 1)) & 1u) << j;
          }
        }
        if (dep) dirs |= out_dirs<TZ, TY, TX>(i, dep);
      }
    }
  }
  if (QM && blockers) {
    uint32_t ups = 0;
#pragma unroll
    for (int k = 0; k < G::PER; ++k) {
      const int i = threadIdx.x + k * kThreads;
      if (mk[k] && G::on_edge(i)) ups |= out_dirs<TZ, TY, TX>(i, mk[k]);
    }
    const uint64_t both = block_or64((uint64_t)ups << 32 | dirs);
    if (threadIdx.x == 0) blockers[t] = (uint32_t)(both >> 32) & ~0x3fffu;
    return (uint32_t)both;
  }
  return block_or32(dirs);
}

// mark_neighbours for a sweep run colour by colour: a neighbour of the later
// colour runs later in this same sweep (it is marked for `sweep`), others in
// the next sweep (marked for sweep + 1; an edge neighbour has the same colour
// and may have read the halo already in this same launch); newly marked
// tiles are counted in counters[1 + s % 64] of their sweep s
__device__ void mark_neighbours_col(uint32_t dirs, const TileCoord& c, const Tiling& tl,
                                    uint32_t* stamp, uint32_t* counters, uint32_t sweep,
                                    uint32_t colour) {
  bool now = false, later = false;
  if (threadIdx.x < 27 && ((dirs >> threadIdx.x) & 1u)) {
    const int dz = (int)threadIdx.x / 9 - 1, dy = ((int)threadIdx.x / 3) % 3 - 1,
              dx = (int)threadIdx.x % 3 - 1;
    const int nz = c.tz + dz, ny = c.ty + dy, nx = c.tx + dx;
    if ((dz | dy | dx) != 0 && nz >= 0 && nz < tl.ntz && ny >= 0 && ny < tl.nty && nx >= 0 &&
        nx < tl.ntx) {
      const uint32_t u = ((uint32_t)nz * tl.nty + ny) * tl.ntx + nx;
      const uint32_t next = tile_colour(nz, ny, nx) > colour ? sweep : sweep + 1;
      const bool newly = atomicMax(&stamp[u], next) < next;
      now = newly && next == sweep;
      later = newly && next != sweep;
    }
  }
  if (threadIdx.x < 64) {
    const uint64_t a = __ballot(now), b = __ballot(later);
    if (threadIdx.x == 0 && a) atomicAdd(&counters[1 + (sweep & 63)], (uint32_t)__popcll(a));
    if (threadIdx.x == 0 && b)
      atomicAdd(&counters[1 + ((sweep + 1) & 63)], (uint32_t)__popcll(b));
  }
}

// One sweep (colour 2: every tile) or one colour of a sweep: the tiles of
// colour `colour` marked for this sweep run.  A coloured sweep runs colour
// 0, then colour 1, so a tile of colour 1 sees what its face and corner
// neighbours changed earlier in the same sweep.
template <int TZ, int TY, int TX>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_repair(
    Box box, Tiling tl, const uint16_t* __restrict__ mask,
    uint32_t* __restrict__ sub, uint32_t* stamp, uint32_t* counters,
    uint32_t sweep, uint32_t colour) {
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t t = colour < 2 ? colour_tile(b, colour, tl) : b;
  if (t >= tl.ntiles) return;
  TileCoord c;
  const uint32_t dirs = repair_body<TZ, TY, TX, false, true>(box, tl, mask, sub, stamp, counters,
                                                relax_total(counters), sweep, t, c);
  if (!dirs) return;
  if (colour < 2) mark_neighbours_col(dirs, c, tl, stamp, counters, sweep, colour);
  else mark_neighbours(dirs, c, tl, stamp, counters, sweep + 1);
}

// Device-driven repair of a single field: a persistent grid takes tiles from
// the repair queue until nothing is listed or running.  A tile run reloads
// the halo, relaxes, writes what changed, releases it and lists the
// neighbour tiles that depend on a changed boundary point; then the run
// stops counting as pending.  Subbins only rise and stay below the least
// fixed point, so the result does not depend on the order of the runs.
// One sweep over a work list: a persistent grid takes the listed tiles
// through a cursor; each reloads its halo, relaxes, writes what changed and
// lists the neighbour tiles that depend on a changed boundary point for the
// next sweep.  An empty list costs one atomic per workgroup.  The run is
// out of line for the reason given at repair_run below.

template <int TZ, int TY, int TX>
__device__ __noinline__ uint32_t sweep_run(Box box, Tiling tl, const uint16_t* __restrict__ mask,
                                           uint32_t* __restrict__ sub, const uint32_t* stamp,
                                           uint32_t* counters, uint32_t sweep, uint32_t t) {
  TileCoord c;
  return repair_body<TZ, TY, TX, false, true>(box, tl, mask, sub, stamp, counters, relax_total(counters),
                                 sweep, t, c);
}

template <int TZ, int TY, int TX>
__global__ __launch_bounds__(kThreads) void k_sweep_list(
    Box box, Tiling tl, const uint16_t* __restrict__ mask, uint32_t* __restrict__ sub,
    uint32_t* stamp, uint32_t* counters, uint32_t* lists, uint32_t sweep) {
  __shared__ uint32_t s_it;
  const uint32_t n = counters[1 + (sweep & 63)];
  const uint32_t* in = lists + (sweep & 1) * tl.ntiles;
  for (;;) {
    if (threadIdx.x == 0) s_it = atomicAdd(&counters[kCursorWord + (sweep & 63)], 1u);
    __syncthreads();
    const uint32_t it = s_it;
    __syncthreads();
    if (it >= n) break;
    const uint32_t t = in[it];
    const uint32_t dirs = sweep_run<TZ, TY, TX>(box, tl, mask, sub, stamp, counters, sweep, t);
    if (dirs) mark_list1(dirs, tile_coord<TZ, TY, TX>(t, tl), tl, stamp, counters, lists,
                         sweep + 1);
  }
}

// ---------------------------------------------------------- point worklists
// The paper's schedule of the repair, for comparison [Sec. IV-D, the loop of
// Alg. 1]: worklists of single points instead of tiles.  Iteration `it`
// recomputes the points listed for it from their lower neighbours in global
// memory and lists, for iteration it + 1, the upper neighbours of those that
// rose, each at most once per iteration (a per-point stamp holds the last
// iteration the point was listed for).  The two lists alternate; the list
// lengths sit in a 64-slot ring of counters.  Subbins only rise and stay
// below the least fixed point, so concurrent reads of stale values are
// harmless: a point that reads a value before it rises is listed again.

// list every point with a same-bin lower neighbour for iteration 0
__global__ __launch_bounds__(kThreads) void k_point_seed(const uint16_t* __restrict__ mask,
                                                         uint32_t n, uint32_t* wl,
                                                         uint32_t* ring) {
  for (uint32_t base = blockIdx.x * kThreads; base < n; base += gridDim.x * kThreads) {
    const uint32_t i = base + threadIdx.x;
    const bool go = i < n && mask[i] != 0;
    const uint64_t b = __ballot(go);
    if (!b) continue;  // wave-uniform
    uint32_t pos = 0;
    if (lane() == 0) pos = atomicAdd(&ring[0], (uint32_t)__popcll(b));
    pos = (uint32_t)__builtin_amdgcn_readfirstlane((int)pos);
    if (go) wl[pos + lane_prefix(b)] = i;
  }
}

__global__ __launch_bounds__(kThreads) void k_point_iter(Box box, const uint16_t* __restrict__ mask,
                                                         uint32_t* sub, const uint32_t* win,
                                                         uint32_t* wout, uint32_t* ring,
                                                         uint32_t* pstamp, uint32_t it) {
  const uint32_t nin = ring[it & 63];
  const uint32_t nx = (uint32_t)box.nx, nxy = (uint32_t)box.nx * (uint32_t)box.ny;
  for (uint32_t base = blockIdx.x * kThreads; base < nin; base += gridDim.x * kThreads) {
    const uint32_t e = base + threadIdx.x;
    bool rose = false;
    uint32_t p = 0;
    int z = 0, y = 0, x = 0;
    if (e < nin) {
      p = win[e];
      z = (int)(p / nxy);
      y = (int)((p / nx) % (uint32_t)box.ny);
      x = (int)(p % nx);
      const uint32_t m = mask[p];
      const uint32_t cur = sub[p];
      uint32_t best = cur;
#pragma unroll
      for (int j = 0; j < 14; ++j) {
        if ((m >> j) & 1u) {  // a flagged neighbour lies in the grid
          const uint32_t q = p + (uint32_t)(kOff[j][0] * (int)nxy + kOff[j][1] * (int)nx + kOff[j][2]);
          const uint32_t c = sub[q] + ((j & 1) ? 0u : 1u);
          best = c > best ? c : best;
        }
      }
      if (best > cur) {
        atomicMax(&sub[p], best);
        rose = true;
      }
    }
    // list the upper neighbours of the points that rose: q at offset j from
    // p whose flags name p (flag j ^ 1)
#pragma unroll
    for (int j = 0; j < 14; ++j) {
      bool app = false;
      uint32_t q = 0;
      if (rose) {
        const int zz = z + kOff[j][0], yy = y + kOff[j][1], xx = x + kOff[j][2];
        if (zz >= 0 && zz < box.nz && yy >= 0 && yy < box.ny && xx >= 0 && xx < box.nx) {
          q = ((uint32_t)zz * (uint32_t)box.ny + (uint32_t)yy) * nx + (uint32_t)xx;
          app = ((mask[q] >> (j ^ 1)) & 1u) && atomicMax(&pstamp[q], it + 1) < it + 1;
        }
      }
      const uint64_t b = __ballot(app);
      if (b) {
        const int leader = __builtin_ctzll(b);
        uint32_t pos = 0;
        if (lane() == leader) pos = atomicAdd(&ring[(it + 1) & 63], (uint32_t)__popcll(b));
        pos = (uint32_t)__builtin_amdgcn_readlane((int)pos, leader);
        if (app) wout[pos + lane_prefix(b)] = q;
      }
    }
  }
}

// The tiles listed for sweep `sweep` become the first items of the queue.
__global__ __launch_bounds__(kThreads) void k_seed_queue(const uint32_t* counters,
                                                         const uint32_t* lists, uint32_t ntiles,
                                                         uint32_t sweep, QueueRef Q) {
  const uint32_t n = counters[1 + (sweep & 63)];
  const uint32_t* in = lists + (sweep & 1) * ntiles;
  for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    q_push(Q, in[i], sweep);
}

// One queued tile run, kept out of line: inlined into the worker loop, the
// per-thread halo offsets of the body were hoisted out of the loop and kept
// live across it (180 VGPRs instead of 67).  Its LDS arrays are its own, so
// their accesses still compile to ds_* instructions.
template <int TZ, int TY, int TX>
__device__ __noinline__ uint32_t repair_run(Box box, Tiling tl, const uint16_t* __restrict__ mask,
                                            uint32_t* __restrict__ sub, uint32_t* counters,
                                            uint32_t t, uint32_t* blockers) {
  TileCoord c;
  return repair_body<TZ, TY, TX, true, true>(box, tl, mask, sub, nullptr, counters,
                                       relax_total(counters), 0, t, c, blockers);
}

template <int TZ, int TY, int TX>
__global__ __launch_bounds__(kThreads) void k_repair_q(
    Box box, Tiling tl, const uint16_t* __restrict__ mask, uint32_t* __restrict__ sub,
    uint32_t* counters, QueueRef Q) {
  __shared__ uint32_t s_item, s_depth, s_first;
  unsigned long long runs = 0, parks = 0;
  uint32_t deepest = 0;
  // nothing listed (the usual end of the work-list sweeps): leave at once
  // without taking tickets
  if (__hip_atomic_load(&Q.q->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t it;
      bool first = false;
      for (;;) {
        it = q_pop(Q);
        if (it == kNoTile) break;
        const TileCoord c = tile_coord<TZ, TY, TX>(it, tl);
        if (q_claim(Q, it, c, tl, 0, parks, first)) break;
      }
      s_item = it;
      s_first = first;
      s_depth = it == kNoTile ? 0u
                              : __hip_atomic_load(&Q.depth[it], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t t = s_item, d = s_depth;
    if (t == kNoTile) break;
    // ends with block barriers: s_item may be rewritten after it
    const uint32_t dirs = repair_run<TZ, TY, TX>(box, tl, mask, sub, counters, t,
                                                 s_first ? Q.blockers : nullptr);
    const TileCoord c = tile_coord<TZ, TY, TX>(t, tl);
    if (threadIdx.x < 64) {
      q_finish(dirs, t, c, tl, Q, 0, d + 1);
      if (threadIdx.x == 0) {
        ++runs;
        deepest = d > deepest ? d : deepest;
      }
    }
  }
  if (threadIdx.x == 0 && runs + parks) {
    atomicAdd(&Q.q->runs, runs);
    atomicAdd(&Q.q->parks, parks);
    atomicMax(&Q.q->max_depth, deepest);
  }
}

// ------------------------------------------------------------------ batches
// Persistent kernels: a fixed grid drains the batch-wide items of one phase.

// mark the neighbour tiles in `dirs` (27-bit set, see out_dirs) of a tile of
// a batch field for sweep `next` and append the newly marked ones (as
// batch-wide tile items) to that sweep's work list; each tile is listed at
// most once per sweep
__device__ void mark_list(uint32_t dirs, const TileCoord& c, const Tiling& tl, uint32_t* stamp,
                          uint32_t t0, uint32_t* lens, uint32_t* list, uint32_t next) {
  if (threadIdx.x >= 64) return;
  bool newly = false;
  uint32_t item = 0;
  if (threadIdx.x < 27 && ((dirs >> threadIdx.x) & 1u)) {
    int dz = (int)threadIdx.x / 9 - 1, dy = ((int)threadIdx.x / 3) % 3 - 1,
        dx = (int)threadIdx.x % 3 - 1;
    int nz = c.tz + dz, ny = c.ty + dy, nx = c.tx + dx;
    if ((dz | dy | dx) != 0 && nz >= 0 && nz < tl.ntz && ny >= 0 && ny < tl.nty &&
        nx >= 0 && nx < tl.ntx) {
      uint32_t u = ((uint32_t)nz * tl.nty + ny) * tl.ntx + nx;
      newly = atomicMax(&stamp[u], next) < next;
      item = t0 + u;
    }
  }
  const uint64_t m = __ballot(newly);
  if (!m) return;
  uint32_t pos = 0;
  if (threadIdx.x == 0) pos = atomicAdd(&lens[next % kRing], (uint32_t)__popcll(m));
  pos = __shfl(pos, 0, 64);
  if (newly) list[pos + lane_prefix(m)] = item;
}

__global__ __launch_bounds__(kThreads) void k_zero_p(const BatchDesc* bd) {
  const uint64_t n = bd->zero_words;
  uint32_t* base = bd->zero_base;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kThreads)
    base[i] = 0;
}

__global__ __launch_bounds__(kThreads) void k_zero_n(uint32_t* w, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kThreads)
    w[i] = 0;
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_minmax_p(const BatchDesc* bd, const Job* jobs) {
  constexpr int g0 = K == 4 ? 0 : 2;
  const uint32_t i1 = bd->item0[PH_MM][g0 + 2];
  const int j0 = (int)bd->job0[g0], j1 = (int)bd->job0[g0 + 2];
  for (uint32_t it = bd->item0[PH_MM][g0] + blockIdx.x; it < i1; it += gridDim.x) {
    const Job& J = jobs[find_job<&Job::mm0>(jobs, j0, j1, it)];
    __syncthreads();
    minmax_body<K>((const typename Traits<K>::Raw*)J.x, J.box.n, J.part, it - J.mm0,
                   (uint32_t)J.mm_blocks);
  }
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_params_p(const BatchDesc* bd, const Job* jobs) {
  constexpr int g0 = K == 4 ? 0 : 2;
  const int j1 = (int)bd->job0[g0 + 2];
  for (int j = (int)bd->job0[g0] + (int)blockIdx.x; j < j1; j += (int)gridDim.x) {
    const Job& J = jobs[j];
    __syncthreads();
    params_body<K>(J.mode, J.eb, J.part, J.mm_blocks, J.prm, J.stream, J.cap, J.ndim,
                   J.dims[0], J.dims[1], J.ndim == 3 ? J.dims[2] : 1);
  }
}

template <int K, int TZ, int TY, int TX>
__global__ __launch_bounds__(kThreads) void k_tile0_p(const BatchDesc* bd, const Job* jobs,
                                                      int g) {
  BatchCounters* bc = bd->bc;
  uint32_t* list1 = bd->lists + bd->tiles;  // sweep 1: odd list
  const uint32_t i1 = bd->item0[PH_T][g + 1];
  const int j0 = (int)bd->job0[g], j1 = (int)bd->job0[g + 1];
  for (uint32_t it = bd->item0[PH_T][g] + blockIdx.x; it < i1; it += gridDim.x) {
    const Job& J = jobs[find_job<&Job::t0>(jobs, j0, j1, it)];
    __syncthreads();
    TileCoord c;
    const uint32_t dirs = tile0_body<K, TZ, TY, TX>(
        (const typename Traits<K>::Raw*)J.x, J.box, J.tl, J.prm,
        (typename Traits<K>::Bin*)J.bins, J.mask, J.sub, &bc->err, bc->relax_iters,
        it - J.t0, c);
    mark_list(dirs, c, J.tl, J.stamp, J.t0, bc->lens, list1, 1);
  }
}

// One run of batch tile `t` of job J: the batch's 2D shape S2 or 3D shape S3.
template <int S2, int S3>
__device__ __forceinline__ uint32_t batch_repair_run(const Job& J, uint32_t* err,
                                                     unsigned long long* itot, uint32_t sweep,
                                                     uint32_t t, TileCoord& c) {
  if (J.tl.tz == 1)
    return repair_body<1, kTile2[S2][1], kTile2[S2][2]>(J.box, J.tl, J.mask, J.sub, J.stamp, err,
                                                        itot, sweep, t, c);
  return repair_body<kTile3[S3][0], kTile3[S3][1], kTile3[S3][2]>(J.box, J.tl, J.mask, J.sub,
                                                                  J.stamp, err, itot, sweep, t,
                                                                  c);
}

// One sweep over the tiles listed for it, of fields of both tile shapes.
template <int S2, int S3>
__global__ __launch_bounds__(kThreads) void k_repair_p(const BatchDesc* bd, const Job* jobs,
                                                       uint32_t sweep) {
  __shared__ uint32_t s_it;
  BatchCounters* bc = bd->bc;
  const uint32_t* list_in = bd->lists + (sweep & 1) * bd->tiles;
  uint32_t* list_out = bd->lists + ((sweep + 1) & 1) * bd->tiles;
  const uint32_t n = bc->lens[sweep % kRing];
  const int nj = (int)bd->job0[kGroups];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_it = atomicAdd(&bc->cursors[sweep % kRing], 1u);
    __syncthreads();
    const uint32_t it = s_it;
    if (it >= n) break;
    const uint32_t item = list_in[it];
    const Job& J = jobs[find_job<&Job::t0>(jobs, 0, nj, item)];
    TileCoord c;
    const uint32_t dirs = batch_repair_run<S2, S3>(J, &bc->err, bc->relax_iters, sweep,
                                                   item - J.t0, c);
    if (dirs) mark_list(dirs, c, J.tl, J.stamp, J.t0, bc->lens, list_out, sweep + 1);
  }
}

// Direct grids: one workgroup per item (the grid is the phase's item count
// of the batch), so each kernel keeps the register budget of its body.
template <int K>
__global__ __launch_bounds__(kThreads) void k_minmax_d(const BatchDesc* bd, const Job* jobs) {
  constexpr int g0 = K == 4 ? 0 : 2;
  const uint32_t it = bd->item0[PH_MM][g0] + blockIdx.x;
  const Job& J = jobs[find_job<&Job::mm0>(jobs, (int)bd->job0[g0], (int)bd->job0[g0 + 2], it)];
  minmax_body<K>((const typename Traits<K>::Raw*)J.x, J.box.n, J.part, it - J.mm0,
                 (uint32_t)J.mm_blocks);
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_params_d(const BatchDesc* bd, const Job* jobs) {
  constexpr int g0 = K == 4 ? 0 : 2;
  const Job& J = jobs[bd->job0[g0] + blockIdx.x];
  params_body<K>(J.mode, J.eb, J.part, J.mm_blocks, J.prm, J.stream, J.cap, J.ndim,
                 J.dims[0], J.dims[1], J.ndim == 3 ? J.dims[2] : 1);
}

template <int K, int TZ, int TY, int TX>
__global__ __launch_bounds__(kThreads) void k_tile0_d(const BatchDesc* bd, const Job* jobs,
                                                      int g) {
  const uint32_t it = bd->item0[PH_T][g] + xcd_tile(blockIdx.x, gridDim.x);
  const Job& J = jobs[find_job<&Job::t0>(jobs, (int)bd->job0[g], (int)bd->job0[g + 1], it)];
  TileCoord c;
  const uint32_t dirs = tile0_body<K, TZ, TY, TX>(
      (const typename Traits<K>::Raw*)J.x, J.box, J.tl, J.prm, (typename Traits<K>::Bin*)J.bins,
      J.mask, J.sub, &bd->bc->err, bd->bc->relax_iters, it - J.t0, c);
  mark_list(dirs, c, J.tl, J.stamp, J.t0, bd->bc->lens, bd->lists + bd->tiles, 1);
}

// One sweep: workgroup b takes entry b of the sweep's work list (the grid
// is the list's capacity; workgroups past its length exit at once).
template <int S2, int S3>
__global__ __launch_bounds__(kThreads) void k_repair_d(const BatchDesc* bd, const Job* jobs,
                                                       uint32_t sweep) {
  BatchCounters* bc = bd->bc;
  if (blockIdx.x >= bc->lens[sweep % kRing]) return;
  const uint32_t item = bd->lists[(sweep & 1) * bd->tiles + blockIdx.x];
  const Job& J = jobs[find_job<&Job::t0>(jobs, 0, (int)bd->job0[kGroups], item)];
  uint32_t* list_out = bd->lists + ((sweep + 1) & 1) * bd->tiles;
  TileCoord c;
  const uint32_t dirs = batch_repair_run<S2, S3>(J, &bc->err, bc->relax_iters, sweep,
                                                 item - J.t0, c);
  if (dirs) mark_list(dirs, c, J.tl, J.stamp, J.t0, bc->lens, list_out, sweep + 1);
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_minmax(int dtype, const void* x, uint32_t n, double* part,
                         int nblocks, void* zero, size_t zero_bytes, hipStream_t s, Ev ev) {
  const uint32_t nz = (uint32_t)(zero_bytes / 16);
  if (dtype == 0)
    launch_ev(k_minmax<4>, dim3(nblocks), dim3(kThreads), s, ev,
                          (const uint32_t*)x, n, (int64_t*)part, (uint4*)zero, nz);
  else
    launch_ev(k_minmax<8>, dim3(nblocks), dim3(kThreads), s, ev,
                          (const uint64_t*)x, n, (int64_t*)part, (uint4*)zero, nz);
  return hipGetLastError();
}

hipError_t launch_params(int dtype, int mode, double eb, const double* part,
                         int nblocks, Params* prm, uint8_t* stream, size_t cap,
                         int ndim, const int64_t* dims, hipStream_t s, Ev ev) {
  int64_t d2 = ndim == 3 ? dims[2] : 1;
  if (dtype == 0)
    launch_ev(k_params<4>, dim3(1), dim3(kThreads), s, ev, mode, eb,
                          (const int64_t*)part, nblocks, prm, stream, (uint64_t)cap, ndim,
                          dims[0], dims[1], d2);
  else
    launch_ev(k_params<8>, dim3(1), dim3(kThreads), s, ev, mode, eb,
                          (const int64_t*)part, nblocks, prm, stream, (uint64_t)cap, ndim,
                          dims[0], dims[1], d2);
  return hipGetLastError();
}

hipError_t launch_tile0(int dtype, const void* x, Box box, Tiling t, Params* prm, void* bins,
                        uint16_t* mask, uint32_t* sub, uint32_t* stamp,
                        uint32_t* counters, uint32_t* lists, const QueueRef& Q, hipStream_t s,
                        Ev ev, bool coloured) {
  const int nl = coloured ? 2 : 1;
  const dim3 b(kThreads);
  const dim3 g(coloured ? (uint32_t)t.ntz * (uint32_t)t.nty * (uint32_t)((t.ntx + 1) / 2)
                        : t.ntiles);
  for (int l = 0; l < nl; ++l) {
    const Ev e{l == 0 ? ev.a : nullptr, l == nl - 1 ? ev.b : nullptr};
    const uint32_t col = coloured ? (uint32_t)l : 2u;
    LOPC_WITH_TILE(t, {
      if (dtype == 0)
        launch_ev(k_tile0<4, TZ, TY, TX>, g, b, s, e, (const uint32_t*)x, box, t, prm,
                  (int32_t*)bins, mask, sub, stamp, counters, lists, Q, col);
      else
        launch_ev(k_tile0<8, TZ, TY, TX>, g, b, s, e, (const uint64_t*)x, box, t, prm,
                  (int64_t*)bins, mask, sub, stamp, counters, lists, Q, col);
    });
  }
  return hipGetLastError();
}

namespace {
// the caller's result words of an enqueued compression: the stream size
// (also when the buffer was short) and the status code of the ST_* bits
// (precedence as in the synchronous calls)
__global__ void k_report(const Params* prm, const RepairQueue* q, uint64_t* d_size,
                         int32_t* d_status) {
  const uint32_t st = prm->status | (q && q->err ? ST_INTERNAL : 0u);
  const int32_t code = (st & ST_NONFINITE) ? -2 : (st & ST_BOUND) ? -3 : (st & ST_RANGE) ? -4
                       : (st & ST_FORMAT) ? -6 : (st & ST_INTERNAL) ? -9
                       : (st & ST_CAPACITY) ? -5 : 0;
  if (d_size) *d_size = (code == 0 || code == -5) ? prm->stream_size : 0ull;
  if (d_status) *d_status = code;
}
}  // namespace

hipError_t launch_report(const Params* prm, const RepairQueue* q, uint64_t* d_size,
                         int32_t* d_status, hipStream_t s) {
  k_report<<<1, 1, 0, s>>>(prm, q, d_size, d_status);
  return hipGetLastError();
}

hipError_t launch_sweep_list(Box box, Tiling t, const uint16_t* mask, uint32_t* sub,
                             uint32_t* stamp, uint32_t* counters, uint32_t* lists,
                             uint32_t sweep, int grid, hipStream_t s, Ev ev) {
  const dim3 g(grid), b(kThreads);
  LOPC_WITH_TILE(t, launch_ev(k_sweep_list<TZ, TY, TX>, g, b, s, ev, box, t, mask, sub, stamp,
                              counters, lists, sweep));
  return hipGetLastError();
}

int sweep_list_blocks_per_cu(int sid) {
  int b = 0;
  Tiling t{};
  t.sid = sid;
  hipError_t e = hipErrorInvalidValue;
  LOPC_WITH_TILE(t, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &b, k_sweep_list<TZ, TY, TX>, kThreads, 0));
  return e == hipSuccess && b > 0 ? b : 1;
}

hipError_t launch_seed_queue(const uint32_t* counters, const uint32_t* lists, uint32_t ntiles,
                             uint32_t sweep, const QueueRef& Q, hipStream_t s) {
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(256, (ntiles + kThreads - 1) / kThreads));
  k_seed_queue<<<grid, kThreads, 0, s>>>(counters, lists, ntiles, sweep, Q);
  return hipGetLastError();
}

hipError_t launch_repair_q(Box box, Tiling t, const uint16_t* mask, uint32_t* sub,
                           uint32_t* counters, const QueueRef& Q, int grid, hipStream_t s,
                           Ev ev) {
  const dim3 g(grid), b(kThreads);
  LOPC_WITH_TILE(t, launch_ev(k_repair_q<TZ, TY, TX>, g, b, s, ev, box, t, mask, sub, counters,
                              Q));
  return hipGetLastError();
}

// resident workgroups per CU of the single-field repair-queue kernel
int repair_q_blocks_per_cu(int sid) {
  int b = 0;
  Tiling t{};
  t.sid = sid;
  hipError_t e = hipErrorInvalidValue;
  LOPC_WITH_TILE(t, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &b, k_repair_q<TZ, TY, TX>, kThreads, 0));
  return e == hipSuccess && b > 0 ? b : 1;
}

hipError_t launch_repair(Box box, Tiling t, const uint16_t* mask, uint32_t* sub,
                         uint32_t* stamp, uint32_t* counters, uint32_t sweep,
                         hipStream_t s, Ev ev) {
  // both colours, or every tile at once; the events bracket the sweep
  const bool col2 = t.coloured != 0;
  const uint32_t n =
      col2 ? (uint32_t)t.ntz * (uint32_t)t.nty * (uint32_t)((t.ntx + 1) / 2) : t.ntiles;
  const uint32_t nl = col2 ? 2 : 1;
  for (uint32_t l = 0; l < nl; ++l) {
    Ev e{l == 0 ? ev.a : nullptr, l == nl - 1 ? ev.b : nullptr};
    LOPC_WITH_TILE(t, launch_ev(k_repair<TZ, TY, TX>, dim3(n), dim3(kThreads), s, e, box, t,
                                mask, sub, stamp, counters, sweep, col2 ? l : 2u));
  }
  return hipGetLastError();
}

hipError_t launch_point_seed(const uint16_t* mask, uint32_t n, uint32_t* wl, uint32_t* ring,
                             int grid, hipStream_t s, Ev ev) {
  launch_ev(k_point_seed, dim3(grid), dim3(kThreads), s, ev, mask, n, wl, ring);
  return hipGetLastError();
}

hipError_t launch_point_iter(Box box, const uint16_t* mask, uint32_t* sub, const uint32_t* win,
                             uint32_t* wout, uint32_t* ring, uint32_t* pstamp, uint32_t it,
                             int grid, hipStream_t s, Ev ev) {
  launch_ev(k_point_iter, dim3(grid), dim3(kThreads), s, ev, box, mask, sub, win, wout, ring,
            pstamp, it);
  return hipGetLastError();
}

hipError_t launch_zero_p(const BatchDesc* bd, int grid, hipStream_t s) {
  k_zero_p<<<grid, kThreads, 0, s>>>(bd);
  return hipGetLastError();
}

hipError_t launch_zero_n(uint32_t* words, uint64_t nwords, hipStream_t s, Ev ev) {
  if (!nwords) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(1024, (nwords + kThreads - 1) / kThreads);
  launch_ev(k_zero_n, dim3(grid), dim3(kThreads), s, ev, words, nwords);
  return hipGetLastError();
}

hipError_t launch_minmax_p(int dtype, const BatchDesc* bd, const Job* jobs, int grid,
                           hipStream_t s) {
  if (dtype == 0) k_minmax_p<4><<<grid, kThreads, 0, s>>>(bd, jobs);
  else k_minmax_p<8><<<grid, kThreads, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

hipError_t launch_params_p(int dtype, const BatchDesc* bd, const Job* jobs, int grid,
                           hipStream_t s) {
  if (dtype == 0) k_params_p<4><<<grid, kThreads, 0, s>>>(bd, jobs);
  else k_params_p<8><<<grid, kThreads, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

// the tile extents of a batch group (2D groups: shape t2, 3D groups: t3)
static Tiling group_tiling(int group, int t2, int t3) {
  Tiling t{};
  t.sid = (group & 1) ? kTiles2 + t3 : t2;
  return t;
}

hipError_t launch_tile0_p(int group, int t2, int t3, const BatchDesc* bd, const Job* jobs,
                          int grid, hipStream_t s) {
  const Tiling t = group_tiling(group, t2, t3);
  LOPC_WITH_TILE(t, {
    if (group < 2) k_tile0_p<4, TZ, TY, TX><<<grid, kThreads, 0, s>>>(bd, jobs, group);
    else k_tile0_p<8, TZ, TY, TX><<<grid, kThreads, 0, s>>>(bd, jobs, group);
  });
  return hipGetLastError();
}

// the repair kernels of the batch for shape pair (t2, t3)
#define LOPC_WITH_PAIR(t2, t3, ...)                                          \
  do {                                                                       \
    const int pair_ = (t2) * kTiles3 + (t3);                                 \
    switch (pair_) {                                                         \
      case 0: { constexpr int S2 = 0, S3 = 0; __VA_ARGS__; } break;          \
      case 1: { constexpr int S2 = 0, S3 = 1; __VA_ARGS__; } break;          \
      case 2: { constexpr int S2 = 0, S3 = 2; __VA_ARGS__; } break;          \
      case 3: { constexpr int S2 = 1, S3 = 0; __VA_ARGS__; } break;          \
      case 4: { constexpr int S2 = 1, S3 = 1; __VA_ARGS__; } break;          \
      default: { constexpr int S2 = 1, S3 = 2; __VA_ARGS__; } break;         \
    }                                                                        \
  } while (0)
static_assert(kTiles2 == 2 && kTiles3 == 3, "LOPC_WITH_PAIR lists every shape pair");

hipError_t launch_repair_p(int t2, int t3, const BatchDesc* bd, const Job* jobs, uint32_t sweep,
                           int grid, hipStream_t s) {
  LOPC_WITH_PAIR(t2, t3, (k_repair_p<S2, S3><<<grid, kThreads, 0, s>>>(bd, jobs, sweep)));
  return hipGetLastError();
}

hipError_t launch_minmax_d(int dtype, const BatchDesc* bd, const Job* jobs, uint32_t items,
                           hipStream_t s) {
  if (!items) return hipSuccess;
  if (dtype == 0) k_minmax_d<4><<<items, kThreads, 0, s>>>(bd, jobs);
  else k_minmax_d<8><<<items, kThreads, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

hipError_t launch_params_d(int dtype, const BatchDesc* bd, const Job* jobs, uint32_t njobs,
                           hipStream_t s) {
  if (!njobs) return hipSuccess;
  if (dtype == 0) k_params_d<4><<<njobs, kThreads, 0, s>>>(bd, jobs);
  else k_params_d<8><<<njobs, kThreads, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

hipError_t launch_tile0_d(int group, int t2, int t3, const BatchDesc* bd, const Job* jobs,
                          uint32_t items, hipStream_t s) {
  if (!items) return hipSuccess;
  const Tiling t = group_tiling(group, t2, t3);
  LOPC_WITH_TILE(t, {
    if (group < 2) k_tile0_d<4, TZ, TY, TX><<<items, kThreads, 0, s>>>(bd, jobs, group);
    else k_tile0_d<8, TZ, TY, TX><<<items, kThreads, 0, s>>>(bd, jobs, group);
  });
  return hipGetLastError();
}

hipError_t launch_repair_d(int t2, int t3, const BatchDesc* bd, const Job* jobs, uint32_t sweep,
                           uint32_t tiles, hipStream_t s) {
  if (!tiles) return hipSuccess;
  LOPC_WITH_PAIR(t2, t3, (k_repair_d<S2, S3><<<tiles, kThreads, 0, s>>>(bd, jobs, sweep)));
  return hipGetLastError();
}

// resident blocks per CU of the persistent kernels of this file
int batch_blocks_per_cu(int kernel) {
  int b = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (kernel) {
    case PK_ZERO: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_zero_p, kThreads, 0); break;
    case PK_MINMAX: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_minmax_p<8>, kThreads, 0); break;
    case PK_PARAMS: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_params_p<8>, kThreads, 0); break;
    case PK_TILE0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_tile0_p<8, 8, 8, 32>, kThreads, 0); break;
    case PK_REPAIR: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_repair_p<0, 1>, kThreads, 0); break;
    default: break;
  }
  return e == hipSuccess && b > 0 ? b : 1;
}

}  // namespace lopc
