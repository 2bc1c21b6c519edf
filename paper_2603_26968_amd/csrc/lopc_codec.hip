// lopc_codec.hip -- chunk encoder and decoder of liblopc.so (gfx950).
//
// Lossless stages of Sec. III-B / Sec. IV-C on 16 kB chunks: bins go through
// DIFFNB_K BIT_K RZE_1, subbins through BIT_K RZE_K RZE_1.  The BIT_K output
// of a chunk of m words is handled as 64-bit "units": unit u = j*G + g (G =
// m/64) holds bit j of the 64 words of group g, i.e. exactly one __ballot.
// Every RZE variant then works unit-parallel: a unit carries 8 (RZE_1), 2
// (RZE_4) or 1 (RZE_8) bitmap bits, so bitmaps, counts and payload offsets
// come from wave scans over units instead of per-byte work.
//
// Chunk offsets in the stream.  A single field: every workgroup parks its
// record in rows of the workspace that its own chunk has finished with, a
// one-workgroup scan turns the record sizes into offsets and a placement
// kernel copies the records into the stream, so no workgroup waits for
// another.  Batches: a decoupled look-back over a ticket-ordered chunk queue
// (a workgroup only waits for chunks that started before it).  A look-back
// word packs its state and size into 64 bits, so it carries no other data
// and relaxed device-scope atomics suffice: release or acquire at that scope
// would write back / invalidate the per-XCD L2 on every publication.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <algorithm>

#include "lopc_device.h"

namespace lopc {
namespace {

constexpr int kCT = 512;        // threads of a codec workgroup
constexpr int kCW = kCT / 64;   // its waves
constexpr uint32_t kMaxUnits = kChunkBytes / 8;  // 2048
constexpr uint32_t kMaxRounds = kMaxUnits / 64;  // 32

// Scratch of the unit-parallel RZE stages.
struct Scratch {
  uint8_t lv0[kMaxUnits + 16] __attribute__((aligned(16)));  // level-1 bitmap
  uint8_t lv1[256 + 16] __attribute__((aligned(16)));
  uint8_t lv2[32 + 16] __attribute__((aligned(16)));
  uint8_t lv3[16] __attribute__((aligned(16)));
  uint8_t kp0[kMaxUnits];  // kept bytes of the level-1 bitmap
  uint8_t kp1[256];
  uint8_t kp2[32];
  uint32_t rpre[kMaxRounds + 1];  // per-round totals, then exclusive prefix
  uint32_t scan[kCW + 1];
  uint32_t nkept[4];
  uint64_t orv[kCW];
  uint64_t scan64[kCW + 1];
  uint64_t planes;
};

__device__ __forceinline__ uint8_t* lvl(Scratch& sc, int l) {
  return l == 0 ? sc.lv0 : (l == 1 ? sc.lv1 : (l == 2 ? sc.lv2 : sc.lv3));
}
__device__ __forceinline__ uint8_t* kept(Scratch& sc, int l) {
  return l == 0 ? sc.kp0 : (l == 1 ? sc.kp1 : sc.kp2);
}

// Bitmap bytes of RZE level l for `items` items: ceil(items / 8^(l+1)) (each
// level is the bitmap of the one below; nested ceilings compose).  Computed
// rather than tabulated so that nothing lands in a private array.
__device__ __forceinline__ uint32_t lvl_size(uint32_t items, int l) {
  const uint32_t sh = 3u * (uint32_t)(l + 1);
  return (items + (1u << sh) - 1u) >> sh;
}
// the top level: the first whose bitmap has at most 8 bytes
__device__ __forceinline__ int rze_top(uint32_t items) {
  int top = 0;
  while (lvl_size(items, top) > 8) ++top;
  return top;
}

// bit b (0..7) of the result: byte b of v is nonzero
__device__ __forceinline__ uint32_t nonzero_bytes(uint64_t v) {
  uint64_t t = v | (v >> 4);
  t |= t >> 2;
  t |= t >> 1;
  t &= 0x0101010101010101ull;
  return (uint32_t)((t * 0x0102040810204080ull) >> 56);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t c) { return wave_scan_u32(c); }

// Turn the per-round totals sc.rpre[0..rounds) into exclusive prefixes and
// return the grand total.  Call between barriers.
__device__ __forceinline__ uint32_t round_prefix(Scratch& sc, uint32_t rounds) {
  if (threadIdx.x < 64) {
    uint32_t c = threadIdx.x < rounds ? sc.rpre[threadIdx.x] : 0u;
    uint32_t inc = wave_incl_scan(c);
    if (threadIdx.x < rounds) sc.rpre[threadIdx.x] = inc - c;
    if (threadIdx.x == 63) sc.rpre[kMaxRounds] = inc;
  }
  __syncthreads();
  return sc.rpre[kMaxRounds];
}

// One level of the bitmap recursion: bit i of nxt = cur[i] differs from the
// byte before it (0 before the first); the differing bytes go to kp.
__device__ void level_encode(const uint8_t* cur, uint32_t n, uint8_t* nxt,
                             uint8_t* kp, uint32_t& nk, Scratch& sc) {
  const uint32_t nb = (n + 7) / 8;  // <= 256
  uint32_t bits = 0;
  if (threadIdx.x < nb) {
    uint32_t i0 = threadIdx.x * 8;
    uint8_t prev = i0 ? cur[i0 - 1] : (uint8_t)0;
    for (uint32_t b = 0; b < 8 && i0 + b < n; ++b) {
      uint8_t v = cur[i0 + b];
      bits |= (uint32_t)(v != prev) << b;
      prev = v;
    }
    nxt[threadIdx.x] = (uint8_t)bits;
  }
  uint32_t tot;
  uint32_t e = block_excl_scan<uint32_t, kCW>((uint32_t)__popc(bits), sc.scan, tot);
  if (threadIdx.x < nb) {
    uint32_t i0 = threadIdx.x * 8;
    for (uint32_t b = 0; b < 8; ++b)
      if ((bits >> b) & 1) kp[e++] = cur[i0 + b];
  }
  nk = tot;
  __syncthreads();
}

// LDS position of BIT_K unit u (plane u / G, group u % G).  In a full chunk
// (G = 64 or 32, a power of two) the groups of plane j are stored
// XOR-permuted by j, so the 8K lanes that store the planes of one group (a
// row stride of G units) reach distinct LDS banks instead of one; partial
// chunks keep the plain order (mask 0).
struct UnitSwizzle {
  uint32_t shift, mask;
  __device__ __forceinline__ uint32_t operator()(uint32_t u) const {
    return u ^ ((u >> shift) & mask);
  }
};

// RZE_W over the first `len` bytes of the unit array U (zero beyond len)
// into out.  Units from `nua` on are known to be zero (bit planes above the
// highest set bit) and are skipped.  Returns the output length; pt = 1 when
// the input is stored verbatim because the output would not be smaller.
// U may be stored swizzled (sw); the output is in plain byte order.
template <int W>
__device__ uint32_t rze_encode(const uint64_t* U, uint32_t len, uint32_t nua,
                               uint8_t* out, Scratch& sc, int& pt,
                               UnitSwizzle sw = UnitSwizzle{0, 0}) {
  const uint32_t NU = (len + 7) / 8;
  const uint32_t items = len / W;
  const uint32_t rounds = (NU + 63) / 64;
  const uint32_t ra = (min(nua, NU) + 63) / 64;  // rounds that may hold nonzero units
  if (ra < rounds) {
    // bitmap bytes of the zero rounds, and their counts
    const uint32_t nb0 = (items + 7) / 8;
    for (uint32_t i = threadIdx.x; i < (nb0 + 3) / 4 + 1; i += kCT) ((uint32_t*)sc.lv0)[i] = 0;
    if (threadIdx.x >= ra && threadIdx.x < rounds) sc.rpre[threadIdx.x] = 0;
    __syncthreads();
  }
  for (uint32_t r = wave(); r < ra; r += kCW) {
    const uint32_t u = r * 64 + lane();
    const uint64_t v = u < NU ? U[sw(u)] : 0ull;
    uint32_t mi, ci;
    if (W == 1) {
      mi = nonzero_bytes(v);
      ci = __popc(mi);
      if (u < NU) sc.lv0[u] = (uint8_t)mi;
    } else if (W == 4) {
      mi = ((uint32_t)v != 0u) | ((uint32_t)((v >> 32) != 0ull) << 1);
      ci = __popc(mi);
      // lanes 4q+1..4q+3 lie in the row of lane 4q: DPP row shifts left
      uint32_t b = mi | (dpp_u32<0x101, 0xf, true>(mi) << 2) |
                   (dpp_u32<0x102, 0xf, true>(mi) << 4) | (dpp_u32<0x103, 0xf, true>(mi) << 6);
      if ((lane() & 3) == 0 && u < NU) sc.lv0[u / 4] = (uint8_t)b;
    } else {
      mi = v != 0ull;
      ci = mi;
      uint64_t m = __ballot(mi);
      if (lane() == 0) *(uint64_t*)(sc.lv0 + r * 8) = m;
    }
    const uint32_t inc = wave_incl_scan(ci);
    if (lane() == 63) sc.rpre[r] = inc;
  }
  __syncthreads();
  const uint32_t npay = round_prefix(sc, rounds);
  const int top = rze_top(items);
  const uint32_t sz_top = lvl_size(items, top);
  for (int l = 0; l < top; ++l)
    level_encode(lvl(sc, l), lvl_size(items, l), lvl(sc, l + 1), kept(sc, l), sc.nkept[l], sc);
  uint32_t out_len = sz_top + npay * W;
  for (int l = 0; l < top; ++l) out_len += sc.nkept[l];
  if (out_len >= len) {
    const uint8_t* ub = (const uint8_t*)U;
    for (uint32_t i = threadIdx.x; i < len; i += kCT) out[i] = ub[8 * sw(i >> 3) + (i & 7)];
    pt = 1;
    __syncthreads();
    return len;
  }
  pt = 0;
  uint32_t pos = 0;
  {
    const uint8_t* tb = lvl(sc, top);
    for (uint32_t i = threadIdx.x; i < sz_top; i += kCT) out[i] = tb[i];
    pos = sz_top;
  }
  for (int l = top - 1; l >= 0; --l) {
    const uint8_t* kb = kept(sc, l);
    for (uint32_t i = threadIdx.x; i < sc.nkept[l]; i += kCT) out[pos + i] = kb[i];
    pos += sc.nkept[l];
  }
  for (uint32_t r = wave(); r < ra; r += kCW) {
    const uint32_t u = r * 64 + lane();
    const uint64_t v = u < NU ? U[sw(u)] : 0ull;
    uint32_t ci;
    if (W == 1) ci = __popc(nonzero_bytes(v));
    else if (W == 4) ci = ((uint32_t)v != 0u) + ((v >> 32) != 0ull);
    else ci = v != 0ull;
    uint32_t d = pos + W * (sc.rpre[r] + wave_incl_scan(ci) - ci);
    if (u >= NU) continue;
    if (W == 1) {
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        uint8_t x = (uint8_t)(v >> (8 * b));
        if (x) out[d++] = x;
      }
    } else if (W == 4) {
      uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
      if (lo) {
        put_bytes(out + d, lo, 4);
        d += 4;
      }
      if (hi) put_bytes(out + d, hi, 4);
    } else {
      if (v) put_bytes(out + d, v, 8);
    }
  }
  __syncthreads();
  return out_len;
}

// Item bits of unit u (of NU, `items` items in all) taken from its level-0
// bitmap byte b0.
template <int W>
__device__ __forceinline__ uint32_t unit_bits(uint32_t b0, uint32_t u, uint32_t items) {
  if (W == 1) {
    const uint32_t valid = items - u * 8;
    return valid < 8 ? b0 & ((1u << valid) - 1) : b0;
  } else if (W == 4) {
    return (b0 >> (2 * (u % 4))) & 3u;
  } else {
    return (b0 >> (u % 8)) & 1u;
  }
}

// One level of the bitmap recursion undone by one wave (no block barrier),
// for levels of at most 512 bytes (level 1 and above of a 16 kB input):
// child byte i = the last kept byte at or before i (0 if none), the kept
// bytes read from in[pos...); lane l handles parent byte l.  Returns false
// (wave-uniform) if the kept bytes run past in_len.  The 8 child bytes of a
// parent byte m (e kept bytes before it) come from one window of kept
// bytes, read as aligned words and joined by byte-align moves: it starts
// one byte before the first kept byte of m when m's bit 0 is clear (that
// byte fills the leading children), at it otherwise; the selector of child
// b is its inclusive count of set bits minus bit 0 of m, or 0x0c (zero)
// while no kept byte has been seen at all (e = 0).
__device__ bool level_decode_w(const uint8_t* par, uint32_t n, const uint8_t* in,
                               uint32_t& pos, uint32_t in_len, uint8_t* child) {
  const uint32_t np = (n + 7) / 8;  // <= 64
  const uint32_t idx = (uint32_t)lane();
  const uint32_t valid = n - idx * 8;
  uint32_t m = 0;
  if (idx < np) {
    m = par[idx];
    if (valid < 8) m &= (1u << valid) - 1;
  }
  const uint32_t cq = (uint32_t)__popc(m);
  const uint32_t incl = wave_incl_scan(cq);
  const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  if (pos + tot > in_len) return false;
  const uint32_t e = incl - cq;
  if (idx < np) {
    const uint32_t b0 = m & 1u;
    // window: from kept byte e - 1 + b0 (in[pos - 1] when e = 0 and b0 = 0,
    // a byte of the levels above, selected by no child), cq + 1 - b0 bytes
    const uint8_t* p = in + pos + e + b0 - 1;
    const uint32_t mis = (uint32_t)(uintptr_t)p & 3u;
    const uint32_t* wq = (const uint32_t*)(p - mis);
    const uint32_t nd = (mis + cq + 1 - b0 + 3) / 4;  // 1..3 words
    const uint32_t w0 = wq[0];
    const uint32_t w1 = nd > 1 ? wq[1] : 0u;
    const uint32_t w2 = nd > 2 ? wq[2] : 0u;
    const uint32_t x0 = __builtin_amdgcn_alignbyte(w1, w0, mis);
    const uint32_t x1 = __builtin_amdgcn_alignbyte(w2, w1, mis);
    // inclusive counts of set bits per child byte (as in unit_payload)
    const uint32_t slo = ((m & 0xfu) * 0x00204081u) & 0x01010101u;
    const uint32_t shi = (((m >> 4) & 0xfu) * 0x00204081u) & 0x01010101u;
    const uint32_t ilo = slo * 0x01010101u;
    const uint32_t ihi = shi * 0x01010101u + (uint32_t)__popc(m & 0xfu) * 0x01010101u;
    uint32_t sel_lo = ilo - b0 * 0x01010101u, sel_hi = ihi - b0 * 0x01010101u;
    if (e == 0) {  // children before the first kept byte of the level are 0
      sel_lo |= ((~(ilo + 0x7f7f7f7fu) & 0x80808080u) >> 7) * 0x0cu;
      sel_hi |= ((~(ihi + 0x7f7f7f7fu) & 0x80808080u) >> 7) * 0x0cu;
    }
    uint64_t v = (uint64_t)__builtin_amdgcn_perm(x1, x0, sel_lo) |
                 (uint64_t)__builtin_amdgcn_perm(x1, x0, sel_hi) << 32;
    if (valid < 8) v &= (1ull << (8 * valid)) - 1ull;  // bytes past n are zero
    ((uint32_t*)child)[2 * idx] = (uint32_t)v;
    ((uint32_t*)child)[2 * idx + 1] = (uint32_t)(v >> 32);
  }
  pos += tot;
  __builtin_amdgcn_wave_barrier();
  return true;
}

// The payload of one unit: its c kept items at p (c * W bytes, any
// alignment) placed at the items of mask m, the others zero.  Reads the
// aligned words covering those bytes only (never past p + c * W rounded up
// to a word), joins them into the 8 bytes from p with byte-align moves, then
// for W = 1 spreads the bytes with one byte permute per half: the selector
// of output byte b is the number of mask bits below b when bit b is set,
// else 0x0c (the permute's zero byte).
template <int W>
__device__ __forceinline__ uint64_t unit_payload(const uint8_t* p, uint32_t m, uint32_t c) {
  if (!m) return 0;
  const uint32_t mis = (uint32_t)(uintptr_t)p & 3u;
  const uint32_t* q = (const uint32_t*)(p - mis);
  const uint32_t nd = (mis + c * W + 3) / 4;  // 1..3 words
  const uint32_t w0 = q[0];
  const uint32_t w1 = nd > 1 ? q[1] : 0u;
  const uint32_t w2 = nd > 2 ? q[2] : 0u;
  const uint32_t x0 = __builtin_amdgcn_alignbyte(w1, w0, mis);
  const uint32_t x1 = __builtin_amdgcn_alignbyte(w2, w1, mis);
  if (W == 8) return (uint64_t)x0 | (uint64_t)x1 << 32;
  if (W == 4) {
    const uint32_t lo = (m & 1) ? x0 : 0u;
    const uint32_t hi = (m & 2) ? ((m & 1) ? x1 : x0) : 0u;
    return (uint64_t)lo | (uint64_t)hi << 32;
  }
  // bit i of each nibble of m to bit 0 of byte i (the four shifted copies
  // do not overlap, so nothing carries)
  const uint32_t slo = ((m & 0xfu) * 0x00204081u) & 0x01010101u;
  const uint32_t shi = (((m >> 4) & 0xfu) * 0x00204081u) & 0x01010101u;
  // inclusive counts per byte, then exclusive: the selector of a set byte
  const uint32_t ilo = slo * 0x01010101u;
  const uint32_t ihi = shi * 0x01010101u + (uint32_t)__popc(m & 0xfu) * 0x01010101u;
  const uint32_t sel_lo = ((ilo - slo) & (slo * 0xffu)) | ((slo ^ 0x01010101u) * 0x0cu);
  const uint32_t sel_hi = ((ihi - shi) & (shi * 0xffu)) | ((shi ^ 0x01010101u) * 0x0cu);
  return (uint64_t)__builtin_amdgcn_perm(x1, x0, sel_lo) |
         (uint64_t)__builtin_amdgcn_perm(x1, x0, sel_hi) << 32;
}

// Upper levels of an RZE decode, on wave 0 alone: the top bitmap and every
// level down to level 1 (the bitmap of the level-0 bitmap) into sc.lv1, zero
// past its last byte.  Leaves sc.nkept[0] = ok and sc.nkept[1] = offset of
// the level-0 kept bytes (with a single level: of the payload).
__device__ void rze_decode_upper(const uint8_t* in, uint32_t in_len, uint32_t items,
                                 Scratch& sc) {
  const int top = rze_top(items);
  const uint32_t sz_top = lvl_size(items, top);
  bool ok = sz_top <= in_len;
  uint32_t pos = sz_top;
  if (ok && top == 1) {
    if (lane() < 16) sc.lv1[lane()] = (uint32_t)lane() < sz_top ? in[lane()] : (uint8_t)0;
  } else if (ok && top >= 2) {
    // the top level is read in place (its sz_top bytes are the parents)
    ok = level_decode_w(in, lvl_size(items, top - 1), in, pos, in_len, lvl(sc, top - 1));
    for (int l = top - 2; l >= 1 && ok; --l)
      ok = level_decode_w(lvl(sc, l + 1), lvl_size(items, l), in, pos, in_len, lvl(sc, l));
  }
  if (lane() == 0) {
    sc.nkept[0] = ok ? 1u : 0u;
    sc.nkept[1] = pos;
  }
}

// Inverse of rze_encode: in[0, in_len) -> the first `len` bytes of U (units
// rounded up; bytes past len are zero).  Returns false on malformed input;
// never reads outside [in, in + in_len).  If G > 0 the units are bit planes
// of G groups and sc.planes receives the mask of planes holding a nonzero
// unit.  Wave 0 decodes the levels above level 0 (small); then every wave
// expands the level-0 bitmap bytes of its own rounds of 64 units straight
// into registers (a byte's position among the kept bytes is a prefix count
// over level 1) and counts their items; after the per-round counts are
// exchanged, the same lanes fetch their units' payload.  Block barriers:
// after the upper levels, after the round counts, after the payload, after
// the plane mask.
template <int W>
__device__ __forceinline__ bool rze_decode(const uint8_t* in, uint32_t in_len, uint32_t len,
                           uint64_t* U, Scratch& sc, uint32_t G) {
  constexpr int kRPW = (int)(kMaxRounds / kCW);  // rounds per wave at most
  const uint32_t NU = (len + 7) / 8;
  const uint32_t items = len / W;
  const uint32_t rounds = (NU + 63) / 64;
  const int top = rze_top(items);
  const uint32_t n0 = lvl_size(items, 0);  // level-0 bitmap bytes
  if (wave() == 0) rze_decode_upper(in, in_len, items, sc);
  __syncthreads();
  if (!sc.nkept[0]) return false;
  const uint32_t pos1 = sc.nkept[1];
  // level 1 as 64-bit words (bit q: level-0 byte q differs from the one
  // before); bits from n0 on do not count
  const uint64_t* l1 = (const uint64_t*)sc.lv1;
  uint32_t wexcl = 0, pos0 = pos1;
  if (top >= 1) {
    const uint32_t nw = (n0 + 63) / 64;  // <= 32
    uint64_t wd = 0;
    if ((uint32_t)lane() < nw) {
      wd = l1[lane()];
      const uint32_t v = n0 - 64u * (uint32_t)lane();
      if (v < 64) wd &= (1ull << v) - 1ull;
    }
    const uint32_t c = (uint32_t)__popcll(wd);
    const uint32_t inc = wave_scan_u32(c);
    wexcl = inc - c;
    pos0 = pos1 + (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    if (pos0 > in_len) return false;
  }
  uint32_t mi[kRPW], incl[kRPW];
#pragma unroll
  for (int k = 0; k < kRPW; ++k) {
    const uint32_t r = wave() + kCW * k;
    mi[k] = 0;
    incl[k] = 0;
    if (r >= rounds) continue;
    const uint32_t u = r * 64 + lane();
    // the level-1 word holding the bits of this round's level-0 bytes
    // (r / W: one word per round of 8 / W items a unit) and the kept bytes
    // before it
    uint64_t wd = 0;
    uint32_t wb = 0;
    if (top >= 1) {
      const uint32_t wi = r / W;
      wd = l1[wi];
      const uint32_t v = n0 - 64u * wi;
      if (v < 64) wd &= (1ull << v) - 1ull;
      wb = (uint32_t)__builtin_amdgcn_readlane((int)wexcl, (int)wi);
    }
    if (u < NU) {
      const uint32_t q = W == 1 ? u : (W == 4 ? u / 4 : u / 8);  // its level-0 byte
      uint32_t b0;
      if (top == 0) {
        b0 = in[q];  // the top level is level 0 (q < n0 = its size)
      } else {
        const uint32_t e = wb + (uint32_t)__popcll(wd & ((2ull << (q & 63)) - 1ull));
        b0 = e ? in[pos1 + e - 1] : 0u;
      }
      mi[k] = unit_bits<W>(b0, u, items);
    }
    incl[k] = wave_incl_scan((uint32_t)__popc(mi[k]));
    if (lane() == 63) sc.rpre[r] = incl[k];
  }
  __syncthreads();
  // payload offsets of the rounds; the payload must end the input exactly
  const uint32_t rc = (uint32_t)lane() < rounds ? sc.rpre[lane()] : 0u;
  const uint32_t rinc = wave_scan_u32(rc);
  const uint32_t npay = (uint32_t)__builtin_amdgcn_readlane((int)rinc, 63);
  if (pos0 + npay * W != in_len) return false;
  uint64_t pm = 0;
#pragma unroll
  for (int k = 0; k < kRPW; ++k) {
    const uint32_t r = wave() + kCW * k;
    if (r >= rounds) break;
    const uint32_t u = r * 64 + lane();
    if (!__ballot(mi[k] != 0u)) {
      if (u < NU) U[u] = 0;
      continue;
    }
    const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)(rinc - rc), (int)r);
    const uint32_t m = mi[k];
    const uint32_t c = (uint32_t)__popc(m);
    if (u >= NU) continue;
    const uint64_t v = unit_payload<W>(in + pos0 + W * (base + incl[k] - c), m, c);
    U[u] = v;
    if (G && v) pm |= 1ull << (u / G);
  }
  if (G) {
    pm = wave_reduce(pm, OpOr{});
    if (lane() == 0) sc.orv[wave()] = pm;
  }
  __syncthreads();
  if (G) {
    uint64_t m = 0;
    for (int w = 0; w < kCW; ++w) m |= sc.orv[w];
    if (threadIdx.x == 0) sc.planes = m;
    __syncthreads();
  }
  return true;
}

// BIT_K of the chunk's words, given per wave in registers: wv[i] is word
// 64*g + lane of group g = wave + kCW*i.  Planes >= np are zero.
template <int K, int GPW>
__device__ void bit_encode(const typename Traits<K>::Word (&wv)[GPW], uint32_t G,
                           uint32_t np, uint64_t* U, UnitSwizzle sw) {
#pragma unroll
  for (int i = 0; i < GPW; ++i) {
    const uint32_t g = wave() + kCW * i;
    if (g >= G) break;
    uint64_t mine = 0;
    for (uint32_t j = 0; j < np; ++j) {
      uint64_t b = __ballot((wv[i] >> j) & 1);
      if (lane() == (int)j) mine = b;
    }
    if (lane() < 8 * K) U[sw(lane() * G + g)] = mine;
  }
}

// Planes holding a nonzero unit (bit j set: plane j not all zero).
template <int K>
__device__ uint64_t nonzero_planes(const uint64_t* U, uint32_t G, Scratch& sc) {
  uint64_t any = 0;
  if (threadIdx.x < 8 * K) {
    const uint64_t* p = U + threadIdx.x * G;
    for (uint32_t g = 0; g < G; ++g) any |= p[g];
  }
  if (threadIdx.x < 64) {
    uint64_t m = __ballot(any != 0ull);
    if (threadIdx.x == 0) sc.planes = m;
  }
  __syncthreads();
  return sc.planes;
}

__device__ __forceinline__ uint64_t block_or(uint64_t v, Scratch& sc) {
  // wave OR by ballots over the set bits is costly; reduce through LDS
  v = wave_reduce(v, OpOr{});
  if (lane() == 0) sc.orv[wave()] = v;
  __syncthreads();
  uint64_t r = 0;
  for (int w = 0; w < kCW; ++w) r |= sc.orv[w];
  __syncthreads();
  return r;
}

constexpr uint64_t kLbAgg = 1ull << 62, kLbInc = 2ull << 62,
                   kLbVal = (1ull << 62) - 1;

// ------------------------------------------------------------------ encoder
// Record byte r of a chunk: 16-byte header, then the bins part, the subbin
// part and zero padding to a multiple of 4.
__device__ __forceinline__ uint8_t record_byte(uint32_t r, const uint8_t* hdr,
                                               const uint8_t* bp, uint32_t blen,
                                               const uint8_t* sp, uint32_t slen) {
  if (r < kRecordHeaderBytes) return hdr[r];
  r -= kRecordHeaderBytes;
  if (r < blen) return bp[r];
  r -= blen;
  return r < slen ? sp[r] : (uint8_t)0;
}

// Where the record of chunk c of a single field waits for its offset: the
// chunk's rows of the bins, subbins and order-flag arrays, in that order
// (free once the encoder has read the chunk; nothing reads them after it),
// and a separate place for the last chunk, whose rows may be short.  The
// rows hold W*sizeof(Bin) + 4W + 2W bytes: 40 KiB for binary32, 28 KiB for
// binary64.  A record is at most 16 + (bins part) + (subbin part) bytes with
// each part at most the bit-plane bytes of its stage input: 16 + 16 KiB +
// 16 KiB for binary32; for binary64 the subbins (below 2^32) fill at most 32
// of the 64 planes, so that part stays under 8 KiB plus its bitmaps, about
// 24.3 KiB in all.  The encoder still checks the room.
struct RecordSlots {
  uint8_t* seg[3];   // chunk 0's rows
  uint32_t len[3];   // bytes of one chunk's rows in each
  uint8_t* tail;     // the last chunk's place
  uint32_t tail_len;
};

__device__ __forceinline__ uint32_t* slot_word(const RecordSlots& S, uint32_t c, bool last,
                                               uint32_t q) {
  uint32_t r = 4 * q;
  if (last) return (uint32_t*)(S.tail + r);
  if (r < S.len[0]) return (uint32_t*)(S.seg[0] + (size_t)c * S.len[0] + r);
  r -= S.len[0];
  if (r < S.len[1]) return (uint32_t*)(S.seg[1] + (size_t)c * S.len[1] + r);
  r -= S.len[1];
  return (uint32_t*)(S.seg[2] + (size_t)c * S.len[2] + r);
}

__device__ __forceinline__ uint32_t record_size(uint32_t blen, uint32_t slen) {
  return (kRecordHeaderBytes + blen + slen + 3) & ~3u;
}

// Encodes chunk c of a field (Sec. III-B, IV-C).  kSlot: parks the record
// in its slot (single field; offsets and placement follow in their own
// kernels); else writes it into the stream after a decoupled look-back.
template <int K, bool kSlot>
__device__ __forceinline__ void encode_body(uint32_t n, const typename Traits<K>::Bin* __restrict__ bins,
                            const uint32_t* __restrict__ sub, uint64_t* lookback,
                            uint32_t* parts, Params* prm, uint8_t* stream, uint64_t cap,
                            uint32_t nch, uint32_t c, const RecordSlots& S) {
  using Tr = Traits<K>;
  using Word = typename Tr::Word;
  constexpr uint32_t W = kChunkBytes / K;
  constexpr int GPW = (int)(W / 64 / kCW);  // groups per wave
  // LDS: the look-back path keeps the bins part (B) until the end beside
  // the RZE_K output (X): 54,248 bytes, three workgroups per CU.  The slot
  // path parks the bins part as soon as it is known and reuses B for X:
  // about 37.9 KB, four workgroups per CU.
  __shared__ uint64_t U[kMaxUnits];      // bit planes; later the subbin part
  __shared__ uint64_t B[kMaxUnits + 2];  // bins part (slot path: then X)
  __shared__ uint64_t Xb[kSlot ? 1 : kMaxUnits + 2];  // subbins after RZE_K (+16 zero bytes)
  uint64_t* X = kSlot ? B : Xb;
  __shared__ uint32_t s_btail;  // slot path: bytes of the bins part's partial last word
  __shared__ Scratch sc;
  // the record header and the chunk's offset live in sc.orv, which is free
  // once both block_or calls are done
  uint8_t* hdr = (uint8_t*)sc.orv;
  uint64_t& s_excl = sc.orv[2];

  const uint32_t p0 = c * W;
  const uint32_t nc = min(W, n - p0);
  const uint32_t m = (nc + 63) / 64 * 64;
  const uint32_t G = m / 64;
  const uint32_t L = m * K;
  const Word M = (Word)0xAAAAAAAAAAAAAAAAull;

  const UnitSwizzle sw{(uint32_t)__builtin_ctz(W / 64), G == W / 64 ? G - 1 : 0u};

  // The chunk's bins and subbins come in as 16-byte vectors through LDS
  // (U and B are free until the bit planes): four vector loads per thread
  // instead of three word loads per value.
  {
    const uint4* bsrc = (const uint4*)(bins + p0);
    const uint4* ssrc = (const uint4*)(sub + p0);
    constexpr uint32_t VB = 16 / sizeof(typename Tr::Bin), VS = 4;  // values per vector
    const uint32_t nb = nc / VB, ns = nc / VS;
    uint4 vb[(W / VB + kCT - 1) / kCT], vs[(W / VS + kCT - 1) / kCT];
#pragma unroll
    for (int q = 0; q < (int)((W / VB + kCT - 1) / kCT); ++q) {
      const uint32_t i = threadIdx.x + q * kCT;
      vb[q] = i < nb ? bsrc[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < (int)((W / VS + kCT - 1) / kCT); ++q) {
      const uint32_t i = threadIdx.x + q * kCT;
      vs[q] = i < ns ? ssrc[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < (int)((W / VB + kCT - 1) / kCT); ++q) {
      const uint32_t i = threadIdx.x + q * kCT;
      if (i < nb) ((uint4*)U)[i] = vb[q];
    }
#pragma unroll
    for (int q = 0; q < (int)((W / VS + kCT - 1) / kCT); ++q) {
      const uint32_t i = threadIdx.x + q * kCT;
      if (i < ns) ((uint4*)B)[i] = vs[q];
    }
    // the ragged end of a last chunk, one value per thread
    for (uint32_t j = nb * VB + threadIdx.x; j < nc; j += kCT)
      ((typename Tr::Bin*)U)[j] = bins[p0 + j];
    for (uint32_t j = ns * VS + threadIdx.x; j < nc; j += kCT) ((uint32_t*)B)[j] = sub[p0 + j];
  }
  __syncthreads();

  // bins: DIFFNB_K (delta from the previous bin, 0 before the chunk, then
  // negabinary), zero words up to m, BIT_K, RZE_1
  Word wv[GPW], sv[GPW];
  uint64_t orv = 0;
#pragma unroll
  for (int i = 0; i < GPW; ++i) {
    const uint32_t g = wave() + kCW * i;
    const uint32_t j = g * 64 + lane();
    Word v = 0;
    if (j < nc) {
      const typename Tr::Bin* lb = (const typename Tr::Bin*)U;
      Word cur = (Word)lb[j];
      Word prev = j ? (Word)lb[j - 1] : (Word)0;
      Word d = cur - prev;
      v = (d + M) ^ M;
    }
    sv[i] = j < nc ? (Word)((const uint32_t*)B)[j] : (Word)0;
    wv[i] = v;
    orv |= (uint64_t)v;
  }
  orv = block_or(orv, sc);
  uint32_t np = orv ? 64 - (uint32_t)__builtin_clzll(orv) : 0;
  bit_encode<K, GPW>(wv, G, np, U, sw);
  __syncthreads();
  int pt_b = 0, pt_s1 = 0, pt_s2 = 0;
  const uint32_t blen = rze_encode<1>(U, L, np * G, (uint8_t*)B, sc, pt_b, sw);
  const bool last = c == nch - 1;
  const uint32_t room = last ? S.tail_len : S.len[0] + S.len[1] + S.len[2];
  if constexpr (kSlot) {
    // park the whole words of the bins part now (record bytes from 16 on)
    if (kRecordHeaderBytes + blen <= room)
      for (uint32_t q = threadIdx.x; q < blen / 4; q += kCT)
        *slot_word(S, c, last, kRecordHeaderBytes / 4 + q) = ((const uint32_t*)B)[q];
    if (threadIdx.x == 0)
      s_btail = (blen & 3u) ? ((const uint32_t*)B)[blen / 4] & ((1u << (8 * (blen & 3u))) - 1u)
                            : 0u;
    __syncthreads();  // B is free for the RZE_K output
  }

  // subbins: zero words up to m, BIT_K, RZE_K, RZE_1
  orv = 0;
#pragma unroll
  for (int i = 0; i < GPW; ++i) orv |= (uint64_t)sv[i];
  orv = block_or(orv, sc);
  np = orv ? 64 - (uint32_t)__builtin_clzll(orv) : 0;
  bit_encode<K, GPW>(sv, G, np, U, sw);
  __syncthreads();
  const uint32_t smid = rze_encode<K>(U, L, np * G, (uint8_t*)X, sc, pt_s1, sw);
  if (threadIdx.x < 16) ((uint8_t*)X)[smid + threadIdx.x] = 0;  // zero units past smid
  __syncthreads();
  const uint32_t slen = rze_encode<1>(X, smid, (smid + 7) / 8, (uint8_t*)U, sc, pt_s2);

  const uint32_t size = record_size(blen, slen);
  if (threadIdx.x == 0) {
    hdr[0] = (uint8_t)pt_b;
    hdr[1] = (uint8_t)(pt_s1 | (pt_s2 << 1));
    hdr[2] = (uint8_t)nc;
    hdr[3] = (uint8_t)(nc >> 8);
    put_bytes(hdr + 4, blen, 4);
    put_bytes(hdr + 8, smid, 4);
    put_bytes(hdr + 12, slen, 4);
  }
  if constexpr (kSlot) {
    if (threadIdx.x == 0) {
      parts[2 * c] = blen;
      parts[2 * c + 1] = slen;
      if (kHeaderBytes + 4ull * c + 4 <= cap)
        *(uint32_t*)(stream + kHeaderBytes + 4ull * c) = size;
    }
    __syncthreads();  // hdr
    if (size <= room) {
      // the header words, then from the bins part's partial word on (its
      // bytes from s_btail), the subbin part and the padding
      const uint8_t* bt = (const uint8_t*)&s_btail;
      const uint8_t* sp = (const uint8_t*)U;
      const uint32_t nfull = blen / 4, nw = size / 4 - nfull;
      for (uint32_t e = threadIdx.x; e < nw; e += kCT) {
        const uint32_t q = e < kRecordHeaderBytes / 4 ? e : e + nfull;
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t r = 4 * q + b;
          uint32_t v;
          if (r < kRecordHeaderBytes) v = hdr[r];
          else if (r < kRecordHeaderBytes + blen) v = bt[r - kRecordHeaderBytes - 4 * nfull];
          else if (r < kRecordHeaderBytes + blen + slen) v = sp[r - kRecordHeaderBytes - blen];
          else v = 0;
          w |= v << (8 * b);
        }
        *slot_word(S, c, last, q) = w;
      }
    } else if (threadIdx.x == 0) {
      set_status(prm, ST_INTERNAL);
    }
    return;
  }

  // decoupled look-back for this chunk's offset in the stream body: wave 0
  // reads 64 predecessors per round trip (lane l reads chunk c - 1 - l - 64r)
  // and adds the sizes up to the nearest inclusive prefix
  if (threadIdx.x < 64) {
    uint64_t excl = 0;
    if (threadIdx.x == 0)
      __hip_atomic_store(&lookback[c], (c == 0 ? kLbInc : kLbAgg) | size, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    if (c > 0) {
      int64_t j0 = (int64_t)c - 1;
      uint32_t spins = 0;
      for (;;) {
        const int64_t j = j0 - lane();
        uint64_t v = kLbInc;  // before the first chunk: an inclusive prefix of 0
        if (j >= 0)
          v = __hip_atomic_load(&lookback[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t st = v & ~kLbVal;
        const uint64_t inc = __ballot(st == kLbInc);
        const uint64_t open = __ballot(st == 0);
        // lanes up to and including the nearest inclusive one (all if none)
        const uint64_t need = inc ? ((inc & (0ull - inc)) << 1) - 1ull : ~0ull;
        if (open & need) {  // a needed predecessor has not published yet
          if (++spins > (1u << 24)) {  // never reached when every chunk runs
            if (threadIdx.x == 0) set_status(prm, ST_INTERNAL);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        uint64_t x = ((need >> lane()) & 1ull) ? (v & kLbVal) : 0ull;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
        excl += x;
        if (inc) break;
        j0 -= 64;
      }
      if (threadIdx.x == 0)
        __hip_atomic_store(&lookback[c], kLbInc | (excl + size), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) {
      s_excl = excl;
      parts[2 * c] = blen;
      parts[2 * c + 1] = slen;
    }
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
    const uint8_t* bp = (const uint8_t*)B;
    const uint8_t* sp = (const uint8_t*)U;
    for (uint32_t q = threadIdx.x; q < size / 4; q += kCT) {
      uint32_t w = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        w |= (uint32_t)record_byte(4 * q + b, hdr, bp, blen, sp, slen) << (8 * b);
      ((uint32_t*)(stream + dst))[q] = w;
    }
  } else if (threadIdx.x == 0) {
    set_status(prm, ST_CAPACITY);
  }
}

// Single field, one workgroup per chunk: encode and park the record.  This
// kernel and the two after it are skipped entirely when gate is given and
// *gate != 0 (the repair sweeps enqueued before them have not reached the
// fixed point; the host then sweeps on and encodes).
template <int K>
__global__ __launch_bounds__(kCT) void k_encode(
    uint32_t n, const typename Traits<K>::Bin* __restrict__ bins,
    const uint32_t* __restrict__ sub, uint32_t* parts, Params* prm, uint8_t* stream,
    uint64_t cap, uint32_t nch, RecordSlots S, const uint32_t* gate) {
  if (gate && *gate) return;
  encode_body<K, true>(n, bins, sub, nullptr, parts, prm, stream, cap, nch, blockIdx.x, S);
}

// Single field: exclusive offsets of the records in the stream body from
// their part sizes, 4096 chunks per pass (four per thread, read as two
// 16-byte vectors); the stream size.
constexpr int kOT = 1024;  // threads of the offset scan
__global__ __launch_bounds__(kOT) void k_record_offsets(const uint32_t* parts, uint32_t nch,
                                                        uint64_t* offs, Params* prm,
                                                        const uint32_t* gate) {
  if (gate && *gate) return;
  __shared__ uint64_t sh[kOT / 64 + 1];
  uint64_t carry = 0;
  for (uint32_t t0 = 0; t0 < nch; t0 += 4 * kOT) {
    const uint32_t i = t0 + 4 * threadIdx.x;
    uint32_t sz[4];
    if (i + 3 < nch) {
      const uint4 a = ((const uint4*)parts)[i / 2], b = ((const uint4*)parts)[i / 2 + 1];
      sz[0] = record_size(a.x, a.y);
      sz[1] = record_size(a.z, a.w);
      sz[2] = record_size(b.x, b.y);
      sz[3] = record_size(b.z, b.w);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        sz[k] = i + k < nch ? record_size(parts[2 * (i + k)], parts[2 * (i + k) + 1]) : 0u;
    }
    const uint64_t sum = (uint64_t)sz[0] + sz[1] + sz[2] + sz[3];
    uint64_t total;
    uint64_t off = carry + block_excl_scan<uint64_t, kOT / 64>(sum, sh, total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i + k < nch) offs[i + k] = off;
      off += sz[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) prm->stream_size = kHeaderBytes + 4ull * nch + carry;
}

// Single field, one workgroup per chunk: copy the parked record to its
// offset (ST_CAPACITY when the stream buffer is too short for it).
__global__ __launch_bounds__(kThreads) void k_place(const uint32_t* parts, const uint64_t* offs,
                                                    uint32_t nch, RecordSlots S, Params* prm,
                                                    uint8_t* stream, uint64_t cap,
                                                    const uint32_t* gate) {
  if (gate && *gate) return;
  const uint32_t c = blockIdx.x;
  const uint32_t size = record_size(parts[2 * c], parts[2 * c + 1]);
  const uint64_t dst = kHeaderBytes + 4ull * nch + offs[c];
  const bool last = c == nch - 1;
  if (size > (last ? S.tail_len : S.len[0] + S.len[1] + S.len[2])) return;  // flagged already
  if (dst + size > cap) {
    if (threadIdx.x == 0) set_status(prm, ST_CAPACITY);
    return;
  }
  uint32_t* out = (uint32_t*)(stream + dst);
  const uint32_t nw = size / 4;
  for (uint32_t q0 = 0; q0 < nw; q0 += 4 * kThreads) {
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t q = q0 + k * kThreads + threadIdx.x;
      v[k] = q < nw ? *slot_word(S, c, last, q) : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t q = q0 + k * kThreads + threadIdx.x;
      if (q < nw) out[q] = v[k];
    }
  }
}

// ------------------------------------------------------------------ decoder
// Exclusive offsets of the records from the size table; the sizes must add
// up to the stream body exactly.
__device__ __forceinline__ void offsets_body(const uint8_t* stream, uint32_t nch, uint64_t body_bytes,
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

// Single field, one 1024-thread block: the same scan, four sizes per thread
// per pass (one 16-byte read where the table allows; the table starts 4
// bytes past a 16-byte boundary of the stream only if the stream does), and
// the start of the decoder's status word (no separate clear).
constexpr int kOfT = 1024;
__global__ __launch_bounds__(kOfT) void k_offsets(
    const uint8_t* stream, uint32_t nch, uint64_t body_bytes,
    uint64_t* offsets, Params* prm) {
  __shared__ uint64_t sh[kOfT / 64 + 1];
  if (threadIdx.x == 0) prm->status = 0;
  const uint32_t* tab = (const uint32_t*)(stream + kHeaderBytes);
  const bool vec = ((uintptr_t)tab & 15u) == 0;
  uint64_t carry = 0;
  for (uint32_t t0 = 0; t0 < nch; t0 += 4 * kOfT) {
    const uint32_t i = t0 + 4 * threadIdx.x;
    uint32_t sz[4];
    if (vec && i + 3 < nch) {
      const uint4 a = *(const uint4*)(tab + i);
      sz[0] = a.x;
      sz[1] = a.y;
      sz[2] = a.z;
      sz[3] = a.w;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) sz[k] = i + k < nch ? tab[i + k] : 0u;
    }
    const uint64_t sum = (uint64_t)sz[0] + sz[1] + sz[2] + sz[3];
    uint64_t total;
    uint64_t off = carry + block_excl_scan<uint64_t, kOfT / 64>(sum, sh, total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i + k < nch) offsets[i + k] = off;
      off += sz[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && carry != body_bytes) set_status(prm, ST_FORMAT);
}

// Totals of the bins and subbin parts over all chunks (statistics only).
__global__ __launch_bounds__(kThreads) void k_sum_parts(const uint32_t* parts,
                                                        uint32_t nch, Params* prm) {
  __shared__ uint64_t sh[kWaves + 1];
  uint64_t b = 0, u = 0;
  for (uint32_t i = threadIdx.x; i < nch; i += kThreads) {
    b += parts[2 * i];
    u += parts[2 * i + 1];
  }
  uint64_t tb, tu;
  block_excl_scan<uint64_t>(b, sh, tb);
  block_excl_scan<uint64_t>(u, sh, tu);
  if (threadIdx.x == 0) {
    prm->bins_bytes = tb;
    prm->sub_bytes = tu;
  }
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
  while (k > -Tr::kMaxKey && Tr::q(Tr::to_double(Tr::unkey(k - 1)), inv) >= b) {
    --k;
    if (++steps > 8) return false;
  }
  while (Tr::q(Tr::to_double(Tr::unkey(k)), inv) < b) {
    if (k >= Tr::kMaxKey || ++steps > 8) return false;
    ++k;
  }
  if (Tr::q(Tr::to_double(Tr::unkey(k)), inv) != b) return false;
  out = k;
  return true;
}

// copy n bytes from global src (4-byte aligned base) to LDS dst
__device__ __forceinline__ void stage(uint8_t* dst, const uint8_t* src, uint32_t n) {
  const uint32_t nw = (n + 3) / 4;
  const uint32_t* s = (const uint32_t*)src;
  uint32_t* d = (uint32_t*)dst;
  for (uint32_t i0 = 0; i0 < nw; i0 += 4 * kCT) {
    uint32_t v[4];  // four loads in flight per thread
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = i0 + k * kCT + threadIdx.x;
      v[k] = i < nw ? s[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = i0 + k * kCT + threadIdx.x;
      if (i < nw) d[i] = v[k];
    }
  }
}

// BIT_K inverse of the groups g = wave + kCW * i (i < GPW) of G into w[i]
// (word 64g + lane): bit j of w[i] is bit `lane` of unit j * G + g, for the
// planes j of mask pm (the others are zero).  Planes outer, groups inner: the
// reads of one plane sit at fixed distances from one address, so they pair
// up into two-address LDS reads.
template <typename Word, int GPW>
__device__ __forceinline__ void planes_to_words(const uint64_t* planes, uint32_t G, uint64_t pm,
                                                Word (&w)[GPW]) {
  const uint32_t* P32 = (const uint32_t*)planes;
  const uint32_t half = (uint32_t)lane() >> 5, sh = (uint32_t)lane() & 31;
#pragma unroll
  for (int i = 0; i < GPW; ++i) w[i] = 0;
  if (wave() + kCW * (GPW - 1) < G) {  // every group of this wave present
    while (pm) {
      const uint32_t j = (uint32_t)__builtin_ctzll(pm);
      pm &= pm - 1;
      const uint32_t* row = P32 + 2 * (j * G + wave()) + half;
#pragma unroll
      for (int i = 0; i < GPW; ++i) w[i] |= (Word)((row[2 * kCW * i] >> sh) & 1u) << j;
    }
  } else {
    while (pm) {
      const uint32_t j = (uint32_t)__builtin_ctzll(pm);
      pm &= pm - 1;
      const uint32_t* row = P32 + 2 * (j * G + wave()) + half;
#pragma unroll
      for (int i = 0; i < GPW; ++i)
        if (wave() + kCW * i < G) w[i] |= (Word)((row[2 * kCW * i] >> sh) & 1u) << j;
    }
  }
}

// Decodes chunk c of a field (Sec. IV-E); a malformed record sets FORMAT.
template <int K>
__device__ __forceinline__ void decode_body(const uint8_t* __restrict__ stream, uint32_t n,
                            const uint64_t* __restrict__ offsets, Params* prm,
                            typename Traits<K>::Raw* __restrict__ out, uint32_t nch,
                            uint32_t c) {
  using Tr = Traits<K>;
  using Word = typename Tr::Word;
  constexpr uint32_t W = kChunkBytes / K;
  constexpr int GPW = (int)(W / 64 / kCW);  // groups per wave
  __shared__ uint64_t U[kMaxUnits + 2];
  __shared__ uint64_t Mb[kMaxUnits + 2];
  __shared__ Scratch sc;
  __shared__ uint64_t gsum[64 + 1];  // per-group sums of the bin deltas
  __shared__ int64_t s_mm[2][kCW];     // per-wave least / greatest bin
  __shared__ int s_bad;

  const uint32_t p0 = c * W, nc = min(W, n - p0);
  const uint32_t m = (nc + 63) / 64 * 64, G = m / 64, L = m * K;
  const uint64_t body = kHeaderBytes + 4ull * nch;
  // the record's size and offset are read together with the status;
  // offsets inconsistent (one read decides for the block: other chunks may
  // set the flag concurrently)
  const uint32_t rsize = ((const uint32_t*)(stream + kHeaderBytes))[c];
  const uint64_t roff = offsets[c];
  if (threadIdx.x == 0) s_bad = 0;
  __shared__ uint32_t s_fail;
  if (threadIdx.x == 0) s_fail = prm->status & ST_FORMAT;
  __syncthreads();
  if (s_fail) return;
  const uint8_t* rec = stream + body + roff;
  if (rsize < kRecordHeaderBytes || (rsize & 3)) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }
  // a record that fits in Mb (every record of a chunk that compresses at all)
  // comes in with one load per word, its parts are then read from LDS; the
  // header is read (scalar loads) while the words are in flight
  const bool whole = rsize <= 8 * (kMaxUnits + 2);
  if (whole) stage((uint8_t*)Mb, rec, rsize);
  const uint8_t* hd = rec;
  const double inv = __longlong_as_double(*(const long long*)(stream + 56));
  const double winv = 1.0 / inv;
  const uint32_t bfl = hd[0], sfl = hd[1];
  const uint32_t npts = hd[2] | (hd[3] << 8);
  const uint32_t blen = *(const uint32_t*)(hd + 4);
  const uint32_t smid = *(const uint32_t*)(hd + 8);
  const uint32_t slen = *(const uint32_t*)(hd + 12);
  bool ok = !(bfl & ~1u) && !(sfl & ~3u) && npts == nc && blen <= L &&
            smid <= L && slen <= L;
  const uint32_t used = kRecordHeaderBytes + blen + slen;
  ok = ok && ((used + 3) & ~3u) == rsize;
  if (ok && threadIdx.x < rsize - used && hd[used + threadIdx.x] != 0) s_bad = 1;
  __syncthreads();  // s_bad, and the staged record
  ok = ok && !s_bad;
  if (!ok) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }

  // bins: RZE_1 -> BIT_K -> negabinary -> prefix sum (words kept in registers)
  const uint64_t* bsrc = Mb + (whole ? kRecordHeaderBytes / 8 : 0);
  if (!whole) {
    stage((uint8_t*)Mb, rec + kRecordHeaderBytes, blen);
    __syncthreads();
  }
  const uint64_t* planes;
  uint64_t pm0 = 0;
  if (bfl & 1) {
    ok = blen == L;
    planes = bsrc;
    if (ok) pm0 = nonzero_planes<K>(planes, G, sc);
  } else {
    ok = rze_decode<1>((const uint8_t*)bsrc, blen, L, U, sc, G);
    planes = U;
    pm0 = sc.planes;
  }
  if (!ok) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }
  Word wv[GPW];
  int64_t bmin = INT64_MAX, bmax = INT64_MIN;
  {
    planes_to_words<Word, GPW>(planes, G, pm0, wv);
    const Word Mk = (Word)0xAAAAAAAAAAAAAAAAull;
#pragma unroll
    for (int i = 0; i < GPW; ++i) {
      const uint32_t g = wave() + kCW * i;
      const Word w = wv[i];
      // negabinary -> delta; inclusive prefix within the group of 64 words
      Word d = (g * 64 + lane() < nc) ? (Word)((w ^ Mk) - Mk) : (Word)0;
      d = wave_scan<Word>(d);
      wv[i] = d;
      if (lane() == 63 && g < G) gsum[g] = (uint64_t)d;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      uint64_t v = threadIdx.x < G ? gsum[threadIdx.x] : 0ull;
      const uint64_t x = wave_scan_u64(v);
      if (threadIdx.x < G) gsum[threadIdx.x] = x - v;  // exclusive
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < GPW; ++i) {
      const uint32_t g = wave() + kCW * i;
      if (g < G) wv[i] += (Word)gsum[g];
      const int64_t b = K == 4 ? (int64_t)(int32_t)(uint32_t)wv[i] : (int64_t)(uint64_t)wv[i];
      if (g * 64 + lane() < nc) {
        bmin = b < bmin ? b : bmin;
        bmax = b > bmax ? b : bmax;
      }
    }
    // the chunk's bin range (for the floor table below); the wave results
    // are read after the next barrier
    bmin = wave_reduce(bmin, OpMin{});
    bmax = wave_reduce(bmax, OpMax{});
    if (lane() == 0) {
      s_mm[0][wave()] = bmin;
      s_mm[1][wave()] = bmax;
    }
  }

  // subbins: RZE_1 -> RZE_K -> BIT_K (the part goes to U, free now)
  const uint32_t soff = kRecordHeaderBytes + blen;
  const uint32_t shift = soff & 3u;
  if (whole) {
    const uint32_t* src = (const uint32_t*)((const uint8_t*)Mb + (soff - shift));
    for (uint32_t i = threadIdx.x; i < (slen + shift + 3) / 4; i += kCT) ((uint32_t*)U)[i] = src[i];
  } else {
    stage((uint8_t*)U, rec + (soff - shift), slen + shift);
  }
  __syncthreads();
  const uint8_t* sp = (const uint8_t*)U + shift;
  if (sfl & 2) {
    ok = slen == smid;
    if (ok) {
      uint8_t* mb = (uint8_t*)Mb;
      for (uint32_t i = threadIdx.x; i < smid; i += kCT) mb[i] = sp[i];
    }
    __syncthreads();
  } else {
    ok = rze_decode<1>(sp, slen, smid, Mb, sc, 0);
  }
  uint64_t* spare = Mb;  // the buffer not holding the subbin planes
  uint64_t spm = 0;
  if (ok) {
    if (sfl & 1) {
      ok = smid == L;
      planes = Mb;
      spare = U;
      if (ok) spm = nonzero_planes<K>(planes, G, sc);
    } else {
      ok = rze_decode<K>((const uint8_t*)Mb, smid, L, U, sc, G);
      planes = U;
      spm = sc.planes;
    }
  }
  if (!ok) {
    if (threadIdx.x == 0) set_status(prm, ST_FORMAT);
    return;
  }
  // BIT_K inverse of the subbins into registers, word 64g + lane of group
  // g = wave + kCW * i in sv[i] (as the bins)
  Word sv[GPW];
  planes_to_words<Word, GPW>(planes, G, spm, sv);

  // reconstruct (Sec. IV-E).  The bin floors of the chunk's bin range go to
  // a table in the spare buffer when the range is small enough, so that each
  // distinct bin is walked once.
  using Key = typename Tr::Bin;  // order keys fit the signed bin type
  constexpr uint32_t kTab = kChunkBytes / sizeof(Key);
  constexpr Key kNoKey = (Key)((uint64_t)1 << (8 * sizeof(Key) - 1));  // most negative
  for (int w = 0; w < kCW; ++w) {
    bmin = min(bmin, s_mm[0][w]);
    bmax = max(bmax, s_mm[1][w]);
  }
  // the table also holds the floor of bin bmax + 1: the keys of bin b are
  // those from floor(b) up to floor(b + 1) (the bins are monotone in the
  // value), so a point whose next bin has a floor needs no re-quantization
  const bool table = (uint64_t)bmax - (uint64_t)bmin < kTab - 1;
  Key* T = (Key*)spare;
  if (table) {
    const uint32_t R = (uint32_t)((uint64_t)bmax - (uint64_t)bmin) + 2;
    for (uint32_t e = threadIdx.x; e < R; e += kCT) {
      int64_t klo;
      T[e] = bin_floor_key<K>(bmin + (int64_t)e, inv, winv, klo) ? (Key)klo : kNoKey;
    }
  }
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int i = 0; i < GPW; ++i) {
    const uint32_t j = (wave() + kCW * i) * 64 + lane();
    if (j >= nc) continue;
    const int64_t b = K == 4 ? (int64_t)(int32_t)(uint32_t)wv[i] : (int64_t)(uint64_t)wv[i];
    const uint64_t s = (uint64_t)sv[i];
    int64_t klo;
    bool have;
    Key next = kNoKey;  // floor of bin b + 1, when known
    if (table) {
      const uint32_t e = (uint32_t)((uint64_t)b - (uint64_t)bmin);
      const Key t = T[e];
      next = T[e + 1];
      have = t != kNoKey;
      klo = (int64_t)t;
    } else {
      have = bin_floor_key<K>(b, inv, winv, klo);
    }
    typename Tr::Raw v = 0;
    // the room above klo can exceed the int64 range: unsigned difference
    if (!have || s > (uint64_t)Tr::kMaxKey - (uint64_t)klo) {
      bad = true;
    } else {
      v = Tr::unkey(klo + (int64_t)s);
      if (next != kNoKey) {
        // inside bin b iff below the floor of bin b + 1
        if (s >= (uint64_t)((int64_t)next - klo)) bad = true;
      } else if (s && Tr::q(Tr::to_double(v), inv) != b) {
        bad = true;
      }
    }
    out[p0 + j] = v;
  }
  if (bad) set_status(prm, ST_FORMAT);
}

template <int K>
__global__ __launch_bounds__(kCT, 6) void k_decode(
    const uint8_t* __restrict__ stream, uint32_t n,
    const uint64_t* __restrict__ offsets, Params* prm,
    typename Traits<K>::Raw* __restrict__ out) {
  decode_body<K>(stream, n, offsets, prm, out, gridDim.x, blockIdx.x);
}

// ------------------------------------------------------------------ batches
// Encoder over the chunks of every field of one dtype, in ticket order: a
// chunk's look-back only waits for chunks of its field with earlier tickets,
// which workgroups already hold.  Skipped when *gate != 0 (the repair sweeps
// before it have not reached the fixed point: tiles are listed for sweep
// gate_sweep).
template <int K>
__global__ __launch_bounds__(kCT) void k_encode_p(const BatchDesc* bd, const Job* jobs,
                                                  int gate_sweep) {
  constexpr int g0 = K == 4 ? 0 : 2;
  __shared__ uint32_t s_t;
  BatchCounters* bc = bd->bc;
  if (gate_sweep > 0 && bc->lens[gate_sweep % kRing]) return;
  const uint32_t i0 = bd->item0[PH_C][g0], i1 = bd->item0[PH_C][g0 + 2];
  const int j0 = (int)bd->job0[g0], j1 = (int)bd->job0[g0 + 2];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_t = i0 + atomicAdd(&bc->enc_cursor[K == 4 ? 0 : 1], 1u);
    __syncthreads();
    const uint32_t t = s_t;
    if (t >= i1) break;
    const Job& J = jobs[find_job<&Job::c0>(jobs, j0, j1, t)];
    encode_body<K, false>(J.box.n, (const typename Traits<K>::Bin*)J.bins, J.sub, J.lookback,
                          J.parts, J.prm, J.stream, J.cap, J.nch, t - J.c0, RecordSlots{});
  }
}

__device__ int status_of(uint32_t st) {
  if (st & ST_NONFINITE) return -2;
  if (st & ST_BOUND) return -3;
  if (st & ST_RANGE) return -4;
  if (st & ST_FORMAT) return -6;
  if (st & ST_INTERNAL) return -9;
  if (st & ST_CAPACITY) return -5;
  return 0;
}

// Per-field results of a compress batch: stream size and status.
__global__ __launch_bounds__(kThreads) void k_finalize_c(const BatchDesc* bd, const Job* jobs,
                                                         int gate_sweep) {
  if (gate_sweep > 0 && bd->bc->lens[gate_sweep % kRing]) return;
  BatchResult* res = bd->res;
  const uint32_t nj = bd->job0[kGroups];
  for (uint32_t j = blockIdx.x * kThreads + threadIdx.x; j < nj; j += gridDim.x * kThreads) {
    const Job& J = jobs[j];
    const int st = status_of(J.prm->status);
    const uint64_t size = J.prm->stream_size;
    res[j].size = size;
    res[j].status = st;
    for (int b = 0; b < (int)kHeaderBytes; ++b) res[j].header[b] = J.prm->header[b];
    if (J.out_size) *J.out_size = size;
    if (J.out_status) *J.out_status = st;
  }
}

// Header check of a field to decode (the same rules as the host parser),
// then the record offsets from its size table.
__global__ __launch_bounds__(kThreads) void k_dhead_p(const BatchDesc* bd, const Job* jobs) {
  __shared__ int s_ok;
  const int nj = (int)bd->job0[kGroups];
  for (int j = blockIdx.x; j < nj; j += gridDim.x) {
    const Job& J = jobs[j];
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint8_t* h = J.stream;
      auto u64 = [&](int o) {
        uint64_t v = 0;
        for (int b = 0; b < 8; ++b) v |= (uint64_t)h[o + b] << (8 * b);
        return v;
      };
      bool ok = (u64(0) & 0xFFFFFFFFFFFFull) == ((uint64_t)kMagic | ((uint64_t)kVersion << 32));
      ok = ok && h[6] == J.dtype && h[7] == J.ndim && h[32] <= 1 &&
           (uint32_t)u64(36) == kChunkBytes;
      for (int i = 0; i < 3; ++i)
        ok = ok && u64(8 + 8 * i) == (uint64_t)(i < J.ndim ? J.dims[i] : 1);
      const double e = __longlong_as_double((long long)u64(48));
      const double v = __longlong_as_double((long long)u64(56));
      ok = ok && finite64(u64(48)) && e > 0.0 && finite64(u64(56)) && v > 0.0;
      ok = ok && fma(v, e, -1.0) >= 0.0 &&
           fma(__longlong_as_double((long long)u64(56) - 1), e, -1.0) < 0.0;
      if (!ok) set_status(J.prm, ST_FORMAT);
      s_ok = ok;
    }
    __syncthreads();
    if (s_ok)
      offsets_body(J.stream, J.nch, J.stream_size - kHeaderBytes - 4ull * J.nch, J.offsets,
                   J.prm);
  }
}

template <int K>
__global__ __launch_bounds__(kCT, 6) void k_decode_p(const BatchDesc* bd, const Job* jobs) {
  constexpr int g0 = K == 4 ? 0 : 2;
  __shared__ uint32_t s_t;
  BatchCounters* bc = bd->bc;
  const uint32_t i0 = bd->item0[PH_C][g0], i1 = bd->item0[PH_C][g0 + 2];
  const int j0 = (int)bd->job0[g0], j1 = (int)bd->job0[g0 + 2];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_t = i0 + atomicAdd(&bc->dec_cursor[K == 4 ? 0 : 1], 1u);
    __syncthreads();
    const uint32_t t = s_t;
    if (t >= i1) break;
    const Job& J = jobs[find_job<&Job::c0>(jobs, j0, j1, t)];
    decode_body<K>(J.stream, J.box.n, J.offsets, J.prm,
                   (typename Traits<K>::Raw*)J.y, J.nch, t - J.c0);
  }
}

// Per-field results of a decompress batch: field bytes and status.
__global__ __launch_bounds__(kThreads) void k_finalize_d(const BatchDesc* bd, const Job* jobs) {
  BatchResult* res = bd->res;
  const uint32_t nj = bd->job0[kGroups];
  for (uint32_t j = blockIdx.x * kThreads + threadIdx.x; j < nj; j += gridDim.x * kThreads) {
    const Job& J = jobs[j];
    const int st = status_of(J.prm->status);
    const uint64_t size = st ? 0 : (uint64_t)J.box.n * (J.dtype == 0 ? 4u : 8u);
    res[j].size = size;
    res[j].status = st;
    if (J.out_size) *J.out_size = size;
    if (J.out_status) *J.out_status = st;
  }
}

// Direct grids: one workgroup per chunk.  The encoder still takes its chunk
// from the ticket counter, so chunks start in field-major order.
template <int K>
__global__ __launch_bounds__(kCT) void k_encode_d(const BatchDesc* bd, const Job* jobs,
                                                  int gate_sweep) {
  constexpr int g0 = K == 4 ? 0 : 2;
  __shared__ uint32_t s_t;
  BatchCounters* bc = bd->bc;
  if (gate_sweep > 0 && bc->lens[gate_sweep % kRing]) return;
  if (threadIdx.x == 0) s_t = bd->item0[PH_C][g0] + atomicAdd(&bc->enc_cursor[K == 4 ? 0 : 1], 1u);
  __syncthreads();
  const uint32_t t = s_t;
  const Job& J = jobs[find_job<&Job::c0>(jobs, (int)bd->job0[g0], (int)bd->job0[g0 + 2], t)];
  encode_body<K, false>(J.box.n, (const typename Traits<K>::Bin*)J.bins, J.sub, J.lookback,
                        J.parts, J.prm, J.stream, J.cap, J.nch, t - J.c0, RecordSlots{});
}

template <int K>
__global__ __launch_bounds__(kCT, 6) void k_decode_d(const BatchDesc* bd, const Job* jobs) {
  constexpr int g0 = K == 4 ? 0 : 2;
  const uint32_t t = bd->item0[PH_C][g0] + blockIdx.x;
  const Job& J = jobs[find_job<&Job::c0>(jobs, (int)bd->job0[g0], (int)bd->job0[g0 + 2], t)];
  decode_body<K>(J.stream, J.box.n, J.offsets, J.prm, (typename Traits<K>::Raw*)J.y, J.nch,
                 t - J.c0);
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_encode(int dtype, uint32_t n, const void* bins, uint32_t* sub,
                         uint16_t* mask, uint8_t* tail, uint64_t* offs, uint32_t* parts,
                         Params* prm, uint8_t* stream, size_t cap, const uint32_t* gate,
                         hipStream_t s, Ev ev) {
  const uint32_t K = dtype == 0 ? 4 : 8;
  const uint32_t W = kChunkBytes / K;
  const uint32_t nch = (n + W - 1) / W;
  RecordSlots S;
  S.seg[0] = (uint8_t*)bins;
  S.seg[1] = (uint8_t*)sub;
  S.seg[2] = (uint8_t*)mask;
  S.len[0] = W * K;
  S.len[1] = W * 4;
  S.len[2] = W * 2;
  S.tail = tail;
  S.tail_len = kRecordTailBytes;
  if (dtype == 0)
    launch_ev(k_encode<4>, dim3(nch), dim3(kCT), s, Ev{ev.a, nullptr}, n,
                          (const int32_t*)bins, (const uint32_t*)sub, parts, prm, stream,
                          (uint64_t)cap, nch, S, gate);
  else
    launch_ev(k_encode<8>, dim3(nch), dim3(kCT), s, Ev{ev.a, nullptr}, n,
                          (const int64_t*)bins, (const uint32_t*)sub, parts, prm, stream,
                          (uint64_t)cap, nch, S, gate);
  k_record_offsets<<<1, kOT, 0, s>>>(parts, nch, offs, prm, gate);
  launch_ev(k_place, dim3(nch), dim3(kThreads), s, Ev{nullptr, ev.b},
                        (const uint32_t*)parts, (const uint64_t*)offs, nch, S, prm, stream,
                        (uint64_t)cap, gate);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const uint32_t* parts, uint32_t nch, Params* prm,
                            hipStream_t s) {
  k_sum_parts<<<1, kThreads, 0, s>>>(parts, nch, prm);
  return hipGetLastError();
}

hipError_t launch_offsets(const uint8_t* stream, uint32_t nch,
                          uint64_t body_bytes, uint64_t* offsets, Params* prm,
                          hipStream_t s, Ev ev) {
  launch_ev(k_offsets, dim3(1), dim3(kOfT), s, ev, stream, nch,
                        body_bytes, offsets, prm);
  return hipGetLastError();
}

hipError_t launch_decode(int dtype, const uint8_t* stream, uint32_t n,
                         const uint64_t* offsets, Params* prm, void* field,
                         hipStream_t s, Ev ev) {
  uint32_t W = kChunkBytes / (dtype == 0 ? 4 : 8);
  uint32_t nch = (n + W - 1) / W;
  if (dtype == 0)
    launch_ev(k_decode<4>, dim3(nch), dim3(kCT), s, ev, stream, n,
                          offsets, prm, (uint32_t*)field);
  else
    launch_ev(k_decode<8>, dim3(nch), dim3(kCT), s, ev, stream, n,
                          offsets, prm, (uint64_t*)field);
  return hipGetLastError();
}

hipError_t launch_encode_p(int dtype, const BatchDesc* bd, const Job* jobs, int gate_sweep,
                           int grid, hipStream_t s) {
  if (dtype == 0) k_encode_p<4><<<grid, kCT, 0, s>>>(bd, jobs, gate_sweep);
  else k_encode_p<8><<<grid, kCT, 0, s>>>(bd, jobs, gate_sweep);
  return hipGetLastError();
}

hipError_t launch_finalize_c(const BatchDesc* bd, const Job* jobs, int gate_sweep,
                             hipStream_t s) {
  k_finalize_c<<<4, kThreads, 0, s>>>(bd, jobs, gate_sweep);
  return hipGetLastError();
}

hipError_t launch_dhead_p(const BatchDesc* bd, const Job* jobs, int grid, hipStream_t s) {
  k_dhead_p<<<grid, kThreads, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

hipError_t launch_decode_p(int dtype, const BatchDesc* bd, const Job* jobs, int grid,
                           hipStream_t s) {
  if (dtype == 0) k_decode_p<4><<<grid, kCT, 0, s>>>(bd, jobs);
  else k_decode_p<8><<<grid, kCT, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

hipError_t launch_finalize_d(const BatchDesc* bd, const Job* jobs, hipStream_t s) {
  k_finalize_d<<<4, kThreads, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

hipError_t launch_encode_d(int dtype, const BatchDesc* bd, const Job* jobs, int gate_sweep,
                           uint32_t items, hipStream_t s) {
  if (!items) return hipSuccess;
  if (dtype == 0) k_encode_d<4><<<items, kCT, 0, s>>>(bd, jobs, gate_sweep);
  else k_encode_d<8><<<items, kCT, 0, s>>>(bd, jobs, gate_sweep);
  return hipGetLastError();
}

hipError_t launch_decode_d(int dtype, const BatchDesc* bd, const Job* jobs, uint32_t items,
                           hipStream_t s) {
  if (!items) return hipSuccess;
  if (dtype == 0) k_decode_d<4><<<items, kCT, 0, s>>>(bd, jobs);
  else k_decode_d<8><<<items, kCT, 0, s>>>(bd, jobs);
  return hipGetLastError();
}

int codec_blocks_per_cu(int kernel) {
  int b = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (kernel) {
    case PK_ENCODE: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_encode_p<8>, kCT, 0); break;
    case PK_DHEAD: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_dhead_p, kThreads, 0); break;
    case PK_DECODE: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_decode_p<8>, kCT, 0); break;
    default: break;
  }
  return e == hipSuccess && b > 0 ? b : 1;
}

}  // namespace lopc
