// Device helpers shared by the kernels of liblopc.so: wave64 lane/wave ids,
// block scans, per-dtype traits.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include "lopc_internal.h"
#include "lopc_numeric.h"

namespace lopc {

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
  __device__ static int64_t q(double y, double inv) { return q_bin32(y, inv); }
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
  __device__ static int64_t q(double y, double inv) { return q_bin(y, inv); }
};

// ------------------------------------------------------------------ stencil
// Edges of the Freudenthal triangulation: +-d for nonzero d in {0,1}^3,
// listed as (dz, dy, dx); bit j of a point's mask refers to offset j.  Even
// entries point to a higher linear index (raising weight 1), odd ones lower.
constexpr int8_t kOff[14][3] = {
    {0, 0, 1},  {0, 0, -1},  {0, 1, 0},  {0, -1, 0}, {0, 1, 1},
    {0, -1, -1}, {1, 0, 0},  {-1, 0, 0}, {1, 0, 1},  {-1, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, 1, 1},  {-1, -1, -1}};
// The same table as arithmetic, for a j known only at run time (no memory
// access): offset j is +-(x, y, z bits of (j >> 1) + 1), minus for odd j.
__device__ __forceinline__ int off_x(int j) {
  const int e = (j >> 1) + 1;
  return (j & 1) ? -(e & 1) : (e & 1);
}
__device__ __forceinline__ int off_y(int j) {
  const int e = (j >> 1) + 1;
  return (j & 1) ? -((e >> 1) & 1) : ((e >> 1) & 1);
}
__device__ __forceinline__ int off_z(int j) {
  const int e = (j >> 1) + 1;
  return (j & 1) ? -(e >> 2) : (e >> 2);
}
// linear offset of stencil offset j in a row-major box of rows hx, planes hxy
__device__ __forceinline__ int off_lin(int j, int hx, int hxy) {
  const int e = (j >> 1) + 1;
  const int o = (e & 1) + ((e >> 1) & 1) * hx + (e >> 2) * hxy;
  return (j & 1) ? -o : o;
}

// ------------------------------------------------------------------ scans
// Wave-wide inclusive prefix sums through DPP lane moves instead of the LDS
// crossbar: shifts by 1, 2, 4 and 8 lanes inside each row of 16 (lanes
// shifted in from outside the row read 0), then the rows are joined by
// broadcasting lane 15 into rows 1 and 3 and lane 31 into rows 2 and 3.
template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, ZERO);
}
template <int CTRL, int ROWS, bool ZERO>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
  return (uint64_t)dpp_u32<CTRL, ROWS, ZERO>((uint32_t)x) |
         (uint64_t)dpp_u32<CTRL, ROWS, ZERO>((uint32_t)(x >> 32)) << 32;
}
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x) {
  x += dpp_u32<0x111, 0xf, true>(x);  // row_shr:1
  x += dpp_u32<0x112, 0xf, true>(x);  // row_shr:2
  x += dpp_u32<0x114, 0xf, true>(x);  // row_shr:4
  x += dpp_u32<0x118, 0xf, true>(x);  // row_shr:8
  x += dpp_u32<0x142, 0xa, false>(x);  // row_bcast:15
  x += dpp_u32<0x143, 0xc, false>(x);  // row_bcast:31
  return x;
}
__device__ __forceinline__ uint64_t wave_scan_u64(uint64_t x) {
  x += dpp_u64<0x111, 0xf, true>(x);
  x += dpp_u64<0x112, 0xf, true>(x);
  x += dpp_u64<0x114, 0xf, true>(x);
  x += dpp_u64<0x118, 0xf, true>(x);
  x += dpp_u64<0x142, 0xa, false>(x);
  x += dpp_u64<0x143, 0xc, false>(x);
  return x;
}
template <typename V>
__device__ __forceinline__ V wave_scan(V x) {
  if constexpr (sizeof(V) == 8) return (V)wave_scan_u64((uint64_t)x);
  else return (V)wave_scan_u32((uint32_t)x);
}

// The same lane moves for an idempotent operation (or, min, max): a lane
// with no source keeps its own value, and the scan pattern leaves the whole
// wave's result in lane 63, read back as a wave-uniform value.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_keep_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS, typename V>
__device__ __forceinline__ V dpp_keep(V x) {
  if constexpr (sizeof(V) == 8) {
    const uint64_t u = (uint64_t)x;
    return (V)((uint64_t)dpp_keep_u32<CTRL, ROWS>((uint32_t)u) |
               (uint64_t)dpp_keep_u32<CTRL, ROWS>((uint32_t)(u >> 32)) << 32);
  } else {
    return (V)dpp_keep_u32<CTRL, ROWS>((uint32_t)x);
  }
}
template <typename V, typename Op>
__device__ __forceinline__ V wave_reduce(V x, Op op) {
  x = op(x, dpp_keep<0x111, 0xf>(x));
  x = op(x, dpp_keep<0x112, 0xf>(x));
  x = op(x, dpp_keep<0x114, 0xf>(x));
  x = op(x, dpp_keep<0x118, 0xf>(x));
  x = op(x, dpp_keep<0x142, 0xa>(x));
  x = op(x, dpp_keep<0x143, 0xc>(x));
  if constexpr (sizeof(V) == 8) {
    const uint64_t u = (uint64_t)x;
    return (V)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63) |
               (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63)
                   << 32);
  } else {
    return (V)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
  }
}
struct OpOr {
  template <typename V>
  __device__ V operator()(V a, V b) const { return a | b; }
};
struct OpMin {
  template <typename V>
  __device__ V operator()(V a, V b) const { return b < a ? b : a; }
};
struct OpMax {
  template <typename V>
  __device__ V operator()(V a, V b) const { return b > a ? b : a; }
};

// Exclusive scan of v over a block of NW waves; sh needs NW + 1 slots;
// total receives the block sum.  Every thread of the block must call it.
template <typename V, int NW = kWaves>
__device__ V block_excl_scan(V v, V* sh, V& total) {
  V x = wave_scan<V>(v);
  if (lane() == 63) sh[wave()] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    V acc = 0;
    for (int w = 0; w < NW; ++w) {
      V t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[NW] = acc;
  }
  __syncthreads();
  V res = x - v + sh[wave()];
  total = sh[NW];
  __syncthreads();
  return res;
}

// Launch k on s; when a timing event is given the dispatch itself records
// the kernel's start (ev.a) and end (ev.b), else it is an ordinary launch
// (which stream capture records as a plain kernel node).
template <typename... P, typename... A>
inline void launch_ev(void (*k)(P...), dim3 g, dim3 b, hipStream_t s, Ev ev, A... a) {
  if (ev.a || ev.b)
    hipExtLaunchKernelGGL(k, g, b, 0, s, ev.a, ev.b, 0, a...);
  else
    k<<<g, b, 0, s>>>(a...);
}

__device__ __forceinline__ void put_bytes(uint8_t* dst, uint64_t v, int nbytes) {
  for (int i = 0; i < nbytes; ++i) dst[i] = (uint8_t)(v >> (8 * i));
}

}  // namespace lopc
