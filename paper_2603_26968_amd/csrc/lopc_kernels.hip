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

#include "lopc_device.h"

namespace lopc {
namespace {

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
  // mark the 26 neighbour tiles for the next sweep; one atomic per block
  // adds the number of newly marked tiles to one of 64 spread counters
  bool newly = false;
  if (edge && threadIdx.x < 27) {
    int dz = (int)threadIdx.x / 9 - 1, dy = ((int)threadIdx.x / 3) % 3 - 1,
        dx = (int)threadIdx.x % 3 - 1;
    int nz = tz + dz, ny = ty + dy, nx = tx + dx;
    if ((dz | dy | dx) != 0 && nz >= 0 && nz < tl.ntz && ny >= 0 &&
        ny < tl.nty && nx >= 0 && nx < tl.ntx) {
      uint32_t u = ((uint32_t)nz * tl.nty + ny) * tl.ntx + nx;
      uint32_t prev = atomicMax(&stamp[u], sweep + 1);
      newly = prev < sweep + 1;
    }
  }
  if (threadIdx.x < 64) {
    uint64_t m = __ballot(newly);
    if (threadIdx.x == 0 && m)
      atomicAdd(&counters[1 + 64 * (sweep & 1) + (t & 63)], (uint32_t)__popcll(m));
  }
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

}  // namespace lopc
