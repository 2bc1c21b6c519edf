// lopc_verify.hip -- invariant checker of liblopc.so (gfx950): what LOPC
// guarantees of a reconstruction, measured at GPU speed on whole fields.
//
//   - every point within the bound: |x - x'| <= eps (exact: the difference is
//     formed as a double-word sum, Sec. IV-A);
//   - every edge of the triangulation keeps the order of its end points in
//     (value, index) order, ties broken by the lower index (Sec. II, IV-E);
//   - hence every vertex keeps its critical type: no lower link vertex ->
//     minimum, no upper -> maximum, one connected component each -> regular,
//     else saddle (Sec. II); boundary vertices use the in-grid part of the
//     link.
//
// One thread per point; counters are reduced per block and added to the
// caller's workspace words.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lopc_device.h"

namespace lopc {
namespace {

// link adjacency of the stencil kOff: neighbours j and j' of a vertex span a
// triangle with it when kOff[j'] - kOff[j] is itself a stencil offset
struct LinkAdj {
  uint16_t m[14];
};
constexpr bool is_offset(int a, int b, int c) {
  for (int j = 0; j < 14; ++j)
    if (kOff[j][0] == a && kOff[j][1] == b && kOff[j][2] == c) return true;
  return false;
}
constexpr LinkAdj make_adj() {
  LinkAdj r{};
  for (int i = 0; i < 14; ++i) {
    uint16_t m = 0;
    for (int j = 0; j < 14; ++j)
      if (j != i && is_offset(kOff[j][0] - kOff[i][0], kOff[j][1] - kOff[i][1],
                              kOff[j][2] - kOff[i][2]))
        m |= (uint16_t)(1u << j);
    r.m[i] = m;
  }
  return r;
}
__constant__ LinkAdj c_adj = make_adj();

// connected components of a subset of the link
__device__ __forceinline__ int components(uint32_t mask) {
  int n = 0;
  while (mask) {
    uint32_t comp = mask & (0u - mask), prev = 0;
    while (comp != prev) {
      prev = comp;
      uint32_t grow = 0, c = comp;
      while (c) {
        const int j = __builtin_ctz(c);
        c &= c - 1;
        grow |= c_adj.m[j];
      }
      comp |= grow & mask;
    }
    mask &= ~comp;
    ++n;
  }
  return n;
}

// 0 regular, 1 minimum, 2 maximum, 3 saddle (as the tests' helper)
__device__ __forceinline__ int crit_type(uint32_t lower, uint32_t upper) {
  if (!upper) return 2;
  if (!lower) return 1;
  return components(lower) == 1 && components(upper) == 1 ? 0 : 3;
}

// words of the report in the workspace
enum {
  V_POINTS, V_BOUND, V_MAXERR, V_EDGES, V_ORDER, V_CO, V_CR = V_CO + 4, V_MISMATCH = V_CR + 4,
  V_WORDS
};

template <int K>
__global__ __launch_bounds__(kThreads) void k_verify(const typename Traits<K>::Raw* __restrict__ x,
                                                     const typename Traits<K>::Raw* __restrict__ y,
                                                     Box box, double eps,
                                                     unsigned long long* out) {
  using Tr = Traits<K>;
  constexpr int NJ = 14;
  uint64_t nbound = 0, nedge = 0, norder = 0, nmis = 0, npts = 0;
  uint64_t co[4] = {0, 0, 0, 0}, cr[4] = {0, 0, 0, 0};
  double maxerr = 0.0;
  const uint64_t n = box.n;
  for (uint64_t p = (uint64_t)blockIdx.x * kThreads + threadIdx.x; p < n;
       p += (uint64_t)gridDim.x * kThreads) {
    const int xx = (int)(p % (uint64_t)box.nx);
    const int yy = (int)((p / (uint64_t)box.nx) % (uint64_t)box.ny);
    const int zz = (int)(p / ((uint64_t)box.nx * (uint64_t)box.ny));
    const typename Tr::Raw xp = x[p], yp = y[p];
    ++npts;
    // |x - x'| <= eps, exactly: s + e = a - b with s rounded (two-sum)
    {
      const double a = Tr::to_double(xp), b = -Tr::to_double(yp);
      const double s = a + b, bb = s - a, e = (a - (s - bb)) + (b - bb);
      const double as = fabs(s);
      if (as > eps || (as == eps && e != 0.0 && ((e > 0.0) == (s > 0.0)))) ++nbound;
      maxerr = as > maxerr ? as : maxerr;
    }
    const int64_t kx = Tr::key(xp), ky = Tr::key(yp);
    uint32_t lox = 0, hix = 0, loy = 0, hiy = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int qz = zz + kOff[j][0], qy = yy + kOff[j][1], qx = xx + kOff[j][2];
      if (qz < 0 || qz >= box.nz || qy < 0 || qy >= box.ny || qx < 0 || qx >= box.nx) continue;
      const uint64_t q = ((uint64_t)qz * box.ny + qy) * box.nx + qx;
      const int64_t kxq = Tr::key(x[q]), kyq = Tr::key(y[q]);
      // odd j: the neighbour has the lower index, so it is lower on a tie
      const bool lx = kxq < kx || (kxq == kx && (j & 1));
      const bool ly = kyq < ky || (kyq == ky && (j & 1));
      lox |= (uint32_t)lx << j;
      hix |= (uint32_t)!lx << j;
      loy |= (uint32_t)ly << j;
      hiy |= (uint32_t)!ly << j;
      if (!(j & 1)) {  // each edge once, from its lower-index end
        ++nedge;
        norder += lx != ly;
      }
    }
    const int tx = crit_type(lox, hix), ty = crit_type(loy, hiy);
    ++co[tx];
    ++cr[ty];
    nmis += tx != ty;
  }
  // block reduction through LDS, then one atomic per word
  __shared__ unsigned long long red[V_WORDS][kWaves];
  uint64_t v[V_WORDS] = {npts, nbound, 0, nedge, norder, co[0], co[1], co[2], co[3],
                         cr[0], cr[1], cr[2], cr[3], nmis};
  v[V_MAXERR] = (uint64_t)__double_as_longlong(maxerr);
#pragma unroll
  for (int w = 0; w < V_WORDS; ++w) {
    uint64_t a = v[w];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      const uint64_t o = __shfl_xor(a, d, 64);
      a = w == V_MAXERR ? (o > a ? o : a) : a + o;  // non-negative doubles order as integers
    }
    if (lane() == 0) red[w][wave()] = a;
  }
  __syncthreads();
  if (threadIdx.x < V_WORDS) {
    const int w = threadIdx.x;
    uint64_t a = red[w][0];
    for (int q = 1; q < kWaves; ++q)
      a = w == V_MAXERR ? (red[w][q] > a ? red[w][q] : a) : a + red[w][q];
    if (w == V_MAXERR) atomicMax(&out[w], (unsigned long long)a);
    else if (a) atomicAdd(&out[w], (unsigned long long)a);
  }
}

}  // namespace

hipError_t launch_verify(int dtype, const void* x, const void* y, Box box, double eps,
                         unsigned long long* out, int blocks, hipStream_t s) {
  if (dtype == 0)
    k_verify<4><<<blocks, kThreads, 0, s>>>((const uint32_t*)x, (const uint32_t*)y, box, eps, out);
  else
    k_verify<8><<<blocks, kThreads, 0, s>>>((const uint64_t*)x, (const uint64_t*)y, box, eps, out);
  return hipGetLastError();
}

}  // namespace lopc
