// Scalar arithmetic of liblopc.so that must be bit-exact: order keys and the
// quantizer.  Host+device so that a CPU harness can check the same source.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lopc {

#define LOPC_HD __host__ __device__ __forceinline__

// ------------------------------------------------------------------ values
// Order key: monotone in the value, -0 == +0, consecutive representable
// values have consecutive keys.
LOPC_HD int64_t key32(uint32_t u) {
  return (u >> 31) ? -(int64_t)(u & 0x7fffffffu) : (int64_t)u;
}
LOPC_HD int64_t key64(uint64_t u) {
  return (u >> 63) ? -(int64_t)(u & 0x7fffffffffffffffull) : (int64_t)u;
}
LOPC_HD uint32_t unkey32(int64_t k) {
  return k >= 0 ? (uint32_t)k : (0x80000000u | (uint32_t)(-k));
}
LOPC_HD uint64_t unkey64(int64_t k) {
  return k >= 0 ? (uint64_t)k : (0x8000000000000000ull | (uint64_t)(-k));
}
LOPC_HD bool finite32(uint32_t u) {
  return (u & 0x7f800000u) != 0x7f800000u;
}
LOPC_HD bool finite64(uint64_t u) {
  return (u & 0x7ff0000000000000ull) != 0x7ff0000000000000ull;
}

// Quantizer (Sec. IV-A): nearest integer to the exact real y*inv, ties to
// even, saturated to +-(2^62 + 1).  The rounded product p and the exact
// residual r = fma(y, inv, -p) give the real product p + r exactly.  Rounding
// is monotone and half-integers below 2^52 are representable, so the real
// product lies on the same side of every half-integer as p, or p is that
// half-integer: rint(p) (ties to even) is the answer unless p is a
// half-integer, and then the sign of r decides (r == 0: a true tie, which
// rint already resolved to even).  From 2^52 on p is an integer and the
// fraction of the real product is in r.
LOPC_HD int64_t q_bin(double y, double inv) {
  const double two52 = 4503599627370496.0;
  const double two62 = 4611686018427387904.0;
  const int64_t sat = 4611686018427387905ll;
  double p = y * inv;
  if (!(fabs(p) <= two62)) return p < 0 ? -sat : sat;
  if (fabs(p) < two52) {
    double q = rint(p);
    if (fabs(p - q) == 0.5) {
      const double r = fma(y, inv, -p);
      if (r != 0.0) q = r > 0.0 ? p + 0.5 : p - 0.5;
    }
    return (int64_t)q;
  }
  double r = fma(y, inv, -p);
  const bool neg = p < 0.0;
  const double a = fabs(p);
  const double rr = neg ? -r : r;
  // a is an integer; the fraction of the magnitude is in rr
  double t = fabs(rr);
  double ft = floor(t);
  double frt = t - ft;
  int64_t cand = rr >= 0.0 ? (int64_t)a + (int64_t)ft : (int64_t)a - (int64_t)ft;
  int64_t step = rr >= 0.0 ? 1 : -1;
  if (frt > 0.5 || (frt == 0.5 && (cand & 1))) cand += step;
  int64_t q = cand;
  if (q > sat) q = sat;
  return neg ? -q : q;
}

// The same function for float32 fields, whose bins must lie within
// +-(2^31 - 2): exact for |y*inv| < 2^31 with 32-bit integer conversions;
// larger products return +-2^31, which is outside the float32 bin range.
LOPC_HD int64_t q_bin32(double y, double inv) {
  const double two31 = 2147483648.0;
  const double p = y * inv;
  if (!(fabs(p) < two31)) return p < 0.0 ? -(int64_t)two31 : (int64_t)two31;
  double q = rint(p);
  if (fabs(p - q) == 0.5) {
    const double r = fma(y, inv, -p);
    if (r != 0.0) q = r > 0.0 ? p + 0.5 : p - 0.5;
  }
  return (int64_t)(int32_t)q;
}

}  // namespace lopc
