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
// residual r = fma(y, inv, -p) give the real product p + r exactly.  The
// rounding is done on the magnitude a = |p| (residual rr = +-r), where the
// fraction a - floor(a) is exact; rounding p can only cross a half-integer h
// if a == h, and then the sign of rr decides.
LOPC_HD int64_t q_bin(double y, double inv) {
  const double two52 = 4503599627370496.0;
  const double two62 = 4611686018427387904.0;
  const int64_t sat = 4611686018427387905ll;
  double p = y * inv;
  if (!(fabs(p) <= two62)) return p < 0 ? -sat : sat;
  double r = fma(y, inv, -p);
  const bool neg = p < 0.0;
  const double a = fabs(p);
  const double rr = neg ? -r : r;
  int64_t q;
  if (a < two52) {
    double fl = floor(a);
    double fr = a - fl;
    q = (int64_t)fl;
    bool up = fr > 0.5 || (fr == 0.5 && (rr > 0.0 || (rr == 0.0 && (q & 1))));
    q += up ? 1 : 0;
  } else {
    // a is an integer; the fraction of the magnitude is in rr
    double t = fabs(rr);
    double ft = floor(t);
    double frt = t - ft;
    int64_t cand = rr >= 0.0 ? (int64_t)a + (int64_t)ft : (int64_t)a - (int64_t)ft;
    int64_t step = rr >= 0.0 ? 1 : -1;
    if (frt > 0.5 || (frt == 0.5 && (cand & 1))) cand += step;
    q = cand;
  }
  if (q > sat) q = sat;
  return neg ? -q : q;
}

// The same function for float32 fields, whose bins must lie within
// +-(2^31 - 2): exact for |y*inv| < 2^31 with 32-bit integer conversions;
// larger products return +-2^31, which is outside the float32 bin range.
LOPC_HD int64_t q_bin32(double y, double inv) {
  const double two31 = 2147483648.0;
  double p = y * inv;
  const bool neg = p < 0.0;
  const double a = fabs(p);
  if (!(a < two31)) return neg ? -(int64_t)two31 : (int64_t)two31;
  double r = fma(y, inv, -p);
  const double rr = neg ? -r : r;
  const double fl = floor(a);
  const double fr = a - fl;
  int32_t q = (int32_t)fl;
  bool up = fr > 0.5 || (fr == 0.5 && (rr > 0.0 || (rr == 0.0 && (q & 1))));
  int64_t v = (int64_t)q + (up ? 1 : 0);
  return neg ? -v : v;
}

}  // namespace lopc
