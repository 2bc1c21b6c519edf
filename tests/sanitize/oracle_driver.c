/* Driver for the sanitizer build of the CPU oracle (test infrastructure):
 * compresses and decompresses seeded fields of both dtypes, 2D and 3D, with
 * ragged chunks, ties and a long falling chain, checks that every value
 * comes back within the bound, then feeds the decoder corrupted copies of
 * the streams (single-bit flips, truncations) that must be rejected or
 * decoded without any access outside the buffers.  Built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py; exits
 * non-zero on the first failed check (the sanitizers abort on their own). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/lopc_ref.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) { /* splitmix64 */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double next_unit(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

static int fail(const char* what, int code) {
  fprintf(stderr, "oracle_driver: %s (%d)\n", what, code);
  return 1;
}

/* kind 0: smooth + noise, 1: integer ties, 2: falling chain */
static int one_case(int dtype, int ndim, const int64_t* dims, int kind, double eb, int mode) {
  size_t n = 1;
  for (int i = 0; i < ndim; ++i) n *= (size_t)dims[i];
  const size_t k = dtype == 0 ? 4 : 8;
  void* x = malloc(n * k);
  void* y = malloc(n * k);
  for (size_t i = 0; i < n; ++i) {
    double v;
    if (kind == 0) v = sin(0.01 * (double)i) + 1e-3 * (next_unit() - 0.5);
    else if (kind == 1) v = (double)(next_u64() % 5) * 0.25;
    else v = (double)(n - i) / (double)n;
    if (dtype == 0) ((float*)x)[i] = (float)v;
    else ((double*)x)[i] = v;
  }
  size_t cap = 0, size = 0;
  int st = lopc_ref_compress_bound(dtype, ndim, dims, &cap);
  if (st) return fail("compress_bound", st);
  uint8_t* s = malloc(cap);
  st = lopc_ref_compress(x, dtype, ndim, dims, eb, mode, s, cap, &size);
  if (st) return fail("compress", st);
  st = lopc_ref_decompress(s, size, y, n * k);
  if (st) return fail("decompress", st);
  double eps, inv;
  int dt2, nd2;
  int64_t d2[3];
  st = lopc_ref_stream_info(s, size, &dt2, &nd2, d2, &eps, &inv);
  if (st) return fail("stream_info", st);
  for (size_t i = 0; i < n; ++i) {
    const double a = dtype == 0 ? ((float*)x)[i] : ((double*)x)[i];
    const double b = dtype == 0 ? ((float*)y)[i] : ((double*)y)[i];
    if (!(fabs(a - b) <= eps)) return fail("error bound", (int)i);
  }
  /* a capacity one byte short is refused */
  if (size > 0 && lopc_ref_compress(x, dtype, ndim, dims, eb, mode, s, size - 1, &cap) !=
                      LOPC_REF_E_CAPACITY)
    return fail("capacity", 0);
  /* corrupted copies: flips anywhere, and truncations */
  uint8_t* c = malloc(size);
  for (int t = 0; t < 60; ++t) {
    memcpy(c, s, size);
    const size_t pos = (size_t)(next_u64() % size);
    c[pos] ^= (uint8_t)(1u << (next_u64() % 8));
    (void)lopc_ref_decompress(c, size, y, n * k);
    const size_t cut = (size_t)(next_u64() % size);
    (void)lopc_ref_decompress(c, cut, y, n * k);
  }
  free(c);
  free(s);
  free(x);
  free(y);
  return 0;
}

int main(void) {
  static const int64_t shapes[][3] = {{1, 1, 1},   {3, 5, 1},   {64, 64, 1},  {65, 63, 1},
                                      {1, 4097, 1}, {9, 17, 33}, {8, 8, 32},  {17, 9, 65},
                                      {2, 3, 300}, {1, 1, 2049}};
  static const int ndims[] = {2, 2, 2, 2, 2, 3, 3, 3, 3, 3};
  int cases = 0;
  for (int si = 0; si < 10; ++si)
    for (int dtype = 0; dtype < 2; ++dtype)
      for (int kind = 0; kind < 3; ++kind) {
        const double eb = kind == 2 ? 10.0 : (kind == 1 ? 0.3 : 1e-2);
        const int mode = kind == 0 ? 1 : 0;
        if (kind == 0 && shapes[si][0] * shapes[si][1] * shapes[si][2] == 1) continue;
        if (one_case(dtype, ndims[si], shapes[si], kind, eb, mode)) return 1;
        ++cases;
      }
  printf("oracle_driver: %d cases clean\n", cases);
  return 0;
}
