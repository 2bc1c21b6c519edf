/*
 * lopc_ref.h -- CPU oracle of LOPC, the Local-Order-Preserving Compressor
 * (Fallin, Gorski, Agarwal, Wang, Gopalakrishnan, Burtscher, arXiv 2603.26968).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded
 * implementation written from the paper's text so that the GPU library can
 * be checked against it.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the GPU library never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (the readings of the paper that the text leaves open are
 * listed in the design doc of the repository):
 *   - a field is a C-order array, last axis fastest; the "index" of a point
 *     that breaks ties is its linear offset (Alg. 2 compares point indices);
 *   - float32 fields use 32-bit bins and subbins, float64 fields 64-bit ones
 *     (Sec. IV-C names the 4- and 8-byte pipelines);
 *   - every function returns 0 or one of the negative status codes below.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (tests/test_oracle_*.py) except the byte layout of the container, which
 * the paper does not describe; that layout is pinned only by round trips
 * and frozen golden streams ("parity unpinned" against the paper).
 */
#ifndef LOPC_REF_H
#define LOPC_REF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LOPC_REF_OK = 0,
  LOPC_REF_E_ARG = -1,        /* bad shape, dtype, mode or pointer          */
  LOPC_REF_E_NONFINITE = -2,  /* NaN or Inf in the field                    */
  LOPC_REF_E_BOUND = -3,      /* error bound not finite/positive, or NOA on
                                 a constant field (zero range)              */
  LOPC_REF_E_RANGE = -4,      /* a bin number does not fit its integer type */
  LOPC_REF_E_CAPACITY = -5,   /* output buffer too small                    */
  LOPC_REF_E_FORMAT = -6,     /* malformed or corrupt stream                */
  LOPC_REF_E_NOMEM = -8       /* host allocation failed                     */
};

/* dtype: 0 = float32, 1 = float64.  mode: 0 = ABS, 1 = NOA (Sec. IV-A). */

/* Error-bound parameters (Sec. IV-A): eps is the absolute bound (eb for ABS,
 * eb * (max - min) for NOA, all in binary64), inv the smallest binary64 with
 * inv * eps >= 1, so that a bin of width 1/inv never exceeds eps. */
int lopc_ref_error_params(const void* field, int dtype, size_t n, double eb,
                          int mode, double* eps, double* inv);

/* Quantizer Q (Sec. IV-A): nearest integer to the exact real y*inv, ties to
 * even.  Returns LOPC_REF_E_RANGE if |bin| exceeds the dtype's limit
 * (2^31-2 for dtype 0, 2^62 for dtype 1). */
int lopc_ref_quantize(double y, double inv, int dtype, int64_t* bin);

/* Bins of a whole field (Alg. 1, first loop). */
int lopc_ref_bins(const void* field, int dtype, size_t n, double inv,
                  int64_t* bins);

/* Subbins (Alg. 1 and Alg. 2, Sec. IV-B): the least fixed point of
 *   s(p) = max(0, max over same-bin neighbours n that precede p of
 *                 s(n) + [index(n) > index(p)]),
 * computed by one pass over the points in ascending (value, index) order. */
int lopc_ref_subbins(const void* field, int dtype, int ndim,
                     const int64_t* dims, const int64_t* bins, uint64_t* subbins);

/* Lowest value of dtype whose bin is b (decoding rule, Sec. IV-E). */
int lopc_ref_bin_floor(int64_t b, double inv, int dtype, double* lo);

/* Decoding of one point: the value s representable steps above the bin floor,
 * i.e. subbin 0 is the lowest value of the bin, subbin 1 the next (Sec. IV-E). */
int lopc_ref_reconstruct(int64_t b, uint64_t s, double inv, int dtype,
                         double* value);

/* Lossless stages on byte strings (Sec. IV-C).  k = word size in bytes.
 *   DIFFNB_k: in-place on an array of int64 words: delta from the previous
 *             word (0 before the first), then two's complement -> negabinary,
 *             all modulo 2^(8k).
 *   BIT_k:    bit transposition of m words (m % 64 == 0): plane j holds bit j
 *             of every word, planes stored lowest bit first, LSB-first.
 *   RZE_w:    zero-word elimination with a recursively compressed bitmap; the
 *             return value is the output length, *passthrough is set when the
 *             input is stored verbatim because the output would not be smaller.
 */
void lopc_ref_diffnb(int64_t* words, size_t n, int k);
void lopc_ref_undiffnb(int64_t* words, size_t n, int k);
int lopc_ref_bit(const uint8_t* in, size_t m, int k, uint8_t* out);
int lopc_ref_unbit(const uint8_t* in, size_t m, int k, uint8_t* out);
size_t lopc_ref_rze(const uint8_t* in, size_t len, int w, uint8_t* out,
                    int* passthrough);
int lopc_ref_unrze(const uint8_t* in, size_t in_len, size_t len, int w,
                   uint8_t* out);

/* Whole stream. */
int lopc_ref_compress_bound(int dtype, int ndim, const int64_t* dims,
                            size_t* bytes);
int lopc_ref_compress(const void* field, int dtype, int ndim,
                      const int64_t* dims, double eb, int mode, void* out,
                      size_t cap, size_t* out_size);
int lopc_ref_stream_info(const void* stream, size_t size, int* dtype,
                         int* ndim, int64_t* dims, double* eps, double* inv);
int lopc_ref_decompress(const void* stream, size_t size, void* field,
                        size_t cap);

/* Decoded bins and subbins of a stream (for tests). */
int lopc_ref_decode_codes(const void* stream, size_t size, int64_t* bins,
                          uint64_t* subbins);

#ifdef __cplusplus
}
#endif
#endif
