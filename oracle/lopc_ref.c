/*
 * lopc_ref.c -- CPU oracle of LOPC (arXiv 2603.26968).
 *
 * TEST INFRASTRUCTURE ONLY: a plain single-threaded implementation written
 * from the paper so that the GPU library can be checked against it.  The GPU
 * library never links, loads or calls this file.  Build with
 *   gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared lopc_ref.c -lm
 * so that every floating-point operation is the IEEE binary64 operation it
 * reads as (no contraction into fused multiply-adds, no reassociation).
 *
 * Section map:
 *   error bound and quantizer ............ Sec. IV-A
 *   neighbours, order, subbins ........... Sec. II, Sec. IV-B, Alg. 1, Alg. 2
 *   decoding rule ........................ Sec. IV-E (last paragraph)
 *   lossless stages and 16 kB chunks ..... Sec. III-B (PFPL), Sec. IV-C
 *   container (header, chunk table) ...... not in the paper: this project's
 *                                          own layout ("parity unpinned")
 */
#include "lopc_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define CHUNK_BYTES 16384u
#define HEADER_BYTES 64u
#define RECORD_HEADER_BYTES 16u
#define MAGIC 0x43504F4Cu /* "LOPC" */
#define VERSION 1u

/* ------------------------------------------------------------------------ */
/* Values, order keys.                                                       */
/* ------------------------------------------------------------------------ */

static double value_at(const void* f, int dtype, size_t i) {
  if (dtype == 0) return (double)((const float*)f)[i];
  return ((const double*)f)[i];
}

/* Order key: an integer that increases with the value, with -0 and +0 equal;
 * consecutive representable values have consecutive keys. */
static int64_t key_of(double y, int dtype) {
  if (dtype == 0) {
    float v = (float)y;
    uint32_t u;
    memcpy(&u, &v, 4);
    if (u >> 31) return -(int64_t)(u & 0x7fffffffu);
    return (int64_t)u;
  } else {
    uint64_t u;
    memcpy(&u, &y, 8);
    if (u >> 63) return -(int64_t)(u & 0x7fffffffffffffffULL);
    return (int64_t)u;
  }
}

static double value_of_key(int64_t k, int dtype) {
  if (dtype == 0) {
    uint32_t u = k >= 0 ? (uint32_t)k : (0x80000000u | (uint32_t)(-k));
    float v;
    memcpy(&v, &u, 4);
    return (double)v;
  } else {
    uint64_t u = k >= 0 ? (uint64_t)k
                        : (0x8000000000000000ULL | (uint64_t)(-k));
    double v;
    memcpy(&v, &u, 8);
    return v;
  }
}

/* key of the largest finite value */
static int64_t max_finite_key(int dtype) {
  return dtype == 0 ? (int64_t)0x7f7fffff : (int64_t)0x7fefffffffffffffLL;
}

static int64_t bin_limit(int dtype) {
  return dtype == 0 ? (int64_t)2147483646 : (int64_t)4611686018427387904LL;
}

/* ------------------------------------------------------------------------ */
/* Quantizer (Sec. IV-A): bin = nearest integer to y / eps.                  */
/* ------------------------------------------------------------------------ */

/* Exact product of two finite binary64 numbers as sign * P * 2^E with an
 * integer P < 2^106: each operand is an integer mantissa times a power of 2. */
typedef struct {
  int neg;
  unsigned __int128 p;
  int e;
} exact_product;

static void split_double(double d, uint64_t* m, int* e) {
  uint64_t u;
  memcpy(&u, &d, 8);
  int ex = (int)((u >> 52) & 0x7ff);
  uint64_t fr = u & 0xfffffffffffffULL;
  if (ex == 0) { /* zero or subnormal */
    *m = fr;
    *e = -1074;
  } else {
    *m = fr | (1ULL << 52);
    *e = ex - 1075;
  }
}

static exact_product mul_exact(double a, double b) {
  uint64_t ma, mb;
  int ea, eb;
  split_double(a, &ma, &ea);
  split_double(b, &mb, &eb);
  exact_product r;
  r.neg = (signbit(a) != 0) != (signbit(b) != 0);
  r.p = (unsigned __int128)ma * mb;
  r.e = ea + eb;
  return r;
}

/* Nearest integer to the exact real product y*inv, ties to even, saturated
 * to +-(2^62 + 1) when the product is larger than 2^62 in magnitude. */
static int64_t q_sat(double y, double inv) {
  const int64_t sat = 4611686018427387905LL;
  exact_product x = mul_exact(y, inv);
  unsigned __int128 q;
  if (x.p == 0) return 0;
  if (x.e >= 0) {
    if (x.e > 62) return x.neg ? -sat : sat;
    q = x.p << x.e; /* P < 2^106 would overflow only for huge e: checked */
    if (x.e > 0 && (q >> x.e) != x.p) return x.neg ? -sat : sat;
  } else {
    int s = -x.e;
    if (s >= 120) {
      q = 0; /* P < 2^106 <= 2^(s-1): below one half */
    } else {
      unsigned __int128 one = 1;
      unsigned __int128 rem = x.p & ((one << s) - 1);
      unsigned __int128 half = one << (s - 1);
      q = x.p >> s;
      if (rem > half || (rem == half && (q & 1))) q += 1;
    }
  }
  if (q > (unsigned __int128)sat) q = sat;
  return x.neg ? -(int64_t)q : (int64_t)q;
}

/* is the exact product a*b >= 1 ? (a, b > 0) */
static int product_at_least_one(double a, double b) {
  exact_product x = mul_exact(a, b);
  if (x.p == 0) return 0;
  if (x.e >= 0) return 1;
  if (-x.e >= 120) return 0;
  return x.p >= ((unsigned __int128)1 << (-x.e));
}

/* ------------------------------------------------------------------------ */
/* Error bound (Sec. IV-A).                                                  */
/* ------------------------------------------------------------------------ */

int lopc_ref_error_params(const void* field, int dtype, size_t n, double eb,
                          int mode, double* eps, double* inv) {
  if ((dtype != 0 && dtype != 1) || (mode != 0 && mode != 1) || !eps || !inv)
    return LOPC_REF_E_ARG;
  if (n == 0 || !field) return LOPC_REF_E_ARG;
  if (!isfinite(eb) || !(eb > 0)) return LOPC_REF_E_BOUND;
  double lo = 0, hi = 0;
  for (size_t i = 0; i < n; ++i) {
    double y = value_at(field, dtype, i);
    if (!isfinite(y)) return LOPC_REF_E_NONFINITE;
    if (i == 0 || y < lo) lo = y;
    if (i == 0 || y > hi) hi = y;
  }
  double e = eb;
  if (mode == 1) {
    /* NOA: the bound is relative to the value range R = max - min. */
    double range = hi - lo;
    e = eb * range;
  }
  if (!isfinite(e) || !(e > 0)) return LOPC_REF_E_BOUND;
  /* inv: the smallest binary64 whose exact product with eps is >= 1 */
  double v = 1.0 / e;
  if (!isfinite(v)) return LOPC_REF_E_BOUND;
  while (!product_at_least_one(v, e)) v = nextafter(v, INFINITY);
  while (product_at_least_one(nextafter(v, 0.0), e)) v = nextafter(v, 0.0);
  if (!isfinite(v)) return LOPC_REF_E_BOUND;
  *eps = e;
  *inv = v;
  return LOPC_REF_OK;
}

int lopc_ref_quantize(double y, double inv, int dtype, int64_t* bin) {
  if ((dtype != 0 && dtype != 1) || !bin) return LOPC_REF_E_ARG;
  if (!isfinite(y)) return LOPC_REF_E_NONFINITE;
  int64_t q = q_sat(y, inv);
  int64_t lim = bin_limit(dtype);
  if (q > lim || q < -lim) return LOPC_REF_E_RANGE;
  *bin = q;
  return LOPC_REF_OK;
}

int lopc_ref_bins(const void* field, int dtype, size_t n, double inv,
                  int64_t* bins) {
  if (!field || !bins || (dtype != 0 && dtype != 1)) return LOPC_REF_E_ARG;
  for (size_t i = 0; i < n; ++i) {
    int st = lopc_ref_quantize(value_at(field, dtype, i), inv, dtype, &bins[i]);
    if (st) return st;
  }
  return LOPC_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Neighbours (Sec. II): the grid is split into triangles (2D) or            */
/* tetrahedra (3D); two grid points are neighbours when they share an edge.  */
/* With the Freudenthal split along the (+1,+1[,+1]) diagonal the edges of a  */
/* point are the offsets d and -d for every nonzero d in {0,1}^ndim.          */
/* ------------------------------------------------------------------------ */

static int neighbour_offsets(int ndim, int off[14][3]) {
  int cnt = 0;
  for (int a = 0; a <= 1; ++a)
    for (int b = 0; b <= 1; ++b)
      for (int c = 0; c <= 1; ++c) {
        if (ndim == 2 && c) continue;
        if (!a && !b && !c) continue;
        off[cnt][0] = a; off[cnt][1] = b; off[cnt][2] = c; ++cnt;
        off[cnt][0] = -a; off[cnt][1] = -b; off[cnt][2] = -c; ++cnt;
      }
  return cnt; /* 6 in 2D, 14 in 3D */
}

/* ------------------------------------------------------------------------ */
/* Subbins (Sec. IV-B, Alg. 1, Alg. 2).                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t key;
  uint64_t idx;
} ordered_point;

static int cmp_points(const void* a, const void* b) {
  const ordered_point* x = (const ordered_point*)a;
  const ordered_point* y = (const ordered_point*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

int lopc_ref_subbins(const void* field, int dtype, int ndim,
                     const int64_t* dims, const int64_t* bins,
                     uint64_t* subbins) {
  if (!field || !dims || !bins || !subbins) return LOPC_REF_E_ARG;
  if ((dtype != 0 && dtype != 1) || (ndim != 2 && ndim != 3))
    return LOPC_REF_E_ARG;
  int64_t d[3] = {dims[0], dims[1], ndim == 3 ? dims[2] : 1};
  for (int i = 0; i < 3; ++i)
    if (d[i] < 1) return LOPC_REF_E_ARG;
  size_t n = (size_t)d[0] * (size_t)d[1] * (size_t)d[2];

  /* The order that the subbins must reproduce: p precedes q when p's value is
   * smaller, or the values are equal and p's index is smaller (the tie rule
   * that Alg. 2 and the two raising rules of Sec. IV-E imply). */
  ordered_point* ord = (ordered_point*)malloc(n * sizeof(ordered_point));
  if (!ord) return LOPC_REF_E_NOMEM;
  for (size_t i = 0; i < n; ++i) {
    ord[i].key = key_of(value_at(field, dtype, i), dtype);
    ord[i].idx = i;
  }
  qsort(ord, n, sizeof(ordered_point), cmp_points);

  int off[14][3];
  int nn = neighbour_offsets(ndim, off);
  /* Every same-bin neighbour that precedes p comes earlier in this order, so
   * its subbin is final when p is visited: one pass gives the fixed point. */
  for (size_t t = 0; t < n; ++t) {
    uint64_t p = ord[t].idx;
    int64_t pk = ord[t].key;
    int64_t i0 = (int64_t)(p / (uint64_t)(d[1] * d[2]));
    int64_t i1 = (int64_t)((p / (uint64_t)d[2]) % (uint64_t)d[1]);
    int64_t i2 = (int64_t)(p % (uint64_t)d[2]);
    uint64_t s = 0;
    for (int j = 0; j < nn; ++j) {
      int64_t a = i0 + off[j][0], b = i1 + off[j][1], c = i2 + off[j][2];
      if (a < 0 || a >= d[0] || b < 0 || b >= d[1] || c < 0 || c >= d[2])
        continue;
      uint64_t q = (uint64_t)((a * d[1] + b) * d[2] + c);
      if (bins[q] != bins[p]) continue;
      int64_t qk = key_of(value_at(field, dtype, q), dtype);
      int precedes = qk < pk || (qk == pk && q < p);
      if (!precedes) continue;
      /* raising rule: equal to the neighbour's subbin if the neighbour has
       * the lower index, one more if it has the higher index */
      uint64_t cand = subbins[q] + (q > p ? 1u : 0u);
      if (cand > s) s = cand;
    }
    subbins[p] = s;
  }
  free(ord);
  return LOPC_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Decoding (Sec. IV-E): subbin 0 is the lowest representable value of the   */
/* bin, subbin 1 the next lowest, and so on.                                 */
/* ------------------------------------------------------------------------ */

static int bin_floor_key(int64_t b, double inv, int dtype, int64_t* out) {
  if (b > bin_limit(dtype) || b < -bin_limit(dtype)) return LOPC_REF_E_FORMAT;
  /* start near the lower edge (b - 1/2)/inv of the bin, then step to the
   * first representable value whose bin is b.  The rounded edge lies within
   * two representable values of that value (one for float32) at every bin
   * magnitude and bound, so a walk of more than 8 steps means a bin no value
   * of the dtype can have: the stream is malformed. */
  double c = ((double)b - 0.5) / inv;
  if (dtype == 0) c = (double)(float)c;
  if (!isfinite(c)) return LOPC_REF_E_FORMAT;
  int64_t k = key_of(c, dtype);
  int64_t kmax = max_finite_key(dtype);
  int steps = 0;
  while (k > -kmax && q_sat(value_of_key(k - 1, dtype), inv) >= b) {
    --k;
    if (++steps > 8) return LOPC_REF_E_FORMAT;
  }
  while (q_sat(value_of_key(k, dtype), inv) < b) {
    if (k >= kmax) return LOPC_REF_E_FORMAT;
    ++k;
    if (++steps > 8) return LOPC_REF_E_FORMAT;
  }
  if (q_sat(value_of_key(k, dtype), inv) != b) return LOPC_REF_E_FORMAT;
  *out = k;
  return LOPC_REF_OK;
}

int lopc_ref_bin_floor(int64_t b, double inv, int dtype, double* lo) {
  if ((dtype != 0 && dtype != 1) || !lo) return LOPC_REF_E_ARG;
  int64_t k;
  int st = bin_floor_key(b, inv, dtype, &k);
  if (st) return st;
  *lo = value_of_key(k, dtype);
  return LOPC_REF_OK;
}

int lopc_ref_reconstruct(int64_t b, uint64_t s, double inv, int dtype,
                         double* value) {
  if ((dtype != 0 && dtype != 1) || !value) return LOPC_REF_E_ARG;
  int64_t k;
  int st = bin_floor_key(b, inv, dtype, &k);
  if (st) return st;
  int64_t kmax = max_finite_key(dtype);
  /* kmax - k can exceed the int64 range (k near -kmax): take it unsigned */
  if (s > (uint64_t)kmax - (uint64_t)k) return LOPC_REF_E_FORMAT;
  int64_t kk = k + (int64_t)s;
  double v = value_of_key(kk, dtype);
  /* a valid stream never leaves the bin */
  if (q_sat(v, inv) != b) return LOPC_REF_E_FORMAT;
  *value = v;
  return LOPC_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Lossless stages (Sec. III-B on PFPL, Sec. IV-C).                          */
/* ------------------------------------------------------------------------ */

static uint64_t word_mask(int k) {
  return k == 8 ? ~0ULL : ((1ULL << (8 * k)) - 1);
}

/* negabinary digits of v (mod 2^(8k)) as an unsigned word */
static uint64_t to_negabinary(uint64_t v, int k) {
  uint64_t m = 0xAAAAAAAAAAAAAAAAULL & word_mask(k);
  return ((v + m) ^ m) & word_mask(k);
}

static uint64_t from_negabinary(uint64_t v, int k) {
  uint64_t m = 0xAAAAAAAAAAAAAAAAULL & word_mask(k);
  return ((v ^ m) - m) & word_mask(k);
}

void lopc_ref_diffnb(int64_t* w, size_t n, int k) {
  uint64_t prev = 0;
  for (size_t i = 0; i < n; ++i) {
    uint64_t cur = (uint64_t)w[i];
    uint64_t d = (cur - prev) & word_mask(k);
    prev = cur;
    w[i] = (int64_t)to_negabinary(d, k);
  }
}

void lopc_ref_undiffnb(int64_t* w, size_t n, int k) {
  uint64_t acc = 0;
  for (size_t i = 0; i < n; ++i) {
    acc = (acc + from_negabinary((uint64_t)w[i], k)) & word_mask(k);
    /* sign-extend the k-byte value */
    uint64_t v = acc;
    if (k < 8 && (v >> (8 * k - 1)) & 1) v |= ~word_mask(k);
    w[i] = (int64_t)v;
  }
}

static uint64_t get_word(const uint8_t* p, size_t i, int k) {
  uint64_t v = 0;
  for (int j = 0; j < k; ++j) v |= (uint64_t)p[i * k + j] << (8 * j);
  return v;
}

static void put_word(uint8_t* p, size_t i, int k, uint64_t v) {
  for (int j = 0; j < k; ++j) p[i * k + j] = (uint8_t)(v >> (8 * j));
}

int lopc_ref_bit(const uint8_t* in, size_t m, int k, uint8_t* out) {
  if (m % 64) return LOPC_REF_E_ARG;
  memset(out, 0, m * k);
  for (size_t i = 0; i < m; ++i) {
    uint64_t v = get_word(in, i, k);
    for (int j = 0; j < 8 * k; ++j)
      if ((v >> j) & 1) {
        size_t bit = (size_t)j * m + i; /* plane j, position i */
        out[bit / 8] |= (uint8_t)(1u << (bit % 8));
      }
  }
  return LOPC_REF_OK;
}

int lopc_ref_unbit(const uint8_t* in, size_t m, int k, uint8_t* out) {
  if (m % 64) return LOPC_REF_E_ARG;
  for (size_t i = 0; i < m; ++i) {
    uint64_t v = 0;
    for (int j = 0; j < 8 * k; ++j) {
      size_t bit = (size_t)j * m + i;
      if ((in[bit / 8] >> (bit % 8)) & 1) v |= 1ULL << j;
    }
    put_word(out, i, k, v);
  }
  return LOPC_REF_OK;
}

/* RZE_w: a bitmap with one bit per w-byte word (1 = nonzero word) plus the
 * nonzero words.  The bitmap is then compressed again and again with the
 * same idea, except that a byte is dropped when it repeats the byte before
 * it (the byte before the first is 0): each level keeps a bitmap of which
 * bytes changed plus the changed bytes, until the bitmap is at most 8 bytes.
 * Output: the last bitmap, then the kept bytes of each level from the top
 * level down, then the nonzero words. */
#define RZE_MAX_LEVELS 24

static int rze_level_sizes(size_t items, size_t* sz) {
  int lv = 0;
  sz[0] = (items + 7) / 8;
  while (sz[lv] > 8) {
    sz[lv + 1] = (sz[lv] + 7) / 8;
    ++lv;
  }
  return lv; /* index of the top (stored raw) bitmap */
}

size_t lopc_ref_rze(const uint8_t* in, size_t len, int w, uint8_t* out,
                    int* passthrough) {
  size_t items = len / (size_t)w;
  size_t sz[RZE_MAX_LEVELS];
  int top = rze_level_sizes(items, sz);
  uint8_t* bm[RZE_MAX_LEVELS];
  uint8_t* kept[RZE_MAX_LEVELS];
  size_t nkept[RZE_MAX_LEVELS];
  for (int l = 0; l <= top; ++l) {
    bm[l] = (uint8_t*)calloc(sz[l] ? sz[l] : 1, 1);
    kept[l] = (uint8_t*)malloc(sz[l] ? sz[l] : 1);
    nkept[l] = 0;
  }
  uint8_t* payload = (uint8_t*)malloc(len ? len : 1);
  size_t npay = 0;
  for (size_t i = 0; i < items; ++i) {
    int nz = 0;
    for (int j = 0; j < w; ++j) nz |= in[i * w + j] != 0;
    if (nz) {
      bm[0][i / 8] |= (uint8_t)(1u << (i % 8));
      memcpy(payload + npay, in + i * w, (size_t)w);
      npay += (size_t)w;
    }
  }
  for (int l = 0; l < top; ++l) {
    uint8_t prev = 0;
    for (size_t i = 0; i < sz[l]; ++i) {
      if (bm[l][i] != prev) {
        bm[l + 1][i / 8] |= (uint8_t)(1u << (i % 8));
        kept[l][nkept[l]++] = bm[l][i];
      }
      prev = bm[l][i];
    }
  }
  size_t total = sz[top] + npay;
  for (int l = 0; l < top; ++l) total += nkept[l];
  if (total >= len) {
    memcpy(out, in, len);
    *passthrough = 1;
    total = len;
  } else {
    size_t pos = 0;
    memcpy(out + pos, bm[top], sz[top]);
    pos += sz[top];
    for (int l = top - 1; l >= 0; --l) {
      memcpy(out + pos, kept[l], nkept[l]);
      pos += nkept[l];
    }
    memcpy(out + pos, payload, npay);
    *passthrough = 0;
  }
  for (int l = 0; l <= top; ++l) {
    free(bm[l]);
    free(kept[l]);
  }
  free(payload);
  return total;
}

int lopc_ref_unrze(const uint8_t* in, size_t in_len, size_t len, int w,
                   uint8_t* out) {
  size_t items = len / (size_t)w;
  size_t sz[RZE_MAX_LEVELS];
  int top = rze_level_sizes(items, sz);
  size_t pos = 0;
  if (sz[top] > in_len) return LOPC_REF_E_FORMAT;
  uint8_t* cur = (uint8_t*)malloc(sz[top] ? sz[top] : 1);
  memcpy(cur, in, sz[top]);
  pos = sz[top];
  for (int l = top - 1; l >= 0; --l) {
    uint8_t* nxt = (uint8_t*)malloc(sz[l] ? sz[l] : 1);
    uint8_t prev = 0;
    for (size_t i = 0; i < sz[l]; ++i) {
      if ((cur[i / 8] >> (i % 8)) & 1) {
        if (pos >= in_len) {
          free(nxt);
          free(cur);
          return LOPC_REF_E_FORMAT;
        }
        prev = in[pos++];
      }
      nxt[i] = prev;
    }
    free(cur);
    cur = nxt;
  }
  for (size_t i = 0; i < items; ++i) {
    if ((cur[i / 8] >> (i % 8)) & 1) {
      if (pos + (size_t)w > in_len) {
        free(cur);
        return LOPC_REF_E_FORMAT;
      }
      memcpy(out + i * w, in + pos, (size_t)w);
      pos += (size_t)w;
    } else {
      memset(out + i * w, 0, (size_t)w);
    }
  }
  free(cur);
  return pos == in_len ? LOPC_REF_OK : LOPC_REF_E_FORMAT;
}

/* ------------------------------------------------------------------------ */
/* Container.  The paper compresses the bins with DIFFNB_k BIT_k RZE_1 and   */
/* the subbins with BIT_k RZE_k RZE_1 in independent 16 kB chunks; how the   */
/* chunks are laid out in a file is not described, so this layout is the    */
/* project's own:                                                           */
/*   header (64 B) | u32 record size per chunk | records                    */
/*   record = u8 bins flags | u8 subbin flags | u16 points | u32 bins bytes  */
/*            | u32 subbins bytes after RZE_k | u32 subbin bytes |          */
/*            bins part | subbins part | zero padding to a multiple of 4.   */
/* A chunk of n points is padded with zero words to m = 64*ceil(n/64) words  */
/* before BIT (the bins after DIFFNB).                                       */
/* ------------------------------------------------------------------------ */

static void put_u16(uint8_t* p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put_u32(uint8_t* p, uint32_t v) { for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i)); }
static void put_u64(uint8_t* p, uint64_t v) { for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i)); }
static uint16_t get_u16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t get_u32(const uint8_t* p) { uint32_t v = 0; for (int i = 0; i < 4; ++i) v |= (uint32_t)p[i] << (8 * i); return v; }
static uint64_t get_u64(const uint8_t* p) { uint64_t v = 0; for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i); return v; }
static void put_f64(uint8_t* p, double d) { uint64_t u; memcpy(&u, &d, 8); put_u64(p, u); }
static double get_f64(const uint8_t* p) { uint64_t u = get_u64(p); double d; memcpy(&d, &u, 8); return d; }

static int shape_points(int ndim, const int64_t* dims, size_t* n) {
  if ((ndim != 2 && ndim != 3) || !dims) return LOPC_REF_E_ARG;
  size_t t = 1;
  for (int i = 0; i < ndim; ++i) {
    if (dims[i] < 1 || dims[i] > ((int64_t)1 << 40)) return LOPC_REF_E_ARG;
    if (t > ((size_t)1 << 48) / (size_t)dims[i]) return LOPC_REF_E_ARG;
    t *= (size_t)dims[i];
  }
  *n = t;
  return LOPC_REF_OK;
}

int lopc_ref_compress_bound(int dtype, int ndim, const int64_t* dims,
                            size_t* bytes) {
  if ((dtype != 0 && dtype != 1) || !bytes) return LOPC_REF_E_ARG;
  size_t n;
  int st = shape_points(ndim, dims, &n);
  if (st) return st;
  size_t k = dtype == 0 ? 4 : 8, W = CHUNK_BYTES / k;
  size_t nch = (n + W - 1) / W, total = HEADER_BYTES + 4 * nch;
  for (size_t c = 0; c < nch; ++c) {
    size_t nc = (c + 1) * W <= n ? W : n - c * W;
    size_t m = (nc + 63) / 64 * 64;
    total += RECORD_HEADER_BYTES + 2 * m * k;
  }
  *bytes = total;
  return LOPC_REF_OK;
}

/* Encode one chunk of nc points into rec; returns the record size. */
static size_t encode_chunk(const int64_t* bins, const uint64_t* sub, size_t nc,
                           int k, uint8_t* rec) {
  size_t m = (nc + 63) / 64 * 64;
  int64_t* w = (int64_t*)calloc(m, sizeof(int64_t));
  uint8_t* a = (uint8_t*)calloc(m * k, 1);
  uint8_t* b = (uint8_t*)calloc(m * k, 1);
  uint8_t* c = (uint8_t*)calloc(m * k, 1);
  uint8_t bflags = 0, sflags = 0;
  int pt;

  /* bins: DIFFNB_k, zero words up to m, BIT_k, RZE_1 */
  memcpy(w, bins, nc * sizeof(int64_t));
  lopc_ref_diffnb(w, nc, k);
  for (size_t i = 0; i < m; ++i) put_word(a, i, k, (uint64_t)w[i]);
  lopc_ref_bit(a, m, k, b);
  uint8_t* out = rec + RECORD_HEADER_BYTES;
  size_t blen = lopc_ref_rze(b, m * k, 1, out, &pt);
  if (pt) bflags |= 1;
  out += blen;

  /* subbins: zero words up to m, BIT_k, RZE_k, RZE_1 */
  memset(a, 0, m * k);
  for (size_t i = 0; i < nc; ++i) put_word(a, i, k, sub[i]);
  lopc_ref_bit(a, m, k, b);
  size_t smid = lopc_ref_rze(b, m * k, k, c, &pt);
  if (pt) sflags |= 1;
  size_t slen = lopc_ref_rze(c, smid, 1, out, &pt);
  if (pt) sflags |= 2;

  rec[0] = bflags;
  rec[1] = sflags;
  put_u16(rec + 2, (uint16_t)nc);
  put_u32(rec + 4, (uint32_t)blen);
  put_u32(rec + 8, (uint32_t)smid);
  put_u32(rec + 12, (uint32_t)slen);
  size_t size = RECORD_HEADER_BYTES + blen + slen;
  while (size % 4) rec[size++] = 0;
  free(w);
  free(a);
  free(b);
  free(c);
  return size;
}

int lopc_ref_compress(const void* field, int dtype, int ndim,
                      const int64_t* dims, double eb, int mode, void* outv,
                      size_t cap, size_t* out_size) {
  if (!field || !out_size || (dtype != 0 && dtype != 1)) return LOPC_REF_E_ARG;
  if (mode != 0 && mode != 1) return LOPC_REF_E_ARG;
  size_t n;
  int st = shape_points(ndim, dims, &n);
  if (st) return st;
  double eps, inv;
  st = lopc_ref_error_params(field, dtype, n, eb, mode, &eps, &inv);
  if (st) return st;
  int64_t* bins = (int64_t*)malloc(n * sizeof(int64_t));
  uint64_t* sub = (uint64_t*)malloc(n * sizeof(uint64_t));
  if (!bins || !sub) {
    free(bins);
    free(sub);
    return LOPC_REF_E_NOMEM;
  }
  st = lopc_ref_bins(field, dtype, n, inv, bins);
  if (!st) st = lopc_ref_subbins(field, dtype, ndim, dims, bins, sub);
  if (st) {
    free(bins);
    free(sub);
    return st;
  }
  size_t k = dtype == 0 ? 4 : 8, W = CHUNK_BYTES / k;
  size_t nch = (n + W - 1) / W;
  size_t bound;
  lopc_ref_compress_bound(dtype, ndim, dims, &bound);
  uint8_t* s = (uint8_t*)calloc(bound, 1);
  if (!s) {
    free(bins);
    free(sub);
    return LOPC_REF_E_NOMEM;
  }
  put_u32(s + 0, MAGIC);
  put_u16(s + 4, VERSION);
  s[6] = (uint8_t)dtype;
  s[7] = (uint8_t)ndim;
  for (int i = 0; i < 3; ++i)
    put_u64(s + 8 + 8 * i, (uint64_t)(i < ndim ? dims[i] : 1));
  s[32] = (uint8_t)mode;
  put_u32(s + 36, CHUNK_BYTES);
  put_f64(s + 40, eb);
  put_f64(s + 48, eps);
  put_f64(s + 56, inv);
  size_t pos = HEADER_BYTES + 4 * nch;
  for (size_t c = 0; c < nch; ++c) {
    size_t nc = (c + 1) * W <= n ? W : n - c * W;
    size_t r = encode_chunk(bins + c * W, sub + c * W, nc, (int)k, s + pos);
    put_u32(s + HEADER_BYTES + 4 * c, (uint32_t)r);
    pos += r;
  }
  free(bins);
  free(sub);
  *out_size = pos;
  if (pos > cap || !outv) {
    free(s);
    return LOPC_REF_E_CAPACITY;
  }
  memcpy(outv, s, pos);
  free(s);
  return LOPC_REF_OK;
}

int lopc_ref_stream_info(const void* sv, size_t size, int* dtype, int* ndim,
                         int64_t* dims, double* eps, double* inv) {
  const uint8_t* s = (const uint8_t*)sv;
  if (!s || size < HEADER_BYTES) return LOPC_REF_E_FORMAT;
  if (get_u32(s) != MAGIC || get_u16(s + 4) != VERSION) return LOPC_REF_E_FORMAT;
  int dt = s[6], nd = s[7];
  if ((dt != 0 && dt != 1) || (nd != 2 && nd != 3)) return LOPC_REF_E_FORMAT;
  if (s[32] > 1 || get_u32(s + 36) != CHUNK_BYTES) return LOPC_REF_E_FORMAT;
  int64_t d[3];
  for (int i = 0; i < 3; ++i) d[i] = (int64_t)get_u64(s + 8 + 8 * i);
  if (nd == 2 && d[2] != 1) return LOPC_REF_E_FORMAT;
  size_t n;
  if (shape_points(nd, d, &n)) return LOPC_REF_E_FORMAT;
  double e = get_f64(s + 48), v = get_f64(s + 56);
  if (!isfinite(e) || !(e > 0) || !isfinite(v) || !(v > 0))
    return LOPC_REF_E_FORMAT;
  /* inv must be the smallest binary64 with inv * eps >= 1 */
  if (!product_at_least_one(v, e) || product_at_least_one(nextafter(v, 0.0), e))
    return LOPC_REF_E_FORMAT;
  if (dtype) *dtype = dt;
  if (ndim) *ndim = nd;
  if (dims)
    for (int i = 0; i < 3; ++i) dims[i] = d[i];
  if (eps) *eps = e;
  if (inv) *inv = v;
  return LOPC_REF_OK;
}

/* Decode one record into bins and subbins of nc points. */
static int decode_chunk(const uint8_t* rec, size_t rsize, size_t nc, int k,
                        int64_t* bins, uint64_t* sub) {
  if (rsize < RECORD_HEADER_BYTES || rsize % 4) return LOPC_REF_E_FORMAT;
  size_t m = (nc + 63) / 64 * 64, L = m * k;
  uint8_t bfl = rec[0], sfl = rec[1];
  size_t blen = get_u32(rec + 4), smid = get_u32(rec + 8), slen = get_u32(rec + 12);
  if ((bfl & ~1u) || (sfl & ~3u) || get_u16(rec + 2) != nc) return LOPC_REF_E_FORMAT;
  if (blen > L || smid > L || slen > L) return LOPC_REF_E_FORMAT;
  size_t used = RECORD_HEADER_BYTES + blen + slen;
  if ((used + 3) / 4 * 4 != rsize) return LOPC_REF_E_FORMAT;
  for (size_t i = used; i < rsize; ++i)
    if (rec[i]) return LOPC_REF_E_FORMAT;
  const uint8_t* bp = rec + RECORD_HEADER_BYTES;
  const uint8_t* sp = bp + blen;
  uint8_t* a = (uint8_t*)malloc(L);
  uint8_t* b = (uint8_t*)malloc(L);
  int64_t* w = (int64_t*)malloc(m * sizeof(int64_t));
  int st = LOPC_REF_OK;

  /* bins */
  if (bfl & 1) {
    if (blen != L) st = LOPC_REF_E_FORMAT;
    else memcpy(a, bp, L);
  } else {
    st = lopc_ref_unrze(bp, blen, L, 1, a);
  }
  if (!st) {
    lopc_ref_unbit(a, m, k, b);
    for (size_t i = 0; i < m; ++i) w[i] = (int64_t)get_word(b, i, k);
    lopc_ref_undiffnb(w, nc, k);
    for (size_t i = 0; i < nc; ++i) bins[i] = w[i];
  }
  /* subbins */
  if (!st) {
    if (sfl & 2) {
      if (slen != smid) st = LOPC_REF_E_FORMAT;
      else memcpy(b, sp, smid);
    } else {
      st = lopc_ref_unrze(sp, slen, smid, 1, b);
    }
  }
  if (!st) {
    if (sfl & 1) {
      if (smid != L) st = LOPC_REF_E_FORMAT;
      else memcpy(a, b, L);
    } else {
      st = lopc_ref_unrze(b, smid, L, k, a);
    }
  }
  if (!st) {
    lopc_ref_unbit(a, m, k, b);
    for (size_t i = 0; i < nc; ++i) sub[i] = get_word(b, i, k);
  }
  free(a);
  free(b);
  free(w);
  return st;
}

static int walk_stream(const uint8_t* s, size_t size, int64_t* bins,
                       uint64_t* sub, void* field, size_t cap) {
  int dt, nd;
  int64_t d[3];
  double eps, inv;
  int st = lopc_ref_stream_info(s, size, &dt, &nd, d, &eps, &inv);
  if (st) return st;
  size_t n = (size_t)d[0] * (size_t)d[1] * (size_t)d[2];
  size_t k = dt == 0 ? 4 : 8, W = CHUNK_BYTES / k;
  size_t nch = (n + W - 1) / W;
  if (field && cap < n * k) return LOPC_REF_E_CAPACITY;
  if (size < HEADER_BYTES + 4 * nch) return LOPC_REF_E_FORMAT;
  size_t pos = HEADER_BYTES + 4 * nch;
  int64_t cb[CHUNK_BYTES / 4];
  uint64_t cs[CHUNK_BYTES / 4];
  for (size_t c = 0; c < nch; ++c) {
    size_t r = get_u32(s + HEADER_BYTES + 4 * c);
    if (r > size - pos) return LOPC_REF_E_FORMAT;
    size_t nc = (c + 1) * W <= n ? W : n - c * W;
    st = decode_chunk(s + pos, r, nc, (int)k, cb, cs);
    if (st) return st;
    for (size_t i = 0; i < nc; ++i) {
      size_t p = c * W + i;
      if (bins) bins[p] = cb[i];
      if (sub) sub[p] = cs[i];
      if (field) {
        double v;
        st = lopc_ref_reconstruct(cb[i], cs[i], inv, dt, &v);
        if (st) return st;
        if (dt == 0) ((float*)field)[p] = (float)v;
        else ((double*)field)[p] = v;
      }
    }
    pos += r;
  }
  return pos == size ? LOPC_REF_OK : LOPC_REF_E_FORMAT;
}

int lopc_ref_decompress(const void* stream, size_t size, void* field,
                        size_t cap) {
  if (!stream || !field) return LOPC_REF_E_ARG;
  return walk_stream((const uint8_t*)stream, size, NULL, NULL, field, cap);
}

int lopc_ref_decode_codes(const void* stream, size_t size, int64_t* bins,
                          uint64_t* subbins) {
  if (!stream || !bins || !subbins) return LOPC_REF_E_ARG;
  return walk_stream((const uint8_t*)stream, size, bins, subbins, NULL, 0);
}
