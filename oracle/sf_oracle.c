/*
 * sf_oracle.c -- plain, slow, obviously correct CPU definitions of SFBcast,
 * SFReduce and SFFetchAndOp (paper Section 3.2).  TEST INFRASTRUCTURE ONLY:
 * used by the tests, the package smoke check and the benchmark's CPU
 * baseline, never by the product path.  See sf_oracle.h for the contract.
 *
 * Readings of points the paper leaves open (each is also listed with the
 * design notes of the project):
 *  - the root takes part in every Reduce as an operand (Section 4.1: the
 *    transpose product adds leaf contributions back onto y);
 *  - FP SUM order: canonical pairwise sum over the root's leaves in ascending
 *    leaf index, then root + T with the root as the left operand;
 *  - MAX/MIN compare under a total order in which -0 < +0;
 *  - MAXLOC: larger value wins, ties go to the smaller index (MPI rule);
 *  - Reduce REPLACE with several leaves: the last leaf in leaf order wins;
 *  - integer SUM wraps around (computed in unsigned arithmetic);
 *  - Bcast with op != REPLACE: leaf = op(leaf, root), leaf on the left.
 */
#include "sf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double v;
  int32_t i;
  int32_t pad;
} orc_pair;

/* ---------------------------------------------------------------- helpers */

static int64_t elem_size(int dtype) {
  switch (dtype) {
    case ORC_F64: return 8;
    case ORC_F32: return 4;
    case ORC_I32: return 4;
    case ORC_I64: return 8;
    case ORC_PAIR: return 16;
    case ORC_F16: return 2;
    case ORC_BF16: return 2;
    default: return -1;
  }
}

/* ------------------------------------------------ 16-bit binary formats */
/* A binary floating-point format with p significand bits (the leading one
 * included), w exponent bits and bias = 2^(w-1) - 1: normal numbers
 * (1.f) 2^E for E in [1 - bias, bias], subnormals f 2^(1 - bias - (p - 1)).
 * binary16: p 11, w 5; bfloat16: p 8, w 8 (IEEE 754-2008, Section 3). */
typedef struct {
  int p, w;
} orc_fmt;
static const orc_fmt FMT_F16 = {11, 5};
static const orc_fmt FMT_BF16 = {8, 8};

static double fmt_decode(orc_fmt f, uint16_t h) {
  const int bias = (1 << (f.w - 1)) - 1, fb = f.p - 1;
  const int ex = (h >> fb) & ((1 << f.w) - 1);
  const double m = (double)(h & ((1u << fb) - 1));
  double v;
  if (ex == 0)
    v = ldexp(m, 1 - bias - fb);
  else if (ex == (1 << f.w) - 1)
    v = m != 0 ? NAN : INFINITY;
  else
    v = ldexp(m + ldexp(1.0, fb), ex - bias - fb);
  return (h >> 15) & 1 ? -v : v;
}

/* The representable value nearest to x (ties to the even significand),
 * +-infinity when that exceeds the largest finite value: scale |x| so that
 * the format's last significand place is 1, round to an integer, scale back.
 * The quantum is 2^(E - (p - 1)) for |x| in [2^E, 2^(E+1)), never below the
 * subnormal quantum. */
static double fmt_round(orc_fmt f, double x) {
  const int bias = (1 << (f.w - 1)) - 1, fb = f.p - 1;
  if (x == 0 || isnan(x) || isinf(x)) return x;
  int e;
  (void)frexp(fabs(x), &e); /* |x| in [2^(e-1), 2^e) */
  int q = (e - 1) - fb;
  if (q < 1 - bias - fb) q = 1 - bias - fb;
  const double r = nearbyint(ldexp(fabs(x), -q)); /* exact scaling; default mode: ties to even */
  double v = ldexp(r, q);
  if (v >= ldexp(1.0, bias + 1)) v = INFINITY;
  return signbit(x) ? -v : v;
}

static uint16_t fmt_encode(orc_fmt f, double x) {
  const int bias = (1 << (f.w - 1)) - 1, fb = f.p - 1;
  const double v = fmt_round(f, x);
  const uint16_t sign = signbit(v) ? 0x8000 : 0;
  const double a = fabs(v);
  if (isnan(v)) return (uint16_t)(((1u << f.w) - 1) << fb | 1u << (fb - 1));
  if (isinf(v)) return (uint16_t)(sign | ((1u << f.w) - 1) << fb);
  if (a < ldexp(1.0, 1 - bias)) return (uint16_t)(sign | (uint16_t)ldexp(a, bias - 1 + fb)); /* subnormal or 0 */
  int e;
  (void)frexp(a, &e);
  const int E = e - 1;
  const uint32_t mant = (uint32_t)(ldexp(a, -E) * ldexp(1.0, fb)) - (1u << fb);
  return (uint16_t)(sign | (uint32_t)(E + bias) << fb | mant);
}

uint16_t orc_to_f16(double x) { return fmt_encode(FMT_F16, x); }
uint16_t orc_to_bf16(double x) { return fmt_encode(FMT_BF16, x); }
double orc_from_f16(uint16_t h) { return fmt_decode(FMT_F16, h); }
double orc_from_bf16(uint16_t h) { return fmt_decode(FMT_BF16, h); }

static int is_half(int dtype) { return dtype == ORC_F16 || dtype == ORC_BF16; }
static orc_fmt half_fmt(int dtype) { return dtype == ORC_F16 ? FMT_F16 : FMT_BF16; }

/* Total order on doubles with -0 < +0 (no NaN in the inputs). */
static int less_f64(double a, double b) {
  if (a < b) return 1;
  if (a > b) return 0;
  return signbit(a) && !signbit(b);
}
static int less_f32(float a, float b) {
  if (a < b) return 1;
  if (a > b) return 0;
  return signbit(a) && !signbit(b);
}

/* MAXLOC: is a strictly better than b? */
static int pair_better(const orc_pair *a, const orc_pair *b) {
  if (less_f64(b->v, a->v)) return 1;
  if (less_f64(a->v, b->v)) return 0;
  return a->i < b->i;
}

/* MINLOC: is a strictly better than b (smaller value, then smaller index)? */
static int pair_better_min(const orc_pair *a, const orc_pair *b) {
  if (less_f64(a->v, b->v)) return 1;
  if (less_f64(b->v, a->v)) return 0;
  return a->i < b->i;
}

/* dst = op(dst, src) for one element; dst is the left operand. */
static void apply_op(int dtype, int op, void *dst, const void *src) {
  if (op == ORC_REPLACE) {
    if (dtype == ORC_PAIR) {
      ((orc_pair *)dst)->v = ((const orc_pair *)src)->v;
      ((orc_pair *)dst)->i = ((const orc_pair *)src)->i;
    } else {
      memcpy(dst, src, (size_t)elem_size(dtype));
    }
    return;
  }
  switch (dtype) {
    case ORC_F64: {
      double a = *(double *)dst, b = *(const double *)src;
      if (op == ORC_SUM) a = a + b;
      else if (op == ORC_PROD) a = a * b;
      else if (op == ORC_MAX) a = less_f64(a, b) ? b : a;
      else if (op == ORC_MIN) a = less_f64(b, a) ? b : a;
      *(double *)dst = a;
      break;
    }
    case ORC_F32: {
      float a = *(float *)dst, b = *(const float *)src;
      if (op == ORC_SUM) a = a + b;
      else if (op == ORC_PROD) a = a * b;
      else if (op == ORC_MAX) a = less_f32(a, b) ? b : a;
      else if (op == ORC_MIN) a = less_f32(b, a) ? b : a;
      *(float *)dst = a;
      break;
    }
    case ORC_I32: {
      int32_t a = *(int32_t *)dst, b = *(const int32_t *)src;
      if (op == ORC_SUM) a = (int32_t)((uint32_t)a + (uint32_t)b);
      else if (op == ORC_PROD) a = (int32_t)((uint32_t)a * (uint32_t)b);
      else if (op == ORC_MAX) a = a < b ? b : a;
      else if (op == ORC_MIN) a = b < a ? b : a;
      *(int32_t *)dst = a;
      break;
    }
    case ORC_I64: {
      int64_t a = *(int64_t *)dst, b = *(const int64_t *)src;
      if (op == ORC_SUM) a = (int64_t)((uint64_t)a + (uint64_t)b);
      else if (op == ORC_PROD) a = (int64_t)((uint64_t)a * (uint64_t)b);
      else if (op == ORC_MAX) a = a < b ? b : a;
      else if (op == ORC_MIN) a = b < a ? b : a;
      *(int64_t *)dst = a;
      break;
    }
    case ORC_F16:
    case ORC_BF16: {
      /* the exact sum / product (exact in binary64 for binary16; for
       * bfloat16 binary64's 53 bits >= 2 x 8 + 2 make the rounding through
       * binary64 equal to a single rounding) rounded once to the format */
      const orc_fmt f = half_fmt(dtype);
      const uint16_t ha = *(uint16_t *)dst, hb = *(const uint16_t *)src;
      const double a = fmt_decode(f, ha), b = fmt_decode(f, hb);
      uint16_t r = ha;
      if (op == ORC_SUM) r = fmt_encode(f, a + b);
      else if (op == ORC_PROD) r = fmt_encode(f, a * b);
      else if (op == ORC_MAX) r = less_f64(a, b) ? hb : ha;
      else if (op == ORC_MIN) r = less_f64(b, a) ? hb : ha;
      *(uint16_t *)dst = r;
      break;
    }
    case ORC_PAIR: {
      orc_pair *a = (orc_pair *)dst;
      const orc_pair *b = (const orc_pair *)src;
      if ((op == ORC_MAXLOC && pair_better(b, a)) || (op == ORC_MINLOC && pair_better_min(b, a))) {
        a->v = b->v;
        a->i = b->i;
      }
      break;
    }
  }
}

static int op_valid(int dtype, int op) {
  if (dtype == ORC_PAIR) return op == ORC_REPLACE || op == ORC_MAXLOC || op == ORC_MINLOC;
  return op == ORC_REPLACE || op == ORC_SUM || op == ORC_MAX || op == ORC_MIN || op == ORC_PROD;
}

static int check_graph(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
                       int dtype, int bs) {
  if (nroots < 0 || nleaves < 0 || bs < 1 || elem_size(dtype) < 0) return -1;
  if (nleaves > 0 && !iroot) return -1;
  for (int64_t i = 0; i < nleaves; i++) {
    if (iroot[i] < 0 || iroot[i] >= nroots) return -1;
    if (ilocal && ilocal[i] < 0) return -1;
  }
  return 0;
}

/* ---------------------------------------------------- canonical pairwise */

static int64_t largest_pow2_below(int64_t n) { /* n >= 2 */
  int64_t m = 1;
  while (m * 2 < n) m *= 2;
  return m;
}

static double pw_f64_topdown(const double *x, int64_t n) {
  if (n == 1) return x[0];
  int64_t m = largest_pow2_below(n);
  double a = pw_f64_topdown(x, m);
  double b = pw_f64_topdown(x + m, n - m);
  return a + b;
}
static float pw_f32_topdown(const float *x, int64_t n) {
  if (n == 1) return x[0];
  int64_t m = largest_pow2_below(n);
  float a = pw_f32_topdown(x, m);
  float b = pw_f32_topdown(x + m, n - m);
  return a + b;
}

static double pw_f64_bottomup(const double *x, int64_t n) {
  double *w = (double *)malloc((size_t)n * sizeof(double));
  memcpy(w, x, (size_t)n * sizeof(double));
  int64_t len = n;
  while (len > 1) {
    int64_t half = 0;
    for (int64_t j = 0; j + 1 < len; j += 2) w[half++] = w[j] + w[j + 1];
    if (len % 2) w[half++] = w[len - 1];
    len = half;
  }
  double s = w[0];
  free(w);
  return s;
}
static float pw_f32_bottomup(const float *x, int64_t n) {
  float *w = (float *)malloc((size_t)n * sizeof(float));
  memcpy(w, x, (size_t)n * sizeof(float));
  int64_t len = n;
  while (len > 1) {
    int64_t half = 0;
    for (int64_t j = 0; j + 1 < len; j += 2) w[half++] = w[j] + w[j + 1];
    if (len % 2) w[half++] = w[len - 1];
    len = half;
  }
  float s = w[0];
  free(w);
  return s;
}

/* The canonical pairwise tree with products instead of sums (top-down). */
static double pwprod_f64(const double *x, int64_t n) {
  if (n == 1) return x[0];
  int64_t m = largest_pow2_below(n);
  return pwprod_f64(x, m) * pwprod_f64(x + m, n - m);
}
static float pwprod_f32(const float *x, int64_t n) {
  if (n == 1) return x[0];
  int64_t m = largest_pow2_below(n);
  return pwprod_f32(x, m) * pwprod_f32(x + m, n - m);
}

/* The canonical pairwise tree (top-down) over n >= 1 elements of a 16-bit
 * format, every node combined by apply_op (rounded to the format). */
static uint16_t pw_half(int dtype, int op, const uint16_t *x, int64_t n) {
  if (n == 1) return x[0];
  int64_t m = largest_pow2_below(n);
  uint16_t a = pw_half(dtype, op, x, m);
  uint16_t b = pw_half(dtype, op, x + m, n - m);
  apply_op(dtype, op, &a, &b);
  return a;
}

double orc_pairwise_f64(const double *x, int64_t n, int form) {
  if (n < 1) return 0.0;
  return form == ORC_PW_BOTTOMUP ? pw_f64_bottomup(x, n) : pw_f64_topdown(x, n);
}
float orc_pairwise_f32(const float *x, int64_t n, int form) {
  if (n < 1) return 0.0f;
  return form == ORC_PW_BOTTOMUP ? pw_f32_bottomup(x, n) : pw_f32_topdown(x, n);
}

/* ------------------------------------------------------------------ Bcast */

int orc_bcast(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
              int dtype, int bs, int op, const void *rootdata, void *leafdata) {
  if (check_graph(nroots, nleaves, ilocal, iroot, dtype, bs) || !op_valid(dtype, op)) return -1;
  int64_t es = elem_size(dtype), us = es * bs;
  const char *root = (const char *)rootdata;
  char *leaf = (char *)leafdata;
  for (int64_t i = 0; i < nleaves; i++) {
    int64_t slot = ilocal ? ilocal[i] : i;
    for (int c = 0; c < bs; c++)
      apply_op(dtype, op, leaf + slot * us + c * es, root + iroot[i] * us + c * es);
  }
  return 0;
}

/* ----------------------------------------------------------------- Reduce */

/* Floating-point SUM and PROD go through the pairwise tree; every other op
 * folds in leaf order (its result does not depend on the order). */
static int tree_op(int dtype, int op) {
  return (op == ORC_SUM || op == ORC_PROD) && (dtype == ORC_F64 || dtype == ORC_F32 || is_half(dtype));
}

/* Leaf lists L_r in ascending leaf index, as a counting sort: start[r] is
 * the first position of root r in order[], order[] holds leaf indices. */
static void build_leaf_lists(int64_t nroots, int64_t nleaves, const int64_t *iroot,
                             int64_t **start_out, int64_t **order_out) {
  int64_t *start = (int64_t *)calloc((size_t)nroots + 1, sizeof(int64_t));
  int64_t *fill = (int64_t *)calloc((size_t)nroots + 1, sizeof(int64_t));
  int64_t *order = (int64_t *)malloc((size_t)(nleaves > 0 ? nleaves : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < nleaves; i++) start[iroot[i] + 1]++;
  for (int64_t r = 0; r < nroots; r++) start[r + 1] += start[r];
  for (int64_t r = 0; r < nroots; r++) fill[r] = start[r];
  for (int64_t i = 0; i < nleaves; i++) order[fill[iroot[i]]++] = i;
  free(fill);
  *start_out = start;
  *order_out = order;
}

int orc_reduce(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
               int dtype, int bs, int op, const void *leafdata, void *rootdata, int pw_form) {
  if (check_graph(nroots, nleaves, ilocal, iroot, dtype, bs) || !op_valid(dtype, op)) return -1;
  int64_t es = elem_size(dtype), us = es * bs;
  const char *leaf = (const char *)leafdata;
  char *root = (char *)rootdata;
  int64_t *start, *order;
  build_leaf_lists(nroots, nleaves, iroot, &start, &order);
  int64_t maxdeg = 0;
  for (int64_t r = 0; r < nroots; r++)
    if (start[r + 1] - start[r] > maxdeg) maxdeg = start[r + 1] - start[r];
  void *tmp = malloc((size_t)(maxdeg > 0 ? maxdeg : 1) * 8);

  for (int64_t r = 0; r < nroots; r++) {
    int64_t deg = start[r + 1] - start[r];
    if (deg == 0) continue;
    const int64_t *Lr = order + start[r];
    for (int c = 0; c < bs; c++) {
      char *dst = root + r * us + c * es;
      if (tree_op(dtype, op)) {
        /* root op PW(leaves in ascending leaf index) */
        for (int64_t k = 0; k < deg; k++) {
          int64_t slot = ilocal ? ilocal[Lr[k]] : Lr[k];
          memcpy((char *)tmp + k * es, leaf + slot * us + c * es, (size_t)es);
        }
        if (is_half(dtype)) {
          uint16_t t = pw_half(dtype, op, (const uint16_t *)tmp, deg);
          apply_op(dtype, op, dst, &t);
        } else if (dtype == ORC_F64) {
          if (op == ORC_SUM) {
            double t = orc_pairwise_f64((const double *)tmp, deg, pw_form);
            *(double *)dst = *(double *)dst + t;
          } else {
            double t = pwprod_f64((const double *)tmp, deg);
            *(double *)dst = *(double *)dst * t;
          }
        } else {
          if (op == ORC_SUM) {
            float t = orc_pairwise_f32((const float *)tmp, deg, pw_form);
            *(float *)dst = *(float *)dst + t;
          } else {
            float t = pwprod_f32((const float *)tmp, deg);
            *(float *)dst = *(float *)dst * t;
          }
        }
      } else {
        /* order-free ops (and REPLACE: the last leaf wins) folded in leaf order */
        for (int64_t k = 0; k < deg; k++) {
          int64_t slot = ilocal ? ilocal[Lr[k]] : Lr[k];
          apply_op(dtype, op, dst, leaf + slot * us + c * es);
        }
      }
    }
  }
  free(tmp);
  free(start);
  free(order);
  return 0;
}

/* ------------------------------------------------------------ FetchAndOp */

int orc_fetch_and_op(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
                     int dtype, int bs, int op, void *rootdata, const void *leafdata, void *leafupdate) {
  if (check_graph(nroots, nleaves, ilocal, iroot, dtype, bs)) return -1;
  if (dtype == ORC_PAIR || is_half(dtype) || !(op == ORC_SUM || op == ORC_MAX || op == ORC_MIN)) return -1;
  int64_t es = elem_size(dtype), us = es * bs;
  char *root = (char *)rootdata;
  const char *leaf = (const char *)leafdata;
  char *upd = (char *)leafupdate;
  for (int64_t i = 0; i < nleaves; i++) {
    int64_t slot = ilocal ? ilocal[i] : i;
    for (int c = 0; c < bs; c++) {
      char *r = root + iroot[i] * us + c * es;
      memcpy(upd + slot * us + c * es, r, (size_t)es);
      apply_op(dtype, op, r, leaf + slot * us + c * es);
    }
  }
  return 0;
}

/* ------------------------------------------------ multi-SF, Gather, Scatter */

/* The multi-SF of Section 3.2, item 2, built as the paper describes: every
 * root r is split into deg(r) new roots placed at its old offset, the
 * exclusive prefix of the degrees (the degrees being the Reduce SUM of ones),
 * and a fetch-and-add in leaf order with the roots starting at their offset
 * and every leaf adding 1 hands leaf i its new root mroot[i]. */
int orc_multi_sf(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot, int64_t *mroot) {
  if (check_graph(nroots, nleaves, ilocal, iroot, ORC_I64, 1) || (nleaves > 0 && !mroot)) return -1;
  int64_t *deg = (int64_t *)calloc((size_t)(nroots > 0 ? nroots : 1), sizeof(int64_t));
  int64_t *off = (int64_t *)malloc((size_t)(nroots > 0 ? nroots : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < nleaves; i++) deg[iroot[i]] += 1;
  int64_t acc = 0;
  for (int64_t r = 0; r < nroots; r++) {
    off[r] = acc;
    acc += deg[r];
  }
  for (int64_t i = 0; i < nleaves; i++) {  /* fetch, then add 1 */
    mroot[i] = off[iroot[i]];
    off[iroot[i]] += 1;
  }
  free(deg);
  free(off);
  return 0;
}

/* SFGather: multiroot[mroot[i]] = leaf[l_i] for every leaf i (whole units). */
int orc_gather(int64_t nleaves, const int64_t *ilocal, const int64_t *mroot, int dtype, int bs,
               const void *leafdata, void *multirootdata) {
  if (nleaves < 0 || bs < 1 || elem_size(dtype) == 0 || (nleaves > 0 && !mroot)) return -1;
  int64_t us = elem_size(dtype) * bs;
  for (int64_t i = 0; i < nleaves; i++) {
    int64_t slot = ilocal ? ilocal[i] : i;
    memcpy((char *)multirootdata + mroot[i] * us, (const char *)leafdata + slot * us, (size_t)us);
  }
  return 0;
}

/* SFScatter, the reverse: leaf[l_i] = multiroot[mroot[i]]; other slots untouched. */
int orc_scatter(int64_t nleaves, const int64_t *ilocal, const int64_t *mroot, int dtype, int bs,
                const void *multirootdata, void *leafdata) {
  if (nleaves < 0 || bs < 1 || elem_size(dtype) == 0 || (nleaves > 0 && !mroot)) return -1;
  int64_t us = elem_size(dtype) * bs;
  for (int64_t i = 0; i < nleaves; i++) {
    int64_t slot = ilocal ? ilocal[i] : i;
    memcpy((char *)leafdata + slot * us, (const char *)multirootdata + mroot[i] * us, (size_t)us);
  }
  return 0;
}

/* --------------------------------------------- sparse products (Section 4.1) */

/* y = A x (+ y when accumulate), A in CSR: row i's entries k in
 * [rowptr[i], rowptr[i+1]) in stored order, each a[k] * x[colidx[k]]
 * added to a running sum that starts at 0 (then added to y[i]). */
int orc_csr_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *colidx, const double *a, const double *x,
                 double *y, int accumulate) {
  if (nrows < 0 || !rowptr) return -1;
  for (int64_t i = 0; i < nrows; i++) {
    double s = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) s = s + a[k] * x[colidx[k]];
    y[i] = accumulate ? y[i] + s : s;
  }
  return 0;
}

/* y = A^T x (+ y when accumulate): every entry a[k] of row i adds
 * a[k] * x[i] to y[colidx[k]], rows and entries in stored order. */
int orc_csr_spmv_t(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx, const double *a,
                   const double *x, double *y, int accumulate) {
  if (nrows < 0 || ncols < 0 || !rowptr) return -1;
  if (!accumulate)
    for (int64_t j = 0; j < ncols; j++) y[j] = 0.0;
  for (int64_t i = 0; i < nrows; i++)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) y[colidx[k]] = y[colidx[k]] + a[k] * x[i];
  return 0;
}
