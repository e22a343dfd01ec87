/*
 * sf_oracle_omp.c -- the oracle's definitions run on several host threads
 * (OpenMP), for the CPU baseline of the benchmark only: TEST INFRASTRUCTURE,
 * never linked, loaded or called by the product path.
 *
 * It includes the sequential oracle (sf_oracle.c) and adds variants whose
 * results are identical to it bit for bit, because every root still sees its
 * leaves in ascending leaf index:
 *   orc_bcast_omp        -- the leaves split among threads (each leaf writes
 *                           its own slot, Section 3.1: stars are disjoint);
 *   orc_reduce_omp       -- the roots split among threads, each root folding
 *                           its leaf list L_r (built once, in leaf order)
 *                           exactly as orc_reduce does;
 *   orc_fetch_and_op_omp -- the roots split among threads, each root taking
 *                           its leaves one by one in leaf order.
 * Build with -fopenmp -O2 -fno-fast-math -ffp-contract=off.
 */
#include "sf_oracle.c"

#include <omp.h>

int orc_omp_threads(void) { return omp_get_max_threads(); }

int orc_bcast_omp(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
                  int dtype, int bs, int op, const void *rootdata, void *leafdata) {
  if (check_graph(nroots, nleaves, ilocal, iroot, dtype, bs) || !op_valid(dtype, op)) return -1;
  int64_t es = elem_size(dtype), us = es * bs;
  const char *root = (const char *)rootdata;
  char *leaf = (char *)leafdata;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nleaves; i++) {
    int64_t slot = ilocal ? ilocal[i] : i;
    for (int c = 0; c < bs; c++)
      apply_op(dtype, op, leaf + slot * us + c * es, root + iroot[i] * us + c * es);
  }
  return 0;
}

int orc_reduce_omp(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
                   int dtype, int bs, int op, const void *leafdata, void *rootdata) {
  if (check_graph(nroots, nleaves, ilocal, iroot, dtype, bs) || !op_valid(dtype, op)) return -1;
  int64_t es = elem_size(dtype), us = es * bs;
  const char *leaf = (const char *)leafdata;
  char *root = (char *)rootdata;
  int64_t *start, *order;
  build_leaf_lists(nroots, nleaves, iroot, &start, &order);
  int64_t maxdeg = 0;
  for (int64_t r = 0; r < nroots; r++)
    if (start[r + 1] - start[r] > maxdeg) maxdeg = start[r + 1] - start[r];
#pragma omp parallel
  {
    void *tmp = malloc((size_t)(maxdeg > 0 ? maxdeg : 1) * 8);
#pragma omp for schedule(dynamic, 1024)
    for (int64_t r = 0; r < nroots; r++) {
      int64_t deg = start[r + 1] - start[r];
      if (deg == 0) continue;
      const int64_t *Lr = order + start[r];
      for (int c = 0; c < bs; c++) {
        char *dst = root + r * us + c * es;
        if (tree_op(dtype, op)) {
          for (int64_t k = 0; k < deg; k++) {
            int64_t slot = ilocal ? ilocal[Lr[k]] : Lr[k];
            memcpy((char *)tmp + k * es, leaf + slot * us + c * es, (size_t)es);
          }
          if (is_half(dtype)) {
            uint16_t t = pw_half(dtype, op, (const uint16_t *)tmp, deg);
            apply_op(dtype, op, dst, &t);
          } else if (dtype == ORC_F64) {
            double t = op == ORC_SUM ? orc_pairwise_f64((const double *)tmp, deg, ORC_PW_TOPDOWN)
                                     : pwprod_f64((const double *)tmp, deg);
            *(double *)dst = op == ORC_SUM ? *(double *)dst + t : *(double *)dst * t;
          } else {
            float t = op == ORC_SUM ? orc_pairwise_f32((const float *)tmp, deg, ORC_PW_TOPDOWN)
                                    : pwprod_f32((const float *)tmp, deg);
            *(float *)dst = op == ORC_SUM ? *(float *)dst + t : *(float *)dst * t;
          }
        } else {
          for (int64_t k = 0; k < deg; k++) {
            int64_t slot = ilocal ? ilocal[Lr[k]] : Lr[k];
            apply_op(dtype, op, dst, leaf + slot * us + c * es);
          }
        }
      }
    }
    free(tmp);
  }
  free(start);
  free(order);
  return 0;
}

int orc_fetch_and_op_omp(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
                         int dtype, int bs, int op, void *rootdata, const void *leafdata, void *leafupdate) {
  if (check_graph(nroots, nleaves, ilocal, iroot, dtype, bs)) return -1;
  if (dtype == ORC_PAIR || !(op == ORC_SUM || op == ORC_MAX || op == ORC_MIN)) return -1;
  int64_t es = elem_size(dtype), us = es * bs;
  char *root = (char *)rootdata;
  const char *leaf = (const char *)leafdata;
  char *upd = (char *)leafupdate;
  int64_t *start, *order;
  build_leaf_lists(nroots, nleaves, iroot, &start, &order);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < nroots; r++) {
    for (int64_t k = start[r]; k < start[r + 1]; k++) {
      int64_t i = order[k];
      int64_t slot = ilocal ? ilocal[i] : i;
      for (int c = 0; c < bs; c++) {
        char *rp = root + r * us + c * es;
        memcpy(upd + slot * us + c * es, rp, (size_t)es);
        apply_op(dtype, op, rp, leaf + slot * us + c * es);
      }
    }
  }
  free(start);
  free(order);
  return 0;
}
