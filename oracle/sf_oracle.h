/*
 * sf_oracle.h -- plain CPU definitions of the star-forest (SF) communication
 * operations, used ONLY as test infrastructure (pytest, the package smoke
 * check and the CPU baseline leg of the benchmark).  The product path never
 * links, loads or calls this code, and this code shares nothing with it: its
 * own enums, its own header, its own loops.
 *
 * Notation follows the paper ("The PetscSF Scalable Communication Layer"):
 *   leaf i in [0, nleaves) lives at slot l_i = ilocal[i] (or i when ilocal is
 *   NULL) and is connected to root r_i = iroot[i] in [0, nroots)
 *   (Section 3.1, PetscSFSetGraph).  L_r = { i : r_i = r } in ascending i.
 *   Data are arrays of units; a unit is bs contiguous elements of one
 *   type (Section 3.2: the unit argument is the type of a vertex's data).
 *
 * Arithmetic is carried out in the unit's own type, since the unit (an MPI
 * datatype in the paper) fixes the precision of MPI_SUM and friends.  Build
 * with -O2 -fno-fast-math -ffp-contract=off so every floating-point operation
 * happens exactly as written (no contraction to FMA, no reassociation).
 *
 * Every function returns 0 on success and -1 on an invalid argument.
 */
#ifndef SF_ORACLE_H
#define SF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types.  ORC_PAIR is the MAXLOC / MINLOC pair {double v; int32 i; int32 pad}
 * with a 16-byte extent; pad is never read or written.  ORC_F16 (IEEE
 * binary16) and ORC_BF16 (bfloat16: binary32's sign and exponent with 7
 * fraction bits) are stored as their 16-bit patterns; every SUM, PROD of
 * them is the exact result rounded once to the format (nearest, ties to
 * even, overflow to infinity), MAX / MIN pick an operand. */
enum { ORC_F64 = 0, ORC_F32 = 1, ORC_I32 = 2, ORC_I64 = 3, ORC_PAIR = 4, ORC_F16 = 5, ORC_BF16 = 6 };

/* Operations (MPI_Op analogues, Section 3.2). */
enum { ORC_REPLACE = 0, ORC_SUM = 1, ORC_MAX = 2, ORC_MIN = 3, ORC_MAXLOC = 4, ORC_MINLOC = 5, ORC_PROD = 6 };

/* Forms of the canonical pairwise sum (see orc_pairwise_*). */
enum { ORC_PW_TOPDOWN = 0, ORC_PW_BOTTOMUP = 1 };

/* SFBcast (Section 3.2, item 1): for every leaf i,
 *   leaf[l_i] = root[r_i]                 (op == REPLACE)
 *   leaf[l_i] = op(leaf[l_i], root[r_i])  (SUM / MAX / MIN / MAXLOC)
 * Slots that are not any l_i are left untouched (holes, Section 3.1). */
int orc_bcast(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
              int dtype, int bs, int op, const void *rootdata, void *leafdata);

/* SFReduce (Section 3.2, item 1, leaves to roots): for every root r with a
 * non-empty L_r, combine the root's value with the values of its leaves:
 *   FP SUM : root[r] = root[r] + PW(leaf[l_i] : i in L_r)  (pairwise, leaf order)
 *   int SUM: two's-complement wrap-around
 *   MAX/MIN: total order with -0 < +0 (NaN never occurs in the inputs)
 *   MAXLOC : larger value wins, equal values -> smaller index wins
 *   MINLOC : smaller value wins, equal values -> smaller index wins
 *   FP PROD: root[r] = root[r] * PWprod(leaf[l_i] : i in L_r) (the same tree
 *            as the sum, with products); int PROD: wrap-around
 *   REPLACE: the last leaf of L_r wins
 * Roots with an empty L_r are left untouched.  pw_form selects which of the
 * two equivalent formulations of PW is used (they must agree bitwise; PROD
 * always uses the top-down form). */
int orc_reduce(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
               int dtype, int bs, int op, const void *leafdata, void *rootdata, int pw_form);

/* SFFetchAndOp (Section 3.2, item 2): for i = 0, 1, ..., nleaves-1 in turn,
 *   leafupdate[l_i] = root[r_i];  root[r_i] = op(root[r_i], leaf[l_i]).
 * op is SUM, MAX or MIN; dtype is not ORC_PAIR. */
int orc_fetch_and_op(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot,
                     int dtype, int bs, int op, void *rootdata, const void *leafdata, void *leafupdate);

/* The multi-SF of Section 3.2, item 2: mroot[i] = the new root of leaf i,
 * from a fetch-and-add in leaf order with roots starting at the exclusive
 * prefix of the degrees and leaves adding 1.  There are nleaves new roots. */
int orc_multi_sf(int64_t nroots, int64_t nleaves, const int64_t *ilocal, const int64_t *iroot, int64_t *mroot);

/* SFGather: multiroot[mroot[i]] = leaf[l_i]; SFScatter: leaf[l_i] =
 * multiroot[mroot[i]] (whole units, any dtype; pad bytes of pairs move too). */
int orc_gather(int64_t nleaves, const int64_t *ilocal, const int64_t *mroot, int dtype, int bs,
               const void *leafdata, void *multirootdata);
int orc_scatter(int64_t nleaves, const int64_t *ilocal, const int64_t *mroot, int dtype, int bs,
                const void *multirootdata, void *leafdata);

/* Sparse products of Section 4.1 (CSR, f64): y = A x and y = A^T x, plus y
 * when accumulate; sums in stored order (see sf_oracle.c). */
int orc_csr_spmv(int64_t nrows, const int64_t *rowptr, const int32_t *colidx, const double *a, const double *x,
                 double *y, int accumulate);
int orc_csr_spmv_t(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx, const double *a,
                   const double *x, double *y, int accumulate);

/* Canonical pairwise sum PW of x[0..n), n >= 1:
 *   PW(x) = x[0] if n == 1, else PW(x[0..m)) + PW(x[m..n)),
 *   m = the largest power of two strictly below n          (ORC_PW_TOPDOWN)
 * or, equivalently, repeated levels that add neighbours (2j, 2j+1) with an
 * unpaired last element passed up unchanged                 (ORC_PW_BOTTOMUP). */
/* Round x to binary16 / bfloat16 (round to nearest, ties to even) and
 * return the 16-bit pattern; decode a pattern.  Exposed for the pins. */
uint16_t orc_to_f16(double x);
uint16_t orc_to_bf16(double x);
double orc_from_f16(uint16_t h);
double orc_from_bf16(uint16_t h);

double orc_pairwise_f64(const double *x, int64_t n, int form);
float orc_pairwise_f32(const float *x, int64_t n, int form);

#ifdef __cplusplus
}
#endif
#endif
