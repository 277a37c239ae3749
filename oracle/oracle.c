/*
 * oracle.c -- plain CPU FP64 reference for the tiled Cholesky hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP library against an
 * obviously correct, slow implementation.  It shares no code, header, table
 * or helper with the HIP library.
 *
 * What it computes (Methods, "Tiled Cholesky Decomposition"): for a symmetric
 * positive-definite A, the lower-triangular L with positive diagonal such
 * that A = L L^T.  The tiled right-looking algorithm of the paper (POTRF,
 * TRSM, SYRK, GEMM on tiles, Fig. 1) is a regrouping of the same scalar
 * operations, so in exact arithmetic it yields exactly this L.  The oracle is
 * therefore the plain unblocked definition, written in the right-looking
 * (outer-product) order that the tiled algorithm blocks.
 *
 * Conventions (the paper is silent on them; readings are listed in the
 * design notes):
 *   - storage is row-major, element (i,j) at a[i*lda + j], lda >= n;
 *   - only the lower triangle including the diagonal is read and written,
 *     in place; the strict upper triangle is never touched;
 *   - a pivot d <= 0 or NaN at column j stops the factorization with
 *     info = j + 1 (LAPACK potrf convention); columns < j then hold L;
 *   - all arithmetic is IEEE FP64, compiled with -ffp-contract=off so that
 *     no fused multiply-add changes the rounding sequence.
 *
 * Parallelism: OpenMP over independent rows inside one column step; every
 * element sees the identical, sequential subtraction sequence, so results
 * are bitwise independent of the thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stddef.h>

#define AT(p, i, j, ld) ((p)[(size_t)(i) * (size_t)(ld) + (size_t)(j)])

/*
 * Right-looking unblocked Cholesky (Methods: POTRF definition, applied with
 * tile size 1, which turns TRSM into a division and SYRK/GEMM into the rank-1
 * trailing update).
 *   for j: d = a_jj; l_jj = sqrt(d); l_ij = a_ij / l_jj (i > j);
 *          a_ik -= l_ij * l_kj for j < k <= i.
 * Returns 0; *info as described above.
 */
int oracle_potrf(double* a, int64_t n, int64_t lda, int64_t* info) {
  *info = 0;
  for (int64_t j = 0; j < n; ++j) {
    double d = AT(a, j, j, lda);
    if (!(d > 0.0)) { *info = j + 1; return 0; }
    double ljj = sqrt(d);
    AT(a, j, j, lda) = ljj;
    for (int64_t i = j + 1; i < n; ++i) AT(a, i, j, lda) = AT(a, i, j, lda) / ljj;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = j + 1; i < n; ++i) {
      const double lij = AT(a, i, j, lda);
      double* ai = &AT(a, i, 0, lda);
      for (int64_t k = j + 1; k <= i; ++k) ai[k] = ai[k] - lij * AT(a, k, j, lda);
    }
  }
  return 0;
}

/*
 * Row-oriented (Crout) form of the same factorization: every entry receives
 * the subtractions l_ik * l_jk for k = 0, 1, ..., j-1 in ascending k, which is
 * exactly the order the right-looking form applies them in, so both forms
 * are bitwise equal.  Used as an independent second reading of the
 * definition and for speed on large inputs (rows are independent within a
 * column).
 */
int oracle_potrf_crout(double* a, int64_t n, int64_t lda, int64_t* info) {
  *info = 0;
  for (int64_t j = 0; j < n; ++j) {
    const double* lj = &AT(a, j, 0, lda);
    double d = AT(a, j, j, lda);
    for (int64_t k = 0; k < j; ++k) d = d - lj[k] * lj[k];
    if (!(d > 0.0)) { *info = j + 1; return 0; }
    const double ljj = sqrt(d);
    AT(a, j, j, lda) = ljj;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < n; ++i) {
      double* li = &AT(a, i, 0, lda);
      double s = li[j];
      for (int64_t k = 0; k < j; ++k) s = s - li[k] * lj[k];
      li[j] = s / ljj;
    }
  }
  return 0;
}

/*
 * Solve A X = B with A = L L^T (the paper's motivating use: SPD systems via
 * the Cholesky factor).  Forward substitution L Y = B, then backward
 * substitution L^T X = Y, sequential in the summation index.  L is read from
 * the lower triangle of l (row-major, lda); B is n x nrhs row-major with
 * leading dimension ldb and is overwritten by X.  Columns of B are independent.
 */
void oracle_solve(const double* l, int64_t n, int64_t lda, double* b, int64_t nrhs, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nrhs; ++c) {
    for (int64_t i = 0; i < n; ++i) {
      double s = AT(b, i, c, ldb);
      for (int64_t k = 0; k < i; ++k) s = s - AT(l, i, k, lda) * AT(b, k, c, ldb);
      AT(b, i, c, ldb) = s / AT(l, i, i, lda);
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = AT(b, i, c, ldb);
      for (int64_t k = i + 1; k < n; ++k) s = s - AT(l, k, i, lda) * AT(b, k, c, ldb);
      AT(b, i, c, ldb) = s / AT(l, i, i, lda);
    }
  }
}

/* Number of OpenMP threads the two parallel loops above use. */
int oracle_num_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    t = omp_get_num_threads();
  }
  return t;
}
