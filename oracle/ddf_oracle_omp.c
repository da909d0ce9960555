/*
 * The oracle's plain FP64 loops spread over host cores with OpenMP.  TEST INFRASTRUCTURE ONLY:
 * the benchmark times them as the many-core CPU baseline; the tests pin them to the serial
 * oracle (ddf_oracle.c).
 *
 * Each loop is the serial oracle's, parallel over independent rows:
 *   - the product over rows of A (each row's sum in the serial order, so bitwise equal);
 *   - the adjoint product A^T G over rows of the transposed pattern (the same terms summed in
 *     row order of A^T, which the serial column-scatter also follows per entry of GX), and
 *     the value gradient over rows of A;
 *   - forward substitution over the rows of one dependence level at a time (each row's
 *     operations in the serial order, so bitwise equal);
 *   - the transposed solve L^T Lam = G over the rows of one reverse level of U = L^T at a time,
 *     each row of U summed in column order, then the value gradient over rows of L.
 * The level sets and the transposed pattern are inputs (computed once, outside the timing).
 * Compiled with -O2 -ffp-contract=off -fopenmp.
 */
#include <stdint.h>

/* Y = A X, rows in parallel. */
void omp_spmv(int32_t n_rows, const int32_t *rp, const int32_t *ci, const double *v, int32_t k,
              const double *X, double *Y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t r = 0; r < k; r++) {
            double acc = 0.0;
            for (int64_t e = rp[i]; e < rp[i + 1]; e++) acc += v[e] * X[(int64_t)ci[e] * k + r];
            Y[i * k + r] = acc;
        }
    }
}

/* GX = A^T G over the rows of the transposed pattern (rpT, ciT: rows of A; perm: value index
 * of each transposed entry); GV[e] = sum_r G[i,r] X[col_e,r] over the rows of A. */
void omp_spmv_adj(int32_t n_rows, int32_t n_cols, const int32_t *rp, const int32_t *ci, const double *v,
                  const int32_t *rpT, const int32_t *ciT, const int64_t *perm, int32_t k, const double *X,
                  const double *G, double *GX, double *GV) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cols; c++) {
        for (int64_t r = 0; r < k; r++) {
            double acc = 0.0;
            for (int64_t e = rpT[c]; e < rpT[c + 1]; e++) acc += v[perm[e]] * G[(int64_t)ciT[e] * k + r];
            GX[c * k + r] = acc;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            double s = 0.0;
            for (int64_t r = 0; r < k; r++) s += G[i * k + r] * X[(int64_t)ci[e] * k + r];
            GV[e] = s;
        }
    }
}

/* Forward substitution, level by level (lptr[nlev + 1] ranges of lrows). */
void omp_sptrsv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t k,
                const int64_t *lptr, const int64_t *lrows, int64_t nlev, const double *B, double *X) {
    (void)n;
    for (int64_t l = 0; l < nlev; l++) {
#pragma omp parallel for schedule(static)
        for (int64_t q = lptr[l]; q < lptr[l + 1]; q++) {
            const int64_t i = lrows[q], d = rp[i + 1] - 1;
            for (int64_t r = 0; r < k; r++) {
                double acc = B[i * k + r];
                for (int64_t e = rp[i]; e < d; e++) acc -= v[e] * X[(int64_t)ci[e] * k + r];
                X[i * k + r] = acc / v[d];
            }
        }
    }
}

/* L^T Lam = G on the rows of U = L^T (rpT, ciT, perm; diagonal first in each row), reverse
 * level by reverse level (ulptr ranges of ulrows), then GV[e] = -sum_r Lam[i,r] X[col_e,r]. */
void omp_sptrsv_adj(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *rpT,
                    const int32_t *ciT, const int64_t *perm, int32_t k, const int64_t *ulptr,
                    const int64_t *ulrows, int64_t nlev, const double *X, const double *G, double *GB,
                    double *GV) {
    for (int64_t l = 0; l < nlev; l++) {
#pragma omp parallel for schedule(static)
        for (int64_t q = ulptr[l]; q < ulptr[l + 1]; q++) {
            const int64_t i = ulrows[q], d = rpT[i];
            for (int64_t r = 0; r < k; r++) {
                double acc = G[i * k + r];
                for (int64_t e = d + 1; e < rpT[i + 1]; e++) acc -= v[perm[e]] * GB[(int64_t)ciT[e] * k + r];
                GB[i * k + r] = acc / v[perm[d]];
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            double s = 0.0;
            for (int64_t r = 0; r < k; r++) s += GB[i * k + r] * X[(int64_t)ci[e] * k + r];
            GV[e] = -s;
        }
    }
}

/* Threads the parallel loops above use. */
#include <omp.h>
int omp_threads(void) { return omp_get_max_threads(); }
