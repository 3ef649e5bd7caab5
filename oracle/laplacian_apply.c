/*
 * Oracle (test infrastructure only): plain FP64 application of the normalized
 * graph Laplacian A = I - D^{-1/2} S D^{-1/2} (Eq. 1) to a dense block.
 *
 * S is binary (Eq. 1: S_ij = 1 iff nodes i and j are connected), stored as a
 * canonical CSR pattern (row_ptr, col) with no values; dinv[i] = 1/sqrt(deg_i)
 * (0 for an isolated node).  For every row i and column c:
 *
 *     Y[i,c] = X[i,c] - dinv[i] * sum_{j in row i, ascending} dinv[j] * X[j,c]
 *
 * X and Y are addressed with explicit row and column strides (in elements) so
 * that both row-major and column-major NumPy arrays can be passed.  Rows are
 * shared among OpenMP threads; each row's sums are taken in ascending neighbour
 * order, so the result does not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_apply_laplacian(int64_t n, const int64_t *row_ptr, const int32_t *col,
                           const double *dinv, const double *X, int64_t xrs, int64_t xcs,
                           double *Y, int64_t yrs, int64_t ycs, int64_t w)
{
    int failed = 0;
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)(w > 0 ? w : 1));
        if (!s) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            if (!s)
                continue;
            for (int64_t c = 0; c < w; ++c)
                s[c] = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                const int64_t j = col[p];
                const double dj = dinv[j];
                const double *xj = X + j * xrs;
                for (int64_t c = 0; c < w; ++c)
                    s[c] += dj * xj[c * xcs];
            }
            for (int64_t c = 0; c < w; ++c)
                Y[i * yrs + c * ycs] = X[i * xrs + c * xcs] - dinv[i] * s[c];
        }
        free(s);
    }
    return failed ? -1 : 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
