/*
 * FISTA (section 8.1; Beck & Teboulle's FISTA, the paper's reference
 * [fista]) in plain C, FP64, with the two sparse products split over host
 * threads (OpenMP).  The same iteration as oracle/fista.py, written out in C
 * so that the CPU baseline can use every host core:
 *
 *   x_0 = x0, y_1 = x_0, t_1 = 1; for k = 1, 2, ...:
 *     r       = A y_k - b
 *     x_k     = soft(y_k - A^T r / L, tau / L)
 *     t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
 *     y_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1})
 *
 * with soft(z, t) = sign(z) max(|z| - t, 0), the exact minimiser of the
 * separable model of eq. (4) with H = L I (section 2).  A is given as CSR
 * and A^T as the CSR of the transpose (rows of A^T = columns of A); every
 * row sum adds its products in index order and each thread owns whole rows,
 * so the result does not depend on the thread count.  Compile with
 * -ffp-contract=off: the products and sums are then rounded exactly as
 * numpy / scipy round them.
 *
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the bench's CPU
 * baseline call it; the HIP library does not.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static void csr_mv(int64_t rows, const int64_t* rp, const int32_t* ci, const double* v, const double* x,
                   const double* sub, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i) {
        double acc = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc += v[k] * x[ci[k]];
        out[i] = sub ? acc - sub[i] : acc;
    }
}

/* Returns 0, or -1 when memory runs out.  x_io holds x0 on entry and x_iters
 * on exit. */
int oracle_fista_csr(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                     const int64_t* tp, const int32_t* ti, const double* tv, const double* b, double tau,
                     double L, int64_t iters, double* x_io, int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    double* x = x_io;
    double* y = malloc((size_t)n * sizeof(double));
    double* xn = malloc((size_t)n * sizeof(double));
    double* g = malloc((size_t)n * sizeof(double));
    double* r = malloc((size_t)m * sizeof(double));
    if (!y || !xn || !g || !r) {
        free(y);
        free(xn);
        free(g);
        free(r);
        return -1;
    }
    memcpy(y, x, (size_t)n * sizeof(double));
    const double thr = tau / L;
    double t = 1.0;
    for (int64_t it = 0; it < iters; ++it) {
        csr_mv(m, rp, ci, v, y, b, r);
        csr_mv(n, tp, ti, tv, r, NULL, g);
        const double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        const double beta = (t - 1.0) / tn;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            const double z = y[j] - g[j] / L;
            const double az = fabs(z) - thr;
            const double xj = az > 0.0 ? (z > 0.0 ? az : -az) : 0.0;
            xn[j] = xj;
            y[j] = xj + beta * (xj - x[j]);
            x[j] = xj;
        }
        t = tn;
    }
    free(y);
    free(xn);
    free(g);
    free(r);
    return 0;
}

/* Threads an OpenMP region would use. */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
