/*
 * Oracle core: plain FP64 loops for the two operations of the filtered
 * Lanczos procedure that touch the sparse matrix.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU oracle that checks
 * the GPU library; the library never links, loads or calls it.
 *
 * Blocks are row-major n x r (row i's r entries contiguous).  The matrix is
 * CSR with zero-based int32 indices (full symmetric storage, Section 3.2.1).
 * Every loop is the textbook definition; OpenMP only splits rows.
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Y = A X : the sparse matrix times a block of r vectors. */
void oracle_csr_spmm(int32_t n, const int32_t *rowptr, const int32_t *colind,
                     const double *val, int32_t r, const double *X, double *Y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t c = 0; c < r; ++c) {
            double s = 0.0;
            for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                s += val[p] * X[(int64_t)colind[p] * r + c];
            Y[i * (int64_t)r + c] = s;
        }
    }
}

/*
 * Y = p(Ahat) X with p = sum_{k=0..m} b_k T_k and Ahat = (A - c I) / e
 * (Section 2.2, the affine map to [-1,1] and the truncated Chebyshev series).
 *
 * Evaluated by the FORWARD three-term recurrence of the Chebyshev
 * polynomials (Section 2.2): t_0 = x, t_1 = Ahat x,
 * t_{k+1} = 2 Ahat t_k - t_{k-1}, y = sum_k b_k t_k.
 * The GPU library evaluates the same polynomial by Clenshaw's backward
 * recurrence; using the other algorithm here keeps the two independent.
 *
 * work must hold 3 * n * r doubles.
 */
void oracle_cheb_forward(int32_t n, const int32_t *rowptr, const int32_t *colind,
                         const double *val, int32_t r, double c, double e,
                         int32_t m, const double *b, const double *X, double *Y,
                         double *work)
{
    int64_t len = (int64_t)n * r;
    double *t_prev = work, *t_cur = work + len, *t_next = work + 2 * len;

    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < len; ++q) {
        t_cur[q] = X[q];
        Y[q] = b[0] * X[q];
    }
    for (int32_t k = 1; k <= m; ++k) {
        /* t_next = Ahat t_cur (k = 1) or 2 Ahat t_cur - t_prev (k > 1) */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            for (int32_t cc = 0; cc < r; ++cc) {
                double s = 0.0;
                for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                    s += val[p] * t_cur[(int64_t)colind[p] * r + cc];
                double ahat = (s - c * t_cur[i * (int64_t)r + cc]) / e;
                double v = (k == 1) ? ahat : 2.0 * ahat - t_prev[i * (int64_t)r + cc];
                t_next[i * (int64_t)r + cc] = v;
                Y[i * (int64_t)r + cc] += b[k] * v;
            }
        }
        double *tmp = t_prev;
        t_prev = t_cur;
        t_cur = t_next;
        t_next = tmp;
    }
}

int oracle_num_threads(void)
{
    int t = 1;
    #pragma omp parallel
    {
        #pragma omp master
        {
#ifdef _OPENMP
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
