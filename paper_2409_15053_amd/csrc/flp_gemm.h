// Device bodies of the tall-skinny products of the full reorthogonalisation
// (Section 3.2.2), shared by the single-solve kernels and the segmented
// (many solves per launch) kernels of the batched block step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "flp_device.h"
#include "flp_internal.h"

namespace flp {
namespace {

// v_mfma_f64_16x16x4f64: D(16x16) = A(16x4) B(4x16) + C.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it holds D[l/16 + 4 v][l % 16]
// for v = 0..3 (rows interleaved across the four lane groups; checked on
// gfx950 with a one-hot probe).
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A pointer read from a descriptor in memory is a generic (flat) pointer to
// the compiler; recast into the global address space, a load through it that
// is uniform across the wave and not preceded by a store can go through the
// scalar cache.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
    return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global_mut(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Address of column q of a (possibly panelled) matrix; row i is at + i * ld.
__device__ __forceinline__ const double *col_base(const DMat &m, int q) {
    return m.p + (int64_t)(q >> m.lpw) * m.ps + (q & ((1 << m.lpw) - 1));
}

// C = beta C + alpha A B for one block of 4 waves: row block rblk (each wave
// MT row tiles of 16 rows) and column block cblk (NT tiles of 16 columns).
// The k index inside a group of 16 is permuted (k = 4 * (l/16) + step) so
// each lane reads 4 contiguous A entries with two 16-byte loads.  A group of
// 16 k values never straddles a panel.  Loads are unconditional: rows past n
// and columns past c are clamped (they only feed outputs that are not
// written) and B rows past K are zeroed.  A and C may be the same block
// (in-place C = A B): each wave reads all of its rows of A before it writes
// those rows of C.
template <int MT, int NT>
__device__ __forceinline__ void gemm_nn_rows(int n, int K, int c, double alpha, const DMat &A,
                                             const double *__restrict__ B, int64_t ldb, double beta, double *C,
                                             int64_t ldc, bool vec_a, int rblk, int cblk) {
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int row0 = (rblk * 4 + wave) * (16 * MT);
    if (row0 >= n) return;
    const int kq = lane / 16, m = lane % 16;
    dbl4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    int col[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) col[j] = min((cblk * NT + j) * 16 + m, c - 1);
    int64_t roff[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) roff[i] = (int64_t)min(row0 + i * 16 + m, n - 1) * A.ld;
    const int kfull = vec_a ? (K & ~15) : 0;
    int k0 = 0;
    for (; k0 < kfull; k0 += 16) {
        const int kb = k0 + 4 * kq;  // this lane's 4 contiguous k values
        const auto abase = as_global(col_base(A, kb));
        double a[MT][4];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const auto ap = abase + roff[i];
            const dbl2 x0 = *reinterpret_cast<gptr<dbl2>>(ap);
            const dbl2 x1 = *reinterpret_cast<gptr<dbl2>>(ap + 2);
            a[i][0] = x0.x;
            a[i][1] = x0.y;
            a[i][2] = x1.x;
            a[i][3] = x1.y;
        }
        double b[4][NT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < NT; ++j) b[q][j] = as_global(B)[(int64_t)(kb + q) * ldb + col[j]];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[i][j] = mfma16x16x4(a[i][q], b[q][j], acc[i][j]);
    }
    for (; k0 < K; k0 += 16) {  // ragged tail (or unaligned A): scalar loads
        const int kb = k0 + 4 * kq;
        double a[MT][4], b[4][NT];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = min(kb + q, K - 1);
            const auto ap = as_global(col_base(A, kk));
#pragma unroll
            for (int i = 0; i < MT; ++i) a[i][q] = ap[roff[i]];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const double x = as_global(B)[(int64_t)kk * ldb + col[j]];
                b[q][j] = (kb + q < K) ? x : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[i][j] = mfma16x16x4(a[i][q], b[q][j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int cj = (cblk * NT + j) * 16 + m;
            if (cj >= c) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int row = row0 + i * 16 + kq + 4 * v;
                if (row < n) {
                    const auto cp = as_global_mut(C) + (int64_t)row * ldc + cj;
                    double prev = (beta != 0.0) ? beta * *cp : 0.0;
                    *cp = prev + alpha * acc[i][j][v];
                }
            }
        }
}

// C partial (K x c) over one chunk of rows.  Each wave owns NT output
// tiles of 16 A-columns x 16 B-columns, taken in pairs: the pair (2p, 2p+1)
// covers 32 consecutive A columns, lane (k, m) reads columns 2m and 2m+1 of
// the pair with one 16-byte load and feeds the first to tile 2p and the
// second to tile 2p+1 (tile 2p's row i is column 2i of the pair).  The
// block's 4 waves split the chunk's rows and combine through LDS.  A group
// of NT tiles never straddles a panel (16 NT divides the panel width).
// Loads are unconditional: in a group that runs past K the A columns are
// clamped to valid addresses (they only feed discarded output rows), and B
// rows past the chunk are zeroed.
template <int NT, bool VEC, bool CLAMP>
__device__ __forceinline__ void tn_rows(int g0, int r1, int K, int q0, const double *abase, int64_t lda,
                                        const double *__restrict__ B, int64_t ldb, int bcol, int kr, int mc,
                                        dbl4 (&acc)[NT]) {
    constexpr int NP = NT / 2;
    int aoff[NP][2];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        aoff[p][0] = CLAMP ? min(p * 32 + 2 * mc, K - 1 - q0) : p * 32 + 2 * mc;
        aoff[p][1] = CLAMP ? min(p * 32 + 2 * mc + 1, K - 1 - q0) : p * 32 + 2 * mc + 1;
    }
    for (int g = g0; g < r1; g += 4 * 4 * 2) {
        double bv[2];
        dbl2 av[2][NP];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row = g + u * 16 + kr;
            const int rc = min(row, r1 - 1);
            const double x = as_global(B)[(int64_t)rc * ldb + bcol];
            bv[u] = row < r1 ? x : 0.0;
            const auto ar = as_global(abase) + (int64_t)rc * lda;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if constexpr (VEC) {
                    av[u][p] = *reinterpret_cast<gptr<dbl2>>(ar + aoff[p][0]);
                } else {
                    av[u][p].x = ar[aoff[p][0]];
                    av[u][p].y = ar[aoff[p][1]];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                acc[2 * p] = mfma16x16x4(av[u][p].x, bv[u], acc[2 * p]);
                acc[2 * p + 1] = mfma16x16x4(av[u][p].y, bv[u], acc[2 * p + 1]);
            }
    }
}

// One block's partial sums of A^T B over rows [r0, r1): the A tile group
// starting at column q0 (NT tiles of 16 columns) against B tile tb (16
// columns), written to dst (K x c, row-major).  red: LDS of the block.
template <int NT>
__device__ __forceinline__ void tn_mfma_block(int r0, int r1, int K, int c, int q0, int tb, const DMat &A,
                                              const double *__restrict__ B, int64_t ldb, bool aligned, double *dst,
                                              double (*red)[4][WAVE]) {
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int kr = lane / 16, mc = lane % 16;
    const double *abase = col_base(A, q0);
    const int bcol = min(tb * 16 + mc, c - 1);
    dbl4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
    if (q0 + 16 * NT > K)
        tn_rows<NT, false, true>(r0 + wave * 4, r1, K, q0, abase, A.ld, B, ldb, bcol, kr, mc, acc);
    else if (aligned)
        tn_rows<NT, true, false>(r0 + wave * 4, r1, K, q0, abase, A.ld, B, ldb, bcol, kr, mc, acc);
    else
        tn_rows<NT, false, false>(r0 + wave * 4, r1, K, q0, abase, A.ld, B, ldb, bcol, kr, mc, acc);
    // combine the 4 waves one output tile at a time through LDS
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (q0 + (t & ~1) * 16 >= K) break;  // uniform
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave][v][lane] = acc[t][v];
        __syncthreads();
        {
            const int v = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
            double s = red[0][v][l] + red[1][v][l] + red[2][v][l] + red[3][v][l];
            int i = q0 + (t / 2) * 32 + 2 * ((l / 16) + 4 * v) + (t & 1);
            int j = tb * 16 + (l % 16);
            if (i < K && j < c) as_global_mut(dst)[(size_t)i * c + j] = s;
        }
        __syncthreads();
    }
}

// The dot products of one A column (entries col[i * lda]) with the first c
// columns of B over rows [r0, r1), accumulated in row order (EXACT: c == C,
// else c < C and acc[c..C) stay zero).  When the row index is the same
// across the wave (one column per thread), each B row is one wide load
// through the scalar cache.
template <int C, int UNR, bool EXACT = true, typename AP, typename BP>
__device__ __forceinline__ void tn_fma_column(AP col, int64_t lda, int r0, int r1, BP B, int64_t ldb,
                                              double (&acc)[C], int c = C) {
#pragma unroll
    for (int j = 0; j < C; ++j) acc[j] = 0.0;
    int row = r0;
    for (; row + UNR <= r1; row += UNR) {
        double a[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) a[u] = col[(int64_t)(row + u) * lda];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const auto b = B + (int64_t)(row + u) * ldb;
#pragma unroll
            for (int j = 0; j < C; ++j)
                if (EXACT || j < c) acc[j] = fma(a[u], b[j], acc[j]);
        }
    }
    for (; row < r1; ++row) {
        const double a = col[(int64_t)row * lda];
        const auto b = B + (int64_t)row * ldb;
#pragma unroll
        for (int j = 0; j < C; ++j)
            if (EXACT || j < c) acc[j] = fma(a, b[j], acc[j]);
    }
}

}  // namespace
}  // namespace flp
