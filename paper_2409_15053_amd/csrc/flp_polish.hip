// Residual-form polish of FP32-filter solves for gfx950.
//
// A polish sweep of an FP32-filter solve applies the filter to the Ritz
// block X in FP64 accuracy.  With Ahat X = X diag(t) + R (t_j the mapped Ritz
// values, R the scaled FP64 residual block), the polynomial splits as
//   p(Ahat) X = X diag(p(t)) + G,   G_j = g_j(Ahat) r_j,
//   g_j(z) = (p(z) - p(t_j)) / (z - t_j)   (degree m - 1),
// and G is the Clenshaw recurrence of each column's own g_j driven by its
// residual column.  The recurrence runs on FP32 matrix values and FP32
// vectors: its rounding is relative to G, which is the size of the residual
// times the filter's slope, so the FP64 sum above keeps the accuracy the
// FP64 recurrence would give while streaming half the bytes.
//
// Blocks are 32 columns wide (zero-padded); a lane owns 8 consecutive
// columns (two 16-byte pieces), 4 lanes share a matrix row.
#include "flp_internal.h"
#include "flp_device.h"
#include "flp_gather.h"

namespace flp {

namespace {

constexpr int PW = 32;       // columns per block
constexpr int PV = 8;        // columns per lane (two 16-byte pieces)
constexpr int PL = PW / PV;  // lanes per row (a DPP quad: the row's index broadcast stays in registers)
constexpr int PRB = 256 / PL;  // rows per 256-thread block

// R32 = (AX - X diag(lam)) * inv_e for the w real columns of the block
// (block column j is Ritz column cols[j]); zero padding.
__global__ __launch_bounds__(256) void polish_resid_kernel(int n, int w, const double *__restrict__ X,
                                                           const double *__restrict__ AX, int64_t ldc,
                                                           const int *__restrict__ cols,
                                                           const double *__restrict__ lam, double inv_e,
                                                           float *__restrict__ R32) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * PW) return;
    const int64_t row = idx / PW;
    const int j = (int)(idx % PW);
    float v = 0.0f;
    if (j < w) {
        const int64_t q = row * ldc + cols[j];
        v = (float)((AX[q] - lam[j] * X[q]) * inv_e);
    }
    R32[idx] = v;
}

// Y[:, cols[j]] = scale[j] X[:, cols[j]] for j < nl: the locked columns of a
// sweep (their residual is already below the tolerance, so the residual
// term of p(Ahat) x is dropped and p(Ahat) x = p(t) x).
__global__ __launch_bounds__(256) void polish_locked_kernel(int n, int nl, const int *__restrict__ cols,
                                                            const double *__restrict__ scale,
                                                            const double *__restrict__ X, int64_t ldc,
                                                            double *__restrict__ Y) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * nl) return;
    const int64_t row = idx / nl;
    const int j = (int)(idx % nl);
    const int64_t q = row * ldc + cols[j];
    Y[q] = scale[j] * X[q];
}

// One Clenshaw step of the column-wise polynomials g_j:
//   out = a (A U1) + b U1 + coef[j] R - U2
// (U1 == null: the first step, out = coef[j] R; U2 == null: no U2 term).
// LAST: the final step; it writes Y[:, cols[j]] = out_j + ptheta[j] X[:, cols[j]]
// in FP64 for the w real columns.  SELL: rowptr / colind / val are the
// sliced ELL copy (slice offsets; entry k of a row at q0 + k * kSellC); its
// padding adds exact zeros after the row's nonzeros, which it visits in
// their CSR order.  The row sum is gather_row's (each nonzero's index and
// value read once per row, every X load of a group issued before its
// products); WIN: the block's rows of U1 and 8 on each side staged in LDS;
// tiles map to XCDs by chunk_tile.
template <bool LAST, bool SELL, bool WIN>
__global__ __launch_bounds__(256) void polish_step_kernel(int n, const int32_t *__restrict__ rowptr,
                                                          const int32_t *__restrict__ colind,
                                                          const float *__restrict__ val, const float *U1,
                                                          const float *U2, const float *__restrict__ R,
                                                          const float *__restrict__ coef, float a, float b,
                                                          float *out, double *Y, int64_t ldy, int w,
                                                          const double *__restrict__ X, int64_t ldx,
                                                          const int *__restrict__ cols,
                                                          const double *__restrict__ ptheta, int chunk) {
    constexpr int WLD = PW + 4;  // LDS row stride (16 bytes of padding)
    const int r0 = chunk_tile(blockIdx.x, gridDim.x, chunk, PRB) * PRB;
    const int row = r0 + threadIdx.x / PL;
    const int sub = threadIdx.x % PL;
    const int c0 = sub * PV;
    XSource<float, PV, WIN> xs{U1, PW, c0, nullptr, 0, WLD, 0u};
    if constexpr (WIN) {
        __shared__ float win[(PRB + 2 * kWinHalo) * WLD];
        FLP_LDS float *lwin = (FLP_LDS float *)win;
        const int wlo = max(0, r0 - kWinHalo), whi = min(n, r0 + PRB + kWinHalo);
        if (U1) stage_window<float, PW, WLD, PRB + 2 * kWinHalo>(U1, PW, wlo, whi, lwin);
        __syncthreads();
        xs.win = lwin;
        xs.wlo = wlo;
        xs.wlen = (unsigned)(whi - wlo);
    }
    if (row >= n) return;
    float acc[PV], u1[PV], u2[PV], r[PV], o[PV];
#pragma unroll
    for (int j = 0; j < PV; ++j) acc[j] = u1[j] = u2[j] = 0.0f;
    if (U1) {
        gather_row<float, PV, PL, SELL, WIN>(row, sub, rowptr, colind, val, xs, acc);
        xs.load(row, u1);
    }
    if (U2) load_vec<float, PV>(U2 + (int64_t)row * PW + c0, u2);
    load_vec<float, PV>(R + (int64_t)row * PW + c0, r);
#pragma unroll
    for (int j = 0; j < PV; ++j) o[j] = a * acc[j] + b * u1[j] + coef[c0 + j] * r[j] - u2[j];
    if constexpr (!LAST) {
        store_vec<float, PV>(out + (int64_t)row * PW + c0, o);
    } else {
#pragma unroll
        for (int j = 0; j < PV; ++j) {
            const int col = c0 + j;
            if (col < w) {
                const int q = cols[col];
                Y[(int64_t)row * ldy + q] = (double)o[j] + ptheta[col] * X[(int64_t)row * ldx + q];
            }
        }
    }
}

}  // namespace

int polish_block_width() { return PW; }

hipError_t launch_polish_resid(int n, int w, const double *X, const double *AX, int64_t ldc, const int *cols,
                               const double *lam, double inv_e, float *R32, hipStream_t s) {
    if (w < 1 || w > PW) return hipErrorInvalidValue;
    const int64_t total = (int64_t)n * PW;
    hipLaunchKernelGGL(polish_resid_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, w, X, AX, ldc,
                       cols, lam, inv_e, R32);
    return hipGetLastError();
}

hipError_t launch_polish_locked(int n, int nl, const int *cols, const double *scale, const double *X, int64_t ldc,
                                double *Y, hipStream_t s) {
    if (nl <= 0) return hipSuccess;
    const int64_t total = (int64_t)n * nl;
    hipLaunchKernelGGL(polish_locked_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, nl, cols,
                       scale, X, ldc, Y);
    return hipGetLastError();
}

hipError_t launch_polish_step(int n, const int32_t *rowptr, const int32_t *colind, const float *val32,
                              const float *U1, const float *U2, const float *R32, const float *coef, float a,
                              float b, float *out, hipStream_t s, bool sell, int chunk, bool win) {
    const dim3 grid((n + PRB - 1) / PRB);
#define FLP_POLISH(SELL, WIN)                                                                                      \
    hipLaunchKernelGGL((polish_step_kernel<false, SELL, WIN>), grid, dim3(256), 0, s, n, rowptr, colind, val32, U1, \
                       U2, R32, coef, a, b, out, nullptr, 0, 0, nullptr, 0, nullptr, nullptr, chunk)
    if (sell) {
        if (win)
            FLP_POLISH(true, true);
        else
            FLP_POLISH(true, false);
    } else if (win) {
        FLP_POLISH(false, true);
    } else {
        FLP_POLISH(false, false);
    }
#undef FLP_POLISH
    return hipGetLastError();
}

hipError_t launch_polish_last(int n, const int32_t *rowptr, const int32_t *colind, const float *val32,
                              const float *U1, const float *U2, const float *R32, const float *coef, float a,
                              float b, double *Y, int64_t ldy, int w, const double *X, int64_t ldx, const int *cols,
                              const double *ptheta, hipStream_t s, bool sell, int chunk, bool win) {
    if (w < 1 || w > PW) return hipErrorInvalidValue;
    const dim3 grid((n + PRB - 1) / PRB);
#define FLP_POLISH(SELL, WIN)                                                                                     \
    hipLaunchKernelGGL((polish_step_kernel<true, SELL, WIN>), grid, dim3(256), 0, s, n, rowptr, colind, val32, U1, \
                       U2, R32, coef, a, b, nullptr, Y, ldy, w, X, ldx, cols, ptheta, chunk)
    if (sell) {
        if (win)
            FLP_POLISH(true, true);
        else
            FLP_POLISH(true, false);
    } else if (win) {
        FLP_POLISH(false, true);
    } else {
        FLP_POLISH(false, false);
    }
#undef FLP_POLISH
    return hipGetLastError();
}

}  // namespace flp
