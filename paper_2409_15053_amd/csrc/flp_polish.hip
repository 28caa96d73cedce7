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
// Blocks are 32 columns wide (zero-padded); a lane owns 4 consecutive
// columns (one 16-byte piece), 8 lanes share a matrix row.
#include "flp_internal.h"
#include "flp_device.h"

namespace flp {

namespace {

constexpr int PW = 32;       // columns per block
constexpr int PV = 4;        // columns per lane
constexpr int PL = PW / PV;  // lanes per row
constexpr int PRB = 256 / PL;  // rows per 256-thread block

// R32 = (AX - X diag(lam)) * inv_e for the w real columns; zero padding.
__global__ __launch_bounds__(256) void polish_resid_kernel(int n, int w, const double *__restrict__ X,
                                                           const double *__restrict__ AX, int64_t ldc,
                                                           const double *__restrict__ lam, double inv_e,
                                                           float *__restrict__ R32) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)n * PW) return;
    const int64_t row = idx / PW;
    const int j = (int)(idx % PW);
    float v = 0.0f;
    if (j < w) v = (float)((AX[row * ldc + j] - lam[j] * X[row * ldc + j]) * inv_e);
    R32[idx] = v;
}

// One Clenshaw step of the column-wise polynomials g_j:
//   out = a (A U1) + b U1 + coef[j] R - U2
// (U1 == null: the first step, out = coef[j] R; U2 == null: no U2 term).
// LAST: the final step; it writes Y[:, j] = out_j + ptheta[j] X[:, j] in FP64
// for the w real columns.  SELL: rowptr / colind / val are the sliced ELL
// copy (slice offsets; entry k of a row at q0 + k * kSellC); its padding adds
// exact zeros after the row's nonzeros, which it visits in their CSR order.
template <bool LAST, bool SELL>
__global__ __launch_bounds__(256) void polish_step_kernel(int n, const int32_t *__restrict__ rowptr,
                                                          const int32_t *__restrict__ colind,
                                                          const float *__restrict__ val, const float *U1,
                                                          const float *U2, const float *__restrict__ R,
                                                          const float *__restrict__ coef, float a, float b,
                                                          float *out, double *Y, int64_t ldy, int w,
                                                          const double *__restrict__ X, int64_t ldx,
                                                          const double *__restrict__ ptheta) {
    const int row = blockIdx.x * PRB + threadIdx.x / PL;
    if (row >= n) return;
    const int c0 = (threadIdx.x % PL) * PV;
    float acc[PV] = {0.0f, 0.0f, 0.0f, 0.0f};
    float u1[PV] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (U1) {
        int base, stride, cnt;  // entry i of the row at base + i * stride
        if constexpr (SELL) {
            const int sl = row / kSellC;
            base = rowptr[sl] + row % kSellC;
            stride = kSellC;
            cnt = (rowptr[sl + 1] - rowptr[sl]) / kSellC;
        } else {
            base = rowptr[row];
            stride = 1;
            cnt = rowptr[row + 1] - base;
        }
        int i = 0;
        for (; i + 4 <= cnt; i += 4) {
            float v[4];
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = base + (i + u) * stride;
                v[u] = val[q];
                x[u] = *reinterpret_cast<const float4 *>(U1 + (int64_t)colind[q] * PW + c0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc[0] = fmaf(v[u], x[u].x, acc[0]);
                acc[1] = fmaf(v[u], x[u].y, acc[1]);
                acc[2] = fmaf(v[u], x[u].z, acc[2]);
                acc[3] = fmaf(v[u], x[u].w, acc[3]);
            }
        }
        for (; i < cnt; ++i) {
            const int q = base + i * stride;
            const float v = val[q];
            const float4 x = *reinterpret_cast<const float4 *>(U1 + (int64_t)colind[q] * PW + c0);
            acc[0] = fmaf(v, x.x, acc[0]);
            acc[1] = fmaf(v, x.y, acc[1]);
            acc[2] = fmaf(v, x.z, acc[2]);
            acc[3] = fmaf(v, x.w, acc[3]);
        }
        const float4 s = *reinterpret_cast<const float4 *>(U1 + (int64_t)row * PW + c0);
        u1[0] = s.x;
        u1[1] = s.y;
        u1[2] = s.z;
        u1[3] = s.w;
    }
    float u2[PV] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (U2) {
        const float4 s = *reinterpret_cast<const float4 *>(U2 + (int64_t)row * PW + c0);
        u2[0] = s.x;
        u2[1] = s.y;
        u2[2] = s.z;
        u2[3] = s.w;
    }
    const float4 r4 = *reinterpret_cast<const float4 *>(R + (int64_t)row * PW + c0);
    const float r[PV] = {r4.x, r4.y, r4.z, r4.w};
    float o[PV];
#pragma unroll
    for (int j = 0; j < PV; ++j) o[j] = a * acc[j] + b * u1[j] + coef[c0 + j] * r[j] - u2[j];
    if constexpr (!LAST) {
        *reinterpret_cast<float4 *>(out + (int64_t)row * PW + c0) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
        for (int j = 0; j < PV; ++j) {
            const int col = c0 + j;
            if (col < w) Y[(int64_t)row * ldy + col] = (double)o[j] + ptheta[col] * X[(int64_t)row * ldx + col];
        }
    }
}

}  // namespace

int polish_block_width() { return PW; }

hipError_t launch_polish_resid(int n, int w, const double *X, const double *AX, int64_t ldc, const double *lam,
                               double inv_e, float *R32, hipStream_t s) {
    if (w < 1 || w > PW) return hipErrorInvalidValue;
    const int64_t total = (int64_t)n * PW;
    hipLaunchKernelGGL(polish_resid_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, w, X, AX, ldc,
                       lam, inv_e, R32);
    return hipGetLastError();
}

hipError_t launch_polish_step(int n, const int32_t *rowptr, const int32_t *colind, const float *val32,
                              const float *U1, const float *U2, const float *R32, const float *coef, float a,
                              float b, float *out, hipStream_t s, bool sell) {
    if (sell)
        hipLaunchKernelGGL((polish_step_kernel<false, true>), dim3((n + PRB - 1) / PRB), dim3(256), 0, s, n, rowptr,
                           colind, val32, U1, U2, R32, coef, a, b, out, nullptr, 0, 0, nullptr, 0, nullptr);
    else
        hipLaunchKernelGGL((polish_step_kernel<false, false>), dim3((n + PRB - 1) / PRB), dim3(256), 0, s, n, rowptr,
                           colind, val32, U1, U2, R32, coef, a, b, out, nullptr, 0, 0, nullptr, 0, nullptr);
    return hipGetLastError();
}

hipError_t launch_polish_last(int n, const int32_t *rowptr, const int32_t *colind, const float *val32,
                              const float *U1, const float *U2, const float *R32, const float *coef, float a,
                              float b, double *Y, int64_t ldy, int w, const double *X, int64_t ldx,
                              const double *ptheta, hipStream_t s, bool sell) {
    if (w < 1 || w > PW) return hipErrorInvalidValue;
    if (sell)
        hipLaunchKernelGGL((polish_step_kernel<true, true>), dim3((n + PRB - 1) / PRB), dim3(256), 0, s, n, rowptr,
                           colind, val32, U1, U2, R32, coef, a, b, nullptr, Y, ldy, w, X, ldx, ptheta);
    else
        hipLaunchKernelGGL((polish_step_kernel<true, false>), dim3((n + PRB - 1) / PRB), dim3(256), 0, s, n, rowptr,
                           colind, val32, U1, U2, R32, coef, a, b, nullptr, Y, ldy, w, X, ldx, ptheta);
    return hipGetLastError();
}

}  // namespace flp
