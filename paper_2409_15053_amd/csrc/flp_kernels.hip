// Gram-Schmidt and helper kernels of the filtered Lanczos procedure for gfx950 (CDNA4).
//
// * gemm_tn / gemm_nn: the tall-skinny products of the full
//   reorthogonalisation (Section 3.2.2): the update and wide projections on
//   FP64 MFMA (16x16x4), the projection against at most 16 columns on FMA
//   (2 flops per byte: bandwidth-bound either way).
// * small helpers: Gershgorin bounds, counter-based normal generator,
//   block copies, residual norms.
#include "flp_internal.h"
#include "flp_device.h"
#include "flp_gemm.h"

#include <algorithm>

namespace flp {

namespace {

template <int NT>
__global__ __launch_bounds__(256) void gemm_tn_partial_kernel(int n, int K, int c, int chunk_rows, int ngroups, DMat A,
                                                              const double *__restrict__ B, int64_t ldb,
                                                              double *__restrict__ partials, bool aligned, bool sym) {
    __shared__ double red[4][4][WAVE];
    const int ntb = (c + 15) / 16;  // B tiles
    // chunk-major and XCD-aware: the blocks of one row chunk (every tile
    // group of the output) run together on one XCD, so the chunk's rows of
    // A and B come from HBM once and from that XCD's L2 for the other groups
    const int L = xcd_tile(blockIdx.x, gridDim.x);
    const int chunk = L / ngroups, grp = L % ngroups;
    const int q0 = (grp / ntb) * NT * 16, tb = grp % ntb;
    // symmetric result: a group wholly below the diagonal is not computed
    // (the reduction reads its mirror image); uniform over the block
    if (sym && q0 > tb * 16 + 15) return;
    const int r0 = chunk * chunk_rows;
    tn_mfma_block<NT>(r0, min(n, r0 + chunk_rows), K, c, q0, tb, A, B, ldb, aligned, partials + (size_t)chunk * K * c,
                      red);
}

// Sum of the per-chunk partials in a fixed order (deterministic): each
// block owns 64 outputs; its 4 thread rows split the chunks and combine
// through LDS.  sym (a square result whose partials exist on and above the
// diagonal only): entry (i, j) below the diagonal takes the sums of (j, i).
__global__ __launch_bounds__(256) void reduce_partials_kernel(int nchunks, int total, int c,
                                                              const double *__restrict__ partials,
                                                              double *__restrict__ C, int ldc, bool sym) {
    __shared__ double red[4][64];
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    const int o = blockIdx.x * 64 + tx;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (o < total) {
        const int i = o / c, j = o % c;
        const double *p = partials + ((sym && i > j) ? j * c + i : o);
        int q = ty;
        for (; q + 12 < nchunks; q += 16) {
            s0 += p[(size_t)q * total];
            s1 += p[(size_t)(q + 4) * total];
            s2 += p[(size_t)(q + 8) * total];
            s3 += p[(size_t)(q + 12) * total];
        }
        for (; q < nchunks; q += 4) s0 += p[(size_t)q * total];
    }
    red[ty][tx] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (ty == 0 && o < total) C[(size_t)(o / c) * ldc + o % c] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

// C = beta C + alpha A B (see gemm_nn_rows): one block of 4 waves per
// 4 x 16 MT rows and 16 NT columns, blocks renumbered per XCD.
template <int MT, int NT>
__global__ __launch_bounds__(256) void gemm_nn_kernel(int n, int K, int c, double alpha, DMat A,
                                                      const double *__restrict__ B, int64_t ldb, double beta,
                                                      double *C, int64_t ldc, bool vec_a) {
    const int nct = (c + 16 * NT - 1) / (16 * NT);
    const int wg = xcd_tile(blockIdx.x, gridDim.x);
    gemm_nn_rows<MT, NT>(n, K, c, alpha, A, B, ldb, beta, C, ldc, vec_a, wg / nct, wg % nct);
}

}  // namespace

namespace {

// C partial (K x C) over one chunk of rows without MFMA, for B of exactly
// C columns: thread q owns column q of A and accumulates its C dot products
// with B over the chunk's rows in order.  The B row is the same for the
// whole block (the rows are walked in step), so it is read through the
// scalar cache as one wide load; the A loads of a wave are 64 consecutive
// doubles of one row.  With C <= 16 this product does 2C flops per 8-byte A
// element, far below what the FMA units sustain at HBM speed, so it needs
// no matrix cores.
template <int C, int UNR>
__global__ __launch_bounds__(256) void gemm_tn_fma_kernel(int n, int K, int chunk_rows, DMat A,
                                                          const double *__restrict__ B, int64_t ldb,
                                                          double *__restrict__ partials) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= K) return;  // no block-level synchronisation follows: idle columns leave at once
    const int chunk = blockIdx.y;
    const int r0 = chunk * chunk_rows, r1 = min(n, r0 + chunk_rows);
    double acc[C];
    tn_fma_column<C, UNR>(col_base(A, q), A.ld, r0, r1, B, ldb, acc);
    double *d = partials + ((size_t)chunk * K + q) * C;
#pragma unroll
    for (int j = 0; j < C; ++j) d[j] = acc[j];
}

}  // namespace

// The FMA projection serves B of exactly 8 columns against a basis of at
// least 256 columns; the MFMA kernel's row-parallel layout does better below
// that and at 16 columns, where the thread-per-column kernel's 16 FMAs per
// loaded element hold it back.  Measured at n = 1e6 (TB/s, FMA / MFMA):
// c = 8: K = 128 3.5 / 5.4, 256 5.6 / 5.4, 512 6.0 / 5.5, 768 6.1 / 5.6;
// c = 16: K = 128 2.6 / 5.5, 352 3.8 / 5.0, 768 5.0 / 5.4.
static bool tn_use_fma(int K, int c) { return c == 8 && K >= 256; }

TnPlan plan_tn(int n, int K, int c) {
    TnPlan p;
    if (tn_use_fma(K, c)) {
        // FMA path: about 1024 blocks of 256 columns x chunk_rows rows (about
        // 1000-2000 rows each at n = 1e6, the fastest chunking measured), the
        // partial buffer kept near 32M doubles at most
        const int ncb = (K + 255) / 256;
        int nch = std::max(1, std::min(1024, 1024 / ncb));
        int rows = std::max(64, (n + nch - 1) / nch);
        rows = (rows + 63) / 64 * 64;
        while ((size_t)((n + rows - 1) / rows) * K * c > (size_t)(32u << 20)) rows *= 2;
        p.chunk_rows = rows;
        p.nchunks = (n + rows - 1) / rows;
        p.partial_elems = (size_t)p.nchunks * K * c;
        return p;
    }
    const int ntiles = ((K + 127) / 128) * ((c + 15) / 16);
    // aim for ~2048 blocks in total, at least 128 rows per block, and keep
    // the partial buffer near 32M doubles at most
    int nch = std::min(512, std::max(1, 2048 / std::max(1, ntiles)));
    int rows = (n + nch - 1) / nch;
    rows = std::max(rows, 128);
    size_t per = (size_t)K * c;
    while ((size_t)((n + rows - 1) / rows) * per > (size_t)(32u << 20)) rows *= 2;
    rows = (rows + 127) / 128 * 128;
    p.chunk_rows = rows;
    p.nchunks = (n + rows - 1) / rows;
    p.partial_elems = (size_t)p.nchunks * per;
    return p;
}

hipError_t launch_gemm_tn_partial(const TnPlan &pl, int n, int K, int c, DMat A, const double *B, int64_t ldb,
                                  double *partials, hipStream_t s, bool sym) {
    if (tn_use_fma(K, c)) {
        dim3 grid((K + 255) / 256, pl.nchunks);
        hipLaunchKernelGGL((gemm_tn_fma_kernel<8, 8>), grid, dim3(256), 0, s, n, K, pl.chunk_rows, A, B, ldb,
                           partials);
        return hipGetLastError();
    }
    // 16-byte A loads need an even leading dimension and panel stride
    const bool aligned = !(A.ld & 1) && !(A.ps & 1) && !(reinterpret_cast<uintptr_t>(A.p) & 15);
    const int nt = K <= 32 ? 2 : (K <= 64 ? 4 : 8);
    const int ngroups = ((K + 16 * nt - 1) / (16 * nt)) * ((c + 15) / 16);
    dim3 grid(pl.nchunks * ngroups);
#define FLP_TN(NT) \
    hipLaunchKernelGGL((gemm_tn_partial_kernel<NT>), grid, dim3(256), 0, s, n, K, c, pl.chunk_rows, ngroups, A, B, ldb, \
                       partials, aligned, sym && K == c)
    if (nt == 2)
        FLP_TN(2);
    else if (nt == 4)
        FLP_TN(4);
    else
        FLP_TN(8);
#undef FLP_TN
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const TnPlan &pl, int K, int c, const double *partials, double *C, int ldc,
                                  hipStream_t s, bool sym) {
    int total = K * c;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((total + 63) / 64), dim3(256), 0, s, pl.nchunks, total, c,
                       partials, C, ldc, sym && K == c);
    return hipGetLastError();
}

hipError_t launch_gemm_nn(int n, int K, int c, double alpha, DMat A, const double *B, int64_t ldb, double beta,
                          double *C, int64_t ldc, hipStream_t s) {
    if (n <= 0 || c <= 0) return hipSuccess;
    bool vec_a = (A.ld % 2 == 0) && (A.ps % 2 == 0) && ((reinterpret_cast<uintptr_t>(A.p) & 15) == 0);
    if (c <= 16) {
        // row tiles per wave: 2 up to a few hundred basis columns, 8 beyond
        // (more A loads in flight per MFMA chain); at n = 1e6 this streams
        // Q at 5.0-5.6 TB/s from K = 64 to 768, where 4 tiles gave 4.3-5.1
        constexpr int NT = 1;
        if (K >= 320) {
            constexpr int MT = 8;
            int rblocks = (n + 4 * 16 * MT - 1) / (4 * 16 * MT);
            hipLaunchKernelGGL((gemm_nn_kernel<MT, NT>), dim3(rblocks), dim3(256), 0, s, n, K, c, alpha, A, B, ldb,
                               beta, C, ldc, vec_a);
        } else {
            constexpr int MT = 2;
            int rblocks = (n + 4 * 16 * MT - 1) / (4 * 16 * MT);
            hipLaunchKernelGGL((gemm_nn_kernel<MT, NT>), dim3(rblocks), dim3(256), 0, s, n, K, c, alpha, A, B, ldb,
                               beta, C, ldc, vec_a);
        }
    } else {
        constexpr int MT = 2, NT = 4;
        int rblocks = (n + 4 * 16 * MT - 1) / (4 * 16 * MT);
        int nct = (c + 16 * NT - 1) / (16 * NT);
        hipLaunchKernelGGL((gemm_nn_kernel<MT, NT>), dim3(rblocks * nct), dim3(256), 0, s, n, K, c, alpha, A, B,
                           ldb, beta, C, ldc, vec_a);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ helpers

namespace {

// Symmetry check, one thread per row: for each stored a_ij, a_ji is looked
// up by binary search in row j (columns sorted) and compared; the count of
// entries without a matching partner goes to *bad (vector atomics).
__global__ void sym_check_kernel(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                                 const double *__restrict__ val, double tol, unsigned int *bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned int cnt = 0;
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int j = colind[p];
        if (j < 0 || j >= n) {
            ++cnt;
            continue;
        }
        int lo = rowptr[j], hi = rowptr[j + 1] - 1, found = -1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int cm = colind[mid];
            if (cm == i) {
                found = mid;
                break;
            }
            if (cm < i)
                lo = mid + 1;
            else
                hi = mid - 1;
        }
        if (found < 0) {
            ++cnt;
            continue;
        }
        const double a = val[p], b = val[found];
        if (fabs(a - b) > tol * fmax(fabs(a), fabs(b))) ++cnt;
    }
    if (cnt) atomicAdd(bad, cnt);
}

__global__ void gershgorin_kernel(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                                  const double *__restrict__ val, double *__restrict__ part) {
    __shared__ double slo[256], shi[256];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double lo = 1e308, hi = -1e308;
    if (i < n) {
        double d = 0.0, rad = 0.0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (colind[p] == i)
                d += val[p];
            else
                rad += fabs(val[p]);
        }
        lo = d - rad;
        hi = d + rad;
    }
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + w]);
            shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = slo[0];
        part[2 * blockIdx.x + 1] = shi[0];
    }
}

__global__ void minmax_kernel(int m, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double slo[256], shi[256];
    double lo = 1e308, hi = -1e308;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        lo = fmin(lo, part[2 * i]);
        hi = fmax(hi, part[2 * i + 1]);
    }
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + w]);
            shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = slo[0];
        out[1] = shi[0];
    }
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the output function applied
// to a Weyl sequence; used here as a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void randn_kernel(int rows, int cols, double *__restrict__ out, int64_t ld, uint64_t seed,
                             uint64_t sid) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)rows * cols;
    if (idx >= total) return;
    uint64_t key = splitmix64(seed ^ splitmix64(sid));
    uint64_t u1 = splitmix64(key + 2 * (uint64_t)idx);
    uint64_t u2 = splitmix64(key + 2 * (uint64_t)idx + 1);
    // 53-bit uniforms in (0, 1] and [0, 1); Box-Muller
    double a = ((u1 >> 11) + 1) * (1.0 / 9007199254740992.0);
    double b = (u2 >> 11) * (1.0 / 9007199254740992.0);
    double z = sqrt(-2.0 * log(a)) * cospi(2.0 * b);
    out[(idx / cols) * ld + idx % cols] = z;
}

// End of one step of the bounds estimate's single-vector Lanczos, on the
// device: alpha_j = h1[hj] + h2[hj] (the two Gram-Schmidt passes' coefficient
// of q_j, column hj of the projection), beta_j = sqrt(g) with g = ||w||^2,
// and q_{j+1} = w / beta_j (zero after a breakdown, beta_j = 0).  ab[2j],
// ab[2j+1] receive alpha_j, beta_j.
__global__ void lanczos_next_kernel(int n, const double *__restrict__ w, double *__restrict__ q, int64_t ldq,
                                    const double *__restrict__ g, const double *__restrict__ h1,
                                    const double *__restrict__ h2, int hj, int j, double *__restrict__ ab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double beta = sqrt(fmax(g[0], 0.0));
    if (i == 0) {
        ab[2 * j] = h1[hj] + h2[hj];
        ab[2 * j + 1] = beta;
    }
    if (i < n) q[(int64_t)i * ldq] = beta > 0.0 ? w[i] / beta : 0.0;
}

__global__ void copy_block_kernel(int rows, int cols, double scale, const double *__restrict__ src, int64_t lds,
                                  DMat dst, int dcol0, float *__restrict__ dst32, int64_t ldd32) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * cols) return;
    int64_t i = idx / cols;
    int j = (int)(idx % cols);
    double v = scale * src[i * lds + j];
    if (dst.p) {
        int q = dcol0 + j;
        dst.p[(int64_t)(q >> dst.lpw) * dst.ps + i * dst.ld + (q & ((1 << dst.lpw) - 1))] = v;
    }
    if (dst32) dst32[i * ldd32 + j] = (float)v;
}

__global__ void to_float_kernel(int64_t count, const double *__restrict__ src, float *__restrict__ dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = (float)src[i];
}

__global__ void scale_kernel(int64_t count, double a, const double *__restrict__ src, double *__restrict__ dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = a * src[i];
}

// per (chunk, column): sum of squares of AX - lam X over the chunk's rows
__global__ void resid_partial_kernel(int n, int c, const double *__restrict__ AX, int64_t ldax,
                                     const double *__restrict__ X, int64_t ldx, const double *__restrict__ lam,
                                     int rows_per_chunk, double *__restrict__ part) {
    __shared__ double red[256];
    const int chunk = blockIdx.x, j0 = blockIdx.y * 64;
    const int j = j0 + threadIdx.x % 64, rsub = threadIdx.x / 64;
    double s = 0.0;
    if (j < c) {
        double l = lam[j];
        int r0 = chunk * rows_per_chunk, r1 = min(n, r0 + rows_per_chunk);
        for (int i = r0 + rsub; i < r1; i += 4) {
            double d = AX[(int64_t)i * ldax + j] - l * X[(int64_t)i * ldx + j];
            s = fma(d, d, s);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 64 && j < c) {
        double t = red[threadIdx.x] + red[threadIdx.x + 64] + red[threadIdx.x + 128] + red[threadIdx.x + 192];
        part[(size_t)chunk * c + j] = t;
    }
}

__global__ void resid_final_kernel(int nchunks, int c, const double *__restrict__ part, double *__restrict__ out) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c) return;
    double s = 0.0;
    for (int q = 0; q < nchunks; ++q) s += part[(size_t)q * c + j];
    out[j] = sqrt(s);
}

// Partial sums over chunks of rows of the column dot products x_j . y_j
// (the layout of resid_partial_kernel), then their sum in chunk order.
__global__ void coldot_partial_kernel(int n, int c, const double *__restrict__ X, int64_t ldx,
                                      const double *__restrict__ Y, int64_t ldy, int rows_per_chunk,
                                      double *__restrict__ part) {
    __shared__ double red[256];
    const int chunk = blockIdx.x, j0 = blockIdx.y * 64;
    const int j = j0 + threadIdx.x % 64, rsub = threadIdx.x / 64;
    double s = 0.0;
    if (j < c) {
        int r0 = chunk * rows_per_chunk, r1 = min(n, r0 + rows_per_chunk);
        for (int i = r0 + rsub; i < r1; i += 4) s = fma(X[(int64_t)i * ldx + j], Y[(int64_t)i * ldy + j], s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 64 && j < c) {
        double t = red[threadIdx.x] + red[threadIdx.x + 64] + red[threadIdx.x + 128] + red[threadIdx.x + 192];
        part[(size_t)chunk * c + j] = t;
    }
}

__global__ void coldot_final_kernel(int nchunks, int c, const double *__restrict__ part, double *__restrict__ out) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c) return;
    double s = 0.0;
    for (int q = 0; q < nchunks; ++q) s += part[(size_t)q * c + j];
    out[j] = s;
}

__global__ void transpose_out_kernel(int n, int c, const double *__restrict__ src, int64_t lds,
                                     double *__restrict__ dst) {
    __shared__ double t[32][33];
    int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx: rows of src, by: columns
    int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 256 threads: ty 0..7
    for (int k = ty; k < 32; k += 8) {
        int i = bx + k, j = by + tx;
        t[k][tx] = (i < n && j < c) ? src[(int64_t)i * lds + j] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        int j = by + k, i = bx + tx;
        if (i < n && j < c) dst[(int64_t)j * n + i] = t[tx][k];
    }
}

// dst (row-major n x c, ldd) = src (column-major n x c, ld n): the inverse
// of transpose_out_kernel, tile by tile through LDS.
__global__ void transpose_in_kernel(int n, int c, const double *__restrict__ src, double *__restrict__ dst,
                                    int64_t ldd) {
    __shared__ double t[32][33];
    int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx: rows of dst, by: columns
    int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int k = ty; k < 32; k += 8) {
        int j = by + k, i = bx + tx;
        t[tx][k] = (i < n && j < c) ? src[(int64_t)j * n + i] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        int i = bx + k, j = by + tx;
        if (i < n && j < c) dst[(int64_t)i * ldd + j] = t[k][tx];
    }
}

}  // namespace

int gershgorin_blocks(int n) { return (n + 255) / 256; }

hipError_t launch_sym_check(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double tol,
                            unsigned int *bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sym_check_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, rowptr, colind, val, tol, bad);
    return hipGetLastError();
}

hipError_t launch_gershgorin(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double *part,
                             int part_cap, double *out, hipStream_t s) {
    int nb = gershgorin_blocks(n);
    if (nb > part_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gershgorin_kernel, dim3(nb), dim3(256), 0, s, n, rowptr, colind, val, part);
    hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(256), 0, s, nb, part, out);
    return hipGetLastError();
}

hipError_t launch_randn(int rows, int cols, double *out, int64_t ld, uint64_t seed, uint64_t sid, hipStream_t s) {
    int64_t total = (int64_t)rows * cols;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(randn_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rows, cols, out, ld,
                       seed, sid);
    return hipGetLastError();
}

hipError_t launch_copy_block(int rows, int cols, double scale, const double *src, int64_t lds, DMat dst, int dcol0,
                             float *dst32, int64_t ldd32, hipStream_t s) {
    int64_t total = (int64_t)rows * cols;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_block_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rows, cols, scale,
                       src, lds, dst, dcol0, dst32, ldd32);
    return hipGetLastError();
}

hipError_t launch_lanczos_next(int n, const double *w, double *q, int64_t ldq, const double *g, const double *h1,
                               const double *h2, int hj, int j, double *ab, hipStream_t s) {
    hipLaunchKernelGGL(lanczos_next_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, w, q, ldq, g, h1, h2, hj, j,
                       ab);
    return hipGetLastError();
}

hipError_t launch_to_float(int64_t count, const double *src, float *dst, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(to_float_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, src, dst);
    return hipGetLastError();
}

hipError_t launch_scale(int64_t count, double a, const double *src, double *dst, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, a, src, dst);
    return hipGetLastError();
}

int resid_chunks(int n) { return std::max(1, std::min(512, (n + 1023) / 1024)); }

hipError_t launch_resid_norms(int n, int c, const double *AX, int64_t ldax, const double *X, int64_t ldx,
                              const double *lam, double *part, int nchunks, double *out, hipStream_t s) {
    if (c <= 0) return hipSuccess;
    int rpc = (n + nchunks - 1) / nchunks;
    hipLaunchKernelGGL(resid_partial_kernel, dim3(nchunks, (c + 63) / 64), dim3(256), 0, s, n, c, AX, ldax, X, ldx,
                       lam, rpc, part);
    hipLaunchKernelGGL(resid_final_kernel, dim3((c + 255) / 256), dim3(256), 0, s, nchunks, c, part, out);
    return hipGetLastError();
}

hipError_t launch_col_dots(int n, int c, const double *X, int64_t ldx, const double *Y, int64_t ldy, double *part,
                           int nchunks, double *out, hipStream_t s) {
    if (c <= 0) return hipSuccess;
    int rpc = (n + nchunks - 1) / nchunks;
    hipLaunchKernelGGL(coldot_partial_kernel, dim3(nchunks, (c + 63) / 64), dim3(256), 0, s, n, c, X, ldx, Y, ldy,
                       rpc, part);
    hipLaunchKernelGGL(coldot_final_kernel, dim3((c + 255) / 256), dim3(256), 0, s, nchunks, c, part, out);
    return hipGetLastError();
}

hipError_t launch_transpose_in(int n, int c, const double *src, double *dst, int64_t ldd, hipStream_t s) {
    if (n <= 0 || c <= 0) return hipSuccess;
    dim3 grid((n + 31) / 32, (c + 31) / 32);
    hipLaunchKernelGGL(transpose_in_kernel, grid, dim3(256), 0, s, n, c, src, dst, ldd);
    return hipGetLastError();
}

hipError_t launch_transpose_out(int n, int c, const double *src, int64_t lds, double *dst, hipStream_t s) {
    if (n <= 0 || c <= 0) return hipSuccess;
    dim3 grid((n + 31) / 32, (c + 31) / 32);
    hipLaunchKernelGGL(transpose_out_kernel, grid, dim3(256), 0, s, n, c, src, lds, dst);
    return hipGetLastError();
}

}  // namespace flp
