// Segmented block step for gfx950: the full reorthogonalisation (two passes
// of classical Gram-Schmidt, Section 3.2.2) and the block normalisation
// W = Q_{j+1} S_j (Cholesky QR twice, eq. lanczos) of many independent
// solves, with one launch per stage for all of them.
//
// A launch's blocks are split into segments, one per solve, by a prefix of
// block counts (OrthSeg tables); a block finds its segment with the same
// ballot count as the segmented filter step.  The r x r Cholesky factors
// are computed on the device (one lane per solve), so a whole block step
// runs without a host round trip; a solve whose first factorisation finds
// numerically dependent columns is flagged and skipped by the later stages,
// and the host repairs it afterwards.
//
// Stages (c = block width r <= 16, k = basis columns, per solve):
//   seg_tn_*    partial sums of Q^T W (k x c), or of W^T W (c x c), over row chunks
//   seg_reduce  the partial sums in a fixed order -> H1, H2 or G
//   seg_nn      W -= Q H (FP64 MFMA)
//   seg_chol    D_j, Cholesky factor and its inverse (pass 1), or S_j (pass 2)
//   seg_rscale  W <- W R^{-1}; the last one writes Q_{j+1} into the basis
//               and the next filter input instead
#include "flp_internal.h"
#include "flp_device.h"
#include "flp_gemm.h"

namespace flp {

namespace {

// Index of the segment that owns block blk: pre[] is non-decreasing, so the
// segments starting at or before blk are a prefix, counted 64 at a time with
// one load per lane and a ballot; the count is made wave-uniform so the
// segment's descriptor is read through the scalar cache.
__device__ __forceinline__ int seg_of(const int *__restrict__ pre, int nseg, int blk) {
    const int lane = threadIdx.x % WAVE;
    int seg = -1;
    for (int base = 0; base < nseg; base += WAVE) {
        const int i = base + lane;
        const bool le = i < nseg && pre[i] <= blk;
        const unsigned long long m = __ballot(le);
        seg += __popcll(m);
        if (~m != 0ull) break;
    }
    return __builtin_amdgcn_readfirstlane(seg);
}

__device__ __forceinline__ bool flagged(const OrthSeg &e, int c) { return e.out[2 * c * c] != 0.0; }

// Projection partial sums of Q^T W for solves with k > 128 on FMA: one
// basis column per thread, 256 columns per block, the block's rows
// [chunk * chunk_rows, ...) walked in step, so each W row is one wide load
// through the scalar cache.  (This kernel has no LDS and no barrier: with
// either in the same kernel the compiler can no longer prove the W rows
// unmodified and falls back to per-lane vector loads of the same row.)
// Partial sums of chunk t go to part[(t k + q) c + j].
template <int CM, bool EXACT>
__global__ __launch_bounds__(256) void seg_tn_fma_kernel(const OrthSeg *__restrict__ tab,
                                                         const int *__restrict__ pre, int nseg, int c) {
    const int seg = seg_of(pre, nseg, blockIdx.x);
    const OrthSeg &e = tab[seg];
    const int lb = blockIdx.x - pre[seg];
    const int K = e.k;
    const int ncb = (K + 255) / 256;
    const int cb = lb % ncb, chunk = lb / ncb;
    const int q = cb * 256 + threadIdx.x;
    if (q >= K) return;
    const int r0 = chunk * e.chunk_rows, r1 = min(e.n, r0 + e.chunk_rows);
    double acc[CM];
    tn_fma_column<CM, (CM > 8 ? 4 : 8), EXACT>(as_global(col_base(e.Q, q)), e.Q.ld, r0, r1, as_global(e.W), c, acc,
                                               c);
    const auto d = as_global_mut(e.part) + ((size_t)chunk * K + q) * c;
#pragma unroll
    for (int j = 0; j < CM; ++j)
        if (EXACT || j < c) d[j] = acc[j];
}

// Projection partial sums on FP64 MFMA (the layout of the single-solve
// kernel: one B tile of 16 columns, NT A tiles per wave, 4 waves over the
// rows of a chunk combined through LDS): Q^T W for solves with k <= 128
// (NT = 8 covers the basis), or the Gram matrix W^T W (GRAM, NT = 2).
template <bool GRAM>
__global__ __launch_bounds__(256) void seg_tn_mfma_kernel(const OrthSeg *__restrict__ tab,
                                                          const int *__restrict__ pre, int nseg, int c, int chk) {
    constexpr int NT = GRAM ? 2 : 8;
    __shared__ double red[4][4][WAVE];
    const int seg = seg_of(pre, nseg, blockIdx.x);
    const OrthSeg &e = tab[seg];
    if (chk && flagged(e, c)) return;
    const int chunk = blockIdx.x - pre[seg];
    const int K = GRAM ? c : e.k;
    const DMat A = GRAM ? DMat{e.W, c, 0, 30} : e.Q;
    const int rows = GRAM ? e.gchunk_rows : e.chunk_rows;
    const int r0 = chunk * rows;
    // 16-byte A loads: the basis panels always qualify, W when c is even
    const bool aligned = !GRAM || (c % 2 == 0);
    tn_mfma_block<NT>(r0, min(e.n, r0 + rows), K, c, 0, 0, A, e.W, c, aligned, e.part + (size_t)chunk * K * c, red);
}

// Sum of the per-chunk partials in a fixed order: 64 outputs per block, its
// 4 thread rows split the chunks and combine through LDS.  which: 0 -> H1,
// 1 -> H2 (k x c each), 2 -> G (c x c).
__global__ __launch_bounds__(256) void seg_reduce_kernel(const OrthSeg *__restrict__ tab,
                                                         const int *__restrict__ pre, int nseg, int c, int which,
                                                         int chk) {
    __shared__ double red[4][64];
    const int seg = seg_of(pre, nseg, blockIdx.x);
    const OrthSeg &e = tab[seg];
    if (chk && flagged(e, c)) return;
    const int lb = blockIdx.x - pre[seg];
    const int K = which == 2 ? c : e.k;
    const int nch = which == 2 ? e.gnchunks : e.nchunks;
    const auto dst = as_global_mut(which == 2 ? e.G : e.H + (size_t)which * e.k * c);
    const int total = K * c;
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    const int o = lb * 64 + tx;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (o < total) {
        const auto p = as_global(e.part) + o;
        int q = ty;
        for (; q + 12 < nch; q += 16) {
            s0 += p[(size_t)q * total];
            s1 += p[(size_t)(q + 4) * total];
            s2 += p[(size_t)(q + 8) * total];
            s3 += p[(size_t)(q + 12) * total];
        }
        for (; q < nch; q += 4) s0 += p[(size_t)q * total];
    }
    red[ty][tx] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (ty == 0 && o < total) dst[o] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

// W -= Q H_which (k inner), 256 rows per block.
__global__ __launch_bounds__(256) void seg_nn_kernel(const OrthSeg *__restrict__ tab, const int *__restrict__ pre,
                                                     int nseg, int c, int which) {
    const int seg = seg_of(pre, nseg, blockIdx.x);
    const OrthSeg &e = tab[seg];
    const int lb = blockIdx.x - pre[seg];
    gemm_nn_rows<4, 1>(e.n, e.k, c, -1.0, e.Q, e.H + (size_t)which * e.k * c, c, 1.0, e.W, c, true, lb, 0);
}

// The r x r factorisations of one solve on one wavefront, through LDS.
// Pass 1: D_j = sym(diagonal blocks of H1 + H2) to out[0, c^2); the first
// factor R1 of G (upper, row-major) by right-looking Cholesky with the
// block QR's dependent-column rule (a pivot at or below (1e-7 ||W||_F)^2
// marks the column: status 1, the later launches skip the solve and the host
// repairs it), then R1^{-1}.  Pass 2: the second factor R2 (status 2 if it
// breaks down), R2^{-1} and S_j = R2 R1 to out[c^2, 2 c^2).  Lane j computes
// column j of an inverse; the other steps spread the c x c entries over the
// lanes.
__global__ __launch_bounds__(64) void seg_chol_kernel(const OrthSeg *__restrict__ tab, int c, int pass) {
    __shared__ double M[16 * 16], T[16 * 16];
    __shared__ int bad;
    const OrthSeg &e = tab[blockIdx.x];
    const int lane = threadIdx.x;
    const int cc = c * c;
    double *out = e.out;
    double *status = out + 2 * cc;
    if (pass == 2 && *status != 0.0) return;  // uniform: every lane reads the same flag
    if (pass == 1) {
        const double *h1 = e.H + (size_t)(e.k - c) * c;
        const double *h2 = e.H + (size_t)e.k * c + (size_t)(e.k - c) * c;
        for (int t = lane; t < cc; t += WAVE) {
            const int i = t / c, j = t % c;
            const double a = h1[i * c + j] + h2[i * c + j], b = h1[j * c + i] + h2[j * c + i];
            out[t] = 0.5 * (a + b);
        }
    }
    for (int t = lane; t < cc; t += WAVE) M[t] = e.G[t];
    if (lane == 0) bad = 0;
    __syncthreads();
    double thr2 = 1e-300;
    if (pass == 1) {
        double fro2 = 0.0;
        for (int i = 0; i < c; ++i) fro2 += fmax(M[i * c + i], 0.0);
        const double thr = 1e-7 * sqrt(fro2);
        thr2 = fmax(thr * thr, 1e-300);
    }
    // right-looking Cholesky in place: row k of M becomes row k of R
    for (int k = 0; k < c; ++k) {
        const double d = M[k * c + k];
        const bool ok = d > thr2;
        const double rkk = ok ? sqrt(d) : 1.0;
        __syncthreads();
        if (lane == 0) {
            M[k * c + k] = rkk;
            if (!ok) bad = 1;
        }
        for (int j = k + 1 + lane; j < c; j += WAVE) M[k * c + j] = ok ? M[k * c + j] / rkk : 0.0;
        __syncthreads();
        // trailing update of the upper triangle: M[i][j] -= R[k][i] R[k][j]
        for (int t = lane; t < cc; t += WAVE) {
            const int i = t / c, j = t % c;
            if (i > k && j >= i) M[t] -= M[k * c + i] * M[k * c + j];
        }
        __syncthreads();
    }
    // lower triangle of R is zero
    for (int t = lane; t < cc; t += WAVE)
        if (t / c > t % c) M[t] = 0.0;
    __syncthreads();
    if (bad) {
        if (lane == 0) *status = pass == 1 ? 1.0 : 2.0;
        return;
    }
    // Ri = R^{-1}: lane j solves for column j by back substitution
    if (lane < c) {
        const int j = lane;
        for (int i = c - 1; i >= 0; --i) {
            double t = (i == j) ? 1.0 : 0.0;
            if (i <= j)
                for (int k = i + 1; k <= j; ++k) t -= M[i * c + k] * T[k * c + j];
            T[i * c + j] = i <= j ? t / M[i * c + i] : 0.0;
        }
    }
    __syncthreads();
    double *Rk = pass == 1 ? e.R1 : e.R2;
    for (int t = lane; t < cc; t += WAVE) {
        Rk[t] = M[t];
        e.Ri[t] = T[t];
    }
    if (pass == 1) {
        if (lane == 0) *status = 0.0;
        return;
    }
    // S_j = R2 R1 (both upper triangular)
    double *Sj = out + cc;
    for (int t = lane; t < cc; t += WAVE) {
        const int i = t / c, j = t % c;
        double acc = 0.0;
        for (int k = i; k <= j; ++k) acc += M[i * c + k] * e.R1[k * c + j];
        Sj[t] = acc;
    }
}

// W <- W Ri row by row (one row per thread).  final: the result is the new
// basis block Q_{j+1}: it goes to the basis columns k .. k + c - 1 (when
// they exist) and to the next filter input (FP64 and, if present, FP32).
template <int CM, bool EXACT>
__global__ __launch_bounds__(256) void seg_rscale_kernel(const OrthSeg *__restrict__ tab,
                                                         const int *__restrict__ pre, int nseg, int c, int final_) {
    const int seg = seg_of(pre, nseg, blockIdx.x);
    const OrthSeg &e = tab[seg];
    if (flagged(e, c)) return;
    const int row = (blockIdx.x - pre[seg]) * 256 + threadIdx.x;
    if (row >= e.n) return;
    double x[CM], y[CM];
    const auto w = as_global(e.W) + (int64_t)row * c;
#pragma unroll
    for (int j = 0; j < CM; ++j) x[j] = (EXACT || j < c) ? w[j] : 0.0;
    const auto Ri = as_global(e.Ri);
#pragma unroll
    for (int j = 0; j < CM; ++j) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i <= j; ++i)
            if (EXACT || j < c) t = fma(x[i], Ri[i * c + j], t);
        y[j] = t;
    }
    if (!final_) {
        const auto wo = as_global_mut(e.W) + (int64_t)row * c;
#pragma unroll
        for (int j = 0; j < CM; ++j)
            if (EXACT || j < c) wo[j] = y[j];
        return;
    }
    if (e.k + c <= e.qcap) {
#pragma unroll
        for (int j = 0; j < CM; ++j)
            if (EXACT || j < c) as_global_mut(const_cast<double *>(col_base(e.Q, e.k + j)))[(int64_t)row * e.Q.ld] = y[j];
    }
    const auto vo = as_global_mut(e.Vin) + (int64_t)row * c;
#pragma unroll
    for (int j = 0; j < CM; ++j)
        if (EXACT || j < c) vo[j] = y[j];
    if (e.V32) {
        const auto fo = as_global_mut(e.V32) + (int64_t)row * c;
#pragma unroll
        for (int j = 0; j < CM; ++j)
            if (EXACT || j < c) fo[j] = (float)y[j];
    }
}

template <int CM, bool EXACT>
hipError_t launch_seg_orth_t(const OrthPlan &p, int c, hipStream_t s) {
    const OrthSeg *tab = p.tab;
    const int ns = p.nseg;
    const int *pre[kOrthKinds];
    for (int t = 0; t < kOrthKinds; ++t) pre[t] = p.pre + (size_t)t * ns;
    for (int pass = 0; pass < 2; ++pass) {
        if (p.blocks[kOrthFma] > 0)
            hipLaunchKernelGGL((seg_tn_fma_kernel<CM, EXACT>), dim3(p.blocks[kOrthFma]), dim3(256), 0, s, tab,
                               pre[kOrthFma], ns, c);
        if (p.blocks[kOrthMfma] > 0)
            hipLaunchKernelGGL(seg_tn_mfma_kernel<false>, dim3(p.blocks[kOrthMfma]), dim3(256), 0, s, tab,
                               pre[kOrthMfma], ns, c, 0);
        hipLaunchKernelGGL(seg_reduce_kernel, dim3(p.blocks[kOrthRed]), dim3(256), 0, s, tab, pre[kOrthRed], ns, c,
                           pass, 0);
        hipLaunchKernelGGL(seg_nn_kernel, dim3(p.blocks[kOrthRows]), dim3(256), 0, s, tab, pre[kOrthRows], ns, c,
                           pass);
    }
    for (int pass = 1; pass <= 2; ++pass) {
        const int chk = pass == 2;
        hipLaunchKernelGGL(seg_tn_mfma_kernel<true>, dim3(p.blocks[kOrthGram]), dim3(256), 0, s, tab,
                           pre[kOrthGram], ns, c, chk);
        hipLaunchKernelGGL(seg_reduce_kernel, dim3(p.blocks[kOrthGred]), dim3(256), 0, s, tab, pre[kOrthGred], ns,
                           c, 2, chk);
        hipLaunchKernelGGL(seg_chol_kernel, dim3(ns), dim3(WAVE), 0, s, tab, c, pass);
        hipLaunchKernelGGL((seg_rscale_kernel<CM, EXACT>), dim3(p.blocks[kOrthRows]), dim3(256), 0, s, tab,
                           pre[kOrthRows], ns, c, pass == 2 ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_seg_orth(const OrthPlan &p, int c, hipStream_t s) {
    if (p.nseg <= 0) return hipSuccess;
    switch (c) {
    case 1: return launch_seg_orth_t<1, true>(p, c, s);
    case 2: return launch_seg_orth_t<2, true>(p, c, s);
    case 3: return launch_seg_orth_t<4, false>(p, c, s);
    case 4: return launch_seg_orth_t<4, true>(p, c, s);
    case 5: case 6: case 7: return launch_seg_orth_t<8, false>(p, c, s);
    case 8: return launch_seg_orth_t<8, true>(p, c, s);
    case 16: return launch_seg_orth_t<16, true>(p, c, s);
    default:
        if (c >= 9 && c <= 15) return launch_seg_orth_t<16, false>(p, c, s);
        return hipErrorInvalidValue;
    }
}

}  // namespace flp
