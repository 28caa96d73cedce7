// Filter kernels of the filtered Lanczos procedure for gfx950 (CDNA4): one
// Clenshaw step of the Chebyshev filter (Section 2.2) as a CSR SpMM over a
// row-major block of r vectors, with the affine map and the three-term
// update fused into the epilogue; the segmented form advances many solves'
// filters in one launch.
#include "flp_internal.h"
#include "flp_device.h"
#include "flp_gather.h"

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

namespace flp {

namespace {

// LPR lanes share one matrix row; lane `sub` owns columns
// [sub*VEC, sub*VEC + VEC) of the block.  All lanes of a row walk the row's
// nonzeros together (the column index and value loads of a row coalesce to
// one request), and each gathers its VEC contiguous entries of X[col, :].
// SELL: rowptr holds the slice offsets and colind / val the sliced ELL
// arrays (sell_gather).
// WIN: the block first stages the rows of X it and its neighbours within
// kWinHalo rows use (stage_window) and gathers those from LDS; the shape
// must then cover exactly the r = LPR * VEC columns in 16-byte pieces.
template <typename T, typename Tout, int LPR, int VEC, bool NT, bool SELL, bool WIN>
__global__ __launch_bounds__(256) void cheb_step_kernel(
    int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
    const T *__restrict__ val, int r, const T *__restrict__ X, int ldx, const T *__restrict__ V,
    int ldv, const T *__restrict__ Y, int ldy, Tout *__restrict__ out, int ldo, T alpha, T beta,
    T gamma, T delta, int chunk) {
    constexpr int RPB = 256 / LPR;  // rows per block
    constexpr int GW = LPR * VEC;
    constexpr int WLD = GW + 16 / (int)sizeof(T);  // LDS row stride: 16 bytes of padding against bank conflicts
    const int tile = chunk_tile(blockIdx.x, gridDim.x, chunk, RPB);
    const int r0 = tile * RPB;
    const int row = r0 + threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    const int c0 = sub * VEC;
    XSource<T, VEC, WIN> xs{X, ldx, c0, nullptr, 0, WLD, 0u};
    if constexpr (WIN) {
        __shared__ T win[(RPB + 2 * kWinHalo) * WLD];
        FLP_LDS T *lwin = (FLP_LDS T *)win;
        const int wlo = max(0, r0 - kWinHalo), whi = min(n, r0 + RPB + kWinHalo);
        stage_window<T, GW, WLD, RPB + 2 * kWinHalo>(X, ldx, wlo, whi, lwin);
        __syncthreads();
        xs.win = lwin;
        xs.wlo = wlo;
        xs.wlen = (unsigned)(whi - wlo);
    }
    if (row >= n || c0 >= r) return;
    T acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = T(0);
    if constexpr (VEC > 1) {  // the aligned shapes: LPR * VEC = r, every lane of a row active
        gather_row<T, VEC, LPR, SELL, WIN>(row, sub, rowptr, colind, val, xs, acc);
    } else if constexpr (SELL) {
        const int sl = row / kSellC;
        const int o0 = rowptr[sl], o1 = rowptr[sl + 1];
        sell_gather<T, VEC, Unroll<T, VEC>::value, WIN>(o0 + row % kSellC, (o1 - o0) / kSellC, colind, val, xs,
                                                        acc);
    } else {
        const int p0 = rowptr[row], p1 = rowptr[row + 1];
        row_gather<T, VEC, Unroll<T, VEC>::value, WIN>(p0, p1, colind, val, xs, acc);
    }
    T xr[VEC];
    xs.load(row, xr);
    T res[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) res[v] = alpha * acc[v] + beta * xr[v];
    if (V) {
        T vv[VEC];
        load_stream<T, VEC, NT>(V + (int64_t)row * ldv + c0, vv);
#pragma unroll
        for (int v = 0; v < VEC; ++v) res[v] = fma(gamma, vv[v], res[v]);
    }
    if (Y) {
        T yy[VEC];
        load_stream<T, VEC, NT>(Y + (int64_t)row * ldy + c0, yy);
#pragma unroll
        for (int v = 0; v < VEC; ++v) res[v] = fma(delta, yy[v], res[v]);
    }
    if constexpr (sizeof(Tout) == sizeof(T)) {
        store_vec<Tout, VEC>(out + (int64_t)row * ldo + c0, res);
    } else {
        Tout o[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) o[v] = (Tout)res[v];
#pragma unroll
        for (int v = 0; v < VEC; ++v) out[(int64_t)row * ldo + c0 + v] = o[v];
    }
}

template <typename T, typename Tout, int LPR, int VEC, bool NT, bool WIN>
hipError_t cheb_launch(int n, const int32_t *rowptr, const int32_t *colind, const T *val, int r,
                       const T *X, int ldx, const T *V, int ldv, const T *Y, int ldy, Tout *out,
                       int ldo, T alpha, T beta, T gamma, T delta, hipStream_t s, bool sell, int chunk) {
    constexpr int RPB = 256 / LPR;
    int grid = (n + RPB - 1) / RPB;
    if (sell)
        hipLaunchKernelGGL((cheb_step_kernel<T, Tout, LPR, VEC, NT, true, WIN>), dim3(grid), dim3(256), 0, s, n,
                           rowptr, colind, val, r, X, ldx, V, ldv, Y, ldy, out, ldo, alpha, beta, gamma, delta,
                           chunk);
    else
        hipLaunchKernelGGL((cheb_step_kernel<T, Tout, LPR, VEC, NT, false, WIN>), dim3(grid), dim3(256), 0, s, n,
                           rowptr, colind, val, r, X, ldx, V, ldv, Y, ldy, out, ldo, alpha, beta, gamma, delta,
                           chunk);
    return hipGetLastError();
}

// Sliding-window form of the step for matrices whose near neighbours reach
// further than a block (a 3D grid's in-plane +-N and +-2N rows): workgroup b
// takes the rows [k L, k L + L), k = xcd_tile(b, K), in steps of RPB rows
// and keeps the rows [s - halo, s - halo + R), R = RPB + 2 halo, around its
// current step s in a ring of R rows in LDS (dynamic shared memory).  At
// each step only the RPB rows entering the window are loaded (issued before
// the step's sums, written after them into the ring slots of the rows that
// leave), so every gathered column within halo rows of the row is read from
// LDS, however many of the row's nonzeros fall there.  With L a fraction
// 1/m of a grid plane, the rows a plane above and below a row are the ones
// workgroups k +- m (on the same XCD, xcd_tile) load at the same time.
// Same sums as cheb_step_kernel.
template <typename T, typename Tout, int LPR, int VEC, bool NT, bool SELL>
__global__ __launch_bounds__(256) void cheb_slide_kernel(
    int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
    const T *__restrict__ val, int r, const T *__restrict__ X, int ldx, const T *__restrict__ V,
    int ldv, const T *__restrict__ Y, int ldy, Tout *__restrict__ out, int ldo, T alpha, T beta,
    T gamma, T delta, int halo, int range, int nranges) {
    constexpr int RPB = 256 / LPR;
    constexpr int GW = LPR * VEC;
    constexpr int WLD = GW + 16 / (int)sizeof(T);
    constexpr int E = 16 / (int)sizeof(T);
    constexpr int P = GW / E;  // 16-byte pieces per row
    constexpr int NPRE = (RPB * P + 255) / 256;
    extern __shared__ unsigned char slide_smem[];
    FLP_LDS T *ring = (FLP_LDS T *)slide_smem;
    const int R = RPB + 2 * halo;
    const int k = xcd_tile((int)blockIdx.x, nranges);
    const int r0 = k * range;
    const int r1 = min(n, r0 + range);
    if (r0 >= r1) return;  // uniform over the block
    const int sub = threadIdx.x % LPR;
    const int c0 = sub * VEC;
    int lo = r0 - halo, pos = 0;
    {  // the first window: rows [max(0, lo), min(n, lo + R)) at ring rows row - lo
        const int a = max(0, lo), cnt = (min(n, lo + R) - a) * P;
        for (int e = threadIdx.x; e < cnt; e += 256)
            *reinterpret_cast<FLP_LDS flp_f4 *>(ring + (a - lo + e / P) * WLD + (e % P) * E) =
                *reinterpret_cast<const flp_f4 *>(X + (int64_t)(a + e / P) * ldx + (e % P) * E);
    }
    __syncthreads();
    for (int s0 = r0; s0 < r1; s0 += RPB) {
        // rows entering the next window: [lo + R, lo + R + RPB), those below n
        const bool more = s0 + RPB < r1;
        const int nlo = lo + R;
        const int nhi = min(n, nlo + RPB);
        flp_f4 pre[NPRE];
#pragma unroll
        for (int it = 0; it < NPRE; ++it) {
            const int e = (int)threadIdx.x + 256 * it;
            const int x = nlo + e / P;
            if (more && e < RPB * P && x < nhi)
                pre[it] = *reinterpret_cast<const flp_f4 *>(X + (int64_t)x * ldx + (e % P) * E);
        }
        const int row = s0 + (int)threadIdx.x / LPR;
        if (row < r1 && c0 < r) {
            T vv[VEC], yy[VEC];
            if (V) load_stream<T, VEC, NT>(V + (int64_t)row * ldv + c0, vv);
            if (Y) load_stream<T, VEC, NT>(Y + (int64_t)row * ldy + c0, yy);
            XSource<T, VEC, true> xs{X, ldx, c0, ring, lo, WLD, (unsigned)R};
            xs.wpos = pos;
            xs.wring = R;
            T acc[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = T(0);
            gather_row<T, VEC, LPR, SELL, true>(row, sub, rowptr, colind, val, xs, acc);
            T xr[VEC];
            xs.load(row, xr);
            T res[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) res[v] = alpha * acc[v] + beta * xr[v];
            if (V) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) res[v] = fma(gamma, vv[v], res[v]);
            }
            if (Y) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) res[v] = fma(delta, yy[v], res[v]);
            }
            if constexpr (sizeof(Tout) == sizeof(T)) {
                store_vec<Tout, VEC>(out + (int64_t)row * ldo + c0, res);
            } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v) out[(int64_t)row * ldo + c0 + v] = (Tout)res[v];
            }
        }
        __syncthreads();  // every read of this window is done
        if (more) {
            // entering row nlo + i takes the ring slot of leaving row lo + i
#pragma unroll
            for (int it = 0; it < NPRE; ++it) {
                const int e = (int)threadIdx.x + 256 * it;
                const int x = nlo + e / P;
                if (e < RPB * P && x < nhi) {
                    int q = pos + (x - nlo);
                    if (q >= R) q -= R;
                    *reinterpret_cast<FLP_LDS flp_f4 *>(ring + q * WLD + (e % P) * E) = pre[it];
                }
            }
        }
        lo += RPB;
        pos += RPB;
        if (pos >= R) pos -= R;
        __syncthreads();
    }
}

// Workgroups of a sliding-window kernel that are resident at once on the
// current device (compute units x workgroups per unit at `lds` bytes of
// LDS), with the kernel's dynamic LDS limit raised to `lds` on first use.
hipError_t slide_slots(const void *kfn, size_t lds, int *slots) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, size_t>, int> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_tuple(dev, kfn, lds);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *slots = it->second;
        return hipSuccess;
    }
    int cus = 0, maxlds = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
    if (lds > (size_t)maxlds) return hipErrorInvalidValue;
    if ((e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess) return e;
    int per = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kfn, 256, lds)) != hipSuccess) return e;
    *slots = cache[key] = std::max(1, cus * std::max(1, per));
    return hipSuccess;
}

// Rows per workgroup of a sliding-window launch: a plane of `plane` rows cut
// into m equal ranges, m as large as keeps every range's workgroup resident
// at once; without planes (or with more planes than resident workgroups)
// the rows split evenly over the resident workgroups.  Rounded up to whole
// steps of rpb rows, so every step starts on a tile boundary as in
// cheb_step_kernel (a wavefront's rows then lie in one sliced ELL slice).
int slide_range(int n, int plane, int slots, int rpb) {
    int64_t L = ((int64_t)n + slots - 1) / slots;
    if (plane > 0) {
        const int64_t m = (int64_t)slots * plane / n;
        if (m >= 1) L = (plane + m - 1) / m;
    }
    return (int)std::min<int64_t>(((std::max<int64_t>(L, 1) + rpb - 1) / rpb) * rpb, INT32_MAX / 2);
}

template <typename T, typename Tout, int LPR, int VEC, bool NT>
hipError_t slide_launch(int n, const int32_t *rowptr, const int32_t *colind, const T *val, int r, const T *X,
                        int ldx, const T *V, int ldv, const T *Y, int ldy, Tout *out, int ldo, T alpha, T beta,
                        T gamma, T delta, hipStream_t s, bool sell, int halo, int plane) {
    constexpr int RPB = 256 / LPR;
    constexpr int WLD = LPR * VEC + 16 / (int)sizeof(T);
    if (halo < 0 || halo > (1 << 16)) return hipErrorInvalidValue;
    const size_t lds = sizeof(T) * (size_t)(RPB + 2 * halo) * WLD;
    auto kfn = sell ? cheb_slide_kernel<T, Tout, LPR, VEC, NT, true> : cheb_slide_kernel<T, Tout, LPR, VEC, NT, false>;
    int slots = 0;
    hipError_t e = slide_slots((const void *)kfn, lds, &slots);
    if (e != hipSuccess) return e;
    const int range = slide_range(n, plane, slots, RPB);
    const int nr = (int)(((int64_t)n + range - 1) / range);
    hipLaunchKernelGGL(kfn, dim3(nr), dim3(256), lds, s, n, rowptr, colind, val, r, X, ldx, V, ldv, Y, ldy, out,
                       ldo, alpha, beta, gamma, delta, halo, range, nr);
    return hipGetLastError();
}

// Sliced ELL copy of a CSR matrix: thread t fills slot t % kSellC of slice
// t / kSellC (its row's nonzeros in order, then zero weights on the row's
// own column; slots past row n - 1 get column 0 and weight 0).  val64 /
// val32 (either may be null) receive the FP64 / FP32 values.
__global__ __launch_bounds__(256) void sell_fill_kernel(int n, int nslots, const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colind,
                                                        const double *__restrict__ v64,
                                                        const float *__restrict__ v32, const int32_t *__restrict__ off,
                                                        int32_t *__restrict__ col, double *__restrict__ val64,
                                                        float *__restrict__ val32) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= nslots) return;
    const int sl = t / kSellC;
    const int q0 = off[sl] + t % kSellC, w = (off[sl + 1] - off[sl]) / kSellC;
    const int p0 = t < n ? rowptr[t] : 0, len = t < n ? rowptr[t + 1] - p0 : 0;
    for (int k = 0; k < w; ++k) {
        const int q = q0 + k * kSellC;
        const bool real = k < len;
        col[q] = real ? colind[p0 + k] : (t < n ? t : 0);
        if (val64) val64[q] = real ? v64[p0 + k] : 0.0;
        if (val32) val32[q] = real ? v32[p0 + k] : 0.0f;
    }
}

}  // namespace

// Aligned launch shapes (LPR lanes per row x VEC columns per lane) with a
// kernel instance: FP64 in 16-, 32- and 64-byte pieces per lane, FP32 in 16-
// and 32-byte pieces.
#define FLP_SHAPES_F64(X) X(1, 2) X(2, 2) X(4, 2) X(8, 2) X(16, 2) X(1, 4) X(2, 4) X(4, 4) X(8, 4) X(1, 8) X(2, 8) X(4, 8)
#define FLP_SHAPES_F32(X) X(1, 4) X(2, 4) X(4, 4) X(8, 4) X(1, 8) X(2, 8) X(4, 8)

static bool shape_has_kernel(bool fp32, int lpr, int vec) {
#define FLP_HAS(L, V) if (lpr == L && vec == V) return true;
    if (fp32) {
        FLP_SHAPES_F32(FLP_HAS)
    } else {
        FLP_SHAPES_F64(FLP_HAS)
    }
#undef FLP_HAS
    return false;
}

StepShape default_step_shape(int r, bool fp32) {
    const int v16 = fp32 ? 4 : 2;
    if (r % v16 == 0 && shape_has_kernel(fp32, r / v16, v16)) return StepShape{r / v16, v16};
    return StepShape{0, 0};
}

std::vector<StepShape> step_shape_candidates(int r, bool fp32, bool window) {
    std::vector<StepShape> out;
    for (int win = 0; win <= (window ? 1 : 0); ++win)
        for (int nt : {0, 1})
            for (int vec : {2, 4, 8})
                if (r % vec == 0 && shape_has_kernel(fp32, r / vec, vec))
                    out.push_back(StepShape{r / vec, vec, nt, 0, win});
    return out;
}

bool step_shape_ok(int r, bool fp32, StepShape sh) {
    return sh.lpr > 0 && sh.lpr * sh.vec == r && shape_has_kernel(fp32, sh.lpr, sh.vec);
}

// One lane per column on the next power of two >= r lanes: the shape for
// block widths with no aligned kernel (the lanes past column r - 1 leave).
static StepShape one_column_shape(int r) {
    const int l = r == 1 ? 1 : (r == 2 ? 2 : (r <= 4 ? 4 : (r <= 8 ? 8 : (r <= 16 ? 16 : 32))));
    return StepShape{l, 1};
}

StepShape step_launch_shape(int r, bool fp32) {
    const int v16 = fp32 ? 4 : 2;
    if (r % v16 == 0) {
        const StepShape d = default_step_shape(r, fp32);
        if (d.lpr > 0) return d;
    }
    return one_column_shape(r);
}

template <typename T, typename Tout>
hipError_t launch_cheb_step(int n, const int32_t *rowptr, const int32_t *colind, const T *val, int r,
                            const T *X, int ldx, const T *V, int ldv, const T *Y, int ldy, Tout *out,
                            int ldo, T alpha, T beta, T gamma, T delta, hipStream_t s, StepShape sh, bool sell) {
    if (n <= 0) return hipSuccess;
    constexpr bool F32 = sizeof(T) == 4;
    // vector loads need every leading dimension and base aligned to 16 bytes
    constexpr int V16 = 16 / (int)sizeof(T);
    auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    bool aligned16 = (ldx % V16 == 0) && (!V || ldv % V16 == 0) && (!Y || ldy % V16 == 0) &&
                     (ldo % V16 == 0) && (sizeof(Tout) == sizeof(T)) && al(X) && al(V) && al(Y) && al(out);
#define FLP_CHEB_NW(LPR, VEC, NT, WIN) \
    return cheb_launch<T, Tout, LPR, VEC, NT, WIN>(n, rowptr, colind, val, r, X, ldx, V, ldv, Y, ldy, out, ldo, alpha, beta, gamma, delta, s, sell, sh.chunk)
#define FLP_CHEB(LPR, VEC) FLP_CHEB_NW(LPR, VEC, false, false)
    if (aligned16 && r % V16 == 0) {
        if (!step_shape_ok(r, F32, sh)) {
            const int chunk = sh.chunk;
            sh = default_step_shape(r, F32);
            sh.chunk = chunk;
        }
        const int lpr = sh.lpr, vec = sh.vec;
        const bool nt = sh.nt != 0, win = sh.win == 1, slide = sh.win == 2;
#define FLP_TRY(L, VV)                           \
    if (lpr == L && vec == VV) {                 \
        if (slide) {                             \
            if (nt)                              \
                return slide_launch<T, Tout, L, VV, true>(n, rowptr, colind, val, r, X, ldx, V, ldv, Y, ldy, out, ldo, alpha, beta, gamma, delta, s, sell, sh.halo, sh.chunk); \
            return slide_launch<T, Tout, L, VV, false>(n, rowptr, colind, val, r, X, ldx, V, ldv, Y, ldy, out, ldo, alpha, beta, gamma, delta, s, sell, sh.halo, sh.chunk); \
        }                                        \
        if (win) {                               \
            if (nt) {                            \
                FLP_CHEB_NW(L, VV, true, true);  \
            } else {                             \
                FLP_CHEB_NW(L, VV, false, true); \
            }                                    \
        } else if (nt) {                         \
            FLP_CHEB_NW(L, VV, true, false);     \
        } else {                                 \
            FLP_CHEB_NW(L, VV, false, false);    \
        }                                        \
    }
        if constexpr (F32) {
            FLP_SHAPES_F32(FLP_TRY)
        } else {
            FLP_SHAPES_F64(FLP_TRY)
        }
#undef FLP_TRY
    }
    if (r == 1) FLP_CHEB(1, 1);
    if (r == 2) FLP_CHEB(2, 1);
    if (r <= 4) FLP_CHEB(4, 1);
    if (r <= 8) FLP_CHEB(8, 1);
    if (r <= 16) FLP_CHEB(16, 1);
    if (r <= 32) FLP_CHEB(32, 1);
#undef FLP_CHEB
#undef FLP_CHEB_NW
    return hipErrorInvalidValue;
}

template hipError_t launch_cheb_step<double, double>(int, const int32_t *, const int32_t *, const double *, int,
                                                     const double *, int, const double *, int, const double *,
                                                     int, double *, int, double, double, double, double,
                                                     hipStream_t, StepShape, bool);
template hipError_t launch_cheb_step<float, float>(int, const int32_t *, const int32_t *, const float *, int,
                                                   const float *, int, const float *, int, const float *, int,
                                                   float *, int, float, float, float, float, hipStream_t,
                                                   StepShape, bool);
template hipError_t launch_cheb_step<float, double>(int, const int32_t *, const int32_t *, const float *, int,
                                                    const float *, int, const float *, int, const float *, int,
                                                    double *, int, float, float, float, float, hipStream_t,
                                                    StepShape, bool);

void tile_order_host(int tiles, int chunk, int rows_per_tile, int32_t *order) {
    for (int b = 0; b < tiles; ++b) order[b] = chunk_tile(b, tiles, chunk, rows_per_tile);
}

hipError_t launch_sell_fill(int n, const int32_t *rowptr, const int32_t *colind, const double *v64, const float *v32,
                            const int32_t *off, int nslices, int32_t *col, double *val64, float *val32,
                            hipStream_t s) {
    const int nslots = nslices * kSellC;
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(sell_fill_kernel, dim3((nslots + 255) / 256), dim3(256), 0, s, n, nslots, rowptr, colind, v64,
                       v32, off, col, val64, val32);
    return hipGetLastError();
}

// ------------------------------------------------------------------ segmented filter step
//
// One launch advances the filters of many independent solves by one
// Clenshaw step: the launch's tiles are split into segments (one per solve,
// each with its own matrix, vectors and coefficients) by a prefix sum of
// tile counts; a block finds its segment by binary search and then runs the
// same row mapping and fused epilogue as cheb_step_kernel.

namespace {

// Lane `sub` of a row owns columns [sub*VEC, sub*VEC + VEC); when LPR * VEC
// exceeds the block width r (the one-column-per-lane shapes for r that is
// not a power of two), lanes past column r - 1 have no column and leave.
template <typename T, int LPR, int VEC, bool NT, bool WIN>
__global__ __launch_bounds__(256) void cheb_seg_kernel(const SegEntry *__restrict__ tab, int nseg, int r,
                                                       int chunk) {
    constexpr int RPB = 256 / LPR;
    constexpr int WLD = LPR * VEC + 16 / (int)sizeof(T);
    const int tile = chunk_tile(blockIdx.x, gridDim.x, chunk > 0 ? chunk : 0, RPB);  // no plane walk across segments
    // The segment holding this tile: the tile offsets ascend, so the
    // segments starting at or before the tile are a prefix; each wave counts
    // it 64 segments at a time with one load per lane and a ballot.  The
    // count is the same on every lane, so it is made wave-uniform and the
    // segment's descriptor is then read through the scalar cache.
    const int lane = threadIdx.x % WAVE;
    int seg = -1;
    for (int base = 0; base < nseg; base += WAVE) {
        const int i = base + lane;
        const bool le = i < nseg && tab[i].tile0 <= tile;
        const unsigned long long m = __ballot(le);
        seg += __popcll(m);
        if (~m != 0ull) break;
    }
    seg = __builtin_amdgcn_readfirstlane(seg);
    const SegEntry &e = tab[seg];
    const int n = e.n;
    const int r0 = (tile - e.tile0) * RPB;
    const int row = r0 + threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    const int c0 = sub * VEC;
    const T *__restrict__ X = (const T *)e.X;
    const int ldx = e.ldx;
    XSource<T, VEC, WIN> xs{X, ldx, c0, nullptr, 0, WLD, 0u};
    if constexpr (WIN) {  // the whole block lies in one segment
        __shared__ T win[(RPB + 2 * kWinHalo) * WLD];
        FLP_LDS T *lwin = (FLP_LDS T *)win;
        const int wlo = max(0, r0 - kWinHalo), whi = min(n, r0 + RPB + kWinHalo);
        stage_window<T, LPR * VEC, WLD, RPB + 2 * kWinHalo>(X, ldx, wlo, whi, lwin);
        __syncthreads();
        xs.win = lwin;
        xs.wlo = wlo;
        xs.wlen = (unsigned)(whi - wlo);
    }
    if (row >= n || c0 >= r) return;
    const int32_t *__restrict__ rowptr = e.rowptr;
    const int32_t *__restrict__ colind = e.colind;
    const T *__restrict__ val = (const T *)e.val;
    T acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = T(0);
    if constexpr (VEC > 1) {  // aligned shapes: LPR * VEC = r
        if (e.sell)
            gather_row<T, VEC, LPR, true, WIN>(row, sub, rowptr, colind, val, xs, acc);
        else
            gather_row<T, VEC, LPR, false, WIN>(row, sub, rowptr, colind, val, xs, acc);
    } else if (e.sell) {
        const int sl = row / kSellC;
        const int o0 = rowptr[sl], o1 = rowptr[sl + 1];
        sell_gather<T, VEC, Unroll<T, VEC>::value, WIN>(o0 + row % kSellC, (o1 - o0) / kSellC, colind, val, xs,
                                                        acc);
    } else {
        const int p0 = rowptr[row], p1 = rowptr[row + 1];
        row_gather<T, VEC, Unroll<T, VEC>::value, WIN>(p0, p1, colind, val, xs, acc);
    }
    T xr[VEC];
    xs.load(row, xr);
    const T alpha = (T)e.alpha, beta = (T)e.beta, gamma = (T)e.gamma, delta = (T)e.delta;
    T res[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) res[v] = alpha * acc[v] + beta * xr[v];
    if (e.V) {
        T vv[VEC];
        load_stream<T, VEC, NT>((const T *)e.V + (int64_t)row * e.ldv + c0, vv);
#pragma unroll
        for (int v = 0; v < VEC; ++v) res[v] = fma(gamma, vv[v], res[v]);
    }
    if (e.Y) {
        T yy[VEC];
        load_stream<T, VEC, NT>((const T *)e.Y + (int64_t)row * e.ldy + c0, yy);
#pragma unroll
        for (int v = 0; v < VEC; ++v) res[v] = fma(delta, yy[v], res[v]);
    }
    if (e.out_f64) {
        double *o = (double *)e.out + (int64_t)row * e.ldo + c0;
#pragma unroll
        for (int v = 0; v < VEC; ++v) o[v] = (double)res[v];
    } else {
        store_vec<T, VEC>((T *)e.out + (int64_t)row * e.ldo + c0, res);
    }
}

}  // namespace

// Shape of the segmented kernel: the tuned or default aligned shape when
// one exists for r, else one lane per column.  seg_rows_per_tile and
// launch_cheb_seg must agree, so both resolve the shape here.
static StepShape seg_shape(int r, bool fp32, StepShape sh) {
    if (step_shape_ok(r, fp32, sh)) return sh;
    StepShape d = default_step_shape(r, fp32);
    if (d.lpr <= 0) d = one_column_shape(r);
    d.chunk = sh.chunk;
    return d;
}

int seg_rows_per_tile(int r, bool fp32, StepShape sh) { return 256 / seg_shape(r, fp32, sh).lpr; }

StepShape seg_launch_shape(int r, bool fp32, StepShape sh) { return seg_shape(r, fp32, sh); }

hipError_t launch_cheb_seg(bool fp32, int r, const SegEntry *tab, int nseg, int total_tiles, hipStream_t s,
                           StepShape sh) {
    if (nseg <= 0 || total_tiles <= 0) return hipSuccess;
    if (r < 1 || r > 32) return hipErrorInvalidValue;
    sh = seg_shape(r, fp32, sh);
    const int lpr = sh.lpr, vec = sh.vec;
    // every column needs a lane (the kernel drops lanes past column r - 1)
    if (lpr * vec < r) return hipErrorInvalidValue;
    const bool nt = sh.nt != 0;
#define FLP_SEG_NW(T, LPR, VEC, NT, WIN) \
    { \
        hipLaunchKernelGGL((cheb_seg_kernel<T, LPR, VEC, NT, WIN>), dim3(total_tiles), dim3(256), 0, s, tab, nseg, r, \
                           sh.chunk); \
        return hipGetLastError(); \
    }
#define FLP_SEG(T, LPR, VEC) FLP_SEG_NW(T, LPR, VEC, false, false)
#define FLP_SEGT(T, L, VV) \
    if (lpr == L && vec == VV) { \
        if (win) { \
            if (nt) \
                FLP_SEG_NW(T, L, VV, true, true) \
            else \
                FLP_SEG_NW(T, L, VV, false, true) \
        } else if (nt) \
            FLP_SEG_NW(T, L, VV, true, false) \
        else \
            FLP_SEG_NW(T, L, VV, false, false) \
    }
#define FLP_SEG64(L, VV) FLP_SEGT(double, L, VV)
#define FLP_SEG32(L, VV) FLP_SEGT(float, L, VV)
    const bool win = sh.win != 0;
    if (!fp32) {
        FLP_SHAPES_F64(FLP_SEG64)
        if (vec == 1) {
            if (lpr == 1) FLP_SEG(double, 1, 1);
            if (lpr == 2) FLP_SEG(double, 2, 1);
            if (lpr == 4) FLP_SEG(double, 4, 1);
            if (lpr == 8) FLP_SEG(double, 8, 1);
            if (lpr == 16) FLP_SEG(double, 16, 1);
            if (lpr == 32) FLP_SEG(double, 32, 1);
        }
    } else {
        FLP_SHAPES_F32(FLP_SEG32)
        if (vec == 1) {
            if (lpr == 1) FLP_SEG(float, 1, 1);
            if (lpr == 2) FLP_SEG(float, 2, 1);
            if (lpr == 4) FLP_SEG(float, 4, 1);
            if (lpr == 8) FLP_SEG(float, 8, 1);
            if (lpr == 16) FLP_SEG(float, 16, 1);
            if (lpr == 32) FLP_SEG(float, 32, 1);
        }
    }
#undef FLP_SEG64
#undef FLP_SEG32
#undef FLP_SEGT
#undef FLP_SEG
#undef FLP_SEG_NW
    return hipErrorInvalidValue;
}

}  // namespace flp
