// Filter kernels of the filtered Lanczos procedure for gfx950 (CDNA4): one
// Clenshaw step of the Chebyshev filter (Section 2.2) as a CSR SpMM over a
// row-major block of r vectors, with the affine map and the three-term
// update fused into the epilogue; the segmented form advances many solves'
// filters in one launch.
#include "flp_internal.h"
#include "flp_device.h"

#include <algorithm>
#include <type_traits>
#include <vector>

namespace flp {

namespace {

// ------------------------------------------------------------------ filter step
//
// Loads of the streamed operands V and U_{k+2}: with NT, nontemporal (they
// are read once per step, so they need not displace the gathered vector
// from the caches); otherwise as load_vec.
template <typename T, int VEC, bool NT>
__device__ __forceinline__ void load_stream(const T *p, T (&v)[VEC]) {
    if constexpr (NT) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[i] = __builtin_nontemporal_load(p + i);
    } else {
        load_vec<T, VEC>(p, v);
    }
}

// Where a lane reads its VEC entries of a row of the gathered block X.
// With WIN, the rows [wlo, wlo + wlen) (the block's own rows and kWinHalo
// rows on each side) were staged in LDS, ld elements apart; a column inside
// that window is read there (the LDS pipeline), any other from global memory
// (the texture address and data units, which the gathers of a stencil with
// many neighbours keep busy).  Both hold the same values, so the sums do not
// change.
constexpr int kWinHalo = 8;

#define FLP_LDS __attribute__((address_space(3)))
typedef float flp_f4 __attribute__((ext_vector_type(4)));  // a 16-byte piece

// VEC consecutive elements from LDS in 16-byte pieces (ds_read_b128).
template <typename T, int VEC>
__device__ __forceinline__ void load_vec_lds(const FLP_LDS T *p, T (&v)[VEC]) {
    static_assert(VEC * sizeof(T) % 16 == 0, "LDS window reads whole 16-byte pieces");
    constexpr int E = 16 / (int)sizeof(T);
#pragma unroll
    for (int k = 0; k < VEC / E; ++k) {
        const flp_f4 x = *reinterpret_cast<const FLP_LDS flp_f4 *>(p + k * E);
        T t[E];
        __builtin_memcpy(t, &x, 16);
#pragma unroll
        for (int j = 0; j < E; ++j) v[k * E + j] = t[j];
    }
}

template <typename T, int VEC, bool WIN>
struct XSource {
    const T *__restrict__ X;
    int ldx, c0;
    const FLP_LDS T *win;
    int wlo, ld;
    unsigned wlen;
    __device__ __forceinline__ void load(int col, T (&v)[VEC]) const {
        if constexpr (WIN) {
            const unsigned j = (unsigned)(col - wlo);
            if (j < wlen) {
                load_vec_lds<T, VEC>(win + (int)j * ld + c0, v);
                return;
            }
        }
        load_vec<T, VEC>(X + (int64_t)col * ldx + c0, v);
    }
};

// acc += sum over the row's nonzeros p0..p1-1 of val[p] * X[colind[p], c0 ..
// c0 + VEC), in order.  The nonzeros go in groups of UNR with every load of
// a group issued before its products: a slot past the row's end re-reads the
// row's last entry (a valid, cached address) with weight zero, so a short row
// costs one round of dependent loads instead of one per leftover nonzero.
template <typename T, int VEC, int UNR, bool WIN>
__device__ __forceinline__ void row_gather(int p0, int p1, const int32_t *__restrict__ colind,
                                           const T *__restrict__ val, const XSource<T, VEC, WIN> &xs,
                                           T (&acc)[VEC]) {
    for (int p = p0; p < p1; p += UNR) {
        int cc[UNR];
        T aa[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int q = min(p + u, p1 - 1);
            cc[u] = colind[q];
            const T a = val[q];
            aa[u] = (p + u < p1) ? a : T(0);
        }
        T xv[UNR][VEC];
#pragma unroll
        for (int u = 0; u < UNR; ++u) xs.load(cc[u], xv[u]);
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = fma(aa[u], xv[u][v], acc[v]);
    }
}

// nonzeros per group: 8, or 4 when each lane gathers 64 bytes per nonzero
template <typename T, int VEC>
struct Unroll {
    static constexpr int value = VEC * (int)sizeof(T) >= 64 ? 4 : 8;
};

// The same sum for a matrix in sliced ELL form (slices of kSellC rows, each
// padded to its longest row with zero weights on the row's own column;
// entry k of row `row` at q0 + k * kSellC): the row's nonzeros in their CSR
// order, so the sum is bit-identical to row_gather's.
template <typename T, int VEC, int UNR, bool WIN>
__device__ __forceinline__ void sell_gather(int q0, int w, const int32_t *__restrict__ colind,
                                            const T *__restrict__ val, const XSource<T, VEC, WIN> &xs,
                                            T (&acc)[VEC]) {
    for (int k = 0; k < w; k += UNR) {
        int cc[UNR];
        T aa[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int q = q0 + min(k + u, w - 1) * kSellC;
            cc[u] = colind[q];
            const T a = val[q];
            aa[u] = (k + u < w) ? a : T(0);
        }
        T xv[UNR][VEC];
#pragma unroll
        for (int u = 0; u < UNR; ++u) xs.load(cc[u], xv[u]);
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = fma(aa[u], xv[u][v], acc[v]);
    }
}

// Stages rows [wlo, whi) (at most ROWS of them) of X (GW columns, 16-byte
// pieces) in the LDS array win (row stride WLD elements) with all 256
// threads, every global load issued before the first LDS write.
template <typename T, int GW, int WLD, int ROWS>
__device__ __forceinline__ void stage_window(const T *__restrict__ X, int ldx, int wlo, int whi, FLP_LDS T *win) {
    constexpr int E = 16 / (int)sizeof(T);
    constexpr int P = GW / E;  // pieces per row
    constexpr int NIT = (ROWS * P + 255) / 256;
    const int cnt = (whi - wlo) * P;
    flp_f4 buf[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = (int)threadIdx.x + 256 * it;
        if (e < cnt) buf[it] = *reinterpret_cast<const flp_f4 *>(X + (int64_t)(wlo + e / P) * ldx + (e % P) * E);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = (int)threadIdx.x + 256 * it;
        if (e < cnt) *reinterpret_cast<FLP_LDS flp_f4 *>(win + (e / P) * WLD + (e % P) * E) = buf[it];
    }
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Lane J of each row's group of LPR lanes broadcast to the whole group: a
// DPP quad permute for LPR <= 4, a wave shuffle (ds_bpermute) beyond.
template <int LPR, int J>
__device__ __forceinline__ int row_bcast_i(int x) {
    if constexpr (LPR == 1) {
        return x;
    } else if constexpr (LPR == 2) {
        return __builtin_amdgcn_mov_dpp(x, J | (J << 2) | ((J + 2) << 4) | ((J + 2) << 6), 0xF, 0xF, false);
    } else if constexpr (LPR == 4) {
        return __builtin_amdgcn_mov_dpp(x, J * 0x55, 0xF, 0xF, false);
    } else {
        const int lane = (int)(threadIdx.x % WAVE);
        return __shfl(x, (lane & ~(LPR - 1)) + J, WAVE);
    }
}
template <int LPR, int J>
__device__ __forceinline__ int row_bcast(int x) {
    return row_bcast_i<LPR, J>(x);
}
template <int LPR, int J>
__device__ __forceinline__ float row_bcast(float x) {
    return __int_as_float(row_bcast_i<LPR, J>(__float_as_int(x)));
}
template <int LPR, int J>
__device__ __forceinline__ double row_bcast(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)row_bcast_i<LPR, J>((int)(unsigned)u);
    const unsigned hi = (unsigned)row_bcast_i<LPR, J>((int)(unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Slots k0 .. k0 + CNT - 1 of the row's nonzeros (slot k at entry addr(k);
// the row's last slot is kmax, later slots re-read it with weight zero),
// added to acc in slot order.  Lane `sub` reads the index and value of slots
// k0 + sub, k0 + sub + LPR, ... and row_bcast hands each slot's pair to the
// row's LPR lanes, so every nonzero's index and value pass the vector memory
// pipeline once per row rather than once per lane; every X load of the
// group is issued before its products.  WIN: columns inside the LDS window
// are read there (into separate registers, so the global loads of the group
// stay in flight) and the others from global memory; same sums.
template <typename T, int VEC, int LPR, int CNT, bool WIN, typename Addr>
__device__ __forceinline__ void gather_group(int k0, int kmax, int sub, const Addr &addr,
                                             const int32_t *__restrict__ colind, const T *__restrict__ val,
                                             const XSource<T, VEC, WIN> &xs, T (&acc)[VEC]) {
    constexpr int G = (CNT + LPR - 1) / LPR;
    int mc[G];
    T ma[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int k = k0 + sub + LPR * g;
        const int q = addr(min(k, kmax));
        mc[g] = colind[q];
        const T a = val[q];
        ma[g] = k <= kmax ? a : T(0);
    }
    int cc[CNT];
    T aa[CNT];
    static_for<0, CNT>([&](auto U) {
        constexpr int u = decltype(U)::value;
        cc[u] = row_bcast<LPR, u % LPR>(mc[u / LPR]);
        aa[u] = row_bcast<LPR, u % LPR>(ma[u / LPR]);
    });
    T xv[CNT][VEC];
    if constexpr (!WIN) {
#pragma unroll
        for (int u = 0; u < CNT; ++u) load_vec<T, VEC>(xs.X + (int64_t)cc[u] * xs.ldx + xs.c0, xv[u]);
#pragma unroll
        for (int u = 0; u < CNT; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = fma(aa[u], xv[u][v], acc[v]);
    } else {
        bool inw[CNT];
#pragma unroll
        for (int u = 0; u < CNT; ++u) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) xv[u][v] = T(0);
            inw[u] = (unsigned)(cc[u] - xs.wlo) < xs.wlen;
            if (!inw[u]) load_vec<T, VEC>(xs.X + (int64_t)cc[u] * xs.ldx + xs.c0, xv[u]);
        }
#pragma unroll
        for (int u = 0; u < CNT; ++u) {
            T l[VEC];
            const int j = inw[u] ? cc[u] - xs.wlo : 0;
            load_vec_lds<T, VEC>(xs.win + j * xs.ld + xs.c0, l);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = fma(aa[u], inw[u] ? l[v] : xv[u][v], acc[v]);
        }
    }
}

// The row's nonzeros through gather_group: sliced ELL slices have one width
// per slice, the same for every row of a wavefront, so whole groups of UNR
// slots and then one exact tail group cover them; CSR rows go in groups of
// UNR (the last one padded).
template <typename T, int VEC, int LPR, bool SELL, bool WIN>
__device__ __forceinline__ void gather_row(int row, int sub, const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ colind, const T *__restrict__ val,
                                           const XSource<T, VEC, WIN> &xs, T (&acc)[VEC]) {
    constexpr int UNR = Unroll<T, VEC>::value;
    if constexpr (SELL) {
        const int sl = row / kSellC;
        const int o0 = rowptr[sl], o1 = rowptr[sl + 1];
        const int q0 = o0 + row % kSellC;
        const int w = __builtin_amdgcn_readfirstlane((o1 - o0) / kSellC);  // one slice per wavefront
        const auto addr = [q0](int k) { return q0 + k * kSellC; };
        int k = 0;
        for (; k + UNR <= w; k += UNR) gather_group<T, VEC, LPR, UNR, WIN>(k, w - 1, sub, addr, colind, val, xs, acc);
        const int rem = w - k;
        static_for<1, UNR>([&](auto C) {
            if (rem == decltype(C)::value)
                gather_group<T, VEC, LPR, decltype(C)::value, WIN>(k, w - 1, sub, addr, colind, val, xs, acc);
        });
    } else {
        const int p0 = rowptr[row], p1 = rowptr[row + 1];
        const auto addr = [](int k) { return k; };
        for (int p = p0; p < p1; p += UNR) gather_group<T, VEC, LPR, UNR, WIN>(p, p1 - 1, sub, addr, colind, val, xs, acc);
    }
}

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
        const bool nt = sh.nt != 0, win = sh.win != 0;
#define FLP_TRY(L, VV)                           \
    if (lpr == L && vec == VV) {                 \
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
template <typename T, int LPR, int VEC, bool NT>
__global__ __launch_bounds__(256) void cheb_seg_kernel(const SegEntry *__restrict__ tab, int nseg, int r,
                                                       int chunk) {
    constexpr int RPB = 256 / LPR;
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
    const int row = (tile - e.tile0) * RPB + threadIdx.x / LPR;
    const int c0 = (threadIdx.x % LPR) * VEC;
    if (row >= n || c0 >= r) return;
    const int32_t *__restrict__ rowptr = e.rowptr;
    const int32_t *__restrict__ colind = e.colind;
    const T *__restrict__ val = (const T *)e.val;
    const T *__restrict__ X = (const T *)e.X;
    const int ldx = e.ldx;
    const XSource<T, VEC, false> xs{X, ldx, c0, nullptr, 0, 0, 0u};
    T acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = T(0);
    if (e.sell) {
        const int sl = row / kSellC;
        const int o0 = rowptr[sl], o1 = rowptr[sl + 1];
        sell_gather<T, VEC, Unroll<T, VEC>::value, false>(o0 + row % kSellC, (o1 - o0) / kSellC, colind, val, xs,
                                                          acc);
    } else {
        const int p0 = rowptr[row], p1 = rowptr[row + 1];
        row_gather<T, VEC, Unroll<T, VEC>::value, false>(p0, p1, colind, val, xs, acc);
    }
    T xr[VEC];
    load_vec<T, VEC>(X + (int64_t)row * ldx + c0, xr);
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
#define FLP_SEG_NT(T, LPR, VEC, NT) \
    { \
        hipLaunchKernelGGL((cheb_seg_kernel<T, LPR, VEC, NT>), dim3(total_tiles), dim3(256), 0, s, tab, nseg, r, \
                           sh.chunk); \
        return hipGetLastError(); \
    }
#define FLP_SEG(T, LPR, VEC) FLP_SEG_NT(T, LPR, VEC, false)
#define FLP_SEG64(L, VV) \
    if (lpr == L && vec == VV) { \
        if (nt) \
            FLP_SEG_NT(double, L, VV, true) \
        else \
            FLP_SEG_NT(double, L, VV, false) \
    }
#define FLP_SEG32(L, VV) \
    if (lpr == L && vec == VV) { \
        if (nt) \
            FLP_SEG_NT(float, L, VV, true) \
        else \
            FLP_SEG_NT(float, L, VV, false) \
    }
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
#undef FLP_SEG
#undef FLP_SEG_NT
    return hipErrorInvalidValue;
}

}  // namespace flp
