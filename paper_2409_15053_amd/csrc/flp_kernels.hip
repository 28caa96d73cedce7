// Device kernels of the filtered Lanczos procedure for gfx950 (CDNA4).
//
// * cheb_step: one Clenshaw step of the filter (Section 2.2) as a CSR SpMM
//   over a row-major block of r vectors with the affine map and the
//   three-term update fused into the epilogue.
// * gemm_tn / gemm_nn: the tall-skinny products of the full
//   reorthogonalisation (Section 3.2.2): the update and wide projections on
//   FP64 MFMA (16x16x4), the projection against at most 16 columns on FMA
//   (2 flops per byte: bandwidth-bound either way).
// * small helpers: Gershgorin bounds, counter-based normal generator,
//   block copies, residual norms.
#include "flp_internal.h"

#include <algorithm>

namespace flp {

namespace {

constexpr int WAVE = 64;
constexpr int NXCD = 8;

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Renumber so that each XCD receives one contiguous range of tiles:
// neighbouring rows of the matrix then share that XCD's L2 for the gathered
// vector entries.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    int q = G / NXCD, rem = G % NXCD;
    int x = b % NXCD, s = b / NXCD;
    return (x < rem) ? x * (q + 1) + s : rem * (q + 1) + (x - rem) * q + s;
}

template <typename T, int VEC>
struct Vec;
template <>
struct Vec<double, 1> {
    using type = double;
};
template <>
struct Vec<double, 2> {
    using type = double2;
};
template <>
struct Vec<float, 1> {
    using type = float;
};
template <>
struct Vec<float, 2> {
    using type = float2;
};
template <>
struct Vec<float, 4> {
    using type = float4;
};

// Loads and stores of VEC consecutive elements in 16-byte (or narrower)
// pieces; the address is aligned to min(16, VEC * sizeof(T)) bytes.
template <typename T, int VEC>
__device__ __forceinline__ void load_vec(const T *p, T (&v)[VEC]) {
    constexpr int C = 16 / (int)sizeof(T);
    if constexpr (VEC > C) {
        static_assert(VEC % C == 0, "vector width must be a multiple of 16 bytes");
#pragma unroll
        for (int k = 0; k < VEC / C; ++k) {
            T t[C];
            load_vec<T, C>(p + k * C, t);
#pragma unroll
            for (int j = 0; j < C; ++j) v[k * C + j] = t[j];
        }
    } else {
        using V = typename Vec<T, VEC>::type;
        V x = *reinterpret_cast<const V *>(p);
        if constexpr (VEC == 1) {
            v[0] = x;
        } else if constexpr (VEC == 2) {
            v[0] = x.x;
            v[1] = x.y;
        } else {
            v[0] = x.x;
            v[1] = x.y;
            v[2] = x.z;
            v[3] = x.w;
        }
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_vec(T *p, const T (&v)[VEC]) {
    constexpr int C = 16 / (int)sizeof(T);
    if constexpr (VEC > C) {
        static_assert(VEC % C == 0, "vector width must be a multiple of 16 bytes");
#pragma unroll
        for (int k = 0; k < VEC / C; ++k) {
            T t[C];
#pragma unroll
            for (int j = 0; j < C; ++j) t[j] = v[k * C + j];
            store_vec<T, C>(p + k * C, t);
        }
    } else {
        using V = typename Vec<T, VEC>::type;
        V x;
        if constexpr (VEC == 1) {
            x = v[0];
        } else if constexpr (VEC == 2) {
            x.x = v[0];
            x.y = v[1];
        } else {
            x.x = v[0];
            x.y = v[1];
            x.z = v[2];
            x.w = v[3];
        }
        *reinterpret_cast<V *>(p) = x;
    }
}

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

// acc += sum over the row's nonzeros p0..p1-1 of val[p] * X[colind[p], c0 ..
// c0 + VEC), in order.  The nonzeros go in groups of UNR with every load of
// a group issued before its products: a slot past the row's end re-reads the
// row's last entry (a valid, cached address) with weight zero, so a short row
// costs one round of dependent loads instead of one per leftover nonzero.
template <typename T, int VEC, int UNR>
__device__ __forceinline__ void row_gather(int p0, int p1, const int32_t *__restrict__ colind,
                                           const T *__restrict__ val, const T *__restrict__ X, int ldx, int c0,
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
        for (int u = 0; u < UNR; ++u) load_vec<T, VEC>(X + (int64_t)cc[u] * ldx + c0, xv[u]);
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

// LPR lanes share one matrix row; lane `sub` owns columns
// [sub*VEC, sub*VEC + VEC) of the block.  All lanes of a row walk the row's
// nonzeros together (the column index and value loads of a row coalesce to
// one request), and each gathers its VEC contiguous entries of X[col, :].
template <typename T, typename Tout, int LPR, int VEC, bool NT>
__global__ __launch_bounds__(256) void cheb_step_kernel(
    int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
    const T *__restrict__ val, int r, const T *__restrict__ X, int ldx, const T *__restrict__ V,
    int ldv, const T *__restrict__ Y, int ldy, Tout *__restrict__ out, int ldo, T alpha, T beta,
    T gamma, T delta) {
    constexpr int RPB = 256 / LPR;  // rows per block
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int row = tile * RPB + threadIdx.x / LPR;
    const int sub = threadIdx.x % LPR;
    const int c0 = sub * VEC;
    if (row >= n || c0 >= r) return;
    const int p0 = rowptr[row], p1 = rowptr[row + 1];
    T acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = T(0);
    row_gather<T, VEC, Unroll<T, VEC>::value>(p0, p1, colind, val, X, ldx, c0, acc);
    T xr[VEC];
    load_vec<T, VEC>(X + (int64_t)row * ldx + c0, xr);
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

template <typename T, typename Tout, int LPR, int VEC, bool NT>
hipError_t cheb_launch(int n, const int32_t *rowptr, const int32_t *colind, const T *val, int r,
                       const T *X, int ldx, const T *V, int ldv, const T *Y, int ldy, Tout *out,
                       int ldo, T alpha, T beta, T gamma, T delta, hipStream_t s) {
    constexpr int RPB = 256 / LPR;
    int grid = (n + RPB - 1) / RPB;
    hipLaunchKernelGGL((cheb_step_kernel<T, Tout, LPR, VEC, NT>), dim3(grid), dim3(256), 0, s, n, rowptr,
                       colind, val, r, X, ldx, V, ldv, Y, ldy, out, ldo, alpha, beta, gamma, delta);
    return hipGetLastError();
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

std::vector<StepShape> step_shape_candidates(int r, bool fp32) {
    std::vector<StepShape> out;
    for (int nt : {0, 1})
        for (int vec : {2, 4, 8})
            if (r % vec == 0 && shape_has_kernel(fp32, r / vec, vec)) out.push_back(StepShape{r / vec, vec, nt});
    return out;
}

bool step_shape_ok(int r, bool fp32, StepShape sh) {
    return sh.lpr > 0 && sh.lpr * sh.vec == r && shape_has_kernel(fp32, sh.lpr, sh.vec);
}

template <typename T, typename Tout>
hipError_t launch_cheb_step(int n, const int32_t *rowptr, const int32_t *colind, const T *val, int r,
                            const T *X, int ldx, const T *V, int ldv, const T *Y, int ldy, Tout *out,
                            int ldo, T alpha, T beta, T gamma, T delta, hipStream_t s, StepShape sh) {
    if (n <= 0) return hipSuccess;
    constexpr bool F32 = sizeof(T) == 4;
    // vector loads need every leading dimension and base aligned to 16 bytes
    constexpr int V16 = 16 / (int)sizeof(T);
    auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    bool aligned16 = (ldx % V16 == 0) && (!V || ldv % V16 == 0) && (!Y || ldy % V16 == 0) &&
                     (ldo % V16 == 0) && (sizeof(Tout) == sizeof(T)) && al(X) && al(V) && al(Y) && al(out);
#define FLP_CHEB_NT(LPR, VEC, NT) \
    return cheb_launch<T, Tout, LPR, VEC, NT>(n, rowptr, colind, val, r, X, ldx, V, ldv, Y, ldy, out, ldo, alpha, beta, gamma, delta, s)
#define FLP_CHEB(LPR, VEC) FLP_CHEB_NT(LPR, VEC, false)
    if (aligned16 && r % V16 == 0) {
        if (!step_shape_ok(r, F32, sh)) sh = default_step_shape(r, F32);
        const int lpr = sh.lpr, vec = sh.vec;
        const bool nt = sh.nt != 0;
#define FLP_TRY(L, VV) \
    if (lpr == L && vec == VV) {        \
        if (nt) {                       \
            FLP_CHEB_NT(L, VV, true);   \
        } else {                        \
            FLP_CHEB_NT(L, VV, false);  \
        }                               \
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
#undef FLP_CHEB_NT
    return hipErrorInvalidValue;
}

template hipError_t launch_cheb_step<double, double>(int, const int32_t *, const int32_t *, const double *, int,
                                                     const double *, int, const double *, int, const double *,
                                                     int, double *, int, double, double, double, double,
                                                     hipStream_t, StepShape);
template hipError_t launch_cheb_step<float, float>(int, const int32_t *, const int32_t *, const float *, int,
                                                   const float *, int, const float *, int, const float *, int,
                                                   float *, int, float, float, float, float, hipStream_t,
                                                   StepShape);
template hipError_t launch_cheb_step<float, double>(int, const int32_t *, const int32_t *, const float *, int,
                                                    const float *, int, const float *, int, const float *, int,
                                                    double *, int, float, float, float, float, hipStream_t,
                                                    StepShape);

// ------------------------------------------------------------------ segmented filter step
//
// One launch advances the filters of many independent solves by one
// Clenshaw step: the launch's tiles are split into segments (one per solve,
// each with its own matrix, vectors and coefficients) by a prefix sum of
// tile counts; a block finds its segment by binary search and then runs the
// same row mapping and fused epilogue as cheb_step_kernel.

namespace {

template <typename T, int LPR, int VEC, bool NT>
__global__ __launch_bounds__(256) void cheb_seg_kernel(const SegEntry *__restrict__ tab, int nseg) {
    constexpr int RPB = 256 / LPR;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
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
    if (row >= n) return;
    const int32_t *__restrict__ rowptr = e.rowptr;
    const int32_t *__restrict__ colind = e.colind;
    const T *__restrict__ val = (const T *)e.val;
    const T *__restrict__ X = (const T *)e.X;
    const int ldx = e.ldx;
    const int p0 = rowptr[row], p1 = rowptr[row + 1];
    T acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = T(0);
    row_gather<T, VEC, Unroll<T, VEC>::value>(p0, p1, colind, val, X, ldx, c0, acc);
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
    if (d.lpr > 0) return d;
    const int l = r == 1 ? 1 : (r == 2 ? 2 : (r <= 4 ? 4 : (r <= 8 ? 8 : (r <= 16 ? 16 : 32))));
    return StepShape{l, 1};
}

int seg_rows_per_tile(int r, bool fp32, StepShape sh) { return 256 / seg_shape(r, fp32, sh).lpr; }

hipError_t launch_cheb_seg(bool fp32, int r, const SegEntry *tab, int nseg, int total_tiles, hipStream_t s,
                           StepShape sh) {
    if (nseg <= 0 || total_tiles <= 0) return hipSuccess;
    sh = seg_shape(r, fp32, sh);
    const int lpr = sh.lpr, vec = sh.vec;
    const bool nt = sh.nt != 0;
#define FLP_SEG_NT(T, LPR, VEC, NT) \
    { \
        hipLaunchKernelGGL((cheb_seg_kernel<T, LPR, VEC, NT>), dim3(total_tiles), dim3(256), 0, s, tab, nseg); \
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

// ------------------------------------------------------------------ MFMA helpers
//
// v_mfma_f64_16x16x4f64: D(16x16) = A(16x4) B(4x16) + C.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it holds D[l/16 + 4 v][l % 16]
// for v = 0..3 (rows interleaved across the four lane groups; checked on
// gfx950 with a one-hot probe).

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ const double *col_base(const DMat &m, int q) {
    return m.p + (int64_t)(q >> m.lpw) * m.ps + (q & ((1 << m.lpw) - 1));
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
        double2 av[2][NP];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int row = g + u * 16 + kr;
            const int rc = min(row, r1 - 1);
            const double x = B[(int64_t)rc * ldb + bcol];
            bv[u] = row < r1 ? x : 0.0;
            const double *ar = abase + (int64_t)rc * lda;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if constexpr (VEC) {
                    av[u][p] = *reinterpret_cast<const double2 *>(ar + aoff[p][0]);
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

template <int NT>
__global__ __launch_bounds__(256) void gemm_tn_partial_kernel(int n, int K, int c, int chunk_rows, DMat A,
                                                              const double *__restrict__ B, int64_t ldb,
                                                              double *__restrict__ partials, bool aligned) {
    __shared__ double red[4][4][WAVE];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int ntb = (c + 15) / 16;            // B tiles
    const int chunk = blockIdx.x;
    const int tg = blockIdx.y / ntb;          // group of NT A tiles
    const int tb = blockIdx.y % ntb;          // B tile
    const int r0 = chunk * chunk_rows;
    const int r1 = min(n, r0 + chunk_rows);
    const int kr = lane / 16, mc = lane % 16;
    const int q0 = tg * NT * 16;
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
    double *dst = partials + (size_t)chunk * K * c;
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
            if (i < K && j < c) dst[(size_t)i * c + j] = s;
        }
        __syncthreads();
    }
}

// Sum of the per-chunk partials in a fixed order (deterministic): each
// block owns 64 outputs; its 4 thread rows split the chunks and combine
// through LDS.
__global__ __launch_bounds__(256) void reduce_partials_kernel(int nchunks, int total, int c,
                                                              const double *__restrict__ partials,
                                                              double *__restrict__ C, int ldc) {
    __shared__ double red[4][64];
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    const int o = blockIdx.x * 64 + tx;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (o < total) {
        const double *p = partials + o;
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

// C = beta C + alpha A B: each wave computes MT row tiles (16 rows each) x
// NT column tiles (16 columns each).  The k index inside a group of 16 is
// permuted (k = 4 * (l/16) + step) so each lane reads 4 contiguous A
// entries with two 16-byte loads.  A group of 16 k values never straddles a
// panel.  Loads are unconditional: rows past n and columns past c are
// clamped (they only feed outputs that are not written) and B rows past K
// are zeroed.  A and C may be the same block (in-place C = A B): each wave
// reads all of its rows of A before it writes those rows of C.
template <int MT, int NT>
__global__ __launch_bounds__(256) void gemm_nn_kernel(int n, int K, int c, double alpha, DMat A,
                                                      const double *__restrict__ B, int64_t ldb, double beta,
                                                      double *C, int64_t ldc, bool vec_a) {
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int nct = (c + 16 * NT - 1) / (16 * NT);
    const int wg = xcd_tile(blockIdx.x, gridDim.x);
    const int rblk = wg / nct, cblk = wg % nct;
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
        const double *abase = col_base(A, kb);
        double a[MT][4];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const double *ap = abase + roff[i];
            double2 x0 = *reinterpret_cast<const double2 *>(ap);
            double2 x1 = *reinterpret_cast<const double2 *>(ap + 2);
            a[i][0] = x0.x;
            a[i][1] = x0.y;
            a[i][2] = x1.x;
            a[i][3] = x1.y;
        }
        double b[4][NT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < NT; ++j) b[q][j] = B[(int64_t)(kb + q) * ldb + col[j]];
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
            const double *ap = col_base(A, kk);
#pragma unroll
            for (int i = 0; i < MT; ++i) a[i][q] = ap[roff[i]];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const double x = B[(int64_t)kk * ldb + col[j]];
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
                    double *cp = C + (int64_t)row * ldc + cj;
                    double prev = (beta != 0.0) ? beta * *cp : 0.0;
                    *cp = prev + alpha * acc[i][j][v];
                }
            }
        }
}

}  // namespace

namespace {

// C partial (K x c, c <= C) over one chunk of rows without MFMA: thread q
// owns column q of A and accumulates its c dot products with B over the
// chunk's rows in order.  The B row is the same for the whole block (the
// rows are walked in step), so it is read through the scalar cache; the A
// loads of a wave are 64 consecutive doubles of one row.  With c <= 16
// this product does 2c flops per 8-byte A element, far below what the FMA
// units sustain at HBM speed, so it needs no matrix cores.
template <int C, int UNR>
__global__ __launch_bounds__(256) void gemm_tn_fma_kernel(int n, int K, int c, int chunk_rows, DMat A,
                                                          const double *__restrict__ B, int64_t ldb,
                                                          double *__restrict__ partials) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int chunk = blockIdx.y;
    const int r0 = chunk * chunk_rows, r1 = min(n, r0 + chunk_rows);
    const double *col = col_base(A, min(q, K - 1));
    const int64_t lda = A.ld;
    double acc[C];
#pragma unroll
    for (int j = 0; j < C; ++j) acc[j] = 0.0;
    int row = r0;
    for (; row + UNR <= r1; row += UNR) {
        double a[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) a[u] = col[(int64_t)(row + u) * lda];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const double *b = B + (int64_t)(row + u) * ldb;
#pragma unroll
            for (int j = 0; j < C; ++j) acc[j] = fma(a[u], j < c ? b[min(j, c - 1)] : 0.0, acc[j]);
        }
    }
    for (; row < r1; ++row) {
        const double a = col[(int64_t)row * lda];
        const double *b = B + (int64_t)row * ldb;
#pragma unroll
        for (int j = 0; j < C; ++j) acc[j] = fma(a, j < c ? b[min(j, c - 1)] : 0.0, acc[j]);
    }
    if (q < K) {
        double *d = partials + ((size_t)chunk * K + q) * c;
#pragma unroll
        for (int j = 0; j < C; ++j)
            if (j < c) d[j] = acc[j];
    }
}

}  // namespace

TnPlan plan_tn(int n, int K, int c) {
    TnPlan p;
    if (c <= 16) {
        // FMA path: about 2048 blocks of 256 columns x chunk_rows rows, the
        // partial buffer kept near 32M doubles at most
        const int ncb = (K + 255) / 256;
        int nch = std::max(1, std::min(2048, 2048 / ncb));
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
                                  double *partials, hipStream_t s) {
    if (c <= 16) {
        dim3 grid((K + 255) / 256, pl.nchunks);
        if (c <= 4)
            hipLaunchKernelGGL((gemm_tn_fma_kernel<4, 8>), grid, dim3(256), 0, s, n, K, c, pl.chunk_rows, A, B, ldb,
                               partials);
        else if (c <= 8)
            hipLaunchKernelGGL((gemm_tn_fma_kernel<8, 8>), grid, dim3(256), 0, s, n, K, c, pl.chunk_rows, A, B, ldb,
                               partials);
        else
            hipLaunchKernelGGL((gemm_tn_fma_kernel<16, 4>), grid, dim3(256), 0, s, n, K, c, pl.chunk_rows, A, B,
                               ldb, partials);
        return hipGetLastError();
    }
    // 16-byte A loads need an even leading dimension and panel stride
    const bool aligned = !(A.ld & 1) && !(A.ps & 1) && !(reinterpret_cast<uintptr_t>(A.p) & 15);
    const int nt = K <= 32 ? 2 : (K <= 64 ? 4 : 8);
    dim3 grid(pl.nchunks, ((K + 16 * nt - 1) / (16 * nt)) * ((c + 15) / 16));
#define FLP_TN(NT) \
    hipLaunchKernelGGL((gemm_tn_partial_kernel<NT>), grid, dim3(256), 0, s, n, K, c, pl.chunk_rows, A, B, ldb, partials, \
                       aligned)
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
                                  hipStream_t s) {
    int total = K * c;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((total + 63) / 64), dim3(256), 0, s, pl.nchunks, total, c,
                       partials, C, ldc);
    return hipGetLastError();
}

hipError_t launch_gemm_nn(int n, int K, int c, double alpha, DMat A, const double *B, int64_t ldb, double beta,
                          double *C, int64_t ldc, hipStream_t s) {
    if (n <= 0 || c <= 0) return hipSuccess;
    bool vec_a = (A.ld % 2 == 0) && (A.ps % 2 == 0) && ((reinterpret_cast<uintptr_t>(A.p) & 15) == 0);
    if (c <= 16) {
        constexpr int MT = 4, NT = 1;
        int rblocks = (n + 4 * 16 * MT - 1) / (4 * 16 * MT);
        hipLaunchKernelGGL((gemm_nn_kernel<MT, NT>), dim3(rblocks), dim3(256), 0, s, n, K, c, alpha, A, B, ldb, beta,
                           C, ldc, vec_a);
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

}  // namespace

int gershgorin_blocks(int n) { return (n + 255) / 256; }

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

hipError_t launch_transpose_out(int n, int c, const double *src, int64_t lds, double *dst, hipStream_t s) {
    if (n <= 0 || c <= 0) return hipSuccess;
    dim3 grid((n + 31) / 32, (c + 31) / 32);
    hipLaunchKernelGGL(transpose_out_kernel, grid, dim3(256), 0, s, n, c, src, lds, dst);
    return hipGetLastError();
}

}  // namespace flp
