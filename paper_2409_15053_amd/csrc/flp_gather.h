// Row gathers of the sparse-matrix-times-block kernels (the filter steps
// and the polish recurrence): for one matrix row, acc = sum over its
// nonzeros, in their CSR order, of val * X[col, c0 .. c0 + VEC), with the
// row's LPR lanes each owning VEC consecutive columns of the block.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "flp_device.h"
#include "flp_internal.h"

namespace flp {
namespace {

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
// change.  kWinHalo: the fixed window's reach (flp_internal.h).

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
    // The window may sit in a ring of wring rows (the sliding window of a
    // workgroup that walks consecutive tiles): row wlo + j is at ring row
    // (wpos + j) mod wring.  A plain window has wpos = 0 and no wrap.
    int wpos = 0, wring = 1 << 30;
    __device__ __forceinline__ int ring_row(int j) const {
        const int p = wpos + j;
        return p >= wring ? p - wring : p;
    }
    __device__ __forceinline__ void load(int col, T (&v)[VEC]) const {
        if constexpr (WIN) {
            const unsigned j = (unsigned)(col - wlo);
            if (j < wlen) {
                load_vec_lds<T, VEC>(win + ring_row((int)j) * ld + c0, v);
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
            const int j = xs.ring_row(inw[u] ? cc[u] - xs.wlo : 0);
            load_vec_lds<T, VEC>(xs.win + j * xs.ld + xs.c0, l);
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                // select the values, not their addresses (a select of two
                // array elements' addresses keeps the arrays in scratch)
                const T lv = l[v], gv = xv[u][v];
                acc[v] = fma(aa[u], inw[u] ? lv : gv, acc[v]);
            }
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

}  // namespace
}  // namespace flp
