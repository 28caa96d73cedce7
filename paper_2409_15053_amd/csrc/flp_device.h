// Device-side helpers shared by the filter and the Gram-Schmidt kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace flp {
namespace {

constexpr int WAVE = 64;
constexpr int NXCD = 8;

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Renumber so that each XCD receives one contiguous range of tiles:
// neighbouring rows of the matrix then share that XCD's L2 for the gathered
// vector entries.
__host__ __device__ __forceinline__ int xcd_tile(int b, int G) {
    int q = G / NXCD, rem = G % NXCD;
    int x = b % NXCD, s = b / NXCD;
    return (x < rem) ? x * (q + 1) + s : rem * (q + 1) + (x - rem) * q + s;
}

// Pencil walk over planes of PT consecutive tiles (PT >= NXCD): the tiles
// form Z = G / PT planes (the z-planes of a 3D grid when PT tiles hold one
// N^2 plane of rows) plus a tail.  Each plane is cut into NXCD column ranges
// (pencils); the enumeration takes pencil 0 plane by plane, then pencil 1,
// ..., then the tail in order, and XCD x receives one contiguous stretch of
// it (the positions xcd_tile gives its blocks).  An XCD thus walks its
// pencil through the planes: a row's neighbours in the planes below and
// above (the +-N^2, +-2N^2 columns of a stencil) were gathered by the same
// XCD a few planes earlier, and the few planes of its pencil in flight fit
// that XCD's L2, where the plain row order has a whole plane per XCD step.
// Bijective on [0, G).
__host__ __device__ __forceinline__ int plane_tile(int b, int G, int PT) {
    const int e = xcd_tile(b, G);
    const int Z = G / PT;
    if (PT < NXCD || Z == 0 || e >= Z * PT) return e;
    const int col = e / Z;                    // Z lo(p) <= e < Z lo(p+1)  <=>  lo(p) <= e / Z < lo(p+1)
    const int pc = (NXCD * col + NXCD - 1) / PT, p = pc < NXCD - 1 ? pc : NXCD - 1;
    const int lo = p * PT / NXCD, w = (p + 1) * PT / NXCD - lo;
    const int local = e - Z * lo;
    return (local / w) * PT + lo + local % w;
}

// The tile a block processes.  chunk == 0: xcd_tile (one contiguous range of
// tiles per XCD).  chunk > 0: the tiles are cut into chunks of `chunk`
// consecutive tiles dealt to the XCDs in turn (chunk q on XCD q % 8).
// Blocks dispatched together then cover one contiguous stretch of rows on
// all XCDs at once, so rows far apart in a row's neighbour list (a 3D
// grid's +-plane neighbours) are gathered while still in the shared
// Infinity Cache, and rows up to a chunk apart share an XCD's L2.  The last
// G mod (8 chunk) tiles keep block order.  chunk < 0: plane_tile with planes
// of -chunk matrix rows (rows_per_tile rows per tile).  Bijective on [0, G).
__host__ __device__ __forceinline__ int chunk_tile(int b, int G, int chunk, int rows_per_tile) {
    if (chunk < 0) return plane_tile(b, G, (-chunk + rows_per_tile / 2) / rows_per_tile);
    if (chunk == 0) return xcd_tile(b, G);
    const int span = NXCD * chunk;
    const int full = (G / span) * span;
    if (b >= full) return b;
    const int x = b % NXCD, s = b / NXCD;
    return (s / chunk) * span + x * chunk + s % chunk;
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

}  // namespace
}  // namespace flp
