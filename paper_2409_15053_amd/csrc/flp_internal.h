// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/flp.h"

namespace flp {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
#define FLP_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            ::flp::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return FLP_E_DEVICE;                                                 \
        }                                                                        \
    } while (0)

// ---------------------------------------------------------------- host eigensolver
// Eigenvalues (ascending) of the symmetric N x N row-major M with
// semi-bandwidth bw.  Of the eigenvector matrix (columns = eigenvectors, in
// the order of evals): rows[0..nrows) are written to Zrows (nrows x N
// row-major) and columns cols[0..ncols) to Zcols (N x ncols row-major).
// Returns 0 on success.
int sym_eig(int N, int bw, const double *M, double *evals, const int *rows, int nrows, double *Zrows,
            const int *cols = nullptr, int ncols = 0, double *Zcols = nullptr);

// The rotation log of one sym_eig call, kept so eigenvector columns can be
// produced later without repeating the reduction.
struct EigRot {
    int32_t p;  // plane (p, p+1)
    double c, s;
};
struct EigLog {
    int N = 0;
    std::vector<EigRot> rot;
    std::vector<int> perm;  // sorted position -> unsorted index
    void clear() {
        N = 0;
        rot.clear();
        rot.shrink_to_fit();
        perm.clear();
    }
};
// Caps the threads one eigensolver call started from the calling thread may
// use (default 16).
void set_eig_threads(int n);

// sym_eig that also returns its rotation log in *keep
int sym_eig_keep(int N, int bw, const double *M, double *evals, const int *rows, int nrows, double *Zrows,
                 EigLog *keep);
// columns cols[0..ncols) (sorted order) of the eigenvector matrix of a kept
// log, written to Zcols (N x ncols row-major)
void eig_log_cols(const EigLog &L, const int *cols, int ncols, double *Zcols);

// ---------------------------------------------------------------- tall matrices
// A tall n x K matrix stored plainly (row-major, leading dimension ld) or
// as column panels of 2^lpw columns, each panel a row-major n x 2^lpw block
// placed ps elements after the previous one.  Element (i, q) lives at
// p[(q >> lpw) * ps + i * ld + (q & (2^lpw - 1))].
struct DMat {
    double *p;
    int64_t ld;
    int64_t ps;
    int lpw;
};
inline DMat plain_mat(const double *p, int64_t ld) { return DMat{const_cast<double *>(p), ld, 0, 30}; }
inline DMat panel_mat(const double *p, int64_t n, int lpw) {
    return DMat{const_cast<double *>(p), int64_t(1) << lpw, n << lpw, lpw};
}

// ---------------------------------------------------------------- kernel launchers
// All take a stream and return hipError_t from the launch.

// Launch shape of a filter step: lpr lanes share one matrix row and each
// owns vec consecutive columns of the block (lpr * vec = r), so a 256-thread
// block covers 256 / lpr rows; nt = 1 reads the streamed operands (V and
// U_{k+2}) with nontemporal loads.  {0, 0, 0} selects the default (16-byte
// pieces, ordinary loads).  chunk: the tile-to-XCD mapping (chunk_tile in
// flp_device.h; 0 = one contiguous range per XCD).  Every shape sums each
// output element in the same order, so all of them give bit-identical
// results.
// Rows on either side of a block's own that the fixed LDS window holds.
constexpr int kWinHalo = 8;

struct StepShape {
    int lpr = 0, vec = 0, nt = 0, chunk = 0;
    // 1: each block stages its rows of the gathered block, +-8 rows, in LDS;
    // 2: sliding window of +-halo rows per workgroup (cheb_slide_kernel),
    // chunk then being the plane length its row ranges are fitted to (0: none)
    int win = 0;
    int halo = 0;
};
// Host evaluation of the tile-to-XCD traversal the filter kernels use:
// order[b] = the row tile that block b of a `tiles`-block launch processes
// (chunk as in StepShape::chunk; rows_per_tile rows per tile).
void tile_order_host(int tiles, int chunk, int rows_per_tile, int32_t *order);
StepShape default_step_shape(int r, bool fp32);
// window: also the LDS-window variants (single-solve kernel only)
std::vector<StepShape> step_shape_candidates(int r, bool fp32, bool window);
bool step_shape_ok(int r, bool fp32, StepShape sh);

// out = alpha * (A X) + beta * X + gamma * V + delta * Y, row-major blocks of
// r columns with leading dimensions; V / Y may be NULL (their terms skipped).
// T = float or double selects the matrix values and the vector type; the
// output type is Tout.  sell: A is in sliced ELL form (rowptr = the slice
// offsets, colind / val = the sliced arrays; see launch_sell_fill).
template <typename T, typename Tout>
hipError_t launch_cheb_step(int n, const int32_t *rowptr, const int32_t *colind, const T *val,
                            int r, const T *X, int ldx, const T *V, int ldv, const T *Y, int ldy,
                            Tout *out, int ldo, T alpha, T beta, T gamma, T delta,
                            hipStream_t s, StepShape sh = StepShape{}, bool sell = false);

// Sliced ELL (SELL-C with C = kSellC rows per slice, rows in their original
// order): slice i holds entries off[i] .. off[i + 1] - 1, its width
// w_i = (off[i + 1] - off[i]) / kSellC, entry k of its row j at
// off[i] + k * kSellC + j; rows shorter than w_i are padded with weight 0 on
// their own column.  off (nslices + 1 entries, built on the host from
// rowptr) is the caller's; the fill writes col and the FP64 / FP32 values
// (val64 / val32 may be null) from the CSR arrays.
constexpr int kSellC = 64;
hipError_t launch_sell_fill(int n, const int32_t *rowptr, const int32_t *colind, const double *v64, const float *v32,
                            const int32_t *off, int nslices, int32_t *col, double *val64, float *val32,
                            hipStream_t s);

// One segment of a segmented filter step: the current Clenshaw launch of
// one solve in a batch (out = alpha AX + beta X + gamma V + delta Y).
struct SegEntry {
    const int32_t *rowptr;
    const int32_t *colind;
    const void *val;  // double or float, as the launch's type
    const void *X;
    const void *V;    // may be null
    const void *Y;    // may be null
    void *out;
    int n, tile0;     // rows; first tile of this segment in the launch
    int ldx, ldv, ldy, ldo;
    int out_f64;      // 1: output in FP64 (last step of an FP32 filter)
    int sell;         // 1: rowptr / colind / val are a sliced ELL copy (launch_sell_fill)
    double alpha, beta, gamma, delta;
};
// rows per tile of the segmented kernel for block width r and value type
int seg_rows_per_tile(int r, bool fp32, StepShape sh = StepShape{});
// the shape the segmented kernel runs for block width r: sh when it is a
// supported shape with lpr * vec = r, else the default 16-byte shape, else
// one column per lane on the next power of two >= r lanes (the lanes past
// column r - 1 leave at once)
StepShape seg_launch_shape(int r, bool fp32, StepShape sh = StepShape{});
// the untuned shape of the single-solve kernel for r columns (aligned blocks)
StepShape step_launch_shape(int r, bool fp32);
// One launch over nseg segments (tab: device array sorted by tile0).
hipError_t launch_cheb_seg(bool fp32, int r, const SegEntry *tab, int nseg, int total_tiles, hipStream_t s,
                           StepShape sh = StepShape{});

// Residual-form polish (FP32 recurrences of the divided-difference
// polynomials on the residual block, 32 columns per block; see flp_polish.hip).
// Block column j is Ritz column cols[j] (a device array); chunk: the tile-to-
// XCD mapping (chunk_tile); win: stage each block's rows of the recurrence's
// input (and 8 on each side) in LDS (StepShape::win).
int polish_block_width();
hipError_t launch_polish_resid(int n, int w, const double *X, const double *AX, int64_t ldc, const int *cols,
                               const double *lam, double inv_e, float *R32, hipStream_t s);
hipError_t launch_polish_locked(int n, int nl, const int *cols, const double *scale, const double *X, int64_t ldc,
                                double *Y, hipStream_t s);
hipError_t launch_polish_step(int n, const int32_t *rowptr, const int32_t *colind, const float *val32,
                              const float *U1, const float *U2, const float *R32, const float *coef, float a,
                              float b, float *out, hipStream_t s, bool sell = false, int chunk = 0,
                              bool win = false);
hipError_t launch_polish_last(int n, const int32_t *rowptr, const int32_t *colind, const float *val32,
                              const float *U1, const float *U2, const float *R32, const float *coef, float a,
                              float b, double *Y, int64_t ldy, int w, const double *X, int64_t ldx, const int *cols,
                              const double *ptheta, hipStream_t s, bool sell = false, int chunk = 0,
                              bool win = false);

// One solve's part of a segmented block step (full reorthogonalisation of
// the filtered block W against the basis Q, then W = Q_{j+1} S_j by
// Cholesky QR twice) with block width c <= 16; every pointer is device memory.
struct OrthSeg {
    int n;                        // rows
    int k;                        // basis columns so far (Q_1 .. Q_j)
    int qcap;                     // basis capacity in columns
    int chunk_rows, nchunks;      // row chunks of the projection partial sums
    int gchunk_rows, gnchunks;    // row chunks of the Gram partial sums
    int pad;
    DMat Q;                       // basis (panelled)
    double *W;                    // n x c, ld c: the filtered block
    double *H;                    // H1 then H2, k x c each (row-major)
    double *G;                    // c x c Gram matrix
    double *R1, *R2, *Ri;         // c x c: first and second factor, current inverse
    double *part;                 // partial sums: max(nchunks k, gnchunks c) c doubles
    double *out;                  // D_j (c x c), S_j (c x c), status (0 ok, 1 dependent columns, 2 breakdown)
    double *Vin;                  // next filter input, n x c
    float *V32;                   // its FP32 copy (or null)
};
// Launch kinds of a segmented block step: projection on FMA (solves with
// k > 128) or MFMA (k <= 128), Gram matrix, reduction of k x c, reduction
// of c x c, blocks of 256 rows.  A solve has no blocks in a kind it skips.
enum { kOrthFma = 0, kOrthMfma, kOrthGram, kOrthRed, kOrthGred, kOrthRows, kOrthKinds };
// Launch bookkeeping of one segmented block step: the device table, one
// prefix array of first blocks per kind (nseg each, kind-major) and each
// kind's block count.
struct OrthPlan {
    const OrthSeg *tab;
    const int *pre;
    int nseg;
    int blocks[kOrthKinds];
};
// The 14 or 16 launches of one block step for every solve in the plan.
hipError_t launch_seg_orth(const OrthPlan &p, int c, hipStream_t s);

// Partial sums for C = A^T B over row chunks: A n x K (lda), B n x c (ldb).
// partials[chunk][K * c] (row-major K x c).  Returns the number of chunks
// used via *nchunks (caller sizes partials with plan_tn()).
struct TnPlan {
    int chunk_rows;
    int nchunks;
    size_t partial_elems;  // nchunks * K * c
};
TnPlan plan_tn(int n, int K, int c);
// sym (K == c and A^T B symmetric, as B = A or B = M A with M symmetric):
// only the tile groups on or above the diagonal are computed, and the
// reduction (with the same flag) mirrors them.
hipError_t launch_gemm_tn_partial(const TnPlan &pl, int n, int K, int c, DMat A, const double *B, int64_t ldb,
                                  double *partials, hipStream_t s, bool sym = false);
// C (K x c, ldc) = sum over chunks of partials (deterministic order).
hipError_t launch_reduce_partials(const TnPlan &pl, int K, int c, const double *partials, double *C,
                                  int ldc, hipStream_t s, bool sym = false);

// C (n x c, ldc) = beta * C + alpha * A (n x K, lda) B (K x c, ldb); B on device.
hipError_t launch_gemm_nn(int n, int K, int c, double alpha, DMat A, const double *B, int64_t ldb, double beta,
                          double *C, int64_t ldc, hipStream_t s);

// Gershgorin: lo/hi per block into part (2 * nblocks doubles), then reduced
// to out[0] = min(a_ii - R_i), out[1] = max(a_ii + R_i).
hipError_t launch_gershgorin(int n, const int32_t *rowptr, const int32_t *colind, const double *val,
                             double *part, int part_cap, double *out, hipStream_t s);
int gershgorin_blocks(int n);
// *bad += entries a_ij of A without a stored a_ji within tol (relative); *bad
// must be zeroed first.  Columns must be sorted within each row.
hipError_t launch_sym_check(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double tol,
                            unsigned int *bad, hipStream_t s);

// N(0,1) entries from a counter-based generator: out[i] for i < count, with
// leading-dimension layout rows x cols (ld).
hipError_t launch_randn(int rows, int cols, double *out, int64_t ld, uint64_t seed, uint64_t stream_id,
                        hipStream_t s);

// dst columns [dcol0, dcol0 + cols) = scale * src (rows x cols, lds) when
// dst.p is non-NULL; optional FP32 copy dst32 (rows x cols, ldd32).
hipError_t launch_copy_block(int rows, int cols, double scale, const double *src, int64_t lds, DMat dst, int dcol0,
                             float *dst32, int64_t ldd32, hipStream_t s);
hipError_t launch_to_float(int64_t count, const double *src, float *dst, hipStream_t s);
// alpha_j, beta_j and q_{j+1} of a single-vector Lanczos step (bounds
// estimate); q_j's coefficients at h1[hj], h2[hj]
hipError_t launch_lanczos_next(int n, const double *w, double *q, int64_t ldq, const double *g, const double *h1,
                               const double *h2, int hj, int j, double *ab, hipStream_t s);
hipError_t launch_scale(int64_t count, double a, const double *src, double *dst, hipStream_t s);

// resid[j] = || AX[:, j] - lam[j] X[:, j] ||_2 for row-major n x c blocks
// (partials of squares per block, reduced in a second pass).
hipError_t launch_resid_norms(int n, int c, const double *AX, int64_t ldax, const double *X,
                              int64_t ldx, const double *lam, double *part, int nchunks,
                              double *out, hipStream_t s);
// out[j] = x_j . y_j for the first c columns of X and Y (n rows), summed
// over resid_chunks(n) row chunks in a fixed order (part: nchunks x c).
hipError_t launch_col_dots(int n, int c, const double *X, int64_t ldx, const double *Y, int64_t ldy, double *part,
                           int nchunks, double *out, hipStream_t s);
int resid_chunks(int n);

// dst (row-major n x c, ldd) = src (column-major n x c, ld n)
hipError_t launch_transpose_in(int n, int c, const double *src, double *dst, int64_t ldd, hipStream_t s);
// dst (column-major n x c, ld n) = src (row-major n x c, lds)
hipError_t launch_transpose_out(int n, int c, const double *src, int64_t lds, double *dst,
                                hipStream_t s);

}  // namespace flp
