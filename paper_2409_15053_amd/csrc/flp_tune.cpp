// Autotuner for the filter step.
//
// The Clenshaw step is a CSR SpMM whose best launch shape depends on the
// matrix (row length, n) and on how much of the step's working set stays in
// the 256 MB Infinity Cache between steps.  Two choices are tuned:
//   * the shape: lanes per matrix row and columns per lane, i.e. rows per
//     wavefront (64 / lanes) and bytes gathered per lane per nonzero;
//   * the column-group width of a single solve's filter: the block of r
//     columns can be filtered as r / gw independent groups of gw columns,
//     which re-reads the matrix per group but can keep a group's whole
//     recurrence resident in the cache.
// Each candidate is timed on the caller's matrix over a ring of six steps
// (the pattern of the real recurrence: gather one buffer, read V and a
// second buffer, write the third), after one untimed ring; among those within
// 3 % of the fastest the widest column group is kept.  Results are cached
// per device, precision, r, grouping allowed, storage, size class (n to a
// quarter octave, nonzeros per row to a quarter) and plane length (below).
// The order in which the row tiles are handed to the XCDs is tuned too
// (chunk_tile): for a single solve this includes a pencil walk over planes
// of P rows, P being the nearest neighbour distance of at least 1024 rows in
// a middle row of the matrix (a 3D grid's N^2).  Every shape and
// width computes each output element with the same operations in the same
// order, so tuning never changes results, only speed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "flp_host.h"

namespace flp {

namespace {

std::atomic<int> g_mode{1};  // 1: tune on first use, 0: fixed defaults
// tile-to-XCD mappings tried (chunk_tile): one contiguous range per XCD, or
// chunks of this many tiles dealt to the XCDs in turn; a single solve's
// filter also tries the pencil walk over the matrix's planes (plane_rows)
constexpr int kTileChunks[] = {0, 4, 32};
// smallest neighbour distance (in rows) taken for a plane of a grid
constexpr int kMinPlaneRows = 1024;
// LDS a sliding-window workgroup may hold: two fit one compute unit
constexpr int64_t kSlideLdsBytes = 80 * 1024;
std::mutex g_mu;
StepShape g_force_shape{};
int g_force_gw = 0;
bool g_force_chunk = false;

using Key = std::tuple<int, int, int, int64_t, int64_t, int, int, int>;
std::map<Key, FilterTune> &cache() {
    static std::map<Key, FilterTune> c;
    return c;
}

// Launches one ring of `steps` filter steps over gw columns with the given
// shape; buffers hold n x gw (row-major, ld gw) elements of the filter type.
int ring(const flp_csr *A, const float *val32, bool fp32, int gw, StepShape sh, void *const U[3], const void *V,
         int ldv, int steps, hipStream_t s, bool sell) {
    for (int j = 0; j < steps; ++j) {
        ClenshawStep st{};
        st.X = U[j % 3];
        st.ldx = gw;
        st.V = V;
        st.ldv = ldv;
        st.Y = U[(j + 2) % 3];
        st.ldy = gw;
        st.out = U[(j + 1) % 3];
        st.ldo = gw;
        st.out_f64 = !fp32;
        st.alpha = 2.0;
        st.beta = -1.0;
        st.gamma = 0.5;
        st.delta = -1.0;
        CKR(launch_plan_step(A, val32, gw, st, fp32, s, sh, sell));
    }
    return FLP_OK;
}

}  // namespace

namespace {

// The distinct distances |col - row| of the nonzeros (up to 64) of the
// matrix's middle row, ascending; empty for matrices under 2048 rows.
int row_offsets(const flp_csr *A, bool sell, hipStream_t s, std::vector<int> *out) {
    out->clear();
    const int n = A->n;
    if (n < 2 * kMinPlaneRows) return FLP_OK;
    const int row = n / 2;
    int32_t rp[2] = {0, 0};
    std::vector<int32_t> cols;
    if (sell) {  // rowptr holds slice offsets; entry k of the row at off + row % C + k C
        const int sl = row / kSellC;
        CK(hipMemcpyAsync(rp, A->rowptr + sl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        const int w = std::min(64, (rp[1] - rp[0]) / kSellC);
        cols.resize(w);
        for (int k = 0; k < w; ++k)
            CK(hipMemcpyAsync(&cols[k], A->colind + rp[0] + row % kSellC + (int64_t)k * kSellC, sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
    } else {
        CK(hipMemcpyAsync(rp, A->rowptr + row, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        const int w = std::min(64, rp[1] - rp[0]);
        cols.resize(std::max(0, w));
        if (w > 0)
            CK(hipMemcpyAsync(cols.data(), A->colind + rp[0], sizeof(int32_t) * w, hipMemcpyDeviceToHost, s));
    }
    CK(hipStreamSynchronize(s));
    for (int32_t c : cols) out->push_back(std::abs(c - row));
    std::sort(out->begin(), out->end());
    out->erase(std::unique(out->begin(), out->end()), out->end());
    return FLP_OK;
}

// Halos a sliding-window shape may take: the distances beyond the fixed
// window's reach and below the plane length (all of them without planes)
// whose window of RPB + 2 halo rows of gw elements (plus 16 bytes of
// padding each) fits kSlideLdsBytes, ascending.
std::vector<int> slide_halos(const std::vector<int> &offs, int plane, int gw, int lpr, size_t es) {
    const int rpb = 256 / lpr;
    const int64_t rows = kSlideLdsBytes / (int64_t)(es * gw + 16);
    const int64_t cap = (rows - rpb) / 2;
    std::vector<int> h;
    for (int d : offs)
        if (d > kWinHalo && (plane == 0 || d < plane) && d <= cap) h.push_back(d);
    return h;
}

// The longest of them (0: none).
int slide_halo(const std::vector<int> &offs, int plane, int gw, int lpr, size_t es) {
    const std::vector<int> h = slide_halos(offs, plane, gw, lpr, es);
    return h.empty() ? 0 : h.back();
}

int plane_of(const std::vector<int> &offs) {
    for (int d : offs)
        if (d >= kMinPlaneRows) return d;
    return 0;
}

}  // namespace

int plane_rows(const flp_csr *A, bool sell, hipStream_t s, int *out) {
    std::vector<int> offs;
    CKR(row_offsets(A, sell, s, &offs));
    *out = plane_of(offs);
    return FLP_OK;
}

void set_autotune(int mode) { g_mode.store(mode ? 1 : 0); }
int autotune_mode() { return g_mode.load(); }

void force_filter_shape(StepShape sh, int gw, bool chunk) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_force_shape = sh;
    g_force_gw = gw;
    g_force_chunk = chunk;
}

int lookup_filter_tune(const flp_csr *A, int r, bool fp32, FilterTune *out) {
    FilterTune def;
    def.gw = r;
    def.sh = default_step_shape(r, fp32);
    *out = def;
    if (g_mode.load() == 0) return FLP_OK;
    int dev = 0;
    CK(hipGetDevice(&dev));
    const int n = A->n;
    int plane = 0;
    CKR(plane_rows(A, false, nullptr, &plane));
    const int64_t nc = std::lround(4.0 * std::log2((double)n)), zc = std::lround(4.0 * (double)A->nnz / n);
    // a single solve's tuning (either storage) first, then the segmented engine's
    const Key keys[] = {Key{dev, fp32 ? 1 : 0, r, nc, zc, 1, 1, plane}, Key{dev, fp32 ? 1 : 0, r, nc, zc, 1, 0, plane},
                        Key{dev, fp32 ? 1 : 0, r, nc, zc, 0, 1, 0}, Key{dev, fp32 ? 1 : 0, r, nc, zc, 0, 0, 0}};
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Key &key : keys) {
        auto it = cache().find(key);
        if (it != cache().end()) {
            *out = it->second;
            return FLP_OK;
        }
    }
    return FLP_OK;
}

int tune_filter(const flp_csr *A, const float *val32, int r, bool fp32, bool allow_groups, void *const U[3],
                const void *V, int ldv, hipStream_t s, FilterTune *out, bool sell) {
    const int n = A->n;
    FilterTune def;
    def.gw = allow_groups ? filter_group_width(n, A->nnz, r, fp32 ? FLP_PREC_FP32_FILTER : FLP_PREC_FP64) : r;
    def.sh = default_step_shape(def.gw, fp32);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_force_shape.lpr > 0 || g_force_gw > 0 || g_force_chunk) {
            FilterTune f = def;
            if (g_force_gw > 0 && r % g_force_gw == 0 && (allow_groups || g_force_gw == r)) f.gw = g_force_gw;
            if (step_shape_ok(f.gw, fp32, g_force_shape)) {
                f.sh = g_force_shape;
                if (f.sh.win == 2 && f.sh.halo == 0) {  // sliding window fitted to this matrix
                    std::vector<int> offs;
                    CKR(row_offsets(A, sell, s, &offs));
                    f.sh.chunk = plane_of(offs);
                    f.sh.halo = slide_halo(offs, f.sh.chunk, f.gw, f.sh.lpr, fp32 ? sizeof(float) : sizeof(double));
                    if (f.sh.halo == 0) f.sh.win = 1;
                }
            } else {
                f.sh = default_step_shape(f.gw, fp32);
                f.sh.chunk = g_force_shape.chunk;
            }
            *out = f;
            return FLP_OK;
        }
    }
    if (g_mode.load() == 0) {
        *out = def;
        return FLP_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    CK(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) {  // never time inside a capture
        *out = def;
        return FLP_OK;
    }
    int dev = 0;
    CK(hipGetDevice(&dev));
    // a single solve's filter also tries the pencil walk over the matrix's
    // planes (the segmented engine's tiles span many matrices)
    std::vector<int> offs;
    if (allow_groups) CKR(row_offsets(A, sell, s, &offs));
    const int plane = plane_of(offs);
    // size class: n to a quarter octave, nonzeros per row to a quarter; plane
    const Key key{dev, fp32 ? 1 : 0, r, (int64_t)std::lround(4.0 * std::log2((double)n)),
                  (int64_t)std::lround(4.0 * (double)A->nnz / n), allow_groups ? 1 : 0, sell ? 1 : 0, plane};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = cache().find(key);
        if (it != cache().end()) {
            *out = it->second;
            return FLP_OK;
        }
    }
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    // the ring starts from zeros so every candidate sees the same data
    for (int i = 0; i < 3; ++i) CK(hipMemsetAsync(U[i], 0, es * (size_t)n * r, s));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    struct G {
        hipEvent_t a, b;
        ~G() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    constexpr int kSteps = 6;
    std::vector<FilterTune> timed;
    int tried = 0;
    for (int gw = r; gw >= 1; gw /= 2) {
        if (r % gw != 0 || (gw != r && !allow_groups)) continue;
        std::vector<StepShape> cands;
        for (StepShape sh : step_shape_candidates(gw, fp32, true)) {
            for (int ch : kTileChunks) {
                sh.chunk = ch;
                cands.push_back(sh);
            }
            if (plane > 0) {
                sh.chunk = -plane;
                cands.push_back(sh);
            }
        }
        // the sliding window, its halo and row ranges fitted to the matrix
        for (StepShape sh : step_shape_candidates(gw, fp32, false))
            for (int h : slide_halos(offs, plane, gw, sh.lpr, es)) {
                sh.halo = h;
                sh.win = 2;
                sh.chunk = plane;
                cands.push_back(sh);
            }
        for (StepShape sh : cands) {
            // V: the caller's block (gw == r) or a contiguous n x gw group,
            // taken from the unused half of the first buffer
            const void *Vg = gw == r ? V : (const void *)((const char *)U[0] + es * (size_t)n * gw);
            const int ldvg = gw == r ? ldv : gw;
            if (gw != r && gw > r / 2) continue;
            CKR(ring(A, val32, fp32, gw, sh, U, Vg, ldvg, kSteps, s, sell));  // warm-up
            CK(hipEventRecord(e0, s));
            CKR(ring(A, val32, fp32, gw, sh, U, Vg, ldvg, kSteps, s, sell));
            CK(hipEventRecord(e1, s));
            CK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1e3 * ms / kSteps * (r / gw);  // all r columns
            ++tried;
            FilterTune t;
            t.gw = gw;
            t.sh = sh;
            t.us_per_step = us;
            timed.push_back(t);
        }
    }
    // Among the configurations within 3 % of the fastest (closer than the
    // timing noise), the widest column group wins: it reads the matrix the
    // fewest times per step, so it moves the least data; then the fastest.
    FilterTune best = def;
    if (!timed.empty()) {
        double fastest = 1e300;
        for (const auto &t : timed) fastest = std::min(fastest, t.us_per_step);
        bool have = false;
        for (const auto &t : timed) {
            if (t.us_per_step > 1.03 * fastest) continue;
            if (!have || t.gw > best.gw || (t.gw == best.gw && t.us_per_step < best.us_per_step)) best = t;
            have = true;
        }
    }
    best.candidates = tried;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        cache()[key] = best;
    }
    *out = best;
    return FLP_OK;
}

}  // namespace flp
