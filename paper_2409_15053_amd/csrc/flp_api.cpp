// C ABI of the filtered Lanczos procedure (include/flp.h): argument checks
// and forwarding to the host drivers; no exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "flp_host.h"

using namespace flp;

// ====================================================================== C ABI

extern "C" {

void flp_opts_default(flp_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->block = 1;
    o->degree = 0;
    o->eps = kDefaultEps;
    o->tol = kDefaultTol;
    o->check_every = 0;  // chosen from the block size (default_check_every)
    o->prec = FLP_PREC_FP64;
    o->seed = 0;
    o->max_basis = 0;
    o->k0 = kDefaultK0;
    o->start = nullptr;
    o->lmin = 0.0;
    o->lmax = 0.0;
    o->stream = nullptr;
    o->sym_tol = -1.0;
    o->polish_degree = 0;
    o->unfiltered = 0;
    o->format = FLP_FORMAT_AUTO;
}

int flp_build_filter(double alpha, double beta, int32_t degree, double lmin, double lmax, flp_filter **out) {
    return make_filter(alpha, beta, degree, lmin, lmax, kDefaultEps, out);
}

int flp_build_filter_eps(double alpha, double beta, int32_t degree, double lmin, double lmax, double eps,
                         flp_filter **out) {
    return make_filter(alpha, beta, degree, lmin, lmax, eps, out);
}

void flp_filter_free(flp_filter *p) { delete p; }

int32_t flp_filter_degree(const flp_filter *p) {
    if (!p) return fail(FLP_E_ARG, "filter is NULL");
    return p->m;
}

int32_t flp_filter_coeffs(const flp_filter *p, double *coeffs, int32_t cap) {
    if (!p) return fail(FLP_E_ARG, "filter is NULL");
    if (coeffs) {
        int k = std::min<int>(cap, p->m + 1);
        for (int i = 0; i < k; ++i) coeffs[i] = p->b[i];
    }
    return p->m + 1;
}

int flp_filter_info(const flp_filter *p, double *o6) {
    if (!p || !o6) return fail(FLP_E_ARG, "NULL argument");
    o6[0] = p->lmin;
    o6[1] = p->lmax;
    o6[2] = p->c;
    o6[3] = p->e;
    o6[4] = p->a1;
    o6[5] = p->b1;
    return FLP_OK;
}

int flp_filter_eval(const flp_filter *p, const double *z, double *o, int32_t count) {
    if (!p || (count > 0 && (!z || !o)) || count < 0) return fail(FLP_E_ARG, "bad argument");
    for (int i = 0; i < count; ++i) o[i] = cheb_scalar(p->b, z[i]);
    return FLP_OK;
}

int32_t flp_filter_divided(const flp_filter *p, double t, double *coeffs, int32_t cap) {
    if (!p || !coeffs || cap < 0) return fail(FLP_E_ARG, "bad argument");
    std::vector<double> c;
    cheb_divided(p->b, t, c);
    for (int i = 0; i < (int)c.size() && i < cap; ++i) coeffs[i] = c[i];
    return (int32_t)c.size();
}

int flp_filter_apply(const flp_filter *p, const flp_csr *A, const double *V, int64_t ldv, double *W, int64_t ldw,
                     int32_t r, int32_t prec, int32_t format, void *stream) {
    if (!p) return fail(FLP_E_ARG, "filter is NULL");
    CKR(check_csr(A));
    if (r < 1 || r > 32) return fail(FLP_E_ARG, "r must be in [1, 32]");
    if (!V || !W) return fail(FLP_E_ARG, "V and W must be non-NULL");
    if (ldv < r || ldw < r || ldv > INT32_MAX || ldw > INT32_MAX)
        return fail(FLP_E_ARG, "leading dimensions must be in [r, 2^31)");
    // the blocks' extents: rows 0..n-1, columns 0..r-1
    const double *vend = V + (size_t)(A->n - 1) * ldv + r;
    const double *wend = W + (size_t)(A->n - 1) * ldw + r;
    if (V < wend && W < vend) return fail(FLP_E_ARG, "W must not overlap V");
    if (prec != FLP_PREC_FP64 && prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    if (format != FLP_FORMAT_AUTO && format != FLP_FORMAT_CSR && format != FLP_FORMAT_SELL)
        return fail(FLP_E_ARG, "bad storage format");
    try {
        return filter_apply_impl(p, A, V, (int)ldv, W, (int)ldw, r, prec, (hipStream_t)stream, format);
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    }
}

int flp_filter_launch_shape(int32_t r, int32_t prec, int32_t segmented, flp_tune_info *out) {
    if (!out) return fail(FLP_E_ARG, "out is NULL");
    if (r < 1 || r > 32) return fail(FLP_E_ARG, "r must be in [1, 32]");
    if (prec != FLP_PREC_FP64 && prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    const bool fp32 = prec == FLP_PREC_FP32_FILTER;
    const StepShape sh = segmented ? seg_launch_shape(r, fp32) : step_launch_shape(r, fp32);
    std::memset(out, 0, sizeof(*out));
    out->group_width = r;
    out->lanes_per_row = sh.lpr;
    out->cols_per_lane = sh.vec;
    out->rows_per_wave = 64 / sh.lpr;
    out->streaming_loads = sh.nt;
    return FLP_OK;
}

int flp_tile_order(int32_t tiles, int32_t tile_chunk, int32_t rows_per_tile, int32_t *order) {
    if (tiles < 0 || rows_per_tile < 1 || (tiles > 0 && !order))
        return fail(FLP_E_ARG, "tiles >= 0, rows_per_tile >= 1 and order non-NULL required");
    tile_order_host(tiles, tile_chunk, rows_per_tile, order);
    return FLP_OK;
}

int flp_tune_filter(const flp_csr *A, int32_t r, int32_t prec, int32_t format, void *stream, flp_tune_info *out) {
    if (!out) return fail(FLP_E_ARG, "out is NULL");
    CKR(check_csr(A));
    if (r < 1 || r > 32) return fail(FLP_E_ARG, "r must be in [1, 32]");
    if (prec != FLP_PREC_FP64 && prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    if (format != FLP_FORMAT_AUTO && format != FLP_FORMAT_CSR && format != FLP_FORMAT_SELL)
        return fail(FLP_E_ARG, "bad storage format");
    try {
        hipStream_t s = (hipStream_t)stream;
        Workspace &w = ws();
        const bool fp32 = prec == FLP_PREC_FP32_FILTER;
        const size_t es = fp32 ? sizeof(float) : sizeof(double);
        const int n = A->n;
        for (auto &u : w.U) CK(ensure(u, es * (size_t)n * r));
        CK(ensure(w.Vg, es * (size_t)n * r));
        CK(hipMemsetAsync(w.Vg.p, 0, es * (size_t)n * r, s));
        const float *v32 = nullptr;
        if (fp32) CKR(ensure_val32(A, w.val32, &w.val32_src, &w.val32_nnz, &v32, s));
        void *U[3] = {w.U[0].p, w.U[1].p, w.U[2].p};
        const flp_csr *fA = A;
        const float *fv32 = v32;
        bool sell = false;
        CKR(workspace_storage(A, v32, fp32, format, s, &fA, &fv32, &sell));
        FilterTune tn;
        CKR(tune_filter(fA, fv32, r, fp32, true, U, w.Vg.p, r, s, &tn, sell));
        CK(hipStreamSynchronize(s));
        StepShape sh = step_shape_ok(tn.gw, fp32, tn.sh) ? tn.sh : default_step_shape(tn.gw, fp32);
        out->group_width = tn.gw;
        out->lanes_per_row = sh.lpr > 0 ? sh.lpr : tn.gw;
        out->cols_per_lane = sh.lpr > 0 ? sh.vec : 1;
        out->rows_per_wave = 64 / out->lanes_per_row;
        out->candidates = tn.candidates;
        out->streaming_loads = sh.lpr > 0 ? sh.nt : 0;
        out->us_per_step = tn.candidates > 0 ? tn.us_per_step : 0.0;
        out->tile_chunk = tn.sh.chunk;
        out->lds_window = sh.lpr > 0 ? sh.win : 0;
        out->window_halo = out->lds_window == 2 ? sh.halo : (out->lds_window == 1 ? kWinHalo : 0);
        return FLP_OK;
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    }
}

void flp_set_autotune(int32_t on) { set_autotune(on); }

void flp_set_filter_shape(int32_t lanes_per_row, int32_t cols_per_lane, int32_t group_width,
                          int32_t streaming_loads, int32_t tile_chunk, int32_t lds_window) {
    const bool chunk = tile_chunk != FLP_TILE_CHUNK_TUNED;
    force_filter_shape(StepShape{std::max(0, (int)lanes_per_row), std::max(0, (int)cols_per_lane),
                                 streaming_loads ? 1 : 0, chunk ? (int)tile_chunk : 0,
                                 lds_window == 2 ? 2 : (lds_window ? 1 : 0)},
                       std::max(0, (int)group_width), chunk);
}

int flp_spmm(const flp_csr *A, const double *X, int32_t ldx, double *Y, int32_t ldy, int32_t r, void *stream) {
    CKR(check_csr(A));
    if (r < 1 || r > 32 || ldx < r || ldy < r || !X || !Y) return fail(FLP_E_ARG, "bad block arguments");
    CK(launch_cheb_step<double, double>(A->n, A->rowptr, A->colind, A->val, r, X, ldx, nullptr, 0, nullptr, 0, Y,
                                        ldy, 1.0, 0.0, 0.0, 0.0, (hipStream_t)stream));
    return FLP_OK;
}

int flp_block_orth(const double *Q, int64_t ldq, int32_t k, int32_t n, double *W, int32_t r, double *H,
                   void *stream) {
    if (!Q || !W || k < 1 || n < 1 || r < 1 || r > 16 || ldq < k) return fail(FLP_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    double *hdev = nullptr;
    CKR(small_dev((size_t)2 * k * r + 64, &hdev));
    CKR(cgs2(plain_mat(Q, ldq), k, n, W, r, hdev, s));
    if (H) {
        std::vector<double> h((size_t)2 * k * r);
        CK(hipMemcpyAsync(h.data(), hdev, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        for (size_t i = 0; i < (size_t)k * r; ++i) H[i] = h[i] + h[(size_t)k * r + i];
    }
    return FLP_OK;
}

int flp_block_qr(double *W, int32_t n, int32_t r, double *S, void *stream) {
    if (!W || !S || n < 1 || r < 1 || r > 16 || r > n) return fail(FLP_E_ARG, "bad arguments");
    std::vector<double> Sv;
    bool replaced = false;
    CKR(block_qr_impl(W, n, r, nullptr, 0, Sv, 12345, 1, (hipStream_t)stream, &replaced));
    if (replaced) return fail(FLP_E_ARG, "block is numerically rank deficient");
    std::memcpy(S, Sv.data(), sizeof(double) * r * r);
    return FLP_OK;
}

int flp_estimate_bounds(const flp_csr *A, int32_t k0, uint64_t seed, double *lmin, double *lmax, void *stream) {
    CKR(check_csr(A));
    if (!lmin || !lmax) return fail(FLP_E_ARG, "NULL output");
    return estimate_bounds_impl(A, k0 > 0 ? k0 : kDefaultK0, seed, lmin, lmax, (hipStream_t)stream);
}

int flp_solve(const flp_csr *A, double alpha, double beta, const flp_opts *opts, flp_result **out) {
    if (!out) return fail(FLP_E_ARG, "out is NULL");
    *out = nullptr;
    CKR(check_csr(A));
    flp_opts o;
    flp_opts_default(&o);
    if (opts) o = *opts;
    try {
        return solve_impl(A, alpha, beta, o, out);
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(FLP_E_DEVICE, "unexpected exception");
    }
}

int flp_solve_sliced(const flp_csr *A, double alpha, double beta, int32_t nslices, const flp_opts *opts,
                     flp_result **out) {
    if (!out) return fail(FLP_E_ARG, "out is NULL");
    *out = nullptr;
    CKR(check_csr(A));
    flp_opts o;
    flp_opts_default(&o);
    if (opts) o = *opts;
    try {
        return solve_sliced_impl(A, alpha, beta, nslices, o, out);
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(FLP_E_DEVICE, "unexpected exception");
    }
}

void flp_result_free(flp_result *res) {
    if (!res) return;
    delete[] res->evals;
    delete[] res->resid;
    if (res->evecs) (void)dev_free(res->evecs);
    delete res;
}

int flp_result_copy_evecs(const flp_result *res, double *dst, void *stream) {
    if (!res || !dst) return fail(FLP_E_ARG, "NULL argument");
    if (res->count == 0) return FLP_OK;
    CK(hipMemcpyAsync(dst, res->evecs, sizeof(double) * (size_t)res->n * res->count, hipMemcpyDeviceToDevice,
                      (hipStream_t)stream));
    return FLP_OK;
}

int flp_solve_batch(int32_t count, const flp_csr *const *A, const double *alpha, const double *beta,
                    const flp_opts *opts, int32_t use_graph, flp_result **results, int32_t *codes,
                    flp_batch_stats *stats) {
    if (count < 1 || !A || !alpha || !beta || !results || !codes) return fail(FLP_E_ARG, "bad batch arguments");
    try {
        return solve_batch_impl(count, A, alpha, beta, opts, use_graph, results, codes, stats);
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(FLP_E_DEVICE, "unexpected exception");
    }
}

int flp_host_sym_eig(int32_t N, int32_t bw, const double *M, double *evals, double *evecs) {
    if (N < 1 || !M || !evals || bw < 0) return fail(FLP_E_ARG, "bad arguments");
    try {
        std::vector<int> cols;
        if (evecs) {
            cols.resize(N);
            for (int i = 0; i < N; ++i) cols[i] = i;
        }
        int rc = sym_eig(N, bw, M, evals, nullptr, 0, nullptr, evecs ? cols.data() : nullptr, evecs ? N : 0, evecs);
        if (rc != 0) return fail(FLP_E_ARG, "eigensolver did not converge");
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    }
    return FLP_OK;
}

void flp_set_allocator(flp_alloc_fn alloc, flp_free_fn free_fn, void *ctx) { set_allocator(alloc, free_fn, ctx); }

int flp_check_symmetric(const flp_csr *A, double tol, void *stream) {
    CKR(check_csr(A));
    try {
        return check_symmetric(A, tol, (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    }
}

void flp_release_workspace(void) {
    ws().release_all();
    release_single_bufs();
    release_dev_cache();
}

const char *flp_last_error(void) { return last_error_cstr(); }

const char *flp_version(void) { return "flp-mi355x 0.1"; }

int32_t flp_abi_sizes(int64_t *sizes, int32_t cap) {
    const int64_t s[] = {(int64_t)sizeof(flp_csr),       (int64_t)sizeof(flp_opts),
                         (int64_t)sizeof(flp_stats),     (int64_t)sizeof(flp_result),
                         (int64_t)sizeof(flp_tune_info), (int64_t)sizeof(flp_batch_stats),
                         (int64_t)sizeof(flp_server_opts)};
    const int32_t n = (int32_t)(sizeof(s) / sizeof(s[0]));
    for (int32_t i = 0; sizes && i < n && i < cap; ++i) sizes[i] = s[i];
    return n;
}

}  // extern "C"
