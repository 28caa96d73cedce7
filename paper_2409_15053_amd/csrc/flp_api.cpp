// C ABI and host orchestration of the filtered Lanczos procedure.
//
// The device work (filter SpMMs, reorthogonalisation GEMMs, norms) runs in
// the kernels of flp_kernels.hip; this file sequences them on one stream,
// keeps the small projected matrices on the host and solves their
// eigenproblems with the banded symmetric eigensolver of flp_eigen.cpp, as
// the paper does (Section 3.2.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "flp_internal.h"

namespace flp {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

constexpr double kDefaultEps = 0.31227;
constexpr int kDefaultCheck = 30;
constexpr int kDefaultK0 = 40;
constexpr double kDefaultTol = 1e-9;
constexpr int kMaxDegree = 100000;
constexpr int64_t kDefaultMaxBasis = 3072;

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ workspace

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

hipError_t ensure(Buf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return e;
    }
    b.bytes = want;
    return hipSuccess;
}

struct Workspace {
    Buf U[3];      // Clenshaw vectors
    Buf V32;       // FP32 copy of the filter input
    Buf val32;     // FP32 copy of the matrix values
    Buf partials;  // gemm_tn partial sums
    Buf small;     // small device matrices
    Buf W;         // block being orthogonalised
    Buf Vin;       // contiguous filter input
    Buf Q;         // Lanczos basis
    Buf Y, AY, X, AX;  // Rayleigh-Ritz blocks
    Buf resid_part;
    const double *val32_src = nullptr;  // val the FP32 copy was made from
    int64_t val32_nnz = 0;
};

Workspace &ws() {
    static Workspace w[64];
    int dev = 0;
    (void)hipGetDevice(&dev);
    return w[dev & 63];
}

#define CK(...)                                                                        \
    do {                                                                               \
        hipError_t e_ = (__VA_ARGS__);                                                 \
        if (e_ != hipSuccess) {                                                        \
            if (e_ == hipErrorOutOfMemory)                                             \
                return fail(FLP_E_NOMEM, std::string(#__VA_ARGS__) + ": out of device memory"); \
            return fail(FLP_E_DEVICE, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)

#define CKR(...)                       \
    do {                               \
        int rc_ = (__VA_ARGS__);       \
        if (rc_ != FLP_OK) return rc_; \
    } while (0)

// ------------------------------------------------------------------ CSR checks

int check_csr(const flp_csr *A) {
    if (!A) return fail(FLP_E_ARG, "A is NULL");
    if (A->n <= 0) return fail(FLP_E_ARG, "n must be positive");
    if (A->nnz < 0 || A->nnz >= (int64_t(1) << 31)) return fail(FLP_E_ARG, "nnz must be in [0, 2^31)");
    if (!A->rowptr || (A->nnz > 0 && (!A->colind || !A->val)))
        return fail(FLP_E_ARG, "CSR pointers must be non-NULL");
    return FLP_OK;
}

}  // namespace
}  // namespace flp

using namespace flp;

// ====================================================================== filter

struct flp_filter {
    double alpha, beta;  // as given
    double lmin, lmax, c, e;
    double a1, b1;       // mapped, clamped interval
    int m;
    std::vector<double> b;
};

namespace flp {
namespace {

// p(z) = sum b_i T_i(z), Clenshaw (Section 2.2) on a scalar.
double cheb_scalar(const std::vector<double> &b, double z) {
    double u1 = 0.0, u2 = 0.0;
    for (int k = (int)b.size() - 1; k >= 1; --k) {
        double u = b[k] + 2.0 * z * u1 - u2;
        u2 = u1;
        u1 = u;
    }
    return b[0] + z * u1 - u2;
}

// b_0..b_m of the indicator of [a, b] in [-1, 1] (closed form of Section 2.2).
void indicator_coeffs(double a1, double b1, int m, std::vector<double> &out) {
    double ta = std::acos(a1), tb = std::acos(b1);
    out.assign(m + 1, 0.0);
    out[0] = (ta - tb) / M_PI;
    for (int i = 1; i <= m; ++i) out[i] = 2.0 * (std::sin(i * ta) - std::sin(i * tb)) / (i * M_PI);
}

// Smallest m >= 1 with ||p_m - phi||_mu < eps ||phi||_mu (eq. optimaldegree);
// the squared error falls by (pi/2) b_m^2 per degree from
// ||phi||^2 - pi b_0^2, with ||phi||^2 = acos(a) - acos(b).
int auto_degree(double a1, double b1, double eps) {
    double ta = std::acos(a1), tb = std::acos(b1);
    double phi2 = ta - tb;
    double b0 = phi2 / M_PI;
    double err2 = phi2 - M_PI * b0 * b0;
    const double lim = eps * std::sqrt(phi2);
    for (int m = 1; m <= 2000; ++m) {
        double bm = 2.0 * (std::sin(m * ta) - std::sin(m * tb)) / (m * M_PI);
        err2 -= 0.5 * M_PI * bm * bm;
        if (std::sqrt(std::max(err2, 0.0)) < lim) return m;
    }
    return 2000;
}

int make_filter(double alpha, double beta, int degree, double lmin, double lmax, double eps, flp_filter **out) {
    if (!out) return fail(FLP_E_ARG, "out is NULL");
    *out = nullptr;
    if (!(std::isfinite(alpha) && std::isfinite(beta) && std::isfinite(lmin) && std::isfinite(lmax)))
        return fail(FLP_E_ARG, "non-finite interval or bounds");
    if (!(alpha < beta)) return fail(FLP_E_ARG, "alpha must be < beta");
    if (!(lmin < lmax)) return fail(FLP_E_ARG, "lmin must be < lmax");
    if (degree > kMaxDegree) return fail(FLP_E_ARG, "degree too large");
    if (!(eps > 0.0 && eps < 1.0)) return fail(FLP_E_ARG, "eps must be in (0, 1)");
    double lo = std::max(alpha, lmin), hi = std::min(beta, lmax);
    if (!(lo <= hi)) return fail(FLP_E_INTERVAL, "[alpha, beta] does not meet [lmin, lmax]");
    auto *f = new flp_filter;
    f->alpha = alpha;
    f->beta = beta;
    f->lmin = lmin;
    f->lmax = lmax;
    f->c = 0.5 * (lmin + lmax);
    f->e = 0.5 * (lmax - lmin);
    f->a1 = std::min(std::max((lo - f->c) / f->e, -1.0), 1.0);
    f->b1 = std::min(std::max((hi - f->c) / f->e, -1.0), 1.0);
    f->m = degree > 0 ? degree : auto_degree(f->a1, f->b1, eps);
    indicator_coeffs(f->a1, f->b1, f->m, f->b);
    *out = f;
    return FLP_OK;
}

// ------------------------------------------------------------------ filter apply
//
// Clenshaw's backward recurrence for W = p(Ahat) V (Section 2.2):
//   U_{m+1} = U_{m+2} = 0,  U_k = b_k V + 2 Ahat U_{k+1} - U_{k+2},
//   W = b_0 V + Ahat U_1 - U_2,   Ahat X = (A X - c X) / e.
// U_m = b_m V is folded into the first product, so there are exactly m
// products with A, each one launch with the update fused in.
template <typename T>
int clenshaw(const flp_filter *p, int n, const int32_t *rowptr, const int32_t *colind, const T *val, int r,
             const T *V, int ldv, double *W, int ldw, T *U0, T *U1, T *U2, hipStream_t s) {
    const int m = p->m;
    const std::vector<double> &b = p->b;
    const double c = p->c, e = p->e;
    const int ld = r;
    if (m == 0) {
        CK(launch_cheb_step<T, double>(n, rowptr, colind, val, r, V, ldv, nullptr, 0, nullptr, 0, W, ldw, T(0),
                                       T(b[0]), T(0), T(0), s));
        return FLP_OK;
    }
    if (m == 1) {
        CK(launch_cheb_step<T, double>(n, rowptr, colind, val, r, V, ldv, nullptr, 0, nullptr, 0, W, ldw,
                                       T(b[1] / e), T(b[0] - c * b[1] / e), T(0), T(0), s));
        return FLP_OK;
    }
    T *ring[3] = {U0, U1, U2};
    // U_{m-1} = b_{m-1} V + (2 b_m / e) (A V - c V)
    T *u_k1 = ring[0];  // holds U_{k+1}
    CK(launch_cheb_step<T, T>(n, rowptr, colind, val, r, V, ldv, nullptr, 0, nullptr, 0, u_k1, ld,
                              T(2.0 * b[m] / e), T(b[m - 1] - 2.0 * c * b[m] / e), T(0), T(0), s));
    T *u_k2 = nullptr;  // U_{k+2}; U_m = b_m V is folded into the V coefficient
    int slot = 1;
    for (int k = m - 2; k >= 1; --k) {
        T *out = ring[slot];
        slot = (slot + 1) % 3;
        if (k == m - 2) {
            CK(launch_cheb_step<T, T>(n, rowptr, colind, val, r, u_k1, ld, V, ldv, nullptr, 0, out, ld,
                                      T(2.0 / e), T(-2.0 * c / e), T(b[k] - b[m]), T(0), s));
        } else {
            CK(launch_cheb_step<T, T>(n, rowptr, colind, val, r, u_k1, ld, V, ldv, u_k2, ld, out, ld, T(2.0 / e),
                                      T(-2.0 * c / e), T(b[k]), T(-1), s));
        }
        u_k2 = u_k1;
        u_k1 = out;
    }
    // W = b_0 V + Ahat U_1 - U_2
    if (m == 2) {
        CK(launch_cheb_step<T, double>(n, rowptr, colind, val, r, u_k1, ld, V, ldv, nullptr, 0, W, ldw, T(1.0 / e),
                                       T(-c / e), T(b[0] - b[2]), T(0), s));
    } else {
        CK(launch_cheb_step<T, double>(n, rowptr, colind, val, r, u_k1, ld, V, ldv, u_k2, ld, W, ldw, T(1.0 / e),
                                       T(-c / e), T(b[0]), T(-1), s));
    }
    return FLP_OK;
}

// Filter bytes per SpMM step: matrix once, gathered input once, V, U_{k+2}
// and the output once each.
double filter_step_bytes(int n, int64_t nnz, int r, int prec) {
    double wv = prec == FLP_PREC_FP32_FILTER ? 4.0 : 8.0;
    return (double)nnz * (wv + 4.0) + 4.0 * (n + 1) + 4.0 * n * r * wv;
}

int ensure_val32(const flp_csr *A, const float **out, hipStream_t s) {
    if (A->val32) {
        *out = A->val32;
        return FLP_OK;
    }
    Workspace &w = ws();
    if (w.val32_src != A->val || w.val32_nnz != A->nnz || !w.val32.p) {
        CK(ensure(w.val32, sizeof(float) * std::max<int64_t>(A->nnz, 1)));
        CK(launch_to_float(A->nnz, A->val, (float *)w.val32.p, s));
        w.val32_src = A->val;
        w.val32_nnz = A->nnz;
    }
    *out = (const float *)w.val32.p;
    return FLP_OK;
}

// Width of the column groups the filter runs on.  The Clenshaw recurrence
// acts on each column independently, so a block of r columns can be
// filtered as several narrower groups, each through all m steps.  A group
// whose per-step working set (matrix + V + three recurrence vectors) fits
// in the 256 MB Infinity Cache streams from that cache instead of HBM for
// steps 2..m; this costs one extra matrix read per extra group and pays off
// only when the narrower set fits and the full block does not.
int filter_group_width(int n, int64_t nnz, int r, int prec) {
    const double budget = 232e6;
    const double wv = prec == FLP_PREC_FP32_FILTER ? 4.0 : 8.0;
    const int vec = prec == FLP_PREC_FP32_FILTER ? 4 : 2;  // 16-byte loads
    auto footprint = [&](int w) { return (double)nnz * (wv + 4.0) + 4.0 * (n + 1) + 4.0 * n * w * wv; };
    if (footprint(r) <= budget) return r;
    for (int w = r / 2; w >= vec; w /= 2) {
        if (r % w != 0 || w % vec != 0) continue;
        if (footprint(w) <= budget) return w;
    }
    return r;
}

// W = p(Ahat) V with the workspace's Clenshaw buffers (V, W: n x r with
// leading dimensions ldv, ldw), filtered in column groups.
int filter_apply_impl(const flp_filter *p, const flp_csr *A, const double *V, int ldv, double *W, int ldw, int r,
                      int prec, hipStream_t s) {
    Workspace &w = ws();
    const int n = A->n;
    const int gw = filter_group_width(n, A->nnz, r, prec);
    if (prec == FLP_PREC_FP32_FILTER) {
        const float *v32 = nullptr;
        CKR(ensure_val32(A, &v32, s));
        size_t vb = sizeof(float) * (size_t)n * r;
        for (auto &u : w.U) CK(ensure(u, sizeof(float) * (size_t)n * gw));
        CK(ensure(w.V32, vb));
        CK(launch_copy_block(n, r, 1.0, V, ldv, DMat{nullptr, 0, 0, 0}, 0, (float *)w.V32.p, r, s));
        for (int j0 = 0; j0 < r; j0 += gw)
            CKR(clenshaw<float>(p, n, A->rowptr, A->colind, v32, gw, (const float *)w.V32.p + j0, r, W + j0, ldw,
                                (float *)w.U[0].p, (float *)w.U[1].p, (float *)w.U[2].p, s));
        return FLP_OK;
    }
    for (auto &u : w.U) CK(ensure(u, sizeof(double) * (size_t)n * gw));
    for (int j0 = 0; j0 < r; j0 += gw)
        CKR(clenshaw<double>(p, n, A->rowptr, A->colind, A->val, gw, V + j0, ldv, W + j0, ldw, (double *)w.U[0].p,
                             (double *)w.U[1].p, (double *)w.U[2].p, s));
    return FLP_OK;
}

// ------------------------------------------------------------------ small dense helpers (host)

// Upper Cholesky G = R^T R (r x r row-major).  Columns whose pivot falls
// below thr^2 are flagged bad: their row of R becomes e_i (placeholder) and
// later columns ignore them.
void cholesky_flag(int r, const double *G, double thr2, std::vector<double> &R, std::vector<int> &bad) {
    R.assign((size_t)r * r, 0.0);
    bad.assign(r, 0);
    for (int i = 0; i < r; ++i) {
        double d = G[i * r + i];
        for (int k = 0; k < i; ++k) d -= R[k * r + i] * R[k * r + i];
        if (!(d > thr2)) {
            bad[i] = 1;
            R[i * r + i] = 1.0;
            continue;
        }
        double rii = std::sqrt(d);
        R[i * r + i] = rii;
        for (int j = i + 1; j < r; ++j) {
            double t = G[i * r + j];
            for (int k = 0; k < i; ++k) t -= R[k * r + i] * R[k * r + j];
            R[i * r + j] = t / rii;
        }
    }
}

// inverse of an upper-triangular r x r
void upper_inverse(int r, const std::vector<double> &R, std::vector<double> &Ri) {
    Ri.assign((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j) {
        Ri[j * r + j] = 1.0 / R[j * r + j];
        for (int i = j - 1; i >= 0; --i) {
            double t = 0.0;
            for (int k = i + 1; k <= j; ++k) t += R[i * r + k] * Ri[k * r + j];
            Ri[i * r + j] = -t / R[i * r + i];
        }
    }
}

void matmul_upper(int r, const std::vector<double> &A, const std::vector<double> &B, std::vector<double> &C) {
    C.assign((size_t)r * r, 0.0);
    for (int i = 0; i < r; ++i)
        for (int k = 0; k < r; ++k)
            for (int j = 0; j < r; ++j) C[i * r + j] += A[i * r + k] * B[k * r + j];
}

// ------------------------------------------------------------------ device helpers

// Host -> device copy that is complete when it returns (the source may be a
// temporary host vector).
hipError_t h2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

int small_dev(size_t elems, double **out) {
    Workspace &w = ws();
    CK(ensure(w.small, elems * sizeof(double)));
    *out = (double *)w.small.p;
    return FLP_OK;
}

// C (K x c, host or device) = A^T B with A n x K (lda), B n x c (ldb).
// dev_out: device K x c row-major; host_out (optional) receives a copy
// (synchronises the stream).
int gram_tn(int n, int K, int c, DMat A, const double *B, int64_t ldb, double *dev_out,
            double *host_out, hipStream_t s) {
    Workspace &w = ws();
    TnPlan pl = plan_tn(n, K, c);
    CK(ensure(w.partials, pl.partial_elems * sizeof(double)));
    CK(launch_gemm_tn_partial(pl, n, K, c, A, B, ldb, (double *)w.partials.p, s));
    CK(launch_reduce_partials(pl, K, c, (double *)w.partials.p, dev_out, c, s));
    if (host_out) {
        CK(hipMemcpyAsync(host_out, dev_out, sizeof(double) * (size_t)K * c, hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
    }
    return FLP_OK;
}

// Two passes of classical Gram-Schmidt of W (n x r, ld r) against
// the first k columns of Q.  H1, H2 (k x r each) stay on the device in hdev[0..2kr).
int cgs2(DMat Q, int k, int n, double *W, int r, double *hdev, hipStream_t s) {
    for (int pass = 0; pass < 2; ++pass) {
        double *H = hdev + (size_t)pass * k * r;
        CKR(gram_tn(n, k, r, Q, W, r, H, nullptr, s));
        CK(launch_gemm_nn(n, k, r, -1.0, Q, H, r, 1.0, W, r, s));
    }
    return FLP_OK;
}

// Block normalisation W = Qn S by Cholesky QR twice (eq. lanczos: S upper
// triangular, non-negative diagonal).  Columns that are numerically
// dependent are replaced by random vectors orthogonalised against Q (when
// given) and the rest of the block; their rows of S are zero.  The Gram
// matrix carries an absolute rounding error of about u ||W||_F^2, so a
// Cholesky pivot sqrt(d_i) is only resolved down to ~1e-8 ||W||_F: a column
// counts as dependent when sqrt(d_i) < 1e-7 ||W||_F.  S: host r x r
// row-major.
int block_qr_impl(double *W, int n, int r, const DMat *Q, int k, std::vector<double> &S,
                  uint64_t seed, uint64_t sid, hipStream_t s, bool *replaced, int depth = 0) {
    if (depth > 3) return fail(FLP_E_DEVICE, "block QR: could not repair a rank-deficient block");
    double *dev = nullptr;
    CKR(small_dev((size_t)2 * std::max<int64_t>(k, r) * r + 4 * (size_t)r * r + 64, &dev));
    double *gdev = dev, *rdev = dev + r * r, *hdev = dev + 2 * r * r;
    std::vector<double> G((size_t)r * r), R1, R2, Ri;
    std::vector<int> bad, bad2;
    // pass 1
    CKR(gram_tn(n, r, r, plain_mat(W, r), W, r, gdev, G.data(), s));
    double fro2 = 0.0;
    for (int i = 0; i < r; ++i) fro2 += std::max(G[i * r + i], 0.0);
    const double thr = 1e-7 * std::sqrt(fro2);
    cholesky_flag(r, G.data(), std::max(thr * thr, 1e-300), R1, bad);
    int nbad = 0;
    for (int i = 0; i < r; ++i) nbad += bad[i];
    upper_inverse(r, R1, Ri);
    CK(h2d(rdev, Ri.data(), sizeof(double) * r * r, s));
    CK(launch_gemm_nn(n, r, r, 1.0, plain_mat(W, r), rdev, r, 0.0, W, r, s));
    if (nbad == 0) {
        // pass 2 on the (nearly) orthonormal block
        CKR(gram_tn(n, r, r, plain_mat(W, r), W, r, gdev, G.data(), s));
        cholesky_flag(r, G.data(), 1e-300, R2, bad2);
        for (int i = 0; i < r; ++i)
            if (bad2[i]) return fail(FLP_E_DEVICE, "block QR: second Cholesky pass broke down");
        upper_inverse(r, R2, Ri);
        CK(h2d(rdev, Ri.data(), sizeof(double) * r * r, s));
        CK(launch_gemm_nn(n, r, r, 1.0, plain_mat(W, r), rdev, r, 0.0, W, r, s));
        matmul_upper(r, R2, R1, S);
        CK(hipStreamSynchronize(s));
        return FLP_OK;
    }
    // repair: the good columns of W are now orthonormal; dependent ones are
    // replaced by random vectors, the block is re-orthogonalised against Q and
    // normalised again: W_orig ~= Qn (S2 S1) with S1 = R1 minus its bad rows.
    if (replaced) *replaced = true;
    std::vector<double> S1 = R1;
    for (int i = 0; i < r; ++i)
        if (bad[i])
            for (int j = 0; j < r; ++j) S1[i * r + j] = 0.0;
    for (int i = 0; i < r; ++i)
        if (bad[i]) CK(launch_randn(n, 1, W + i, r, seed, sid * 131 + depth * 17 + i + 1, s));
    if (Q && k > 0) CKR(cgs2(*Q, k, n, W, r, hdev, s));
    std::vector<double> S2;
    CKR(block_qr_impl(W, n, r, Q, k, S2, seed, sid + 7777, s, nullptr, depth + 1));
    matmul_upper(r, S2, S1, S);
    return FLP_OK;
}

// ------------------------------------------------------------------ bounds

int estimate_bounds_impl(const flp_csr *A, int k0, uint64_t seed, double *lmin, double *lmax, hipStream_t s) {
    Workspace &w = ws();
    const int n = A->n;
    int k = std::max(1, std::min(k0, n));
    const int ldb = (k + 2) & ~1;
    CK(ensure(w.Q, sizeof(double) * (size_t)n * ldb));
    CK(ensure(w.W, sizeof(double) * (size_t)n * 2));
    double *Qb = (double *)w.Q.p, *wv = (double *)w.W.p;
    double *dev = nullptr;
    CKR(small_dev((size_t)4 * ldb + 64, &dev));
    // start vector
    CK(launch_randn(n, 1, wv, 1, seed, 0xB0B0, s));
    double g = 0.0;
    CKR(gram_tn(n, 1, 1, plain_mat(wv, 1), wv, 1, dev, &g, s));
    if (!(g > 0.0)) return fail(FLP_E_DEVICE, "bounds: zero start vector");
    CK(launch_copy_block(n, 1, 1.0 / std::sqrt(g), wv, 1, plain_mat(Qb, ldb), 0, nullptr, 0, s));
    std::vector<double> al, be;
    std::vector<double> h1(k), h2(k);
    double beta_k = 0.0;
    int steps = 0;
    for (int j = 0; j < k; ++j) {
        // w = A q_j
        CK(launch_cheb_step<double, double>(n, A->rowptr, A->colind, A->val, 1, Qb + j, ldb, nullptr, 0, nullptr,
                                            0, wv, 1, 1.0, 0.0, 0.0, 0.0, s));
        CKR(cgs2(plain_mat(Qb, ldb), j + 1, n, wv, 1, dev, s));
        CK(hipMemcpyAsync(h1.data(), dev, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(h2.data(), dev + (j + 1), sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s));
        CKR(gram_tn(n, 1, 1, plain_mat(wv, 1), wv, 1, dev + 2 * ldb, &g, s));
        al.push_back(h1[j] + h2[j]);
        double bj = std::sqrt(std::max(g, 0.0));
        be.push_back(bj);
        steps = j + 1;
        beta_k = bj;
        if (bj == 0.0 || j == k - 1) break;
        CK(launch_copy_block(n, 1, 1.0 / bj, wv, 1, plain_mat(Qb, ldb), j + 1, nullptr, 0, s));
    }
    // Ritz values of the tridiagonal and the last eigenvector row
    std::vector<double> T((size_t)steps * steps, 0.0);
    for (int i = 0; i < steps; ++i) {
        T[(size_t)i * steps + i] = al[i];
        if (i + 1 < steps) {
            T[(size_t)i * steps + i + 1] = be[i];
            T[(size_t)(i + 1) * steps + i] = be[i];
        }
    }
    std::vector<double> theta(steps), last(steps);
    int row = steps - 1;
    if (sym_eig(steps, 1, T.data(), theta.data(), &row, 1, last.data()) != 0)
        return fail(FLP_E_DEVICE, "bounds: tridiagonal eigensolver did not converge");
    double rho_lo = std::fabs(beta_k * last[0]);
    double rho_hi = std::fabs(beta_k * last[steps - 1]);
    double delta = 1e-3 * (theta[steps - 1] - theta[0]);
    double lo = theta[0] - rho_lo - delta;
    double hi = theta[steps - 1] + rho_hi + delta;
    // Gershgorin enclosure
    int nb = gershgorin_blocks(n);
    CK(ensure(w.partials, sizeof(double) * (2 * (size_t)nb + 8)));
    CKR(small_dev((size_t)4 * ldb + 64, &dev));
    CK(launch_gershgorin(n, A->rowptr, A->colind, A->val, (double *)w.partials.p, nb, dev, s));
    double gg[2];
    CK(hipMemcpyAsync(gg, dev, sizeof(gg), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    *lmin = std::max(lo, gg[0]);
    *lmax = std::min(hi, gg[1]);
    if (!(*lmin < *lmax)) {
        // a matrix with a single distinct eigenvalue: widen symmetrically
        double mid = 0.5 * (*lmin + *lmax), rad = std::max(1e-12, 1e-8 * std::fabs(mid));
        *lmin = mid - rad;
        *lmax = mid + rad;
    }
    return FLP_OK;
}

// ------------------------------------------------------------------ solve

// Y (n x c, ld ldc) <- Y R^{-1} with Y^T Y = R^T R (one Cholesky QR pass);
// tmp is an n x c work block.
int orthonormalize_cols(int n, int c, double *&Y, double *&tmp, int ldc, double *sdev, hipStream_t s) {
    std::vector<double> G((size_t)c * c), R, Ri;
    std::vector<int> bad;
    CKR(gram_tn(n, c, c, plain_mat(Y, ldc), Y, ldc, sdev, G.data(), s));
    cholesky_flag(c, G.data(), 1e-300, R, bad);
    for (int i = 0; i < c; ++i)
        if (bad[i]) return fail(FLP_E_DEVICE, "Ritz block lost rank");
    upper_inverse(c, R, Ri);
    std::vector<double> Rp((size_t)c * ldc, 0.0);
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) Rp[(size_t)i * ldc + j] = Ri[(size_t)i * c + j];
    CK(h2d(sdev, Rp.data(), sizeof(double) * Rp.size(), s));
    CK(launch_gemm_nn(n, c, c, 1.0, plain_mat(Y, ldc), sdev, ldc, 0.0, tmp, ldc, s));
    std::swap(Y, tmp);
    return FLP_OK;
}

// Rayleigh-Ritz with A on the orthonormal block Y (eq. rayleigh, eq. proj):
// G = Y^T A Y = Z diag(lam) Z^T, X = Y Z, AX = (A Y) Z and the residual
// norms ||A x_j - lam_j x_j|| (host, unscaled).  lam ascending.
int rayleigh_ritz(const flp_csr *A, int n, int c, const double *Y, double *AY, double *X, double *AX, int ldc,
                  double *sdev, std::vector<double> &lam, std::vector<double> &res, hipStream_t s) {
    Workspace &w = ws();
    for (int j0 = 0; j0 < c; j0 += 16) {
        int cw = std::min(16, c - j0);
        CK(launch_cheb_step<double, double>(n, A->rowptr, A->colind, A->val, cw, Y + j0, ldc, nullptr, 0, nullptr,
                                            0, AY + j0, ldc, 1.0, 0.0, 0.0, 0.0, s));
    }
    std::vector<double> G((size_t)c * c);
    CKR(gram_tn(n, c, c, plain_mat(Y, ldc), AY, ldc, sdev, G.data(), s));
    std::vector<double> Gs((size_t)c * c);
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) Gs[(size_t)i * c + j] = 0.5 * (G[(size_t)i * c + j] + G[(size_t)j * c + i]);
    lam.assign(c, 0.0);
    std::vector<double> ZG((size_t)c * c);
    std::vector<int> rows(c);
    for (int i = 0; i < c; ++i) rows[i] = i;
    if (sym_eig(c, c - 1, Gs.data(), lam.data(), rows.data(), c, ZG.data()) != 0)
        return fail(FLP_E_DEVICE, "eigensolver for the Rayleigh-Ritz matrix did not converge");
    std::vector<double> Zp((size_t)c * ldc, 0.0);
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) Zp[(size_t)i * ldc + j] = ZG[(size_t)i * c + j];
    CK(h2d(sdev, Zp.data(), sizeof(double) * Zp.size(), s));
    CK(launch_gemm_nn(n, c, c, 1.0, plain_mat(Y, ldc), sdev, ldc, 0.0, X, ldc, s));
    CK(launch_gemm_nn(n, c, c, 1.0, plain_mat(AY, ldc), sdev, ldc, 0.0, AX, ldc, s));
    double *lamd = sdev + (size_t)c * ldc;
    double *rdev = lamd + ldc;
    CK(h2d(lamd, lam.data(), sizeof(double) * c, s));
    int nch = resid_chunks(n);
    CK(ensure(w.resid_part, sizeof(double) * (size_t)nch * c));
    CK(launch_resid_norms(n, c, AX, ldc, X, ldc, lamd, (double *)w.resid_part.p, nch, rdev, s));
    res.assign(c, 0.0);
    CK(hipMemcpyAsync(res.data(), rdev, sizeof(double) * c, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return FLP_OK;
}

int solve_impl(const flp_csr *A, double alpha, double beta, const flp_opts &o, flp_result **out) {
    const double t_start = now();
    hipStream_t s = (hipStream_t)o.stream;
    Workspace &w = ws();
    const int n = A->n;
    const int r = o.block;
    if (r < 1 || r > 16) return fail(FLP_E_ARG, "block size must be in [1, 16]");
    if (r > n) return fail(FLP_E_ARG, "block size exceeds n");
    if (!(std::isfinite(alpha) && std::isfinite(beta)) || !(alpha < beta))
        return fail(FLP_E_ARG, "need finite alpha < beta");
    if (o.prec != FLP_PREC_FP64 && o.prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    flp_stats st{};

    // PREPROC: spectrum bounds
    double lmin, lmax;
    double t0 = now();
    if (o.lmin < o.lmax) {
        lmin = o.lmin;
        lmax = o.lmax;
    } else {
        CKR(estimate_bounds_impl(A, o.k0 > 0 ? o.k0 : kDefaultK0, o.seed, &lmin, &lmax, s));
    }
    st.t_pre = now() - t0;

    flp_filter *pf = nullptr;
    CKR(make_filter(alpha, beta, o.degree, lmin, lmax, o.eps > 0 ? o.eps : kDefaultEps, &pf));
    std::unique_ptr<flp_filter> filt(pf);
    const double tau = 0.5 * std::min(cheb_scalar(filt->b, filt->a1), cheb_scalar(filt->b, filt->b1));
    const double tol_p = o.prec == FLP_PREC_FP32_FILTER ? 1e-5 : 1e-10;
    const int check_every = o.check_every > 0 ? o.check_every : kDefaultCheck;

    int64_t maxb = o.max_basis > 0 ? o.max_basis : kDefaultMaxBasis;
    maxb = std::min<int64_t>(maxb, n);
    const int max_steps = std::max<int>(1, (int)(maxb / r));
    // Lanczos basis: column panels of 128 columns, each a contiguous
    // row-major n x 128 block (the reorthogonalisation streams whole panels)
    const int lpw = 7;
    const int64_t npanels = ((int64_t)max_steps * r + (1 << lpw) - 1) >> lpw;
    CK(ensure(w.Q, sizeof(double) * (size_t)n * (size_t)(npanels << lpw)));
    CK(ensure(w.W, sizeof(double) * (size_t)n * r));
    CK(ensure(w.Vin, sizeof(double) * (size_t)n * r));
    double *W = (double *)w.W.p, *Vin = (double *)w.Vin.p;
    const DMat Q = panel_mat((double *)w.Q.p, n, lpw);
    double *hdev = nullptr;
    CKR(small_dev((size_t)2 * (npanels << lpw) * r + 4 * r * r + 64, &hdev));

    // start block
    if (o.start) {
        CK(h2d(W, o.start, sizeof(double) * (size_t)n * r, s));
    } else {
        CK(launch_randn(n, r, W, r, o.seed, 0x51A7, s));
    }
    std::vector<double> Sj;
    CKR(block_qr_impl(W, n, r, nullptr, 0, Sj, o.seed, 1, s, nullptr));
    CK(launch_copy_block(n, r, 1.0, W, r, Q, 0, nullptr, 0, s));
    CK(launch_copy_block(n, r, 1.0, W, r, plain_mat(Vin, r), 0, nullptr, 0, s));

    hipEvent_t ev[4];
    for (auto &e : ev) CK(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};

    std::vector<double> D_all, S_all;  // per step r x r
    std::vector<double> h1((size_t)r * r), h2((size_t)r * r);
    int steps = 0, prev_count = -1;
    bool converged = false;
    std::vector<int> cand;
    std::vector<double> theta;
    int kfinal = 0;
    const double step_bytes = filter_step_bytes(n, A->nnz, r, o.prec);
    while (steps < max_steps) {
        const int k = (steps + 1) * r;  // basis columns so far
        CK(hipEventRecord(ev[0], s));
        CKR(filter_apply_impl(filt.get(), A, Vin, r, W, r, r, o.prec, s));
        CK(hipEventRecord(ev[1], s));
        st.filter_bytes += step_bytes * filt->m;
        st.mv += (int64_t)r * filt->m;
        CKR(cgs2(Q, k, n, W, r, hdev, s));
        CK(hipMemcpyAsync(h1.data(), hdev + (size_t)(k - r) * r, sizeof(double) * r * r, hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(h2.data(), hdev + (size_t)k * r + (size_t)(k - r) * r, sizeof(double) * r * r,
                          hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) {
                double a = h1[i * r + j] + h2[i * r + j], b = h1[j * r + i] + h2[j * r + i];
                D_all.push_back(0.5 * (a + b));
            }
        CKR(block_qr_impl(W, n, r, &Q, k, Sj, o.seed, 1000 + steps, s, nullptr));
        S_all.insert(S_all.end(), Sj.begin(), Sj.end());
        CK(hipEventRecord(ev[2], s));
        CK(hipEventSynchronize(ev[2]));
        float ms_mv = 0, ms_orth = 0;
        CK(hipEventElapsedTime(&ms_mv, ev[0], ev[1]));
        CK(hipEventElapsedTime(&ms_orth, ev[1], ev[2]));
        st.t_mv += ms_mv * 1e-3;
        st.t_orth += ms_orth * 1e-3;
        ++steps;
        const bool last = steps == max_steps || (int64_t)(steps + 1) * r > n;
        if (steps % check_every == 0 || last) {
            double tc = now();
            const int K = k;
            std::vector<double> T((size_t)K * K, 0.0);
            for (int b = 0; b < steps; ++b) {
                for (int i = 0; i < r; ++i)
                    for (int j = 0; j < r; ++j) {
                        T[(size_t)(b * r + i) * K + b * r + j] = D_all[(size_t)b * r * r + i * r + j];
                        if (b + 1 < steps) {
                            double sv = S_all[(size_t)b * r * r + i * r + j];  // S_b(i, j)
                            T[(size_t)((b + 1) * r + i) * K + b * r + j] = sv;
                            T[(size_t)(b * r + j) * K + (b + 1) * r + i] = sv;
                        }
                    }
            }
            theta.assign(K, 0.0);
            std::vector<int> rows(r);
            for (int i = 0; i < r; ++i) rows[i] = K - r + i;
            std::vector<double> Zl((size_t)r * K);
            if (sym_eig(K, r, T.data(), theta.data(), rows.data(), r, Zl.data()) != 0)
                return fail(FLP_E_DEVICE, "eigensolver for T_k did not converge");
            // rho_i = || S_k E_k^T w_i ||
            double big = 1e-300;
            for (double t : theta) big = std::max(big, std::fabs(t));
            cand.clear();
            bool ok = true;
            for (int i = 0; i < K; ++i) {
                if (theta[i] < tau) continue;
                cand.push_back(i);
                double rho2 = 0.0;
                for (int a = 0; a < r; ++a) {
                    double t = 0.0;
                    for (int b = 0; b < r; ++b) t += Sj[a * r + b] * Zl[(size_t)b * K + i];
                    rho2 += t * t;
                }
                if (std::sqrt(rho2) > tol_p * big) ok = false;
            }
            st.t_check += now() - tc;
            if ((ok && (int)cand.size() == prev_count) || last) {
                converged = ok && (int)cand.size() == prev_count;
                kfinal = K;
                break;
            }
            prev_count = (int)cand.size();
        }
        CK(launch_copy_block(n, r, 1.0, W, r, Q, k, nullptr, 0, s));
        CK(launch_copy_block(n, r, 1.0, W, r, plain_mat(Vin, r), 0, nullptr, 0, s));
    }
    st.iters = steps;
    st.basis_cols = kfinal;

    // ---- Rayleigh-Ritz with A on the candidate Ritz vectors
    double tr = now();
    const double anorm = std::max(std::fabs(lmin), std::fabs(lmax));
    auto *res = new flp_result;
    std::memset(res, 0, sizeof(*res));
    res->n = n;
    res->lmin = lmin;
    res->lmax = lmax;
    res->alpha = alpha;
    res->beta = beta;
    res->degree = filt->m;
    res->converged = converged ? 1 : 0;
    std::unique_ptr<flp_result, void (*)(flp_result *)> guard(res, flp_result_free);
    const int c = (int)cand.size();
    if (c > 0) {
        const int K = kfinal;
        // full eigenvectors of T_k for the candidates
        std::vector<double> T((size_t)K * K, 0.0);
        for (int b = 0; b < steps; ++b)
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < r; ++j) {
                    T[(size_t)(b * r + i) * K + b * r + j] = D_all[(size_t)b * r * r + i * r + j];
                    if (b + 1 < steps) {
                        double sv = S_all[(size_t)b * r * r + i * r + j];
                        T[(size_t)((b + 1) * r + i) * K + b * r + j] = sv;
                        T[(size_t)(b * r + j) * K + (b + 1) * r + i] = sv;
                    }
                }
        std::vector<int> rows(K);
        for (int i = 0; i < K; ++i) rows[i] = i;
        std::vector<double> Z((size_t)K * K), th(K);
        double tc = now();
        if (sym_eig(K, r, T.data(), th.data(), rows.data(), K, Z.data()) != 0)
            return fail(FLP_E_DEVICE, "eigensolver for T_k did not converge");
        st.t_check += now() - tc;
        const int ldc = (c + 1) & ~1;
        std::vector<double> Wc((size_t)K * ldc, 0.0);
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < c; ++j) Wc[(size_t)i * ldc + j] = Z[(size_t)i * K + cand[j]];
        CK(ensure(w.Y, sizeof(double) * (size_t)n * ldc));
        CK(ensure(w.AY, sizeof(double) * (size_t)n * ldc));
        CK(ensure(w.X, sizeof(double) * (size_t)n * ldc));
        CK(ensure(w.AX, sizeof(double) * (size_t)n * ldc));
        double *Y = (double *)w.Y.p, *AY = (double *)w.AY.p, *X = (double *)w.X.p, *AX = (double *)w.AX.p;
        double *sdev = nullptr;
        CKR(small_dev((size_t)std::max(K, c) * ldc * 2 + 4 * (size_t)ldc + 64, &sdev));
        CK(h2d(sdev, Wc.data(), sizeof(double) * Wc.size(), s));
        // Ritz vectors of p(A): Y = Q_k W_C (eq. proj)
        CK(launch_gemm_nn(n, K, c, 1.0, Q, sdev, ldc, 0.0, Y, ldc, s));
        CKR(orthonormalize_cols(n, c, Y, X, ldc, sdev, s));
        std::vector<double> lam, rres;
        CKR(rayleigh_ritz(A, n, c, Y, AY, X, AX, ldc, sdev, lam, rres, s));
        // FP32 filter: FP64 polish sweeps (X <- p(A) X, orthonormalise, RR
        // with A) until the in-interval residuals meet the tolerance
        auto worst = [&](int &i0, int &i1) {
            i0 = 0;
            while (i0 < c && lam[i0] < alpha) ++i0;
            i1 = i0;
            while (i1 < c && lam[i1] <= beta) ++i1;
            double m = 0.0;
            for (int j = i0; j < i1; ++j) m = std::max(m, rres[j] / anorm);
            return m;
        };
        const double tol = o.tol > 0 ? o.tol : kDefaultTol;
        int i0 = 0, i1 = 0;
        if (o.prec == FLP_PREC_FP32_FILTER) {
            while (worst(i0, i1) > tol && st.polish_sweeps < 3) {
                for (auto &u : w.U) CK(ensure(u, sizeof(double) * (size_t)n * 16));
                for (int j0 = 0; j0 < c; j0 += 16) {
                    int cw = std::min(16, c - j0);
                    CKR(filter_apply_impl(filt.get(), A, X + j0, ldc, Y + j0, ldc, cw, FLP_PREC_FP64, s));
                }
                st.filter_bytes += filter_step_bytes(n, A->nnz, 16, FLP_PREC_FP64) * filt->m * ((c + 15) / 16);
                CKR(orthonormalize_cols(n, c, Y, X, ldc, sdev, s));
                CKR(orthonormalize_cols(n, c, Y, X, ldc, sdev, s));
                CKR(rayleigh_ritz(A, n, c, Y, AY, X, AX, ldc, sdev, lam, rres, s));
                ++st.polish_sweeps;
            }
        }
        worst(i0, i1);
        const int cnt = i1 - i0;
        res->count = cnt;
        if (cnt > 0) {
            res->evals = new double[cnt];
            res->resid = new double[cnt];
            for (int j = 0; j < cnt; ++j) {
                res->evals[j] = lam[i0 + j];
                res->resid[j] = rres[i0 + j] / anorm;
            }
            CK(hipMalloc(&res->evecs, sizeof(double) * (size_t)n * cnt));
            CK(launch_transpose_out(n, cnt, X + i0, ldc, res->evecs, s));
            CK(hipStreamSynchronize(s));
        }
    }
    st.t_rr = now() - tr;
    st.t_total = now() - t_start;
    res->stats = st;
    *out = guard.release();
    return converged ? FLP_OK : FLP_E_NOCONV;
}

}  // namespace
}  // namespace flp

// ====================================================================== C ABI

extern "C" {

void flp_opts_default(flp_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->block = 1;
    o->degree = 0;
    o->eps = kDefaultEps;
    o->tol = kDefaultTol;
    o->check_every = kDefaultCheck;
    o->prec = FLP_PREC_FP64;
    o->seed = 0;
    o->max_basis = 0;
    o->k0 = kDefaultK0;
    o->start = nullptr;
    o->lmin = 0.0;
    o->lmax = 0.0;
    o->stream = nullptr;
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

int flp_filter_apply(const flp_filter *p, const flp_csr *A, const double *V, double *W, int32_t r, int32_t prec,
                     void *stream) {
    if (!p) return fail(FLP_E_ARG, "filter is NULL");
    CKR(check_csr(A));
    if (r < 1 || r > 32) return fail(FLP_E_ARG, "r must be in [1, 32]");
    if (!V || !W) return fail(FLP_E_ARG, "V and W must be non-NULL");
    if (V == W) return fail(FLP_E_ARG, "W must not alias V");
    if (prec != FLP_PREC_FP64 && prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    return filter_apply_impl(p, A, V, r, W, r, r, prec, (hipStream_t)stream);
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

void flp_result_free(flp_result *res) {
    if (!res) return;
    delete[] res->evals;
    delete[] res->resid;
    if (res->evecs) (void)hipFree(res->evecs);
    delete res;
}

int flp_result_copy_evecs(const flp_result *res, double *dst, void *stream) {
    if (!res || !dst) return fail(FLP_E_ARG, "NULL argument");
    if (res->count == 0) return FLP_OK;
    CK(hipMemcpyAsync(dst, res->evecs, sizeof(double) * (size_t)res->n * res->count, hipMemcpyDeviceToDevice,
                      (hipStream_t)stream));
    return FLP_OK;
}

int flp_host_sym_eig(int32_t N, int32_t bw, const double *M, double *evals, double *evecs) {
    if (N < 1 || !M || !evals || bw < 0) return fail(FLP_E_ARG, "bad arguments");
    try {
        std::vector<int> rows;
        if (evecs) {
            rows.resize(N);
            for (int i = 0; i < N; ++i) rows[i] = i;
        }
        int rc = sym_eig(N, bw, M, evals, evecs ? rows.data() : nullptr, evecs ? N : 0, evecs);
        if (rc != 0) return fail(FLP_E_ARG, "eigensolver did not converge");
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    }
    return FLP_OK;
}

void flp_release_workspace(void) {
    Workspace &w = ws();
    Buf *all[] = {&w.U[0], &w.U[1], &w.U[2], &w.V32, &w.val32, &w.partials, &w.small, &w.W,
                  &w.Vin,   &w.Q,    &w.Y,    &w.AY,  &w.X,     &w.AX,       &w.resid_part};
    for (Buf *b : all) {
        if (b->p) (void)hipFree(b->p);
        b->p = nullptr;
        b->bytes = 0;
    }
    w.val32_src = nullptr;
    w.val32_nnz = 0;
}

const char *flp_last_error(void) { return g_last_error.c_str(); }

const char *flp_version(void) { return "flp-mi355x 0.1"; }

}  // extern "C"
