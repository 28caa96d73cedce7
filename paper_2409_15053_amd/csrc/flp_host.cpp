// Host-side helpers of the filtered Lanczos procedure: workspace, filter
// construction and the Clenshaw launch plan (Section 2.2), two-pass
// Gram-Schmidt and block QR (Sections 2.3, 3.2.2), spectrum bounds, and
// Rayleigh-Ritz with A (eq. rayleigh, eq. proj).  The device work runs in
// the kernels of flp_kernels.hip; the small projected problems are solved on
// the host with the banded eigensolver of flp_eigen.cpp, as in the paper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "flp_host.h"

namespace flp {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ device memory
//
// Every device allocation of the library goes through dev_alloc/dev_free:
// the library's own cache over hipMalloc, or the caller's functions set by
// flp_set_allocator.  Each allocation remembers which allocator made it, so
// memory is always returned to its own allocator even if the setting
// changes in between.  A free synchronises the device first (work still
// queued on any of the library's streams may use the block), as hipFree
// would.
//
// The cache: blocks of 1 MiB and more are rounded up to 2 MiB and, when
// freed, kept per device (up to kDevCacheBytes) for the next request they fit
// within 25 %.  The batched engine and the server allocate and release tens
// of GB per batch (bases, recurrence vectors, Ritz blocks); returning them to
// the driver every time made later batches stall for seconds.
// flp_release_workspace() hands the cached blocks back.

namespace {
struct Allocator {
    flp_alloc_fn alloc = nullptr;
    flp_free_fn free = nullptr;
    void *ctx = nullptr;
};
struct Block {
    int device;
    size_t bytes;  // 0: not cached (small, straight hipMalloc)
};
constexpr size_t kCacheMin = (size_t)1 << 20;
constexpr size_t kCacheGrain = (size_t)2 << 20;
constexpr size_t kDevCacheBytes = (size_t)64 << 30;
std::mutex g_alloc_mu;
Allocator g_alloc;
std::unordered_map<void *, Allocator> &custom_allocs() {
    static std::unordered_map<void *, Allocator> m;
    return m;
}
std::unordered_map<void *, Block> &own_blocks() {
    static std::unordered_map<void *, Block> m;
    return m;
}
struct DevCache {
    std::multimap<size_t, void *> free;  // size -> block
    size_t bytes = 0;
};
std::map<int, DevCache> &dev_cache() {
    static std::map<int, DevCache> m;
    return m;
}
}  // namespace

std::shared_mutex &capture_mutex() {
    static std::shared_mutex m;
    return m;
}

void set_allocator(flp_alloc_fn alloc, flp_free_fn free, void *ctx) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = (alloc && free) ? Allocator{alloc, free, ctx} : Allocator{};
}

hipError_t dev_alloc(void **p, size_t bytes) {
    Allocator a;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        a = g_alloc;
    }
    if (a.alloc) {
        *p = a.alloc(bytes, a.ctx);
        if (!*p) return hipErrorOutOfMemory;
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        custom_allocs()[*p] = a;
        return hipSuccess;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (bytes < kCacheMin) {
        e = hipMalloc(p, bytes);
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_alloc_mu);
            own_blocks()[*p] = Block{dev, 0};
        }
        return e;
    }
    const size_t want = (bytes + kCacheGrain - 1) / kCacheGrain * kCacheGrain;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        DevCache &c = dev_cache()[dev];
        auto it = c.free.lower_bound(want);
        if (it != c.free.end() && it->first <= want + want / 4) {
            *p = it->second;
            own_blocks()[*p] = Block{dev, it->first};
            c.bytes -= it->first;
            c.free.erase(it);
            return hipSuccess;
        }
    }
    e = hipMalloc(p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // the cached blocks may be what is in the way
        release_dev_cache();
        e = hipMalloc(p, want);
        if (e != hipSuccess) return e;
    }
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    own_blocks()[*p] = Block{dev, want};
    return hipSuccess;
}

hipError_t dev_free(void *p) {
    if (!p) return hipSuccess;
    Allocator a;
    Block b{0, 0};
    bool custom = false, own = false;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = custom_allocs().find(p);
        if (it != custom_allocs().end()) {
            a = it->second;
            custom_allocs().erase(it);
            custom = true;
        } else {
            auto ob = own_blocks().find(p);
            if (ob != own_blocks().end()) {
                b = ob->second;
                own_blocks().erase(ob);
                own = true;
            }
        }
    }
    if (custom) {
        hipError_t e;
        {
            std::unique_lock<std::shared_mutex> cl(capture_mutex());
            e = hipDeviceSynchronize();
        }
        a.free(p, a.ctx);
        return e;
    }
    if (!own || b.bytes == 0) return hipFree(p);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != b.device) (void)hipSetDevice(b.device);
    hipError_t e;
    {
        std::unique_lock<std::shared_mutex> cl(capture_mutex());
        e = hipDeviceSynchronize();
    }
    if (cur != b.device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        DevCache &c = dev_cache()[b.device];
        if (c.bytes + b.bytes <= kDevCacheBytes) {
            c.free.emplace(b.bytes, p);
            c.bytes += b.bytes;
            return hipSuccess;
        }
    }
    return hipFree(p);
}

void release_dev_cache() {
    std::vector<std::pair<int, void *>> all;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        for (auto &kv : dev_cache()) {
            for (auto &f : kv.second.free) all.emplace_back(kv.first, f.second);
            kv.second.free.clear();
            kv.second.bytes = 0;
        }
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &d : all) {
        (void)hipSetDevice(d.first);
        (void)hipFree(d.second);
    }
    (void)hipSetDevice(cur);
}

// ------------------------------------------------------------------ workspace

Buf::~Buf() { release(); }

void Buf::release() {
    if (p) (void)dev_free(p);
    p = nullptr;
    bytes = 0;
}

hipError_t ensure_grow(Buf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return hipSuccess;
    return ensure(b, std::max(bytes, b.bytes + b.bytes / 2));
}

hipError_t ensure(Buf &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = dev_free(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = dev_alloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return e;
    }
    b.bytes = want;
    return hipSuccess;
}

void Workspace::release_all() {
    Buf *all[] = {&U[0],   &U[1],   &U[2],       &V32,  &Vg,    &val32,    &partials, &small,
                  &W,      &Vin,    &Q,          &Y,    &AY,    &X,        &AX,       &resid_part,
                  &PU[0],  &PU[1],  &PU[2],      &PR,   &PC,    &sell_off, &sell_col, &sell_val};
    for (Buf *b : all) b->release();
    val32_src = nullptr;
    val32_nnz = 0;
    sell_valid = false;
}

namespace {
// Host worker pool for the convergence checks.  Each worker limits the
// eigensolver's own inner threads so that concurrent checks share the cores.
struct HostPool {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    std::vector<std::thread> th;
    bool stop = false;
    HostPool() {
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        const int nw = std::max(2, std::min(16, hw / 2));
        for (int i = 0; i < nw; ++i)
            th.emplace_back([this, hw, nw]() {
                set_eig_threads(std::max(1, std::min(16, hw) / nw));
                for (;;) {
                    std::function<void()> f;
                    {
                        std::unique_lock<std::mutex> lk(mu);
                        cv.wait(lk, [&] { return stop || !q.empty(); });
                        if (stop && q.empty()) return;
                        f = std::move(q.front());
                        q.pop_front();
                    }
                    f();
                }
            });
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto &t : th) t.join();
    }
};
HostPool &host_pool() {
    static HostPool p;
    return p;
}
}  // namespace

void host_pool_submit(std::function<void()> f) {
    HostPool &p = host_pool();
    {
        std::lock_guard<std::mutex> lk(p.mu);
        p.q.push_back(std::move(f));
    }
    p.cv.notify_one();
}

Workspace &ws() {
    // per thread and device: the batched engine's finisher thread works
    // beside its stepping thread
    static thread_local Workspace w[64];
    int dev = 0;
    (void)hipGetDevice(&dev);
    return w[dev & 63];
}

// ------------------------------------------------------------------ CSR checks

int check_csr(const flp_csr *A) {
    if (!A) return fail(FLP_E_ARG, "A is NULL");
    if (A->n <= 0) return fail(FLP_E_ARG, "n must be positive");
    if (A->nnz < 0 || A->nnz >= (int64_t(1) << 31)) return fail(FLP_E_ARG, "nnz must be in [0, 2^31)");
    if (!A->rowptr || (A->nnz > 0 && (!A->colind || !A->val)))
        return fail(FLP_E_ARG, "CSR pointers must be non-NULL");
    return FLP_OK;
}


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

// Chebyshev coefficients c_0..c_{m-1} of g(z) = (p(z) - p(t)) / (z - t) for
// p = sum_k b_k T_k (degree m >= 1): synthetic division by (z - t) in the
// Chebyshev basis.  With z T_0 = T_1 and z T_k = (T_{k+1} + T_{k-1}) / 2,
// matching the coefficients of (z - t) g = p - p(t) from T_m down gives
// c_{m-1} = 2 b_m, c_{j-1} = 2 (b_j + t c_j) - c_{j+1} (j = m-1 .. 2) and
// c_0 = b_1 + t c_1 - c_2 / 2 (the T_0 equation then holds by itself).
void cheb_divided(const std::vector<double> &b, double t, std::vector<double> &c) {
    const int m = (int)b.size() - 1;
    c.assign(std::max(m, 1) + 2, 0.0);
    if (m >= 2) {
        c[m - 1] = 2.0 * b[m];
        for (int j = m - 1; j >= 2; --j) c[j - 1] = 2.0 * (b[j] + t * c[j]) - c[j + 1];
    }
    if (m >= 1) c[0] = b[1] + t * c[1] - 0.5 * c[2];
    c.resize(std::max(m, 1));
}

// b_0..b_m of the indicator of [a, b] in [-1, 1] (closed form of Section 2.2).
static void indicator_coeffs(double a1, double b1, int m, std::vector<double> &out) {
    double ta = std::acos(a1), tb = std::acos(b1);
    out.assign(m + 1, 0.0);
    out[0] = (ta - tb) / M_PI;
    for (int i = 1; i <= m; ++i) out[i] = 2.0 * (std::sin(i * ta) - std::sin(i * tb)) / (i * M_PI);
}

// Smallest m >= 1 with ||p_m - phi||_mu < eps ||phi||_mu (eq. optimaldegree);
// the squared error falls by (pi/2) b_m^2 per degree from
// ||phi||^2 - pi b_0^2, with ||phi||^2 = acos(a) - acos(b).
static int auto_degree(double a1, double b1, double eps) {
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
std::vector<ClenshawStep> clenshaw_plan(const flp_filter *p, int r, const void *V, int ldv, double *W, int ldw,
                                        void *U0, void *U1, void *U2, bool fp32) {
    const int m = p->m;
    const std::vector<double> &b = p->b;
    const double c = p->c, e = p->e;
    const int ld = r;
    std::vector<ClenshawStep> out;
    auto step = [&](const void *X, int ldx, const void *Vv, const void *Y, void *o, int ldo, bool f64, double al,
                    double be, double ga, double de) {
        out.push_back(ClenshawStep{X, ldx, Vv, ldv, Y, ld, o, ldo, f64, al, be, ga, de});
    };
    const bool last_f64 = true;  // W is FP64 in both precisions
    if (m == 1) {
        step(V, ldv, nullptr, nullptr, W, ldw, last_f64, b[1] / e, b[0] - c * b[1] / e, 0.0, 0.0);
        return out;
    }
    void *ring[3] = {U0, U1, U2};
    // U_{m-1} = b_{m-1} V + (2 b_m / e) (A V - c V)
    void *u_k1 = ring[0];
    step(V, ldv, nullptr, nullptr, u_k1, ld, !fp32, 2.0 * b[m] / e, b[m - 1] - 2.0 * c * b[m] / e, 0.0, 0.0);
    void *u_k2 = nullptr;  // U_{k+2}; U_m = b_m V is folded into the V coefficient
    int slot = 1;
    for (int k = m - 2; k >= 1; --k) {
        void *o = ring[slot];
        slot = (slot + 1) % 3;
        if (k == m - 2)
            step(u_k1, ld, V, nullptr, o, ld, !fp32, 2.0 / e, -2.0 * c / e, b[k] - b[m], 0.0);
        else
            step(u_k1, ld, V, u_k2, o, ld, !fp32, 2.0 / e, -2.0 * c / e, b[k], -1.0);
        u_k2 = u_k1;
        u_k1 = o;
    }
    // W = b_0 V + Ahat U_1 - U_2
    if (m == 2)
        step(u_k1, ld, V, nullptr, W, ldw, last_f64, 1.0 / e, -c / e, b[0] - b[2], 0.0);
    else
        step(u_k1, ld, V, u_k2, W, ldw, last_f64, 1.0 / e, -c / e, b[0], -1.0);
    return out;
}

// Launch one planned step with the direct (single-matrix) kernel.
int launch_plan_step(const flp_csr *A, const float *val32, int r, const ClenshawStep &st, bool fp32,
                     hipStream_t s, StepShape sh, bool sell) {
    const int n = A->n;
    if (!fp32) {
        CK(launch_cheb_step<double, double>(n, A->rowptr, A->colind, A->val, r, (const double *)st.X, st.ldx,
                                            (const double *)st.V, st.ldv, (const double *)st.Y, st.ldy,
                                            (double *)st.out, st.ldo, st.alpha, st.beta, st.gamma, st.delta, s,
                                            sh, sell));
    } else if (st.out_f64) {
        CK(launch_cheb_step<float, double>(n, A->rowptr, A->colind, val32, r, (const float *)st.X, st.ldx,
                                           (const float *)st.V, st.ldv, (const float *)st.Y, st.ldy,
                                           (double *)st.out, st.ldo, (float)st.alpha, (float)st.beta,
                                           (float)st.gamma, (float)st.delta, s, sh, sell));
    } else {
        CK(launch_cheb_step<float, float>(n, A->rowptr, A->colind, val32, r, (const float *)st.X, st.ldx,
                                          (const float *)st.V, st.ldv, (const float *)st.Y, st.ldy,
                                          (float *)st.out, st.ldo, (float)st.alpha, (float)st.beta,
                                          (float)st.gamma, (float)st.delta, s, sh, sell));
    }
    return FLP_OK;
}

int build_sell(const flp_csr *A, const float *val32, bool fp32, Buf &boff, Buf &bcol, Buf &bval, flp_csr *out,
               const float **out32, hipStream_t s, double max_pad, bool *built) {
    *built = false;
    const int n = A->n;
    std::vector<int32_t> rp((size_t)n + 1);
    CK(hipMemcpyAsync(rp.data(), A->rowptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    const int nsl = (n + kSellC - 1) / kSellC;
    std::vector<int32_t> off((size_t)nsl + 1);
    int64_t tot = 0;
    for (int i = 0; i < nsl; ++i) {
        int w = 0;
        for (int j = i * kSellC; j < std::min(n, (i + 1) * kSellC); ++j) w = std::max(w, rp[j + 1] - rp[j]);
        off[i] = (int32_t)tot;
        tot += (int64_t)w * kSellC;
        if (tot > INT32_MAX) return fail(FLP_E_ARG, "the sliced ELL copy of A would exceed 2^31 entries");
    }
    off[nsl] = (int32_t)tot;
    if ((double)tot > max_pad * (double)A->nnz + kSellC) return FLP_OK;
    const size_t ents = (size_t)std::max<int64_t>(tot, 1);
    CK(ensure(boff, sizeof(int32_t) * ((size_t)nsl + 1)));
    CK(ensure(bcol, sizeof(int32_t) * ents));
    CK(ensure(bval, (fp32 ? sizeof(float) : sizeof(double)) * ents));
    CK(h2d(boff.p, off.data(), sizeof(int32_t) * ((size_t)nsl + 1), s));
    auto *col = (int32_t *)bcol.p;
    CK(launch_sell_fill(n, A->rowptr, A->colind, fp32 ? nullptr : A->val, fp32 ? val32 : nullptr,
                        (const int32_t *)boff.p, nsl, col, fp32 ? nullptr : (double *)bval.p,
                        fp32 ? (float *)bval.p : nullptr, s));
    CK(hipStreamSynchronize(s));
    *out = *A;
    out->rowptr = (const int32_t *)boff.p;
    out->colind = col;
    out->nnz = tot;
    out->val = fp32 ? nullptr : (const double *)bval.p;
    out->val32 = nullptr;
    *out32 = fp32 ? (const float *)bval.p : nullptr;
    *built = true;
    return FLP_OK;
}

// Filter bytes per SpMM step: matrix once, gathered input once, V, U_{k+2}
// and the output once each.
double filter_step_bytes(int n, int64_t nnz, int r, int prec) {
    double wv = prec == FLP_PREC_FP32_FILTER ? 4.0 : 8.0;
    return (double)nnz * (wv + 4.0) + 4.0 * (n + 1) + 4.0 * n * r * wv;
}

int ensure_val32(const flp_csr *A, Buf &buf, const double **src_cache, int64_t *nnz_cache, const float **out,
                 hipStream_t s) {
    if (A->val32) {
        *out = A->val32;
        return FLP_OK;
    }
    if (*src_cache != A->val || *nnz_cache != A->nnz || !buf.p) {
        CK(ensure(buf, sizeof(float) * std::max<int64_t>(A->nnz, 1)));
        CK(launch_to_float(A->nnz, A->val, (float *)buf.p, s));
        *src_cache = A->val;
        *nnz_cache = A->nnz;
    }
    *out = (const float *)buf.p;
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
// The storage the calling thread's filter products read A in: A itself, or
// its sliced ELL copy in the workspace (built once per matrix and precision,
// then reused) when format asks for it (FLP_FORMAT_AUTO: only if padding
// adds under kSellMaxPad).
int workspace_storage(const flp_csr *A, const float *v32, bool fp32, int format, hipStream_t s,
                      const flp_csr **fA, const float **fv32, bool *sell) {
    Workspace &w = ws();
    *fA = A;
    *fv32 = v32;
    *sell = false;
    if (format == FLP_FORMAT_CSR) return FLP_OK;
    const bool same = w.sell_valid && w.sell_fp32 == fp32 && w.sell_src.n == A->n && w.sell_src.nnz == A->nnz &&
                      w.sell_src.rowptr == A->rowptr && w.sell_src.colind == A->colind &&
                      w.sell_src.val == A->val && w.sell_src.val32 == v32;
    if (!same) {
        w.sell_valid = false;
        bool built = false;
        CKR(build_sell(A, v32, fp32, w.sell_off, w.sell_col, w.sell_val, &w.sell_A, &w.sell_val32, s,
                       format == FLP_FORMAT_SELL ? 1e300 : kSellMaxPad, &built));
        w.sell_src = *A;
        w.sell_src.val32 = v32;
        w.sell_fp32 = fp32;
        w.sell_built = built;
        w.sell_valid = true;
    }
    if (w.sell_built) {
        *sell = true;
        *fA = &w.sell_A;
        *fv32 = w.sell_val32;
    }
    return FLP_OK;
}

int filter_apply_impl(const flp_filter *p, const flp_csr *A, const double *V, int ldv, double *W, int ldw, int r,
                      int prec, hipStream_t s, int format) {
    Workspace &w = ws();
    const int n = A->n;
    const bool fp32 = prec == FLP_PREC_FP32_FILTER;
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    for (auto &u : w.U) CK(ensure(u, es * (size_t)n * r));
    void *U[3] = {w.U[0].p, w.U[1].p, w.U[2].p};
    const float *v32 = nullptr;
    const void *vfull = V;
    int ldfull = ldv;
    if (fp32) {
        CKR(ensure_val32(A, w.val32, &w.val32_src, &w.val32_nnz, &v32, s));
        CK(ensure(w.V32, sizeof(float) * (size_t)n * r));
        CK(launch_copy_block(n, r, 1.0, V, ldv, DMat{nullptr, 0, 0, 0}, 0, (float *)w.V32.p, r, s));
        vfull = w.V32.p;
        ldfull = r;
    }
    const flp_csr *fA = A;
    const float *fv32 = v32;
    bool sell = false;
    CKR(workspace_storage(A, v32, fp32, format, s, &fA, &fv32, &sell));
    FilterTune tn;
    CKR(tune_filter(fA, fv32, r, fp32, true, U, vfull, ldfull, s, &tn, sell));
    const int gw = tn.gw;
    if (gw == r) {
        auto plan = clenshaw_plan(p, r, vfull, ldfull, W, ldw, U[0], U[1], U[2], fp32);
        for (const auto &st : plan) CKR(launch_plan_step(fA, fv32, r, st, fp32, s, tn.sh, sell));
        return FLP_OK;
    }
    // Each column group of V (converted to FP32 in that precision) is staged
    // as a contiguous n x gw block: the filter reads V at every step, and a
    // strided group would pull in the other groups' columns with each line.
    CK(ensure(w.Vg, es * (size_t)n * gw));
    for (int j0 = 0; j0 < r; j0 += gw) {
        if (fp32)
            CK(launch_copy_block(n, gw, 1.0, V + j0, ldv, DMat{nullptr, 0, 0, 0}, 0, (float *)w.Vg.p, gw, s));
        else
            CK(launch_copy_block(n, gw, 1.0, V + j0, ldv, plain_mat((double *)w.Vg.p, gw), 0, nullptr, 0, s));
        auto plan = clenshaw_plan(p, gw, w.Vg.p, gw, W + j0, ldw, U[0], U[1], U[2], fp32);
        for (const auto &st : plan) CKR(launch_plan_step(fA, fv32, gw, st, fp32, s, tn.sh, sell));
    }
    return FLP_OK;
}

int polish_apply(const flp_filter *p, const flp_csr *A, const float *val32, int c, const double *X,
                 const double *AX, int ldc, const std::vector<double> &lam, double *Y, hipStream_t s,
                 double *bytes, const flp_csr *sellA, const float *sell32, const std::vector<double> *rres,
                 double lock_abs, StepShape tile) {
    const int chunk = tile.chunk;
    const bool win = tile.win != 0;
    Workspace &w = ws();
    // the recurrence reads the sliced ELL copy when the solve holds one
    const bool sell = sellA != nullptr;
    const int32_t *mrow = sell ? sellA->rowptr : A->rowptr;
    const int32_t *mcol = sell ? sellA->colind : A->colind;
    const float *mval = sell ? sell32 : val32;
    const int n = A->n, PW = polish_block_width();
    const int mg = std::max(p->m, 1);  // coefficients of the divided differences
    const double cc = p->c, e = p->e;
    // locked columns: residual already at or below lock_abs, so the residual
    // term is dropped and the column is only scaled by p(t_j)
    std::vector<int> active, locked;
    for (int j = 0; j < c; ++j) {
        if (rres && lock_abs > 0.0 && (*rres)[j] <= lock_abs)
            locked.push_back(j);
        else
            active.push_back(j);
    }
    const int na = (int)active.size();
    const int nblk = (na + PW - 1) / PW;
    for (auto &u : w.PU) CK(ensure(u, sizeof(float) * (size_t)n * PW));
    CK(ensure(w.PR, sizeof(float) * (size_t)n * PW));
    const size_t tab_bytes = ((sizeof(float) * (size_t)mg * PW + 255) / 256) * 256;
    // per block: coefficient table, Ritz values and p(t_j) (2 PW doubles),
    // column indices (PW ints); then the locked columns' indices and scales
    const size_t blk_bytes = tab_bytes + sizeof(double) * 2 * PW + sizeof(int) * PW + 256;
    const size_t lock_bytes = (sizeof(int) + sizeof(double)) * (size_t)locked.size() + 256;
    CK(ensure_grow(w.PC, blk_bytes * (size_t)std::max(nblk, 1) + lock_bytes));
    float *U[3] = {(float *)w.PU[0].p, (float *)w.PU[1].p, (float *)w.PU[2].p};
    float *R = (float *)w.PR.p;
    char *pc = (char *)w.PC.p;
    const float a2 = (float)(2.0 / e), b2 = (float)(-2.0 * cc / e), a1 = (float)(1.0 / e), b1 = (float)(-cc / e);
    std::vector<char> host(blk_bytes * (size_t)std::max(nblk, 1) + lock_bytes, 0);
    std::vector<double> g;
    for (int bi = 0; bi < nblk; ++bi) {
        char *hb = host.data() + blk_bytes * bi;
        float *tab = (float *)hb;
        double *lph = (double *)(hb + tab_bytes);
        int *cl = (int *)(hb + tab_bytes + sizeof(double) * 2 * PW);
        const int wc = std::min(PW, na - bi * PW);
        for (int j = 0; j < wc; ++j) {
            const int col = active[bi * PW + j];
            const double t = (lam[col] - cc) / e;
            cheb_divided(p->b, t, g);
            for (int k = 0; k < mg; ++k) tab[(size_t)k * PW + j] = (float)g[k];
            lph[j] = lam[col];
            lph[PW + j] = cheb_scalar(p->b, t);
            cl[j] = col;
        }
    }
    {
        char *hl = host.data() + blk_bytes * (size_t)std::max(nblk, 1);
        int *lc = (int *)hl;
        double *ls = (double *)(hl + ((sizeof(int) * locked.size() + 7) / 8) * 8);
        for (size_t t = 0; t < locked.size(); ++t) {
            lc[t] = locked[t];
            ls[t] = cheb_scalar(p->b, (lam[locked[t]] - cc) / e);
        }
    }
    CK(h2d(pc, host.data(), host.size(), s));
    if (!locked.empty()) {
        char *dl = pc + blk_bytes * (size_t)std::max(nblk, 1);
        const int *lc = (const int *)dl;
        const double *ls = (const double *)(dl + ((sizeof(int) * locked.size() + 7) / 8) * 8);
        CK(launch_polish_locked(n, (int)locked.size(), lc, ls, X, ldc, Y, s));
    }
    for (int bi = 0; bi < nblk; ++bi) {
        char *db = pc + blk_bytes * bi;
        const float *coef = (const float *)db;
        const double *lp = (const double *)(db + tab_bytes);
        const int *cl = (const int *)(db + tab_bytes + sizeof(double) * 2 * PW);
        const int wc = std::min(PW, na - bi * PW);
        CK(launch_polish_resid(n, wc, X, AX, ldc, cl, lp, 1.0 / e, R, s));
        // Clenshaw for sum_k g_k T_k(Ahat) r: u_k = g_k r + 2 Ahat u_{k+1} - u_{k+2}
        // (k = mg-1 .. 1), result g_0 r + Ahat u_1 - u_2, plus p(t_j) x_j
        const float *u1 = nullptr, *u2 = nullptr;
        int next = 0;
        for (int k = mg - 1; k >= 1; --k) {
            float *out = U[next];
            next = (next + 1) % 3;
            CK(launch_polish_step(n, mrow, mcol, mval, u1, u2, R, coef + (size_t)k * PW, a2, b2, out, s, sell,
                                  chunk, win));
            u2 = u1;
            u1 = out;
        }
        CK(launch_polish_last(n, mrow, mcol, mval, u1, u2, R, coef, a1, b1, Y, ldc, wc, X, ldc, cl, lp + PW, s, sell,
                              chunk, win));
    }
    if (bytes) {
        // per step: the matrix in FP32 once, the gathered block, U_{k+2},
        // the residual block and the output (FP32); plus the FP64 in/out of
        // every column (X, AX read and Y written for the active ones, X read
        // and Y written for the locked ones)
        const double step = (double)A->nnz * 8.0 + 4.0 * (n + 1) + 4.0 * (double)n * PW * 4.0;
        *bytes = step * mg * nblk + 8.0 * 3.0 * (double)n * na + 8.0 * 2.0 * (double)n * locked.size();
    }
    return FLP_OK;
}

// ------------------------------------------------------------------ small dense helpers (host)

namespace {
// y += a x over len entries: every entry one multiply and one add, in the
// same order whichever build runs (the AVX2 one, where the CPU has it, has
// no fused multiply-add), so results do not depend on the machine.
inline __attribute__((always_inline)) void axpy_body(int len, double a, const double *__restrict x,
                                                     double *__restrict y) {
#pragma clang fp contract(off)
    for (int j = 0; j < len; ++j) y[j] += a * x[j];
}
__attribute__((target("avx2"))) void axpy_avx2(int len, double a, const double *x, double *y) {
    axpy_body(len, a, x, y);
}
void axpy_base(int len, double a, const double *x, double *y) { axpy_body(len, a, x, y); }
}  // namespace

void host_axpy(int len, double a, const double *x, double *y) {
    static void (*const f)(int, double, const double *, double *) =
        __builtin_cpu_supports("avx2") ? axpy_avx2 : axpy_base;
    f(len, a, x, y);
}

// Upper Cholesky G = R^T R (r x r row-major).  Columns whose pivot falls
// below thr^2 are flagged bad: their row of R becomes e_i (placeholder) and
// later columns ignore them.  Right-looking: once row i of R is final, its
// outer product comes off the rows below it (which hold their part of G
// until their turn), so every entry sees the subtractions of the
// dot-product form in the same order, along rows.
void cholesky_flag(int r, const double *G, double thr2, std::vector<double> &R, std::vector<int> &bad) {
    R.assign((size_t)r * r, 0.0);
    bad.assign(r, 0);
    for (int i = 0; i < r; ++i)
        for (int j = i; j < r; ++j) R[(size_t)i * r + j] = G[(size_t)i * r + j];
    for (int i = 0; i < r; ++i) {
        double *ri = &R[(size_t)i * r];
        const double d = ri[i];
        if (!(d > thr2)) {
            bad[i] = 1;
            ri[i] = 1.0;
            for (int j = i + 1; j < r; ++j) ri[j] = 0.0;
            continue;
        }
        const double rii = std::sqrt(d);
        ri[i] = rii;
        for (int j = i + 1; j < r; ++j) ri[j] /= rii;
        for (int k = i + 1; k < r; ++k) host_axpy(r - k, -ri[k], ri + k, &R[(size_t)k * r + k]);
    }
}

// inverse of an upper-triangular r x r, row by row from the last:
// Ri[i][j] = -(sum over i < k <= j of R[i][k] Ri[k][j]) / R[i][i], the sum
// taken in increasing k along the rows of Ri
void upper_inverse(int r, const std::vector<double> &R, std::vector<double> &Ri) {
    Ri.assign((size_t)r * r, 0.0);
    std::vector<double> acc(r);
    for (int i = r - 1; i >= 0; --i) {
        const double *ri = &R[(size_t)i * r];
        std::fill(acc.begin() + i, acc.end(), 0.0);
        for (int k = i + 1; k < r; ++k) host_axpy(r - k, ri[k], &Ri[(size_t)k * r + k], &acc[k]);
        double *out = &Ri[(size_t)i * r];
        out[i] = 1.0 / ri[i];
        for (int j = i + 1; j < r; ++j) out[j] = -acc[j] / ri[i];
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

int check_symmetric(const flp_csr *A, double tol, hipStream_t s) {
    if (!(tol >= 0.0)) return fail(FLP_E_ARG, "symmetry tolerance must be >= 0");
    double *dev = nullptr;
    CKR(small_dev(8, &dev));
    unsigned int *bad = reinterpret_cast<unsigned int *>(dev);
    CK(hipMemsetAsync(bad, 0, sizeof(unsigned int), s));
    CK(launch_sym_check(A->n, A->rowptr, A->colind, A->val, tol, bad, s));
    unsigned int h = 0;
    CK(hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (h) return fail(FLP_E_NOTSYM, "matrix is not symmetric: " + std::to_string(h) + " entries without a matching transpose entry");
    return FLP_OK;
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
            double *host_out, hipStream_t s, bool sym) {
    Buf &pb = ws().partials;
    TnPlan pl = plan_tn(n, K, c);
    CK(ensure(pb, pl.partial_elems * sizeof(double)));
    CK(launch_gemm_tn_partial(pl, n, K, c, A, B, ldb, (double *)pb.p, s, sym));
    CK(launch_reduce_partials(pl, K, c, (double *)pb.p, dev_out, c, s, sym));
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
                  uint64_t seed, uint64_t sid, hipStream_t s, bool *replaced, int depth) {
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

int estimate_bounds_impl(const flp_csr *A, int k0, uint64_t seed, double *lmin, double *lmax, hipStream_t s,
                         const flp_csr *spmv_A) {
    Workspace &w = ws();
    const int n = A->n;
    int k = std::max(1, std::min(k0, n));
    // The last two Lanczos vectors, row-major n x 2: q_j in column j % 2 (the
    // next vector overwrites q_{j-1}); w = A q_j is orthogonalised twice
    // against both (the three-term recurrence, with its rounding removed
    // twice), which keeps the extreme Ritz values and their residual bounds
    // that the bounds need without the cost of a full basis.
    CK(ensure(w.Q, sizeof(double) * (size_t)n * 2));
    CK(ensure(w.W, sizeof(double) * (size_t)n * 2));
    double *Qw = (double *)w.Q.p, *wv = (double *)w.W.p;
    double *dev = nullptr;
    CKR(small_dev((size_t)2 * k + 64, &dev));
    // start vector
    CK(launch_randn(n, 1, wv, 1, seed, 0xB0B0, s));
    double g = 0.0;
    CKR(gram_tn(n, 1, 1, plain_mat(wv, 1), wv, 1, dev, &g, s));
    if (!(g > 0.0)) return fail(FLP_E_DEVICE, "bounds: zero start vector");
    CK(launch_copy_block(n, 1, 1.0 / std::sqrt(g), wv, 1, plain_mat(Qw, 2), 0, nullptr, 0, s));
    // k steps without a host round trip: the Gram-Schmidt coefficients, the
    // norm and the next vector stay on the device (dev: H1, H2 in [0, 4),
    // ||w||^2 at 8, alpha_j / beta_j pairs from 16)
    double *gdev = dev + 8, *abdev = dev + 16;
    const flp_csr *M = spmv_A ? spmv_A : A;
    for (int j = 0; j < k; ++j) {
        const int cur = j % 2, kk = std::min(j + 1, 2);
        // w = A q_j
        CK(launch_cheb_step<double, double>(n, M->rowptr, M->colind, M->val, 1, Qw + cur, 2, nullptr, 0, nullptr, 0,
                                            wv, 1, 1.0, 0.0, 0.0, 0.0, s, StepShape{}, spmv_A != nullptr));
        CKR(cgs2(plain_mat(Qw, 2), kk, n, wv, 1, dev, s));
        CKR(gram_tn(n, 1, 1, plain_mat(wv, 1), wv, 1, gdev, nullptr, s));
        CK(launch_lanczos_next(n, wv, Qw + (1 - cur), 2, gdev, dev, dev + kk, kk == 1 ? 0 : cur, j, abdev, s));
    }
    std::vector<double> ab(2 * (size_t)k);
    CK(hipMemcpyAsync(ab.data(), abdev, sizeof(double) * ab.size(), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    // the recurrence ends at the first breakdown (beta_j = 0) or after k steps
    std::vector<double> al, be;
    double beta_k = 0.0;
    int steps = 0;
    for (int j = 0; j < k; ++j) {
        al.push_back(ab[2 * j]);
        be.push_back(ab[2 * j + 1]);
        steps = j + 1;
        beta_k = ab[2 * j + 1];
        if (beta_k == 0.0) break;
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
    CKR(small_dev((size_t)2 * k + 64, &dev));
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
    CKR(gram_tn(n, c, c, plain_mat(Y, ldc), Y, ldc, sdev, G.data(), s, true));
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
    for (int j0 = 0; j0 < c; j0 += 32) {
        int cw = std::min(32, c - j0);
        CK(launch_cheb_step<double, double>(n, A->rowptr, A->colind, A->val, cw, Y + j0, ldc, nullptr, 0, nullptr,
                                            0, AY + j0, ldc, 1.0, 0.0, 0.0, 0.0, s));
    }
    std::vector<double> G((size_t)c * c);
    CKR(gram_tn(n, c, c, plain_mat(Y, ldc), AY, ldc, sdev, G.data(), s, true));
    std::vector<double> Gs((size_t)c * c);
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) Gs[(size_t)i * c + j] = 0.5 * (G[(size_t)i * c + j] + G[(size_t)j * c + i]);
    lam.assign(c, 0.0);
    std::vector<double> ZG((size_t)c * c);
    std::vector<int> cols(c);
    for (int i = 0; i < c; ++i) cols[i] = i;
    if (sym_eig(c, c - 1, Gs.data(), lam.data(), nullptr, 0, nullptr, cols.data(), c, ZG.data()) != 0)
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

// Rayleigh-Ritz with A on span(Y) for a block whose columns need not be
// orthonormal (eq. rayleigh, eq. proj on the basis Y C with C^T Y^T Y C = I),
// in place of orthonormalising Y first: with D = diag(Y^T Y)^(-1/2) and the
// Cholesky factor D Y^T Y D = R^T R, the symmetric R^-T D Y^T A Y D R^-1 =
// Z diag(lam) Z^T gives C = D R^-1 Z, X = Y C and AX = (A Y) C.  The
// column scaling makes D Y^T Y D close to the identity for the blocks the
// finish phase meets (orthonormal up to rounding, or a filtered block whose
// columns point along nearly orthogonal eigenvectors with very different
// norms), so the factorisation loses nothing.  Four n x c x c products
// instead of the six of two orthonormalisations and a Rayleigh-Ritz.
// Fails when Y has numerically dependent columns.
namespace {
// f(i) for every i in [0, n), the indices claimed one at a time by up to 16
// threads when work (an operation count) is large enough to pay for them;
// f(i) writes only its own output row, so the result does not depend on
// the thread count.
template <typename F>
void rows_parallel(int n, double work, F f) {
    int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (work < 4e6) nt = 1;
    nt = std::min(nt, n);
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) f(i);
        });
    for (auto &x : th) x.join();
}
}  // namespace

int rayleigh_ritz_gen(const flp_csr *A, int n, int c, const double *Y, double *AY, double *X, double *AX, int ldc,
                      double *sdev, std::vector<double> &lam, std::vector<double> &res, hipStream_t s) {
    Workspace &w = ws();
    for (int j0 = 0; j0 < c; j0 += 32) {
        int cw = std::min(32, c - j0);
        CK(launch_cheb_step<double, double>(n, A->rowptr, A->colind, A->val, cw, Y + j0, ldc, nullptr, 0, nullptr,
                                            0, AY + j0, ldc, 1.0, 0.0, 0.0, 0.0, s));
    }
    std::vector<double> M((size_t)c * c), G((size_t)c * c);
    CKR(gram_tn(n, c, c, plain_mat(Y, ldc), Y, ldc, sdev, M.data(), s, true));
    CKR(gram_tn(n, c, c, plain_mat(Y, ldc), AY, ldc, sdev, G.data(), s, true));
    std::vector<double> d(c);
    for (int i = 0; i < c; ++i) {
        const double m = M[(size_t)i * c + i];
        if (!(m > 0.0) || !std::isfinite(m)) return fail(FLP_E_DEVICE, "Ritz block has a zero or non-finite column");
        d[i] = 1.0 / std::sqrt(m);
    }
    std::vector<double> Ms((size_t)c * c), Gs((size_t)c * c);
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) {
            const size_t ij = (size_t)i * c + j, ji = (size_t)j * c + i;
            Ms[ij] = d[i] * (0.5 * (M[ij] + M[ji])) * d[j];
            Gs[ij] = d[i] * (0.5 * (G[ij] + G[ji])) * d[j];
        }
    std::vector<double> R, Ri;
    std::vector<int> bad;
    cholesky_flag(c, Ms.data(), 1e-24, R, bad);
    for (int i = 0; i < c; ++i)
        if (bad[i]) return fail(FLP_E_DEVICE, "Ritz block lost rank");
    upper_inverse(c, R, Ri);
    // T = Gs Ri (T[i][j] = sum over k <= j of Gs[i][k] Ri[k][j]), then
    // H = Ri^T T (H[i][j] = sum over k <= i of Ri[k][i] T[k][j]); each row
    // of T and of H is its own task, its sums taken in increasing k
    const double cube = (double)c * c * c;
    std::vector<double> T((size_t)c * c, 0.0), H((size_t)c * c, 0.0);
    rows_parallel(c, cube, [&](int i) {
        double *ti = &T[(size_t)i * c];
        for (int k = 0; k < c; ++k) host_axpy(c - k, Gs[(size_t)i * c + k], &Ri[(size_t)k * c + k], ti + k);
    });
    rows_parallel(c, cube, [&](int i) {
        double *hi = &H[(size_t)i * c];
        for (int k = 0; k <= i; ++k) host_axpy(c, Ri[(size_t)k * c + i], &T[(size_t)k * c], hi);
    });
    for (int i = 0; i < c; ++i)
        for (int j = 0; j < i; ++j) {
            const double v = 0.5 * (H[(size_t)i * c + j] + H[(size_t)j * c + i]);
            H[(size_t)i * c + j] = H[(size_t)j * c + i] = v;
        }
    lam.assign(c, 0.0);
    std::vector<double> Z((size_t)c * c);
    std::vector<int> cols(c);
    for (int i = 0; i < c; ++i) cols[i] = i;
    if (sym_eig(c, c - 1, H.data(), lam.data(), nullptr, 0, nullptr, cols.data(), c, Z.data()) != 0)
        return fail(FLP_E_DEVICE, "eigensolver for the Rayleigh-Ritz matrix did not converge");
    // C = D Ri Z (rows of C padded to ldc)
    std::vector<double> Cp((size_t)c * ldc, 0.0);
    rows_parallel(c, cube, [&](int i) {
        double *ci = &Cp[(size_t)i * ldc];
        for (int k = i; k < c; ++k) host_axpy(c, d[i] * Ri[(size_t)i * c + k], &Z[(size_t)k * c], ci);
    });
    CK(h2d(sdev, Cp.data(), sizeof(double) * Cp.size(), s));
    CK(launch_gemm_nn(n, c, c, 1.0, plain_mat(Y, ldc), sdev, ldc, 0.0, X, ldc, s));
    // AX = A X by the sparse product (a read of A and of X per 32 columns)
    // rather than AY C (a dense n x c x c product on the FP64 matrix cores)
    for (int j0 = 0; j0 < c; j0 += 32) {
        int cw = std::min(32, c - j0);
        CK(launch_cheb_step<double, double>(n, A->rowptr, A->colind, A->val, cw, X + j0, ldc, nullptr, 0, nullptr,
                                            0, AX + j0, ldc, 1.0, 0.0, 0.0, 0.0, s));
    }
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

}  // namespace flp
