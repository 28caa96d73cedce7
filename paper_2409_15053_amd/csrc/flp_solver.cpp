// The filtered Lanczos procedure as a per-solve state machine (Sections 2.3
// and 3.2.2): set-up (bounds, filter, start block), one block step after
// each filter application (two-pass Gram-Schmidt, D_j, block QR, periodic
// convergence check), and the final Rayleigh-Ritz with A.  The single-solve
// driver runs one state machine; the batched driver advances many in
// lockstep with one segmented filter launch per Clenshaw step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "flp_host.h"

namespace flp {

namespace {

// T_k (K x K, row-major dense, semi-bandwidth r) from D_1..D_k and S_1..S_{k-1}
// (eq. lanczos).
void assemble_T(const Solve &S, int steps, std::vector<double> &T) {
    const int r = S.r, K = steps * r;
    T.assign((size_t)K * K, 0.0);
    for (int b = 0; b < steps; ++b)
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) {
                T[(size_t)(b * r + i) * K + b * r + j] = S.D_all[(size_t)b * r * r + i * r + j];
                if (b + 1 < steps) {
                    const double sv = S.S_all[(size_t)b * r * r + i * r + j];  // S_b(i, j)
                    T[(size_t)((b + 1) * r + i) * K + b * r + j] = sv;
                    T[(size_t)(b * r + j) * K + (b + 1) * r + i] = sv;
                }
            }
}

}  // namespace

int solve_setup(Solve &S) {
    S.t_start = now();
    const flp_csr *A = S.A;
    const flp_opts &o = S.o;
    hipStream_t s = S.s;
    S.n = A->n;
    S.r = o.block;
    const int n = S.n, r = S.r;
    if (r < 1 || r > 16) return fail(FLP_E_ARG, "block size must be in [1, 16]");
    if (r > n) return fail(FLP_E_ARG, "block size exceeds n");
    if (!(std::isfinite(S.alpha) && std::isfinite(S.beta)) || !(S.alpha < S.beta))
        return fail(FLP_E_ARG, "need finite alpha < beta");
    if (o.prec != FLP_PREC_FP64 && o.prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    const bool fp32 = o.prec == FLP_PREC_FP32_FILTER;
    S.unfiltered = o.unfiltered != 0;
    if (o.format != FLP_FORMAT_AUTO && o.format != FLP_FORMAT_CSR && o.format != FLP_FORMAT_SELL)
        return fail(FLP_E_ARG, "bad storage format");
    if (S.unfiltered && fp32) return fail(FLP_E_ARG, "unfiltered Lanczos runs in FP64 only");
    if (o.warm || o.warm_count != 0) return fail(FLP_E_ARG, "a warm start runs through flp_solve only");
    if (o.sym_tol >= 0.0) CKR(check_symmetric(A, o.sym_tol, s));

    // the filter's storage of A (and, in FP64, the bounds' SpMVs read it too)
    SolveBufs &B = *S.B;
    if (fp32) CKR(ensure_val32(A, B.val32, &B.val32_src, &B.val32_nnz, &S.val32, s));
    S.sell = false;
    if (o.format != FLP_FORMAT_CSR)
        CKR(build_sell(A, S.val32, fp32, B.sell_off, B.sell_col, B.sell_val, &S.SA, &S.sval32, s,
                       o.format == FLP_FORMAT_SELL ? 1e300 : kSellMaxPad, &S.sell));
    S.st.filter_format = S.sell ? FLP_FORMAT_SELL : FLP_FORMAT_CSR;

    // PREPROC: spectrum bounds
    double t0 = now();
    if (o.lmin < o.lmax) {
        S.lmin = o.lmin;
        S.lmax = o.lmax;
    } else {
        CKR(estimate_bounds_impl(A, o.k0 > 0 ? o.k0 : kDefaultK0, o.seed, &S.lmin, &S.lmax, s,
                                 S.sell && !fp32 ? &S.SA : nullptr));
    }
    S.st.t_pre = now() - t0;

    flp_filter *pf = nullptr;
    CKR(make_filter(S.alpha, S.beta, S.unfiltered ? 1 : o.degree, S.lmin, S.lmax, o.eps > 0 ? o.eps : kDefaultEps,
                    &pf));
    S.filt.reset(pf);
    if (S.unfiltered) S.filt->b = {0.0, 1.0};  // p = T_1: one product with Ahat per block step
    // an interval covering the whole mapped spectrum makes the ideal filter
    // the constant 1 on [-1, 1]: p(Ahat) = I separates nothing
    if (!S.unfiltered && S.alpha <= S.lmin && S.beta >= S.lmax)
        return fail(FLP_E_ARG, "[alpha, beta] covers the whole spectrum [lmin, lmax]: the filter is the constant 1 "
                               "(unfiltered Lanczos or a dense solver applies)");
    S.tau = 0.5 * std::min(cheb_scalar(S.filt->b, S.filt->a1), cheb_scalar(S.filt->b, S.filt->b1));
    S.tol_p = fp32 ? 1e-5 : 1e-10;
    S.check_every = o.check_every > 0 ? o.check_every : default_check_every(r);

    int64_t maxb = o.max_basis > 0 ? o.max_basis : S.unfiltered ? kUnfilteredMaxBasis : kDefaultMaxBasis;
    maxb = std::min<int64_t>(maxb, n);
    S.max_steps = std::max<int>(1, (int)(maxb / r));
    // Lanczos basis: column panels of 128 columns, each a contiguous
    // row-major n x 128 block (the reorthogonalisation streams whole panels)
    S.npanels = ((int64_t)S.max_steps * r + (1 << kPanelLog2) - 1) >> kPanelLog2;
    // the basis starts with a few panels and grows as the solve needs them
    // (max_basis columns would mostly stay unused)
    const size_t panel_bytes = (sizeof(double) * (size_t)n) << kPanelLog2;
    CK(ensure(B.Q, panel_bytes * (size_t)std::min<int64_t>(S.npanels, kInitPanels)));
    S.qpanels = std::min<int64_t>(S.npanels, (int64_t)(B.Q.bytes / panel_bytes));
    CK(ensure(B.W, sizeof(double) * (size_t)n * r));
    CK(ensure(B.Vin, sizeof(double) * (size_t)n * r));
    const size_t hcols = (size_t)(S.npanels << kPanelLog2);
    CK(ensure(B.hdev, sizeof(double) * (2 * hcols * r + 4 * (size_t)r * r + 64)));
    S.W = (double *)B.W.p;
    S.Vin = (double *)B.Vin.p;
    S.hdev = (double *)B.hdev.p;
    S.gdev = S.hdev + 2 * hcols * r;
    S.rdev = S.gdev + (size_t)r * r;
    if (!S.pin) CK(hipHostMalloc((void **)&S.pin, sizeof(double) * 4 * (size_t)r * r, hipHostMallocDefault));
    S.Q = panel_mat((double *)B.Q.p, n, kPanelLog2);
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    for (auto &u : B.U) CK(ensure(u, es * (size_t)n * r));
    for (int i = 0; i < 3; ++i) S.U[i] = B.U[i].p;
    if (fp32) {
        CK(ensure(B.V32, sizeof(float) * (size_t)n * r));
        S.V32 = (float *)B.V32.p;
    }
    S.plan = clenshaw_plan(S.filt.get(), r, fp32 ? (const void *)S.V32 : (const void *)S.Vin, r, S.W, r, S.U[0],
                           S.U[1], S.U[2], fp32);

    // start block: orthonormal random (or given) n x r
    if (o.start) {
        CK(h2d(S.W, o.start, sizeof(double) * (size_t)n * r, s));
    } else {
        CK(launch_randn(n, r, S.W, r, o.seed, 0x51A7, s));
    }
    std::vector<double> S0;
    CKR(block_qr_impl(S.W, n, r, nullptr, 0, S0, o.seed, 1, s, nullptr));
    CK(launch_copy_block(n, r, 1.0, S.W, r, S.Q, 0, nullptr, 0, s));
    CK(launch_copy_block(n, r, 1.0, S.W, r, plain_mat(S.Vin, r), 0, S.V32, r, s));
    return FLP_OK;
}

Solve::~Solve() {
    // a check still in flight owns its snapshot (shared with the pool task)
    if (pin) (void)hipHostFree(pin);
}

int ensure_basis(Solve &S, int64_t cols) {
    cols = std::min<int64_t>(cols, S.npanels << kPanelLog2);
    const int64_t need = (cols + (1 << kPanelLog2) - 1) >> kPanelLog2;
    if (need <= S.qpanels) return FLP_OK;
    const int64_t want = std::min(S.npanels, std::max(need, 2 * S.qpanels));
    const size_t panel_bytes = (sizeof(double) * (size_t)S.n) << kPanelLog2;
    void *p = nullptr;
    CK(dev_alloc(&p, panel_bytes * (size_t)want));
    hipError_t e = hipMemcpyAsync(p, S.B->Q.p, panel_bytes * (size_t)S.qpanels, hipMemcpyDeviceToDevice, S.s);
    if (e == hipSuccess) e = hipStreamSynchronize(S.s);
    if (e != hipSuccess) {
        (void)dev_free(p);
        CK(e);
    }
    Buf &q = S.B->Q;
    S.B->retired.emplace_back();
    S.B->retired.back().p = q.p;
    S.B->retired.back().bytes = q.bytes;
    q.p = p;
    q.bytes = panel_bytes * (size_t)want;
    S.qpanels = want;
    S.Q = panel_mat((double *)p, S.n, kPanelLog2);
    return FLP_OK;
}

int step_orth_launch(Solve &S) {
    const int n = S.n, r = S.r;
    CKR(ensure_basis(S, (int64_t)(S.steps + 2) * r));  // the projection's columns and the next block
    hipStream_t s = S.s;
    S.t_step0 = now();
    const int k = (S.steps + 1) * r;  // basis columns so far
    S.st.filter_bytes += filter_step_bytes(n, S.A->nnz, r, S.o.prec) * S.filt->m;
    S.st.mv += (int64_t)r * S.filt->m;
    S.st.orth_bytes += 4.0 * 8.0 * (double)n * k;
    // full reorthogonalisation (Section 3.2.2): two passes of classical Gram-Schmidt
    CKR(cgs2(S.Q, k, n, S.W, r, S.hdev, s));
    const size_t rr = (size_t)r * r;
    CK(hipMemcpyAsync(S.pin, S.hdev + (size_t)(k - r) * r, sizeof(double) * rr, hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(S.pin + rr, S.hdev + (size_t)k * r + (size_t)(k - r) * r, sizeof(double) * rr,
                      hipMemcpyDeviceToHost, s));
    // Gram matrix of the projected block (first Cholesky QR pass)
    CKR(gram_tn(n, r, r, plain_mat(S.W, r), S.W, r, S.gdev, nullptr, s));
    CK(hipMemcpyAsync(S.pin + 2 * rr, S.gdev, sizeof(double) * rr, hipMemcpyDeviceToHost, s));
    return FLP_OK;
}

int step_qr1(Solve &S) {
    const int n = S.n, r = S.r;
    hipStream_t s = S.s;
    const size_t rr = (size_t)r * r;
    const double *h1 = S.pin, *h2 = S.pin + rr, *G = S.pin + 2 * rr;
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) {
            const double a = h1[i * r + j] + h2[i * r + j], b = h1[j * r + i] + h2[j * r + i];
            S.D_all.push_back(0.5 * (a + b));
        }
    // W = Q_{j+1} S_j (eq. lanczos) by Cholesky QR twice
    double fro2 = 0.0;
    for (int i = 0; i < r; ++i) fro2 += std::max(G[i * r + i], 0.0);
    const double thr = 1e-7 * std::sqrt(fro2);
    std::vector<int> bad;
    cholesky_flag(r, G, std::max(thr * thr, 1e-300), S.R1, bad);
    S.slow = false;
    for (int i = 0; i < r; ++i) S.slow = S.slow || bad[i];
    if (S.slow) {
        // numerically dependent columns: the synchronous repair path
        const int k = (S.steps + 1) * r;
        return block_qr_impl(S.W, n, r, &S.Q, k, S.Sj, S.o.seed, 1000 + S.steps, s, nullptr);
    }
    std::vector<double> Ri;
    upper_inverse(r, S.R1, Ri);
    std::memcpy(S.pin + 3 * rr, Ri.data(), sizeof(double) * rr);
    CK(hipMemcpyAsync(S.rdev, S.pin + 3 * rr, sizeof(double) * rr, hipMemcpyHostToDevice, s));
    CK(launch_gemm_nn(n, r, r, 1.0, plain_mat(S.W, r), S.rdev, r, 0.0, S.W, r, s));
    CKR(gram_tn(n, r, r, plain_mat(S.W, r), S.W, r, S.gdev, nullptr, s));
    CK(hipMemcpyAsync(S.pin + 2 * rr, S.gdev, sizeof(double) * rr, hipMemcpyDeviceToHost, s));
    return FLP_OK;
}

int step_qr2(Solve &S) {
    const int n = S.n, r = S.r;
    hipStream_t s = S.s;
    const size_t rr = (size_t)r * r;
    if (!S.slow) {
        std::vector<double> R2, Ri;
        std::vector<int> bad;
        cholesky_flag(r, S.pin + 2 * rr, 1e-300, R2, bad);
        for (int i = 0; i < r; ++i)
            if (bad[i]) return fail(FLP_E_DEVICE, "block QR: second Cholesky pass broke down");
        upper_inverse(r, R2, Ri);
        std::memcpy(S.pin + 3 * rr, Ri.data(), sizeof(double) * rr);
        CK(hipMemcpyAsync(S.rdev, S.pin + 3 * rr, sizeof(double) * rr, hipMemcpyHostToDevice, s));
        CK(launch_gemm_nn(n, r, r, 1.0, plain_mat(S.W, r), S.rdev, r, 0.0, S.W, r, s));
        matmul_upper(r, R2, S.R1, S.Sj);
    }
    S.S_all.insert(S.S_all.end(), S.Sj.begin(), S.Sj.end());
    ++S.steps;
    S.st.t_orth += now() - S.t_step0;
    return FLP_OK;
}

bool at_check(const Solve &S) {
    if (S.steps == S.max_steps || (int64_t)(S.steps + 1) * S.r > S.n) return true;
    // unfiltered Lanczos runs to bases of thousands of columns, where one
    // eigensolve of T_k costs many block steps: its checks are also spaced
    // by a tenth of the basis at least
    if (S.unfiltered && S.checked_step > 0 && 10 * (S.steps - S.checked_step) < S.checked_step) return false;
    return S.steps >= S.check_every && (S.steps + S.check_offset) % S.check_every == 0;
}

namespace {
bool at_last(const Solve &S) { return S.steps == S.max_steps || (int64_t)(S.steps + 1) * S.r > S.n; }
}  // namespace

namespace {
void run_check_body(CheckTask &c);
}  // namespace

// Runs on a pool thread: every failure comes back through c.rc.
void run_check(CheckTask &c) {
    try {
        run_check_body(c);
    } catch (const std::bad_alloc &) {
        c.rc = FLP_E_NOMEM;
        c.msg = "host allocation failed in the convergence check";
    } catch (...) {
        c.rc = FLP_E_DEVICE;
        c.msg = "unexpected exception in the convergence check";
    }
    c.ready.store(true);
}

namespace {
void run_check_body(CheckTask &c) {
    const double t0 = now();
    const int K = c.K, r = c.r;
    std::vector<double> theta(K);
    std::vector<int> rows(r);
    for (int i = 0; i < r; ++i) rows[i] = K - r + i;
    std::vector<double> Zl((size_t)r * K);
    for (double t : c.T)
        if (!std::isfinite(t)) {
            c.rc = FLP_E_DEVICE;
            c.msg = "T_k holds non-finite entries (the filtered block overflowed, or A changed during the solve)";
            c.secs = now() - t0;
            return;
        }
    if (sym_eig_keep(K, r, c.T.data(), theta.data(), rows.data(), r, Zl.data(), &c.eig) != 0) {
        c.rc = FLP_E_DEVICE;
        c.msg = "eigensolver for T_k did not converge";
        c.secs = now() - t0;
        return;
    }
    // rho_i = || S_k E_k^T w_i ||; candidates theta_i >= tau, or for
    // unfiltered Lanczos theta_i in [lo, hi] and its two outside neighbours
    // (with them converged, no Ritz value is still moving into the interval)
    double big = 1e-300;
    for (double t : theta) big = std::max(big, std::fabs(t));
    int ilo = K, ihi = -1;  // unfiltered: first and last index taken (theta ascending)
    if (c.unfiltered) {
        for (int i = 0; i < K; ++i)
            if (theta[i] >= c.lo && theta[i] <= c.hi) {
                ilo = std::min(ilo, i);
                ihi = i;
            }
        if (ihi < 0) {  // none inside: the neighbours around where the interval sits
            ilo = (int)(std::lower_bound(theta.begin(), theta.end(), c.lo) - theta.begin());
            ihi = ilo - 1;
        }
        ilo = std::max(ilo - 1, 0);
        ihi = std::min(ihi + 1, K - 1);
    }
    c.ok = true;
    for (int i = 0; i < K; ++i) {
        if (c.unfiltered ? (i < ilo || i > ihi) : theta[i] < c.tau) continue;
        c.cand.push_back(i);
        double rho2 = 0.0;
        for (int a = 0; a < r; ++a) {
            double t = 0.0;
            for (int b = 0; b < r; ++b) t += c.Sk[a * r + b] * Zl[(size_t)b * K + i];
            rho2 += t * t;
        }
        if (std::sqrt(rho2) > c.tol_p * big) c.ok = false;
    }
    if (c.fp32) {
        // Guards for the FP64 polish: subspace iteration with p damps an
        // error component along eigenvalue mu by |p(mu)| / p(lambda) per
        // sweep, and that ratio nears 1/2 at the interval ends if the
        // transition band next to the candidates is left out.  The Ritz
        // values with tau / 4 <= |theta| < tau are taken, the largest |theta|
        // first, at most a quarter of the candidate count and at least 2r of
        // them: when all fit, the excluded part has |p| < tau / 4 and each
        // sweep gains at least 8x; the cap keeps the block (whose
        // Rayleigh-Ritz costs grow with its width squared) small where the
        // transition band is crowded, as on a 3D Hamiltonian whose band
        // holds more Ritz values than half the candidates, and one sweep
        // still meets the tolerance there (a quarter against a half:
        // 1.21 s against 1.26 s per solve on the 120^3 Hamiltonian, batch
        // of 64 3.04x against 2.83x the plain path).
        std::vector<int> g;
        for (int i = 0; i < K; ++i)
            if (theta[i] < c.tau && std::fabs(theta[i]) >= 0.25 * c.tau) g.push_back(i);
        std::sort(g.begin(), g.end(), [&](int a, int b) { return std::fabs(theta[a]) > std::fabs(theta[b]); });
        const size_t cap = std::max<size_t>(c.cand.size() / 4, 2 * (size_t)r);
        if (g.size() > cap) g.resize(cap);
        // the polish sweeps the block in fixed-width column blocks, each
        // costing a full block's traffic: a last block filled by guards
        // alone is dropped when that keeps at least 3/4 of them and 2r (on
        // the 120^3 Hamiltonian 349 candidates + 67 guards = 13 blocks of
        // 32 instead of 87 guards in 14; one sweep still suffices, and the
        // FP32 solve takes 1.02 s instead of 1.05)
        const size_t pw = (size_t)polish_block_width();
        const size_t tail = (c.cand.size() + g.size()) % pw;
        if (tail != 0 && tail <= g.size() / 4 && g.size() - tail >= 2 * (size_t)r) g.resize(g.size() - tail);
        std::sort(g.begin(), g.end());
        c.guard = g;
    }
    c.secs = now() - t0;
}
}  // namespace

int wait_check(Solve &S) {
    if (!S.check) return FLP_OK;
    std::shared_ptr<CheckTask> c = std::move(S.check);
    S.check.reset();
    while (!c->ready.load()) std::this_thread::sleep_for(std::chrono::microseconds(50));
    S.st.t_check += c->secs;
    if (c->rc != FLP_OK) return fail(c->rc, c->msg);
    // stop rule: every candidate converged and the candidate count unchanged
    // since the previous check, or no room left in the basis
    const int cnt = (int)c->cand.size();
    // (a basis of all n columns spans the whole space: its Ritz pairs are exact)
    const bool settled = cnt == S.prev_count || c->K >= S.n;
    if ((c->ok && settled) || S.check_last) {
        S.converged = c->ok && settled;
        S.kfinal = c->K;
        S.done = true;
        S.cand = std::move(c->cand);
        S.guard = std::move(c->guard);
        S.eig = std::move(c->eig);
        return FLP_OK;
    }
    S.prev_count = cnt;
    return FLP_OK;
}

int step_check(Solve &S, bool async, bool copy_next) {
    // a check that has finished in the background is applied first; one
    // still running after kMaxSpeculative further block steps is waited for
    // (speculative steps are wasted work if it decides convergence)
    if (S.check && (S.check->ready.load() || S.steps - S.checked_step >= kMaxSpeculative)) {
        CKR(wait_check(S));
        if (S.done) return FLP_OK;
    }
    if (at_check(S) && S.checked_step != S.steps) {
        // checks apply in order: one still running is waited for
        CKR(wait_check(S));
        if (S.done) return FLP_OK;
        S.checked_step = S.steps;
        auto c = std::make_shared<CheckTask>();
        c->K = S.steps * S.r;
        c->r = S.r;
        c->tau = S.tau;
        c->unfiltered = S.unfiltered;
        c->lo = S.filt->a1;
        c->hi = S.filt->b1;
        c->tol_p = S.tol_p;
        c->fp32 = S.o.prec == FLP_PREC_FP32_FILTER;
        assemble_T(S, S.steps, c->T);
        c->Sk = S.Sj;
        S.check = c;
        S.check_last = at_last(S);
        if (async && !S.check_last) {
            host_pool_submit([c]() { run_check(*c); });
        } else {
            run_check(*c);
            CKR(wait_check(S));
            if (S.done) return FLP_OK;
        }
    }
    if (!copy_next) return FLP_OK;
    // the new block joins the basis and is the next filter input
    const int n = S.n, r = S.r, k = S.steps * r;
    CK(launch_copy_block(n, r, 1.0, S.W, r, S.Q, k, nullptr, 0, S.s));
    CK(launch_copy_block(n, r, 1.0, S.W, r, plain_mat(S.Vin, r), 0, S.V32, r, S.s));
    return FLP_OK;
}

int solve_after_filter(Solve &S) {
    CKR(step_orth_launch(S));
    CK(hipStreamSynchronize(S.s));
    CKR(step_qr1(S));
    CK(hipStreamSynchronize(S.s));
    CKR(step_qr2(S));
    return step_check(S);
}

int solve_finish(Solve &S, flp_result **out) {
    const double tr = now();
    Workspace &w = ws();
    hipStream_t s = S.s;
    const int n = S.n, r = S.r;
    const flp_csr *A = S.A;
    const double anorm = std::max(std::fabs(S.lmin), std::fabs(S.lmax));
    auto *res = new flp_result;
    std::memset(res, 0, sizeof(*res));
    res->n = n;
    res->lmin = S.lmin;
    res->lmax = S.lmax;
    res->alpha = S.alpha;
    res->beta = S.beta;
    res->degree = S.filt->m;
    res->converged = S.converged ? 1 : 0;
    std::unique_ptr<flp_result, void (*)(flp_result *)> guard(res, flp_result_free);
    S.st.iters = S.kfinal / S.r;  // block steps behind the result (speculative ones after the deciding check are not counted)
    S.st.basis_cols = S.kfinal;
    std::vector<int> sel = S.cand;
    sel.insert(sel.end(), S.guard.begin(), S.guard.end());
    S.st.candidates = (int)S.cand.size();
    S.st.guards = (int)S.guard.size();
    const int c = S.cand.empty() ? 0 : (int)sel.size();
    if (c > 0) {
        const int K = S.kfinal;
        // eigenvectors of T_k for the candidates (eq. proj) and guards, from
        // the rotation log the last convergence check kept
        std::vector<double> Zc((size_t)K * c);
        const double tc = now();
        if (S.eig.N != K) return fail(FLP_E_DEVICE, "internal: no eigen-decomposition of the final T_k");
        eig_log_cols(S.eig, sel.data(), c, Zc.data());
        S.eig.clear();
        S.st.t_check += now() - tc;
        // FP32 filter: room for the separation step below (at most c more columns)
        const bool fp32 = S.o.prec == FLP_PREC_FP32_FILTER;
        const int cap = fp32 ? 2 * c : c;
        const int ldc = (cap + 1) & ~1;
        std::vector<double> Wc((size_t)K * ldc, 0.0);
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < c; ++j) Wc[(size_t)i * ldc + j] = Zc[(size_t)i * c + j];
        const bool own = S.B && S.B->own_ritz;
        Buf &bY = own ? S.B->Y : w.Y, &bAY = own ? S.B->AY : w.AY;
        Buf &bX = own ? S.B->X : w.X, &bAX = own ? S.B->AX : w.AX;
        const size_t blk = sizeof(double) * (size_t)n * ldc;
        CK(own ? ensure(bY, blk) : ensure_grow(bY, blk));
        CK(own ? ensure(bAY, blk) : ensure_grow(bAY, blk));
        CK(own ? ensure(bX, blk) : ensure_grow(bX, blk));
        CK(own ? ensure(bAX, blk) : ensure_grow(bAX, blk));
        double *Y = (double *)bY.p, *AY = (double *)bAY.p, *X = (double *)bX.p, *AX = (double *)bAX.p;
        double *sdev = nullptr;
        CKR(small_dev((size_t)std::max(K, cap) * ldc * 2 + 4 * (size_t)ldc + 64, &sdev));
        CK(h2d(sdev, Wc.data(), sizeof(double) * Wc.size(), s));
        // Ritz vectors of p(A): Y = Q_k W_C
        CK(launch_gemm_nn(n, K, c, 1.0, S.Q, sdev, ldc, 0.0, Y, ldc, s));
        std::vector<double> lam, rres;
        if (!fp32) CKR(rayleigh_ritz_gen(A, n, c, Y, AY, X, AX, ldc, sdev, lam, rres, s));
        const double alpha = S.alpha, beta = S.beta;
        int cur = c;  // Ritz vectors in the block
        auto worst = [&](int &i0, int &i1) {
            i0 = 0;
            while (i0 < cur && lam[i0] < alpha) ++i0;
            i1 = i0;
            while (i1 < cur && lam[i1] <= beta) ++i1;
            double m = 0.0;
            for (int j = i0; j < i1; ++j) m = std::max(m, rres[j] / anorm);
            return m;
        };
        const double tol = S.o.tol > 0 ? S.o.tol : kDefaultTol;
        int i0 = 0, i1 = 0;
        if (fp32) {
            // the polish filter: the solve's own, or one of the requested degree
            const flp_filter *pf = S.filt.get();
            std::unique_ptr<flp_filter> pown;
            if (S.o.polish_degree > 0 && S.o.polish_degree != S.filt->m) {
                flp_filter *q = nullptr;
                CKR(make_filter(S.alpha, S.beta, S.o.polish_degree, S.lmin, S.lmax,
                                S.o.eps > 0 ? S.o.eps : kDefaultEps, &q));
                pown.reset(q);
                pf = q;
            }
            {
                // The first polish sweep starts from the block Y itself: it is
                // an orthonormal basis of the Ritz space of p(Ahat), and the
                // residual form needs only A Y and one shift per column (any
                // shifts give the same p(Ahat) Y; the Rayleigh quotients
                // y_j^T A y_j keep the FP32 residuals small), so no
                // Rayleigh-Ritz step precedes it; mixed pairs are separated
                // after the Rayleigh-Ritz that follows it.
                for (int j0 = 0; j0 < c; j0 += 32) {
                    const int cw = std::min(32, c - j0);
                    CK(launch_cheb_step<double, double>(n, A->rowptr, A->colind, A->val, cw, Y + j0, ldc, nullptr, 0,
                                                        nullptr, 0, AY + j0, ldc, 1.0, 0.0, 0.0, 0.0, s));
                }
                const int nch = resid_chunks(n);
                CK(ensure(w.resid_part, sizeof(double) * (size_t)nch * c));
                CK(launch_col_dots(n, c, Y, ldc, AY, ldc, (double *)w.resid_part.p, nch, sdev, s));
                lam.assign(c, 0.0);
                CK(hipMemcpyAsync(lam.data(), sdev, sizeof(double) * c, hipMemcpyDeviceToHost, s));
                CK(hipStreamSynchronize(s));
                double pbytes = 0.0;
                const double tp = now();
                CKR(polish_apply(pf, A, S.val32, c, Y, AY, ldc, lam, X, s, &pbytes, S.sell ? &S.SA : nullptr,
                                 S.sell ? S.sval32 : nullptr, nullptr, 0.0,
                                 StepShape{0, 0, 0, S.tile_chunk, S.tile_win}));
                CK(hipStreamSynchronize(s));
                S.st.t_polish += now() - tp;
                S.st.polish_bytes += pbytes;
                // Rayleigh-Ritz with A on the polished block X; its Ritz
                // vectors land in Y, then X and Y trade places
                CKR(rayleigh_ritz_gen(A, n, c, X, AY, Y, AX, ldc, sdev, lam, rres, s));
                std::swap(X, Y);
                ++S.st.polish_sweeps;
            }
            int separations = 0;
            for (;;) {
                // A Ritz pair inside [alpha, beta] whose residual is far above
                // what the FP32 filter leaves (about 1e-7) approximates no
                // eigenvector: a guard vector mixing eigenvectors from both
                // sides of the interval whose filter values nearly coincide,
                // which subspace iteration with p cannot split.  Rayleigh-Ritz
                // with A on span{X, A x} for such x does split it (its parts
                // land outside the interval); the block grows by one column
                // per such pair.
                worst(i0, i1);
                std::vector<int> mixed;
                for (int j = i0; j < i1; ++j)
                    if (rres[j] / anorm > kMixedResid) mixed.push_back(j);
                if (!mixed.empty() && separations < kMaxSeparations && cur + (int)mixed.size() <= cap) {
                    CK(launch_copy_block(n, cur, 1.0, X, ldc, plain_mat(Y, ldc), 0, nullptr, 0, s));
                    for (size_t t = 0; t < mixed.size(); ++t)
                        CK(launch_copy_block(n, 1, 1.0, AX + mixed[t], ldc, plain_mat(Y, ldc), cur + (int)t, nullptr,
                                             0, s));
                    cur += (int)mixed.size();
                    CKR(orthonormalize_cols(n, cur, Y, X, ldc, sdev, s));
                    CKR(orthonormalize_cols(n, cur, Y, X, ldc, sdev, s));
                    CKR(rayleigh_ritz(A, n, cur, Y, AY, X, AX, ldc, sdev, lam, rres, s));
                    ++separations;
                    ++S.st.separations;
                    continue;
                }
                if (worst(i0, i1) <= tol || S.st.polish_sweeps >= kMaxPolish) break;
                // polish: X <- p(Ahat) X in FP64 accuracy (residual form, FP32
                // recurrences), orthonormalise, Rayleigh-Ritz with A
                const int c = cur;
                double pbytes = 0.0;
                CK(hipStreamSynchronize(s));  // (already idle: the Rayleigh-Ritz above ends on the host)
                const double tp = now();
                CKR(polish_apply(pf, A, S.val32, c, X, AX, ldc, lam, Y, s, &pbytes, S.sell ? &S.SA : nullptr,
                                 S.sell ? S.sval32 : nullptr, &rres, kLockFrac * tol * anorm,
                                 StepShape{0, 0, 0, S.tile_chunk, S.tile_win}));
                CK(hipStreamSynchronize(s));
                S.st.t_polish += now() - tp;
                S.st.polish_bytes += pbytes;
                CKR(rayleigh_ritz_gen(A, n, c, Y, AY, X, AX, ldc, sdev, lam, rres, s));
                ++S.st.polish_sweeps;
            }
        }
        // a pair inside [alpha, beta] that still misses the tolerance makes the
        // result non-converged (reported, never passed off as an eigenpair)
        if (worst(i0, i1) > tol) {
            S.converged = false;
            res->converged = 0;
        }
        const int cnt = i1 - i0;
        res->count = cnt;
        if (cnt > 0) {
            res->evals = new double[cnt];
            res->resid = new double[cnt];
            for (int j = 0; j < cnt; ++j) {
                res->evals[j] = lam[i0 + j];
                res->resid[j] = rres[i0 + j] / anorm;
            }
            CK(dev_alloc((void **)&res->evecs, sizeof(double) * (size_t)n * cnt));
            CK(launch_transpose_out(n, cnt, X + i0, ldc, res->evecs, s));
            CK(hipStreamSynchronize(s));
        }
    }
    S.st.t_rr = now() - tr;
    S.st.t_total = now() - S.t_start;
    res->stats = S.st;
    *out = guard.release();
    return S.converged ? FLP_OK : FLP_E_NOCONV;
}

size_t finish_bytes(const Solve &S) {
    const size_t c = S.cand.empty() ? 0 : S.cand.size() + S.guard.size();
    if (c == 0) return 0;
    const bool fp32 = S.o.prec == FLP_PREC_FP32_FILTER;
    const size_t ldc = ((fp32 ? 2 * c : c) + 1) & ~(size_t)1;
    const size_t n = (size_t)S.n;
    size_t b = 4 * n * ldc * sizeof(double);  // Y, AY, X, AX
    b += n * c * sizeof(double);              // the result's eigenvectors (at most c)
    if (fp32) b += 4 * n * (size_t)polish_block_width() * sizeof(float);  // polish recurrence and residual
    return b;
}

// ------------------------------------------------------------------ single solve

namespace {
SolveBufs &single_bufs() {
    static thread_local SolveBufs b[64];
    int dev = 0;
    (void)hipGetDevice(&dev);
    return b[dev & 63];
}
}  // namespace

void release_single_bufs() {
    SolveBufs &B = single_bufs();
    Buf *all[] = {&B.Q, &B.W, &B.Vin, &B.U[0], &B.U[1], &B.U[2], &B.V32, &B.val32, &B.hdev};
    for (Buf *b : all) b->release();
    B.val32_src = nullptr;
    B.val32_nnz = 0;
}

// ------------------------------------------------------------------ warm start

namespace {

constexpr int kMaxWarmSweeps = 16;
constexpr int kWarmMinDegree = 20;     // lowest filter degree of the warm sweeps
constexpr int kWarmSettledGuards = 2;  // settled guard pairs past the transition band that certify
constexpr int kWarmFallback = 1;       // solve_warm: not certified, the cold solve runs

// Subspace iteration with the filter from [previous eigenvectors, random
// guards] (flp_opts.warm): X <- p(Ahat) X by the residual form (FP32
// recurrences on the FP64 residuals, FP64 accuracy), orthonormalise, and
// Rayleigh-Ritz with A.  Subspace iteration captures the eigenvectors in the
// order of |p(lambda)|, and every eigenvalue inside [alpha, beta] has
// p >= 2 tau, so once the block holds settled Ritz pairs outside the
// interval with |p| < tau (past the transition band), no eigenvalue of the
// interval is left out.  The call certifies its result when the Ritz pairs
// inside the interval meet the tolerance, their count repeats, and at least
// kWarmSettledGuards pairs outside it have |p| < tau and a residual below
// kMixedResid.  Guard columns: half the warm block (at least 2 block); when
// the pairs inside have nearly converged (1e-6) but no guard has got past
// the band in three sweeps, the band holds more eigenvalues than guards and
// as many random guards again are added (up to twice the first width).
// The filter has degree max(polish_degree or degree, kWarmMinDegree), since
// the band of a low-degree filter holds too many eigenvalues for the guards.
// Returns FLP_OK with *out, kWarmFallback, or an error code.
int solve_warm(const flp_csr *A, double alpha, double beta, const flp_opts &o, flp_result **out) {
    const double t0 = now();
    hipStream_t s = (hipStream_t)o.stream;
    Workspace &w = ws();
    const int n = A->n, k = o.warm_count;
    if (!o.warm || k < 1 || k > n) return fail(FLP_E_ARG, "warm start needs 1 <= warm_count <= n and a block");
    if (o.unfiltered) return fail(FLP_E_ARG, "unfiltered Lanczos takes no warm start");
    if (!(std::isfinite(alpha) && std::isfinite(beta)) || !(alpha < beta))
        return fail(FLP_E_ARG, "need finite alpha < beta");
    if (o.prec != FLP_PREC_FP64 && o.prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    if (o.sym_tol >= 0.0) CKR(check_symmetric(A, o.sym_tol, s));
    const int r = std::max(1, o.block);
    const int g = std::min(n - k, std::max(2 * r, (k + 1) / 2));  // guard columns
    if (g < 1) return kWarmFallback;                              // no room beside the warm block
    flp_stats st{};
    double lmin = o.lmin, lmax = o.lmax;
    if (!(o.lmin < o.lmax)) {
        const double tb = now();
        CKR(estimate_bounds_impl(A, o.k0 > 0 ? o.k0 : kDefaultK0, o.seed, &lmin, &lmax, s));
        st.t_pre = now() - tb;
    }
    flp_filter *pf = nullptr;
    CKR(make_filter(alpha, beta, o.polish_degree > 0 ? o.polish_degree : o.degree, lmin, lmax,
                    o.eps > 0 ? o.eps : kDefaultEps, &pf));
    std::unique_ptr<flp_filter> filt(pf);
    if (filt->m < kWarmMinDegree) {
        flp_filter *pf2 = nullptr;
        CKR(make_filter(alpha, beta, kWarmMinDegree, lmin, lmax, o.eps > 0 ? o.eps : kDefaultEps, &pf2));
        filt.reset(pf2);
    }
    if (alpha <= lmin && beta >= lmax)
        return fail(FLP_E_ARG, "[alpha, beta] covers the whole spectrum [lmin, lmax]: the filter is the constant 1");
    const double tau = 0.5 * std::min(cheb_scalar(filt->b, filt->a1), cheb_scalar(filt->b, filt->b1));
    const double anorm = std::max(std::fabs(lmin), std::fabs(lmax));
    const double tol = o.tol > 0 ? o.tol : kDefaultTol;
    const float *v32 = nullptr;
    CKR(ensure_val32(A, w.val32, &w.val32_src, &w.val32_nnz, &v32, s));
    FilterTune tn;  // the tile-to-XCD mapping tuned for this matrix size, if any
    CKR(lookup_filter_tune(A, std::max(1, o.block), false, &tn));
    const int c0 = k + g, cap = 2 * c0, ldc = (cap + 1) & ~1;
    const size_t blk = sizeof(double) * (size_t)n * ldc;
    CK(ensure_grow(w.Y, blk));
    CK(ensure_grow(w.AY, blk));
    CK(ensure_grow(w.X, blk));
    CK(ensure_grow(w.AX, blk));
    double *Y = (double *)w.Y.p, *AY = (double *)w.AY.p, *X = (double *)w.X.p, *AX = (double *)w.AX.p;
    double *sdev = nullptr;
    CKR(small_dev((size_t)cap * ldc * 2 + 4 * (size_t)ldc + 64, &sdev));
    const double tr = now();
    CK(launch_transpose_in(n, k, o.warm, Y, ldc, s));
    CK(launch_randn(n, g, Y + k, ldc, o.seed, 0x3A21, s));
    std::vector<double> lam, rres;
    CKR(rayleigh_ritz_gen(A, n, c0, Y, AY, X, AX, ldc, sdev, lam, rres, s));
    int cur = c0, prev_count = -1, sweeps = 0, separations = 0, i0 = 0, i1 = 0, last_grow = 0, grown = 0;
    auto inside = [&]() {
        i0 = 0;
        while (i0 < cur && lam[i0] < alpha) ++i0;
        i1 = i0;
        while (i1 < cur && lam[i1] <= beta) ++i1;
        double m = 0.0;
        for (int j = i0; j < i1; ++j) m = std::max(m, rres[j] / anorm);
        return m;
    };
    bool certified = false;
    for (;;) {
        const double worst = inside();
        // Ritz pairs inside the interval far from converged mix eigenvectors
        // from both sides of it: split them as the finish phase does
        std::vector<int> mixed;
        for (int j = i0; j < i1; ++j)
            if (rres[j] / anorm > kMixedResid) mixed.push_back(j);
        if (sweeps > 0 && !mixed.empty() && separations < kMaxSeparations && cur + (int)mixed.size() <= cap) {
            CK(launch_copy_block(n, cur, 1.0, X, ldc, plain_mat(Y, ldc), 0, nullptr, 0, s));
            for (size_t t = 0; t < mixed.size(); ++t)
                CK(launch_copy_block(n, 1, 1.0, AX + mixed[t], ldc, plain_mat(Y, ldc), cur + (int)t, nullptr, 0, s));
            cur += (int)mixed.size();
            CKR(orthonormalize_cols(n, cur, Y, X, ldc, sdev, s));
            CKR(orthonormalize_cols(n, cur, Y, X, ldc, sdev, s));
            CKR(rayleigh_ritz(A, n, cur, Y, AY, X, AX, ldc, sdev, lam, rres, s));
            ++separations;
            ++st.separations;
            continue;
        }
        const int count = i1 - i0;
        int settled = 0;  // settled Ritz pairs outside the interval and past the transition band
        for (int j = 0; j < cur; ++j)
            if ((j < i0 || j >= i1) && rres[j] / anorm <= kMixedResid &&
                std::fabs(cheb_scalar(filt->b, (lam[j] - filt->c) / filt->e)) < tau)
                ++settled;
        if (sweeps >= 2 && worst <= tol && count == prev_count && settled >= kWarmSettledGuards) {
            certified = true;
            break;
        }
        if (sweeps >= kMaxWarmSweeps) break;
        const bool grow = sweeps >= 3 && sweeps - last_grow >= 3 && settled < kWarmSettledGuards &&
                          count == prev_count && worst <= 1e-6 && grown < 2 && cur + g <= cap;
        prev_count = count;
        double pbytes = 0.0;
        CK(hipStreamSynchronize(s));
        const double tp = now();
        CKR(polish_apply(filt.get(), A, v32, cur, X, AX, ldc, lam, Y, s, &pbytes, nullptr, nullptr, &rres,
                         kLockFrac * tol * anorm,
                         StepShape{0, 0, 0, tn.sh.win == 2 ? 0 : tn.sh.chunk, tn.sh.win != 0 ? 1 : 0}));
        CK(hipStreamSynchronize(s));
        st.t_polish += now() - tp;
        st.polish_bytes += pbytes;
        st.mv += (int64_t)cur * filt->m;
        if (grow) {  // the band holds more eigenvalues than guards: g more random guards
            CK(launch_randn(n, g, Y + cur, ldc, o.seed + 1 + grown, 0x3A22, s));
            cur += g;
            last_grow = sweeps + 1;
            ++grown;
        }
        CKR(rayleigh_ritz_gen(A, n, cur, Y, AY, X, AX, ldc, sdev, lam, rres, s));
        ++sweeps;
    }
    if (!certified) return kWarmFallback;
    auto *res = new flp_result;
    std::memset(res, 0, sizeof(*res));
    std::unique_ptr<flp_result, void (*)(flp_result *)> guard(res, flp_result_free);
    res->n = n;
    res->lmin = lmin;
    res->lmax = lmax;
    res->alpha = alpha;
    res->beta = beta;
    res->degree = filt->m;
    res->converged = 1;
    const int cnt = i1 - i0;
    res->count = cnt;
    if (cnt > 0) {
        res->evals = new double[cnt];
        res->resid = new double[cnt];
        for (int j = 0; j < cnt; ++j) {
            res->evals[j] = lam[i0 + j];
            res->resid[j] = rres[i0 + j] / anorm;
        }
        CK(dev_alloc((void **)&res->evecs, sizeof(double) * (size_t)n * cnt));
        CK(launch_transpose_out(n, cnt, X + i0, ldc, res->evecs, s));
        CK(hipStreamSynchronize(s));
    }
    st.polish_sweeps = sweeps;
    st.warm_sweeps = sweeps;
    st.warm_status = 1;
    st.basis_cols = cur;
    st.filter_format = FLP_FORMAT_CSR;
    st.t_rr = now() - tr;
    st.t_total = now() - t0;
    res->stats = st;
    *out = guard.release();
    return FLP_OK;
}

}  // namespace

int solve_impl(const flp_csr *A, double alpha, double beta, const flp_opts &o_in, flp_result **out) {
    flp_opts o = o_in;
    int warm_sweeps = 0;
    const bool warm = o.warm_count > 0 || o.warm != nullptr;
    if (warm) {
        const int rc = solve_warm(A, alpha, beta, o, out);
        if (rc != kWarmFallback) return rc;
        warm_sweeps = kMaxWarmSweeps;
        o.warm = nullptr;
        o.warm_count = 0;
    }
    const int rc = solve_cold(A, alpha, beta, o, out);
    if (warm && *out) {
        (*out)->stats.warm_status = 2;
        (*out)->stats.warm_sweeps = warm_sweeps;
    }
    return rc;
}

int solve_cold(const flp_csr *A, double alpha, double beta, const flp_opts &o, flp_result **out) {
    Solve S;
    S.A = A;
    S.alpha = alpha;
    S.beta = beta;
    S.o = o;
    S.s = (hipStream_t)o.stream;
    S.B = &single_bufs();
    CKR(solve_setup(S));
    const bool fp32 = o.prec == FLP_PREC_FP32_FILTER;
    // filter in cache-sized column groups (the plan is rebuilt for the group
    // width); each group of the input block is first staged as a contiguous
    // n x gw block in the unused tail of the first recurrence buffer, so the
    // V reads of every step touch only that group's bytes
    FilterTune tn;
    void *U[3] = {S.U[0], S.U[1], S.U[2]};
    const flp_csr *fA = S.sell ? &S.SA : A;  // the filter's copy of A
    const float *fv32 = S.sell ? S.sval32 : S.val32;
    CKR(tune_filter(fA, fv32, S.r, fp32, true, U, fp32 ? (const void *)S.V32 : (const void *)S.Vin, S.r, S.s, &tn,
                    S.sell));
    const int gw = tn.gw;
    {
        const StepShape used = step_shape_ok(gw, fp32, tn.sh) ? tn.sh : default_step_shape(gw, fp32);
        S.st.filter_group_width = gw;
        S.st.filter_lanes_per_row = used.lpr;
        S.st.filter_cols_per_lane = used.vec;
        S.st.filter_streaming_loads = used.nt;
        S.st.filter_tile_chunk = tn.sh.chunk;
        S.st.filter_lds_window = used.win;
        S.st.filter_window_halo = used.win == 2 ? used.halo : (used.win == 1 ? kWinHalo : 0);
        // the polish follows the filter's tile mapping and fixed window (its
        // kernel has no sliding form: chunk then holds the plane length)
        S.tile_chunk = used.win == 2 ? 0 : tn.sh.chunk;
        S.tile_win = used.win != 0 ? 1 : 0;
    }
    std::vector<ClenshawStep> gplan;
    void *stage = nullptr;
    if (gw != S.r) {
        const size_t es = fp32 ? sizeof(float) : sizeof(double);
        stage = (char *)S.U[0] + es * (size_t)S.n * gw;  // U buffers hold n x r >= 2 n x gw
        gplan = clenshaw_plan(S.filt.get(), gw, stage, gw, S.W, S.r, S.U[0], S.U[1], S.U[2], fp32);
    }
    hipEvent_t ev[4];
    for (auto &e : ev) CK(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};
    while (!S.done) {
        CK(hipEventRecord(ev[0], S.s));
        // While a convergence check is still running on the host, the step's
        // launches go out in chunks, each issued after the chunk before the
        // previous one has run (the device never waits), and the check is
        // applied as soon as it is ready: when it decides convergence the
        // rest of this speculative step is never issued.
        bool pace = S.check != nullptr;
        int issued = 0, chunk = 0;
        bool stop = false;
        auto after_launch = [&]() -> int {
            if (!pace || ++issued % kPaceLaunches != 0) return FLP_OK;
            hipEvent_t e = ev[2 + (chunk & 1)];
            CK(hipEventRecord(e, S.s));
            if (chunk > 0) CK(hipEventSynchronize(ev[2 + ((chunk - 1) & 1)]));
            ++chunk;
            if (S.check && S.check->ready.load()) {
                CKR(wait_check(S));
                stop = S.done;
                pace = false;  // not converged: the rest of the step goes out at once
            }
            return FLP_OK;
        };
        if (gw == S.r) {
            for (const auto &st : S.plan) {
                CKR(launch_plan_step(fA, fv32, S.r, st, fp32, S.s, tn.sh, S.sell));
                CKR(after_launch());
                if (stop) break;
            }
        } else {
            for (int j0 = 0; j0 < S.r && !stop; j0 += gw) {
                if (fp32)
                    CK(launch_copy_block(S.n, gw, 1.0, S.Vin + j0, S.r, DMat{nullptr, 0, 0, 0}, 0, (float *)stage,
                                         gw, S.s));
                else
                    CK(launch_copy_block(S.n, gw, 1.0, S.Vin + j0, S.r, plain_mat((double *)stage, gw), 0,
                                         nullptr, 0, S.s));
                for (ClenshawStep st : gplan) {
                    if (st.out == (void *)S.W) st.out = S.W + j0;  // the last step writes the group's columns of W
                    CKR(launch_plan_step(fA, fv32, gw, st, fp32, S.s, tn.sh, S.sell));
                    CKR(after_launch());
                    if (stop) break;
                }
            }
        }
        CK(hipEventRecord(ev[1], S.s));
        CK(hipEventSynchronize(ev[1]));
        float ms = 0;
        CK(hipEventElapsedTime(&ms, ev[0], ev[1]));
        S.st.t_mv += ms * 1e-3;
        if (stop) {
            // converged at the check applied above: the part of this step that
            // ran is discarded (its products and bytes still count)
            S.st.filter_bytes += filter_step_bytes(S.n, S.A->nnz, gw, S.o.prec) * issued;
            S.st.mv += (int64_t)gw * issued;
            break;
        }
        CKR(solve_after_filter(S));
    }
    return solve_finish(S, out);
}

}  // namespace flp
