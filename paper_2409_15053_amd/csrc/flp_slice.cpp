// Spectrum slicing on one GPU.
//
// The paper names spectrum slicing as the route to several devices
// (Section 5): [alpha, beta] is cut into sub-intervals and each is an
// independent filtered Lanczos problem.  Here the slices run on one GPU as
// one batch over the shared matrix: every Clenshaw step of every slice goes
// into the same segmented launch, and each slice's basis only has to hold
// its own part of the spectrum, so the Gram-Schmidt work (quadratic in the
// basis size) drops with the number of slices.
//
// Slices have equal width in the angle variable theta = acos(z) of the
// mapped spectrum [-1, 1]: the filter degree rule (eq. optimaldegree) then
// gives every slice the same degree, so all slices take part in every
// launch.  Slice i returns its eigenpairs in [b_i, b_{i+1}]; the merged
// result keeps lambda < b_{i+1} from slice i (lambda <= beta from the last)
// and drops an eigenpair found by both neighbours of a boundary (equal
// eigenvalues to 1e-8 ||A|| and eigenvector overlap above 1/2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "flp_host.h"

namespace flp {

int solve_sliced_impl(const flp_csr *A, double alpha, double beta, int nslices, const flp_opts &o,
                      flp_result **out) {
    const double t0 = now();
    *out = nullptr;
    if (nslices < 1 || nslices > 256) return fail(FLP_E_ARG, "nslices must be in [1, 256]");
    if (o.unfiltered) return fail(FLP_E_ARG, "unfiltered Lanczos runs through flp_solve only");
    if (o.format == FLP_FORMAT_SELL)
        return fail(FLP_E_ARG, "slices share A's CSR arrays (a sliced ELL copy per slice would repeat it)");
    if (!(std::isfinite(alpha) && std::isfinite(beta)) || !(alpha < beta))
        return fail(FLP_E_ARG, "need finite alpha < beta");
    hipStream_t s = (hipStream_t)o.stream;
    // spectrum bounds once, shared by every slice
    double lmin = o.lmin, lmax = o.lmax;
    if (!(lmin < lmax)) CKR(estimate_bounds_impl(A, o.k0 > 0 ? o.k0 : kDefaultK0, o.seed, &lmin, &lmax, s));
    const double a = std::max(alpha, lmin), b = std::min(beta, lmax);
    if (!(a < b)) return fail(FLP_E_INTERVAL, "[alpha, beta] does not meet the spectrum bounds");
    const double c = 0.5 * (lmax + lmin), e = 0.5 * (lmax - lmin);
    auto clampz = [](double z) { return std::max(-1.0, std::min(1.0, z)); };
    const double ta = std::acos(clampz((a - c) / e)), tb = std::acos(clampz((b - c) / e));
    std::vector<double> bnd(nslices + 1);
    bnd[0] = a;
    bnd[nslices] = b;
    for (int i = 1; i < nslices; ++i) bnd[i] = c + e * std::cos(ta + (tb - ta) * i / nslices);
    for (int i = 1; i <= nslices; ++i)
        if (!(bnd[i] > bnd[i - 1])) return fail(FLP_E_ARG, "interval too narrow for that many slices");

    std::vector<const flp_csr *> As(nslices, A);
    std::vector<double> lo(bnd.begin(), bnd.end() - 1), hi(bnd.begin() + 1, bnd.end());
    std::vector<flp_opts> os(nslices, o);
    for (int i = 0; i < nslices; ++i) {
        os[i].lmin = lmin;
        os[i].lmax = lmax;
        os[i].seed = o.seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
        os[i].format = FLP_FORMAT_CSR;
    }
    std::vector<flp_result *> res(nslices, nullptr);
    std::vector<int> codes(nslices, FLP_OK);
    flp_batch_stats bs{};
    struct Free {
        std::vector<flp_result *> &r;
        ~Free() {
            for (auto *p : r) flp_result_free(p);
        }
    } fr{res};
    CKR(solve_batch_impl(nslices, As.data(), lo.data(), hi.data(), os.data(), 1, res.data(), codes.data(), &bs));
    bool converged = true;
    for (int i = 0; i < nslices; ++i) converged = converged && codes[i] == FLP_OK;

    // merge: (slice, index) pairs in ascending eigenvalue order
    const double anorm = std::max(std::fabs(lmin), std::fabs(lmax));
    struct Pick {
        int slice, idx;
        double lam;
    };
    std::vector<Pick> keep;
    for (int i = 0; i < nslices; ++i) {
        const flp_result *r = res[i];
        if (!r) continue;
        for (int j = 0; j < r->count; ++j) {
            const double l = r->evals[j];
            if (i + 1 < nslices && !(l < hi[i])) continue;
            keep.push_back({i, j, l});
        }
    }
    std::sort(keep.begin(), keep.end(), [](const Pick &x, const Pick &y) { return x.lam < y.lam; });
    const int n = A->n;
    // duplicates across a boundary: same eigenvalue, overlapping vectors
    std::vector<char> drop(keep.size(), 0);
    std::vector<double> u(n), v(n);
    for (size_t p = 0; p + 1 < keep.size(); ++p)
        for (size_t q = p + 1; q < keep.size() && keep[q].lam - keep[p].lam <= 1e-8 * anorm; ++q) {
            if (keep[q].slice == keep[p].slice || drop[p] || drop[q]) continue;
            CK(hipMemcpyAsync(u.data(), res[keep[p].slice]->evecs + (size_t)keep[p].idx * n, sizeof(double) * n,
                              hipMemcpyDeviceToHost, s));
            CK(hipMemcpyAsync(v.data(), res[keep[q].slice]->evecs + (size_t)keep[q].idx * n, sizeof(double) * n,
                              hipMemcpyDeviceToHost, s));
            CK(hipStreamSynchronize(s));
            double d = 0.0;
            for (int k = 0; k < n; ++k) d += u[k] * v[k];
            if (std::fabs(d) > 0.5) drop[q] = 1;
        }
    auto *R = new flp_result;
    std::memset(R, 0, sizeof(*R));
    std::unique_ptr<flp_result, void (*)(flp_result *)> guard(R, flp_result_free);
    R->n = n;
    R->lmin = lmin;
    R->lmax = lmax;
    R->alpha = a;
    R->beta = b;
    R->converged = converged ? 1 : 0;
    int cnt = 0;
    for (size_t p = 0; p < keep.size(); ++p) cnt += drop[p] ? 0 : 1;
    R->count = cnt;
    if (cnt > 0) {
        R->evals = new double[cnt];
        R->resid = new double[cnt];
        CK(dev_alloc((void **)&R->evecs, sizeof(double) * (size_t)n * cnt));
        int w = 0;
        for (size_t p = 0; p < keep.size(); ++p) {
            if (drop[p]) continue;
            const flp_result *r = res[keep[p].slice];
            R->evals[w] = r->evals[keep[p].idx];
            R->resid[w] = r->resid[keep[p].idx];
            CK(hipMemcpyAsync(R->evecs + (size_t)w * n, r->evecs + (size_t)keep[p].idx * n, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
            ++w;
        }
        CK(hipStreamSynchronize(s));
    }
    // statistics: work summed over slices, the deepest slice's iterations
    flp_stats &st = R->stats;
    for (int i = 0; i < nslices; ++i) {
        const flp_result *r = res[i];
        if (!r) continue;
        R->degree = std::max(R->degree, r->degree);
        st.iters = std::max(st.iters, r->stats.iters);
        st.mv += r->stats.mv;
        st.basis_cols += r->stats.basis_cols;
        st.polish_sweeps = std::max(st.polish_sweeps, r->stats.polish_sweeps);
        st.t_mv += r->stats.t_mv;
        st.t_orth += r->stats.t_orth;
        st.t_check += r->stats.t_check;
        st.t_rr += r->stats.t_rr;
        st.filter_bytes += r->stats.filter_bytes;
        st.polish_bytes += r->stats.polish_bytes;
        st.t_polish += r->stats.t_polish;
        st.orth_bytes += r->stats.orth_bytes;
    }
    st.t_mv = bs.t_filter;  // the slices share the segmented launches
    st.t_pre = bs.t_setup;
    st.t_total = now() - t0;
    *out = guard.release();
    return converged ? FLP_OK : FLP_E_NOCONV;
}

}  // namespace flp
