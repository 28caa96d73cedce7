// Host symmetric eigensolver for the small projected problems.
//
// The paper solves the eigenproblem of the banded block-tridiagonal T_k on
// the CPU with a special-purpose banded symmetric eigensolver (Section
// 3.2.2).  This one works in two phases, both on adjacent-plane Givens
// rotations:
//   1. band -> tridiagonal: the outermost diagonal is annihilated one entry
//      at a time and the bulge each rotation creates is chased down the band
//      (Rutishauser/Schwarz band reduction), bandwidth b -> b-1 -> ... -> 1,
//      on compact band storage (each column keeps its b+2 lower entries);
//   2. implicit symmetric QR with the Wilkinson shift on the tridiagonal
//      (Golub & Van Loan, "Matrix Computations", Sec. 8.3).
// Every rotation is logged, so eigenvectors are built only where needed:
//   * selected ROWS of the eigenvector matrix Z = J_1 J_2 ... J_t, applied
//     to rows of the identity as the rotations are made (the convergence
//     check needs the last r rows, for the Ritz residual bounds);
//   * selected COLUMNS of Z by replaying the log backwards on columns of the
//     identity, Z e_j = J_1 (J_2 (... (J_t e_j))) (the Ritz vectors need
//     only the candidates' columns).
// Both cost O(#rotations x #selected); the column replay runs in parallel
// threads.
//
// Dense matrices (the Rayleigh-Ritz projections, whose bandwidth is the full
// order) take a different first phase: Householder reduction to tridiagonal
// form (Golub & Van Loan, Alg. 8.3.1), whose cost is O(N^3) with unit-stride
// inner loops, instead of O(N^2 log b) rotations each touching O(b) strided
// entries.  Their eigenvectors are the logged QR rotations replayed on
// identity columns followed by the reflectors.
#include "flp_internal.h"

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

namespace flp {

namespace {

using Rot = EigRot;

// Symmetric band matrix, lower half of half-width w, column-compact:
// entry (i, j), i >= j, i - j <= w, at B[j * (w + 1) + (i - j)].
struct Band {
    int N, w;
    std::vector<double> B;
    double get(int i, int j) const {
        if (i < j) std::swap(i, j);
        const int d = i - j;
        return d > w ? 0.0 : B[(size_t)j * (w + 1) + d];
    }
    void set(int i, int j, double v) {
        if (i < j) std::swap(i, j);
        const int d = i - j;
        if (d <= w) B[(size_t)j * (w + 1) + d] = v;
    }
};

// M' = J^T M J on the plane (p, q = p + 1), J[:,p] = c e_p + s e_q,
// J[:,q] = -s e_p + c e_q, touching only entries within the band.  Entries
// one step outside the band are structurally zero before and after (the
// bulge always sits within w = b + 1 of the diagonal), so they are neither
// read nor written.
inline void rotate_band(Band &M, int p, double c, double s) {
    const int q = p + 1, w = M.w, N = M.N, W1 = w + 1;
    double *B = M.B.data();
    // rows x < p: column x holds (p, x) at distance d = p - x and (q, x) at d + 1
    for (int x = std::max(0, p - w); x < p; ++x) {
        double *col = B + (size_t)x * W1;
        const int d = p - x;
        const double a = col[d];
        if (d + 1 <= w) {
            const double b = col[d + 1];
            col[d] = c * a + s * b;
            col[d + 1] = -s * a + c * b;
        } else {
            col[d] = c * a;
        }
    }
    // rows x > q: column p holds (x, p) at x - p, column q holds (x, q) at x - q
    double *cp = B + (size_t)p * W1, *cq = B + (size_t)q * W1;
    const int xhi = std::min(N - 1, q + w);
    for (int x = q + 1; x <= xhi; ++x) {
        const int dp = x - p, dq = x - q;
        const double b = cq[dq];
        if (dp <= w) {
            const double a = cp[dp];
            cp[dp] = c * a + s * b;
            cq[dq] = -s * a + c * b;
        } else {
            cq[dq] = c * b;
        }
    }
    const double app = cp[0], apq = cp[1], aqq = cq[0];
    cp[0] = c * c * app + 2.0 * c * s * apq + s * s * aqq;
    cq[0] = s * s * app - 2.0 * c * s * apq + c * c * aqq;
    cp[1] = c * s * (aqq - app) + (c * c - s * s) * apq;
}

// Reduce a symmetric band matrix of semi-bandwidth b (stored with w = b + 1
// so the bulge fits) to tridiagonal form in place, logging the rotations.
// Rows of the accumulated rotation product, applied as each rotation is
// made: Zt is N x nr (row p holds the nr tracked rows' entries in column p),
// a rotation on plane (p, p + 1) mixes entries p and p + 1.
inline void rot_rows(double *Zt, int nr, int p, double c, double s) {
    double *a = Zt + (size_t)p * nr;
    double *b = a + nr;
    for (int j = 0; j < nr; ++j) {
        const double u = a[j], v = b[j];
        a[j] = c * u + s * v;
        b[j] = -s * u + c * v;
    }
}

void band_to_tridiag(Band &M, int b, std::vector<Rot> &log, double *Zt, int nr) {
    const int N = M.N;
    for (int bw = b; bw >= 2; --bw) {
        for (int j = 0; j + bw < N; ++j) {
            int k = j, i = j + bw;
            while (i < N) {
                const double x = M.get(i - 1, k);
                const double y = M.get(i, k);
                if (y == 0.0) break;
                const double r = std::sqrt(x * x + y * y);
                const double c = x / r, s = y / r;
                rotate_band(M, i - 1, c, s);
                M.set(i, k, 0.0);
                log.push_back({i - 1, c, s});
                if (nr) rot_rows(Zt, nr, i - 1, c, s);
                // the rotation fills (i-1+bw+1, i-1); chase it with plane (i-1+bw, i+bw)
                k = i - 1;
                i = i + bw;
            }
        }
    }
}

// Implicit QR with Wilkinson shift on the tridiagonal (d, e); e[i] couples
// i and i+1.  On return d holds the eigenvalues (unsorted).  A matrix whose
// largest entry lies far from 1 is scaled to it first (the rotations do not
// depend on the scale): at 1e-200 the squares in the rotations underflow
// and the iteration would not move.
bool tridiag_qr(std::vector<double> &d, std::vector<double> &e, std::vector<Rot> &log, double *Zt, int nr) {
    const int N = (int)d.size();
    if (N <= 1) return true;
    double amax = 0.0;
    for (double x : d) amax = std::max(amax, std::fabs(x));
    for (double x : e) amax = std::max(amax, std::fabs(x));
    if (!std::isfinite(amax)) return false;
    if (amax == 0.0) return true;
    const double scale = (amax < 1e-100 || amax > 1e100) ? 1.0 / amax : 1.0;
    if (scale != 1.0) {
        for (double &x : d) x *= scale;
        for (double &x : e) x *= scale;
    }
    int hi = N - 1;
    long guard = 0;
    const long max_steps = 60L * N + 100;
    while (hi > 0) {
        double tiny = DBL_EPSILON * (std::fabs(d[hi - 1]) + std::fabs(d[hi]));
        if (std::fabs(e[hi - 1]) <= tiny || std::fabs(e[hi - 1]) < DBL_MIN) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0) {
            double t = DBL_EPSILON * (std::fabs(d[lo - 1]) + std::fabs(d[lo]));
            if (std::fabs(e[lo - 1]) <= t || std::fabs(e[lo - 1]) < DBL_MIN) {
                e[lo - 1] = 0.0;
                break;
            }
            --lo;
        }
        if (++guard > max_steps) return false;
        // Wilkinson shift from the trailing 2x2 of the active block
        double dd = 0.5 * (d[hi - 1] - d[hi]);
        double ee = e[hi - 1];
        double den = dd + std::copysign(std::hypot(dd, ee), dd == 0.0 ? 1.0 : dd);
        double mu = d[hi] - ee * ee / den;
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            double r = std::sqrt(x * x + z * z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                c = x / r;
                s = z / r;
            }
            if (k > lo) e[k - 1] = r;
            double a = d[k], b = e[k], dq = d[k + 1];
            d[k] = c * c * a + 2.0 * c * s * b + s * s * dq;
            d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * dq;
            e[k] = c * s * (dq - a) + (c * c - s * s) * b;
            if (k + 1 < hi) {
                z = s * e[k + 1];
                e[k + 1] = c * e[k + 1];
                x = e[k];
            }
            log.push_back({k, c, s});
            if (nr) rot_rows(Zt, nr, k, c, s);
        }
    }
    if (scale != 1.0) {
        for (double &x : d) x /= scale;
        for (double &x : e) x /= scale;
    }
    return true;
}

thread_local int tl_eig_threads = 16;  // inner-thread cap of the calling thread

int nthreads_for(long work, int units) {
    int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    nt = std::min(nt, std::max(1, tl_eig_threads));
    nt = std::min(nt, units);
    if (work < 4000000L) nt = 1;
    return std::max(nt, 1);
}

template <typename F>
void parallel_for(int units, int nt, F f) {
    if (nt <= 1) {
        f(0, units);
        return;
    }
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w) {
        const int u0 = (int)((long)units * w / nt), u1 = (int)((long)units * (w + 1) / nt);
        th.emplace_back(f, u0, u1);
    }
    for (auto &t : th) t.join();
}

// The log replayed backwards on a row-major N x W tile of eigenvector
// columns, then (dense path, A != nullptr) the Householder reflectors from
// the last to the first.  Every column sees the same operations in the same
// order for any W; the width sets how many independent columns share one
// pass over the log, so that each rotation's dependence on the one before
// (they share a row) is hidden behind W columns of work.
template <int W>
inline __attribute__((always_inline)) void vectors_tile(const Rot *log, size_t nlog, const double *A,
                                                        const double *beta, int N, double *tile) {
#pragma clang fp contract(off)
    for (size_t t = nlog; t-- > 0;) {
        const double c = log[t].c, s = log[t].s;
        double *__restrict a = tile + (size_t)log[t].p * W;
        double *__restrict b = a + W;
        for (int j = 0; j < W; ++j) {
            const double u = a[j], v = b[j];
            a[j] = c * u - s * v;
            b[j] = s * u + c * v;
        }
    }
    if (!A) return;
    for (int k = N - 3; k >= 0; --k) {
        const double bt = beta[k];
        if (bt == 0.0) continue;
        const double *v = A + (size_t)k * N + k + 1;
        double *z = tile + (size_t)(k + 1) * W;
        const int len = N - k - 1;
        double acc[W] = {};
        for (int i = 0; i < len; ++i)
            for (int j = 0; j < W; ++j) acc[j] += v[i] * z[(size_t)i * W + j];
        for (int j = 0; j < W; ++j) acc[j] *= bt;
        for (int i = 0; i < len; ++i)
            for (int j = 0; j < W; ++j) z[(size_t)i * W + j] -= acc[j] * v[i];
    }
}

// The same code built for AVX2 where the CPU has it: 4 doubles per vector
// operation instead of 2, with no fused multiply-add, so both builds round
// alike.
template <int W>
__attribute__((target("avx2"))) void vectors_tile_avx2(const Rot *log, size_t nlog, const double *A,
                                                       const double *beta, int N, double *tile) {
    vectors_tile<W>(log, nlog, A, beta, N, tile);
}
template <int W>
void vectors_tile_base(const Rot *log, size_t nlog, const double *A, const double *beta, int N, double *tile) {
    vectors_tile<W>(log, nlog, A, beta, N, tile);
}
bool cpu_avx2() {
    static const bool have = __builtin_cpu_supports("avx2");
    return have;
}

using TileFn = void (*)(const Rot *, size_t, const double *, const double *, int, double *);
template <int W>
TileFn tile_fn() {
    return cpu_avx2() ? &vectors_tile_avx2<W> : &vectors_tile_base<W>;
}

// Columns ids (unsorted eigen-indices) of J_1 J_2 ... J_t, or of
// Q J_1 ... J_t with Q = H_0 H_1 ... H_{N-3} when A holds the reflectors
// (rows of A, beta[k]): identity columns through vectors_tile, tiles of 32,
// 16 or 8 columns (the widest that still gives every thread a tile) claimed
// by the threads in turn.  Z is N x ncols row-major.
void build_cols(const std::vector<Rot> &log, const double *A, const double *beta, int N, const int *ids, int ncols,
                double *Z) {
    const long work = (long)(log.size() + (A ? (size_t)N * N : 0)) * ncols;
    const int nt = nthreads_for(work, (ncols + 7) / 8);
    const int W = ncols >= 32 * nt ? 32 : (ncols >= 16 * nt ? 16 : 8);
    const TileFn fn = W == 32 ? tile_fn<32>() : (W == 16 ? tile_fn<16>() : tile_fn<8>());
    const int ntiles = (ncols + W - 1) / W;
    std::atomic<int> next{0};
    auto work_fn = [&](int, int) {
        std::vector<double> tile((size_t)N * W);
        for (;;) {
            const int t = next.fetch_add(1);
            if (t >= ntiles) return;
            const int c0 = t * W, nc = std::min(W, ncols - c0);
            std::fill(tile.begin(), tile.end(), 0.0);
            for (int j = 0; j < nc; ++j) tile[(size_t)ids[c0 + j] * W + j] = 1.0;
            fn(log.data(), log.size(), A, beta, N, tile.data());
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < nc; ++j) Z[(size_t)i * ncols + c0 + j] = tile[(size_t)i * W + j];
        }
    };
    parallel_for(std::min(nt, ntiles), std::min(nt, ntiles), work_fn);
}

void replay_cols(const std::vector<Rot> &log, int N, const int *ids, int ncols, double *Z) {
    build_cols(log, nullptr, nullptr, N, ids, ncols, Z);
}

// Householder reduction of a dense symmetric N x N matrix (row-major, full
// storage, overwritten) to tridiagonal (d, e).  Step k maps row k's entries
// k+1..N-1 to mu e_1 with H_k = I - beta_k v_k v_k^T (v_k(0) = 1), applied
// to the trailing block as B -= v w^T + w v^T, w = p - (beta p^T v / 2) v,
// p = beta B v (B symmetric: p accumulates the rows of B scaled by the
// entries of v, in row order, so the inner loops run along rows).  v_k is
// left in row k, beta_k in beta[k].
inline __attribute__((always_inline)) void householder_body(int N, double *A, double *d, double *e, double *beta,
                                                            double *p, double *w) {
#pragma clang fp contract(off)
    for (int k = 0; k + 2 < N; ++k) {
        const int len = N - k - 1;
        double *x = A + (size_t)k * N + k + 1;
        double sigma = 0.0;
        for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
        const double x0 = x[0];
        if (sigma == 0.0) {
            e[k] = x0;
            beta[k] = 0.0;
            for (int i = 1; i < len; ++i) x[i] = 0.0;
            x[0] = 1.0;
            continue;
        }
        const double mu = std::sqrt(x0 * x0 + sigma);
        const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
        const double bt = 2.0 * v0 * v0 / (sigma + v0 * v0);
        const double inv = 1.0 / v0;
        x[0] = 1.0;
        for (int i = 1; i < len; ++i) x[i] *= inv;
        e[k] = mu;
        beta[k] = bt;
        // p = beta B v over the trailing block B = A[k+1:, k+1:]
        for (int i = 0; i < len; ++i) p[i] = 0.0;
        for (int j = 0; j < len; ++j) {
            const double *__restrict row = A + (size_t)(k + 1 + j) * N + k + 1;
            double *__restrict pp = p;
            const double xj = x[j];
            for (int i = 0; i < len; ++i) pp[i] += row[i] * xj;
        }
        double pv = 0.0;
        for (int i = 0; i < len; ++i) {
            p[i] *= bt;
            pv += p[i] * x[i];
        }
        const double K = 0.5 * bt * pv;
        for (int i = 0; i < len; ++i) w[i] = p[i] - K * x[i];
        for (int i = 0; i < len; ++i) {
            double *__restrict row = A + (size_t)(k + 1 + i) * N + k + 1;  // row k + 1 + i, x is row k
            const double xi = x[i], wi = w[i];
            const double *__restrict wr = w;
            const double *__restrict xr = x;
            for (int j = 0; j < len; ++j) row[j] -= xi * wr[j] + wi * xr[j];
        }
    }
    for (int k = 0; k < N; ++k) d[k] = A[(size_t)k * N + k];
    if (N >= 2) e[N - 2] = A[(size_t)(N - 2) * N + N - 1];
}
__attribute__((target("avx2"))) void householder_avx2(int N, double *A, double *d, double *e, double *beta,
                                                       double *p, double *w) {
    householder_body(N, A, d, e, beta, p, w);
}
void householder_base(int N, double *A, double *d, double *e, double *beta, double *p, double *w) {
    householder_body(N, A, d, e, beta, p, w);
}

void householder_tridiag(int N, double *A, std::vector<double> &d, std::vector<double> &e,
                         std::vector<double> &beta) {
    d.assign(N, 0.0);
    e.assign(std::max(N - 1, 0), 0.0);
    beta.assign(std::max(N - 2, 0), 0.0);
    std::vector<double> p(N), w(N);
    (cpu_avx2() ? householder_avx2 : householder_base)(N, A, d.data(), e.data(), beta.data(), p.data(), w.data());
}

// Columns ids of Q Z_t, Q = H_0 H_1 ... H_{N-3} (reflectors stored in the
// rows of A by householder_tridiag), Z_t = the QR rotations J_1 ... J_t:
// identity columns, rotations replayed backwards, then the reflectors from
// the last to the first.  Z is N x ncols row-major.
void dense_vectors(const std::vector<Rot> &log, const double *A, const std::vector<double> &beta, int N,
                   const int *ids, int ncols, double *Z) {
    build_cols(log, A, beta.data(), N, ids, ncols, Z);
}

// 1 / (largest |entry|) for a matrix whose entries all lie far from 1 (the
// squares in the rotations and reflector norms would underflow or
// overflow), else 1; 0 for non-finite entries.  Eigenvectors do not depend
// on the scale; eigenvalues are divided by it afterwards.
double far_scale(const std::vector<double> &v) {
    double amax = 0.0;
    for (double x : v) amax = std::max(amax, std::fabs(x));
    if (!std::isfinite(amax)) return 0.0;
    return (amax > 0.0 && (amax < 1e-100 || amax > 1e100)) ? 1.0 / amax : 1.0;
}

// Dense path: eigenvalues ascending in evals, selected columns (indices into
// the ascending order) of the eigenvector matrix in Zcols (N x ncols).
int dense_sym_eig(int N, const double *M, double *evals, const int *cols, int ncols, double *Zcols) {
    std::vector<double> A((size_t)N * N);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) A[(size_t)i * N + j] = 0.5 * (M[(size_t)i * N + j] + M[(size_t)j * N + i]);
    const double sc = far_scale(A);
    if (sc == 0.0) return -2;
    if (sc != 1.0)
        for (double &x : A) x *= sc;
    std::vector<double> d, e, beta;
    householder_tridiag(N, A.data(), d, e, beta);
    std::vector<Rot> log;
    log.reserve((size_t)N * 4);
    if (!tridiag_qr(d, e, log, nullptr, 0)) return -2;
    std::vector<int> perm(N);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int i = 0; i < N; ++i) evals[i] = d[perm[i]] / sc;
    if (ncols > 0 && Zcols) {
        std::vector<int> ids(ncols);
        for (int j = 0; j < ncols; ++j) ids[j] = perm[cols[j]];
        dense_vectors(log, A.data(), beta, N, ids.data(), ncols, Zcols);
    }
    return 0;
}

}  // namespace

void set_eig_threads(int n) { tl_eig_threads = std::max(1, n); }

int sym_eig_keep(int N, int bw, const double *M, double *evals, const int *rows, int nrows, double *Zrows,
                 EigLog *keep) {
    if (N <= 0) return -1;
    bw = std::max(0, std::min(bw, N - 1));
    Band Bd;
    Bd.N = N;
    Bd.w = bw + 1;
    Bd.B.assign((size_t)N * (Bd.w + 1), 0.0);
    for (int j = 0; j < N; ++j)
        for (int d = 0; d <= bw && j + d < N; ++d) {
            const int i = j + d;
            Bd.B[(size_t)j * (Bd.w + 1) + d] = 0.5 * (M[(size_t)i * N + j] + M[(size_t)j * N + i]);
        }
    const double sc = far_scale(Bd.B);
    if (sc == 0.0) return -2;
    if (sc != 1.0)
        for (double &x : Bd.B) x *= sc;
    std::vector<Rot> local;
    std::vector<Rot> &log = keep ? keep->rot : local;
    log.clear();
    log.reserve((size_t)N * 4);
    // the requested rows of the eigenvector matrix, accumulated as the
    // rotations are made (independent of the rotation chain, so they fill
    // its latency)
    const int nr = (nrows > 0 && Zrows) ? nrows : 0;
    std::vector<double> Zt((size_t)N * nr, 0.0);
    for (int i = 0; i < nr; ++i) Zt[(size_t)rows[i] * nr + i] = 1.0;
    if (bw >= 2) band_to_tridiag(Bd, bw, log, Zt.data(), nr);
    std::vector<double> d(N), e(std::max(N - 1, 0));
    for (int i = 0; i < N; ++i) d[i] = Bd.get(i, i);
    for (int i = 0; i + 1 < N; ++i) e[i] = Bd.get(i + 1, i);
    if (!tridiag_qr(d, e, log, Zt.data(), nr)) return -2;
    std::vector<int> perm(N);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int i = 0; i < N; ++i) evals[i] = d[perm[i]] / sc;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < N; ++j) Zrows[(size_t)i * N + j] = Zt[(size_t)perm[j] * nr + i];
    if (keep) {
        keep->N = N;
        keep->perm = perm;
    }
    return 0;
}

void eig_log_cols(const EigLog &L, const int *cols, int ncols, double *Zcols) {
    std::vector<int> ids(ncols);
    for (int j = 0; j < ncols; ++j) ids[j] = L.perm[cols[j]];
    replay_cols(L.rot, L.N, ids.data(), ncols, Zcols);
}

int sym_eig(int N, int bw, const double *M, double *evals, const int *rows, int nrows, double *Zrows,
            const int *cols, int ncols, double *Zcols) {
    if (N <= 0) return -1;
    if (nrows == 0 && std::min(bw, N - 1) >= std::max(24, N / 8)) return dense_sym_eig(N, M, evals, cols, ncols, Zcols);
    if (ncols > 0 && Zcols) {
        EigLog L;
        const int rc = sym_eig_keep(N, bw, M, evals, rows, nrows, Zrows, &L);
        if (rc != 0) return rc;
        eig_log_cols(L, cols, ncols, Zcols);
        return 0;
    }
    return sym_eig_keep(N, bw, M, evals, rows, nrows, Zrows, nullptr);
}

}  // namespace flp
