// Host symmetric eigensolver for the small projected problems.
//
// The paper solves the eigenproblem of the banded block-tridiagonal T_k on
// the CPU with a special-purpose banded symmetric eigensolver (Section
// 3.2.2).  This one works in two phases, both on adjacent-plane Givens
// rotations:
//   1. band -> tridiagonal: the outermost diagonal is annihilated one entry
//      at a time and the bulge each rotation creates is chased down the band
//      (Rutishauser/Schwarz band reduction), bandwidth b -> b-1 -> ... -> 1;
//   2. implicit symmetric QR with the Wilkinson shift on the tridiagonal
//      (Golub & Van Loan, "Matrix Computations", Sec. 8.3).
// Every rotation is logged.  Eigenvector rows are obtained by replaying the
// log on selected rows of the identity: the convergence check only needs
// the last r rows of the eigenvector matrix (for the Ritz residual bounds),
// so it replays on r rows; the final Ritz vectors replay on all rows, in
// parallel over row tiles.
#include "flp_internal.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

namespace flp {

namespace {

struct Rot {
    int32_t p;  // plane (p, p+1)
    double c, s;
};

// M' = J^T M J on rows/columns (p, p+1) restricted to [lo, hi], where
// J[:,p] = c e_p + s e_q and J[:,q] = -s e_p + c e_q.
inline void rotate_dense(double *M, int N, int p, double c, double s, int lo, int hi) {
    const int q = p + 1;
    double *rp = M + (size_t)p * N, *rq = M + (size_t)q * N;
    for (int x = lo; x <= hi; ++x) {
        double a = rp[x], b = rq[x];
        rp[x] = c * a + s * b;
        rq[x] = -s * a + c * b;
    }
    for (int x = lo; x <= hi; ++x) {
        double *row = M + (size_t)x * N;
        double a = row[p], b = row[q];
        row[p] = c * a + s * b;
        row[q] = -s * a + c * b;
    }
}

// Reduce the symmetric matrix M (N x N row-major, semi-bandwidth b) to
// tridiagonal form in place, logging the rotations.
void band_to_tridiag(double *M, int N, int b, std::vector<Rot> &log) {
    for (int bw = b; bw >= 2; --bw) {
        for (int j = 0; j + bw < N; ++j) {
            int k = j, i = j + bw;
            while (i < N) {
                double x = M[(size_t)(i - 1) * N + k];
                double y = M[(size_t)i * N + k];
                if (y == 0.0) break;
                double r = std::hypot(x, y);
                double c = x / r, s = y / r;
                int lo = std::max(0, i - 1 - bw - 1);
                int hi = std::min(N - 1, i + bw + 1);
                rotate_dense(M, N, i - 1, c, s, lo, hi);
                M[(size_t)i * N + k] = 0.0;
                M[(size_t)k * N + i] = 0.0;
                log.push_back({i - 1, c, s});
                // the rotation fills (i-1+bw+1, i-1); chase it with plane (i-1+bw, i+bw)
                k = i - 1;
                i = i + bw;
            }
        }
    }
}

// Implicit QR with Wilkinson shift on the tridiagonal (d, e); e[i] couples
// i and i+1.  On return d holds the eigenvalues (unsorted).
bool tridiag_qr(std::vector<double> &d, std::vector<double> &e, std::vector<Rot> &log) {
    const int N = (int)d.size();
    if (N <= 1) return true;
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
            double r = std::hypot(x, z);
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
        }
    }
    return true;
}

// Rows R of (I J_1 J_2 ... J_t): start from the identity rows and replay the
// log.  Z is nrows x N row-major; rows[i] is the identity row for Z row i.
void replay(const std::vector<Rot> &log, int N, const int *rows, int nrows, double *Z) {
    constexpr int TILE = 8;
    const int ntiles = (nrows + TILE - 1) / TILE;
    auto work = [&](int t0, int t1) {
        std::vector<double> tile((size_t)N * TILE);
        for (int t = t0; t < t1; ++t) {
            int r0 = t * TILE, nr = std::min(TILE, nrows - r0);
            std::fill(tile.begin(), tile.end(), 0.0);
            for (int i = 0; i < nr; ++i) tile[(size_t)rows[r0 + i] * TILE + i] = 1.0;
            for (const Rot &g : log) {
                double *a = &tile[(size_t)g.p * TILE];
                double *b = a + TILE;
                for (int i = 0; i < TILE; ++i) {
                    double u = a[i], v = b[i];
                    a[i] = g.c * u + g.s * v;
                    b[i] = -g.s * u + g.c * v;
                }
            }
            for (int i = 0; i < nr; ++i)
                for (int j = 0; j < N; ++j) Z[(size_t)(r0 + i) * N + j] = tile[(size_t)j * TILE + i];
        }
    };
    int nthreads = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    nthreads = std::min(nthreads, ntiles);
    if (nthreads <= 1 || (long)log.size() * nrows < 2000000L) {
        work(0, ntiles);
        return;
    }
    std::vector<std::thread> th;
    for (int w = 0; w < nthreads; ++w) {
        int t0 = (int)((long)ntiles * w / nthreads), t1 = (int)((long)ntiles * (w + 1) / nthreads);
        th.emplace_back(work, t0, t1);
    }
    for (auto &t : th) t.join();
}

}  // namespace

int sym_eig(int N, int bw, const double *M, double *evals, const int *rows, int nrows,
            double *Z) {
    if (N <= 0) return -1;
    bw = std::max(0, std::min(bw, N - 1));
    std::vector<double> W(M, M + (size_t)N * N);
    std::vector<Rot> log;
    log.reserve((size_t)N * 4);
    if (bw >= 2) band_to_tridiag(W.data(), N, bw, log);
    std::vector<double> d(N), e(std::max(N - 1, 0));
    for (int i = 0; i < N; ++i) d[i] = W[(size_t)i * N + i];
    for (int i = 0; i + 1 < N; ++i) e[i] = 0.5 * (W[(size_t)i * N + i + 1] + W[(size_t)(i + 1) * N + i]);
    if (!tridiag_qr(d, e, log)) return -2;
    std::vector<int> perm(N);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int i = 0; i < N; ++i) evals[i] = d[perm[i]];
    if (nrows > 0 && Z) {
        std::vector<double> tmp((size_t)nrows * N);
        replay(log, N, rows, nrows, tmp.data());
        for (int i = 0; i < nrows; ++i)
            for (int j = 0; j < N; ++j) Z[(size_t)i * N + j] = tmp[(size_t)i * N + perm[j]];
    }
    return 0;
}

}  // namespace flp
