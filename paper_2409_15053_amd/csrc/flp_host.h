// Host-side orchestration shared by the single-solve, batched and serving
// drivers: workspace buffers, filter construction, the Clenshaw launch plan,
// Gram-Schmidt, block QR, bounds, Rayleigh-Ritz and the per-solve state
// machine of the filtered Lanczos procedure.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "flp_internal.h"

// A Chebyshev filter polynomial: degree, coefficients and the spectrum
// bounds of its affine map (Section 3.2.3).
struct flp_filter {
    double alpha, beta;  // as given
    double lmin, lmax, c, e;
    double a1, b1;       // mapped, clamped interval
    int m;
    std::vector<double> b;
};

namespace flp {

constexpr double kDefaultEps = 0.31227;
constexpr int kDefaultCheck = 30;
constexpr int kDefaultK0 = 40;
constexpr double kDefaultTol = 1e-9;
constexpr int kMaxDegree = 100000;
constexpr int64_t kDefaultMaxBasis = 3072;
constexpr int kPanelLog2 = 7;  // Lanczos basis panels of 128 columns

int fail(int code, const std::string &msg);
const char *last_error_cstr();
double now();

#define CK(...)                                                                                  \
    do {                                                                                         \
        hipError_t e_ = (__VA_ARGS__);                                                           \
        if (e_ != hipSuccess) {                                                                  \
            if (e_ == hipErrorOutOfMemory)                                                       \
                return ::flp::fail(FLP_E_NOMEM, std::string(#__VA_ARGS__) + ": out of device memory"); \
            return ::flp::fail(FLP_E_DEVICE, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
        }                                                                                        \
    } while (0)

#define CKR(...)                       \
    do {                               \
        int rc_ = (__VA_ARGS__);       \
        if (rc_ != FLP_OK) return rc_; \
    } while (0)

// ---------------------------------------------------------------- buffers
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    Buf() = default;
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    ~Buf();
    void release();
};
hipError_t ensure(Buf &b, size_t bytes);

// Per-device scratch shared by calls that run one after another.
struct Workspace {
    Buf U[3];      // Clenshaw vectors
    Buf V32;       // FP32 copy of the filter input
    Buf val32;     // FP32 copy of the matrix values
    Buf partials;  // gemm_tn partial sums
    Buf small;     // small device matrices
    Buf W, Vin, Q; // single-solve Lanczos buffers
    Buf Y, AY, X, AX;  // Rayleigh-Ritz blocks
    Buf resid_part;
    const double *val32_src = nullptr;  // val the FP32 copy was made from
    int64_t val32_nnz = 0;
    void release_all();
};
Workspace &ws();

int check_csr(const flp_csr *A);
hipError_t h2d(void *dst, const void *src, size_t bytes, hipStream_t s);
int small_dev(size_t elems, double **out);

// ---------------------------------------------------------------- filter
double cheb_scalar(const std::vector<double> &b, double z);
int make_filter(double alpha, double beta, int degree, double lmin, double lmax, double eps, flp_filter **out);
double filter_step_bytes(int n, int64_t nnz, int r, int prec);
int filter_group_width(int n, int64_t nnz, int r, int prec);
int ensure_val32(const flp_csr *A, Buf &buf, const double **src_cache, int64_t *nnz_cache, const float **out,
                 hipStream_t s);

// One launch of the Clenshaw recurrence (Section 2.2):
// out = alpha (A X) + beta X + gamma V + delta Y on row-major blocks.
struct ClenshawStep {
    const void *X;
    int ldx;
    const void *V;  // may be null
    int ldv;
    const void *Y;  // may be null
    int ldy;
    void *out;
    int ldo;
    bool out_f64;   // output written in FP64 (the last step of an FP32 filter)
    double alpha, beta, gamma, delta;
};
// The m launches that evaluate W = p(Ahat) V for one column group: V, W with
// leading dimensions; U0..U2 three scratch blocks n x r (ld r) of the
// recurrence's type; fp32 selects the FP32 recurrence (V, U in FP32, W FP64).
std::vector<ClenshawStep> clenshaw_plan(const flp_filter *p, int r, const void *V, int ldv, double *W, int ldw,
                                        void *U0, void *U1, void *U2, bool fp32);
int launch_plan_step(const flp_csr *A, const float *val32, int r, const ClenshawStep &st, bool fp32,
                     hipStream_t s);

// W = p(Ahat) V (V, W n x r with leading dimensions) through the
// workspace's Clenshaw buffers.
int filter_apply_impl(const flp_filter *p, const flp_csr *A, const double *V, int ldv, double *W, int ldw, int r,
                      int prec, hipStream_t s);

// ---------------------------------------------------------------- dense helpers
void cholesky_flag(int r, const double *G, double thr2, std::vector<double> &R, std::vector<int> &bad);
void upper_inverse(int r, const std::vector<double> &R, std::vector<double> &Ri);
void matmul_upper(int r, const std::vector<double> &A, const std::vector<double> &B, std::vector<double> &C);

int gram_tn(int n, int K, int c, DMat A, const double *B, int64_t ldb, double *dev_out, double *host_out,
            hipStream_t s);
int cgs2(DMat Q, int k, int n, double *W, int r, double *hdev, hipStream_t s);
int block_qr_impl(double *W, int n, int r, const DMat *Q, int k, std::vector<double> &S, uint64_t seed,
                  uint64_t sid, hipStream_t s, bool *replaced, int depth = 0);
int estimate_bounds_impl(const flp_csr *A, int k0, uint64_t seed, double *lmin, double *lmax, hipStream_t s);
int orthonormalize_cols(int n, int c, double *&Y, double *&tmp, int ldc, double *sdev, hipStream_t s);
int rayleigh_ritz(const flp_csr *A, int n, int c, const double *Y, double *AY, double *X, double *AX, int ldc,
                  double *sdev, std::vector<double> &lam, std::vector<double> &res, hipStream_t s);

// ---------------------------------------------------------------- solve state
// Device buffers one solve keeps across block steps.
struct SolveBufs {
    Buf Q, W, Vin, U[3], V32, val32, hdev;
    const double *val32_src = nullptr;
    int64_t val32_nnz = 0;
};

// One filtered Lanczos solve advanced block step by block step.
struct Solve {
    // inputs
    const flp_csr *A = nullptr;
    double alpha = 0, beta = 0;
    flp_opts o{};
    hipStream_t s = nullptr;
    SolveBufs *B = nullptr;
    // derived
    int n = 0, r = 0;
    double lmin = 0, lmax = 0, tau = 0, tol_p = 0;
    std::unique_ptr<flp_filter> filt;
    int check_every = 0, max_steps = 0;
    int64_t npanels = 0;
    DMat Q{};
    double *W = nullptr, *Vin = nullptr, *hdev = nullptr;
    const float *val32 = nullptr;
    float *V32 = nullptr;
    void *U[3] = {nullptr, nullptr, nullptr};
    std::vector<ClenshawStep> plan;  // the filter's launches for this solve
    // state
    std::vector<double> D_all, S_all, Sj;
    int steps = 0, prev_count = -1, kfinal = 0;
    bool converged = false, done = false;
    std::vector<int> cand;
    flp_stats st{};
    double t_start = 0;
    int code = FLP_OK;  // first error
    // block-step staging: pinned host h1, h2, G, R^{-1} (r x r each) and the
    // device Gram / R^{-1} blocks behind the projection coefficients
    double *pin = nullptr;
    double *gdev = nullptr, *rdev = nullptr;
    std::vector<double> R1;
    bool slow = false;      // this step's block needed the rank repair path
    int checked_step = -1;  // block step whose convergence check has run
    EigLog eig;             // rotation log of the last check's T_k
    double t_step0 = 0.0;   // host time the current block step started
    Solve() = default;
    Solve(const Solve &) = delete;
    Solve &operator=(const Solve &) = delete;
    ~Solve();
};

// bounds, filter, buffers, start block (PREPROC and set-up)
int solve_setup(Solve &S);
// One block step after the filter has produced W, in phases separated by a
// stream synchronisation (the batched driver runs each phase for all solves
// before one shared synchronisation):
//   step_orth_launch: CGS2 against the basis, Gram matrix of W (async);
//   step_qr1:         D_j; first Cholesky factor; apply it; second Gram (async);
//   step_qr2:         second Cholesky factor; apply it; S_j;
//   step_check:       convergence check at the cadence (host only), else the
//                     new block joins the basis and becomes the next input.
int step_orth_launch(Solve &S);
int step_qr1(Solve &S);
int step_qr2(Solve &S);
int step_check(Solve &S);
// the host part of step_check (thread-safe per solve): runs the check when
// this block step is at the cadence and has not been checked yet
int step_check_host(Solve &S);
// all four phases with synchronisations (single solve)
int solve_after_filter(Solve &S);
// Ritz vectors, Rayleigh-Ritz with A, FP32 polish, result
int solve_finish(Solve &S, flp_result **out);

// ---------------------------------------------------------------- engine
// Segment tables of one block step for the active solves: table t lists
// the solves taking part in filter launch t, in order, with tile offsets.
struct Tables {
    int M = 0, cap = 0, r = 0;
    bool fp32 = false;
    std::vector<SegEntry> host;    // M x cap
    std::vector<int> nseg, tiles;  // per launch
    Buf dev;
};

// One request of the batched / serving engine.
struct Job {
    uint64_t id = 0;
    std::unique_ptr<Solve> S;
    std::unique_ptr<SolveBufs> B;
    flp_result *res = nullptr;
    int code = FLP_OK;
    double t_submit = 0, t_done = 0;
    size_t footprint = 0;   // device bytes reserved at admission
    flp_csr A{};            // the caller's matrix descriptor
    std::string msg;        // error message of a failed request
};

// Advances a set of active solves in lockstep: per block step, one
// segmented filter launch per Clenshaw step (replayed from a HIP graph while
// the set is unchanged), then each solve's Gram-Schmidt, block QR and
// convergence check, then Rayleigh-Ritz for the solves that finished.
struct Engine {
    hipStream_t s = nullptr;
    int r = 0, prec = 0;
    bool use_graph = true;
    std::vector<Job *> active;
    Tables T;
    bool tables_valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    flp_batch_stats stats{};
    Engine() = default;
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;
    ~Engine();
    int init(int r, int prec, bool use_graph);
    void add(Job *j);
    // one block step of every active solve; jobs that completed (result or
    // error) leave the active set and are appended to finished
    int step(std::vector<Job *> &finished);
    void graph_reset();
};

// drivers
int solve_impl(const flp_csr *A, double alpha, double beta, const flp_opts &o, flp_result **out);
int solve_batch_impl(int count, const flp_csr *const *A, const double *alpha, const double *beta,
                     const flp_opts *opts, int use_graph, flp_result **results, int *codes, flp_batch_stats *bs);
void release_single_bufs();

}  // namespace flp
