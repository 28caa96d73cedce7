// Host-side orchestration shared by the single-solve, batched and serving
// drivers: workspace buffers, filter construction, the Clenshaw launch plan,
// Gram-Schmidt, block QR, bounds, Rayleigh-Ritz and the per-solve state
// machine of the filtered Lanczos procedure.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
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
// Block steps between convergence checks when the caller leaves it open:
// the paper checks every 30 block steps at block size 3 (Table 2), i.e.
// every 90 basis columns; larger blocks keep that spacing in columns
// (r = 8: 11 steps, r = 16: 6), smaller ones stay at 30 steps.
inline int default_check_every(int r) { return std::min(30, std::max(1, (90 + r / 2) / r)); }
constexpr int kDefaultK0 = 40;
constexpr double kDefaultTol = 1e-9;
constexpr int kMaxDegree = 100000;
constexpr int64_t kDefaultMaxBasis = 3072;
// FLP_FORMAT_AUTO keeps CSR when the sliced ELL copy would store more than
// this many times the nonzeros
constexpr double kSellMaxPad = 1.25;
// Unfiltered Lanczos resolves an interval only once its Ritz values there
// have converged without a filter's help, which takes many more columns.
constexpr int64_t kUnfilteredMaxBasis = 12288;
constexpr int kPanelLog2 = 7;  // Lanczos basis panels of 128 columns
constexpr int64_t kInitPanels = 4;  // basis panels allocated at set-up (more on demand)
constexpr int kMaxPolish = 5;  // FP64 polish sweeps after an FP32-filter solve
// relative residual above which an in-interval Ritz pair of an FP32-filter
// solve counts as a mixture of eigenvectors (converged pairs sit near 1e-7)
constexpr double kMixedResid = 1e-4;
constexpr int kMaxSeparations = 8;  // Rayleigh-Ritz rounds on span{X, A x} for mixed pairs
// A polish sweep locks (only scales by p(t)) Ritz columns whose relative
// residual is already below this fraction of the tolerance
constexpr double kLockFrac = 0.1;
constexpr int kSetupThreads = 8;  // host threads for the set-up of a batch's solves
constexpr int kMaxSpeculative = 2;  // block steps a solve may take past a convergence check in flight
constexpr int kPaceLaunches = 8;    // filter launches per chunk while a check is in flight (single solve)

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
// ensure() that grows by at least half the current size (buffers whose
// demand creeps up: fewer reallocations, each a device-wide wait)
hipError_t ensure_grow(Buf &b, size_t bytes);

// Per-thread, per-device scratch shared by the calls one thread makes.
struct Workspace {
    Buf U[3];      // Clenshaw vectors
    Buf V32;       // FP32 copy of the filter input
    Buf Vg;        // one column group of the filter input, stored contiguously
    Buf PU[3], PR, PC;  // residual-form polish: FP32 recurrence and residual blocks, coefficients
    Buf val32;     // FP32 copy of the matrix values
    Buf partials;  // gemm_tn partial sums
    Buf small;     // small device matrices
    Buf W, Vin, Q; // single-solve Lanczos buffers
    Buf Y, AY, X, AX;  // Rayleigh-Ritz blocks
    Buf resid_part;
    const double *val32_src = nullptr;  // val the FP32 copy was made from
    int64_t val32_nnz = 0;
    // sliced ELL copy of the last matrix flp_filter_apply read in that
    // storage, with the arrays and precision it was built from
    Buf sell_off, sell_col, sell_val;
    flp_csr sell_src{};
    bool sell_fp32 = false, sell_built = false, sell_valid = false;
    flp_csr sell_A{};
    const float *sell_val32 = nullptr;
    void release_all();
};
Workspace &ws();

// Device allocations of the library (hipMalloc/hipFree, or the caller's
// allocator set by flp_set_allocator).
hipError_t dev_alloc(void **p, size_t bytes);
hipError_t dev_free(void *p);
// hands the allocator's cached device blocks back to the driver
void release_dev_cache();
// Held shared by the library's graph captures and exclusively around the
// device synchronisation of a free: a device-wide synchronisation in one
// thread invalidates a capture in progress in another.
std::shared_mutex &capture_mutex();
void set_allocator(flp_alloc_fn alloc, flp_free_fn free, void *ctx);
int check_symmetric(const flp_csr *A, double tol, hipStream_t s);

int check_csr(const flp_csr *A);
hipError_t h2d(void *dst, const void *src, size_t bytes, hipStream_t s);
int small_dev(size_t elems, double **out);

// ---------------------------------------------------------------- filter
double cheb_scalar(const std::vector<double> &b, double z);
// Chebyshev coefficients (m of them) of (p(z) - p(t)) / (z - t), p = sum b_k T_k
void cheb_divided(const std::vector<double> &b, double t, std::vector<double> &c);
int make_filter(double alpha, double beta, int degree, double lmin, double lmax, double eps, flp_filter **out);
double filter_step_bytes(int n, int64_t nnz, int r, int prec);
int filter_group_width(int n, int64_t nnz, int r, int prec);
int ensure_val32(const flp_csr *A, Buf &buf, const double **src_cache, int64_t *nnz_cache, const float **out,
                 hipStream_t s);
struct SolveBufs;
// Sliced ELL copy of A into off / col / val (FP64 values, or FP32 ones from val32
// when fp32): *out describes it (rowptr = slice offsets, nnz = stored
// entries, val = FP64 values or null), *out32 the FP32 values.  If the copy
// would store more than max_pad times A's nonzeros nothing is built and
// *built is false.  Synchronous.
int build_sell(const flp_csr *A, const float *val32, bool fp32, Buf &off, Buf &col, Buf &val, flp_csr *out,
               const float **out32, hipStream_t s, double max_pad, bool *built);

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
                     hipStream_t s, StepShape sh = StepShape{}, bool sell = false);

// ---------------------------------------------------------------- autotuner
struct FilterTune {
    int gw = 0;           // columns per filter launch (column-group width)
    StepShape sh{};       // launch shape of each step
    double us_per_step = 0.0;
    int candidates = 0;   // configurations timed (0: default, not timed)
};
// Picks (gw, shape) for filtering r columns of A by timing candidates (see
// flp_tune.cpp).  U: three device buffers of n x r filter-type elements
// (scratch, overwritten); V: n x r input block (read only, ld ldv).
int tune_filter(const flp_csr *A, const float *val32, int r, bool fp32, bool allow_groups, void *const U[3],
                const void *V, int ldv, hipStream_t s, FilterTune *out, bool sell = false);
// The cached tuning of a filter over r columns for A's size class and plane
// length (a single solve's first, then the segmented engine's), or the
// default shape; never times anything.  Callers use its tile mapping.
int lookup_filter_tune(const flp_csr *A, int r, bool fp32, FilterTune *out);
// The plane length the tuner's pencil walk uses for A: the smallest
// distance |j - i| >= 1024 between the middle row i and one of its columns
// j (a 3D grid's N^2 in natural order), or 0.  sell: A is a sliced ELL copy.
// Synchronises stream s.
int plane_rows(const flp_csr *A, bool sell, hipStream_t s, int *out);
void set_autotune(int mode);
int autotune_mode();
// chunk: sh.chunk is forced too (else only the shape and width)
void force_filter_shape(StepShape sh, int gw, bool chunk);

// W = p(Ahat) V (V, W n x r with leading dimensions) through the
// workspace's Clenshaw buffers.
// format: FLP_FORMAT_CSR, _SELL or _AUTO (the sliced copy is cached in the
// workspace, keyed by A's arrays).
int filter_apply_impl(const flp_filter *p, const flp_csr *A, const double *V, int ldv, double *W, int ldw, int r,
                      int prec, hipStream_t s, int format = FLP_FORMAT_CSR);
// The storage the calling thread's filter products read A in for `format`:
// *fA = A (and *fv32 = v32), or the workspace's sliced ELL copy of A (*sell).
int workspace_storage(const flp_csr *A, const float *v32, bool fp32, int format, hipStream_t s,
                      const flp_csr **fA, const float **fv32, bool *sell);
// Y = p(Ahat) X for c Ritz vectors of A (X, AX = A X, Ritz values lam;
// n x c blocks with leading dimension ldc) by the residual form: X diag(p(t))
// in FP64 plus the divided-difference recurrences on the residuals in FP32
// (val32: FP32 copy of A's values), 32 columns per recurrence.  Columns
// whose residual norm rres[j] (unscaled, as rayleigh_ritz returns it) is at
// or below lock_abs are locked: only scaled by p(t_j) (lock_abs <= 0 or
// rres == NULL: none).  chunk: tile-to-XCD mapping of the recurrence.
// Returns the algorithmic bytes moved.
int polish_apply(const flp_filter *p, const flp_csr *A, const float *val32, int c, const double *X,
                 const double *AX, int ldc, const std::vector<double> &lam, double *Y, hipStream_t s,
                 double *bytes,
                 const flp_csr *sellA = nullptr, const float *sell32 = nullptr,
                 const std::vector<double> *rres = nullptr, double lock_abs = 0.0, StepShape tile = StepShape{});

// ---------------------------------------------------------------- dense helpers
// y += a x over len doubles (host; an AVX2 build where the CPU has one,
// rounding alike to the plain build)
void host_axpy(int len, double a, const double *x, double *y);
void cholesky_flag(int r, const double *G, double thr2, std::vector<double> &R, std::vector<int> &bad);
void upper_inverse(int r, const std::vector<double> &R, std::vector<double> &Ri);
void matmul_upper(int r, const std::vector<double> &A, const std::vector<double> &B, std::vector<double> &C);

// sym: K == c and A^T B symmetric (B = A, or B = M A with M symmetric): the
// blocks below the diagonal are skipped and mirrored.
int gram_tn(int n, int K, int c, DMat A, const double *B, int64_t ldb, double *dev_out, double *host_out,
            hipStream_t s, bool sym = false);
int cgs2(DMat Q, int k, int n, double *W, int r, double *hdev, hipStream_t s);
int block_qr_impl(double *W, int n, int r, const DMat *Q, int k, std::vector<double> &S, uint64_t seed,
                  uint64_t sid, hipStream_t s, bool *replaced, int depth = 0);
// Spectrum bounds (PREPROC): k0 Lanczos steps, each new vector
// orthogonalised twice against the two before it, Ritz values widened by
// their residual bounds, clamped into the Gershgorin enclosure.  spmv_A: a
// sliced ELL copy of A with FP64 values for the products, or NULL (CSR A).
int estimate_bounds_impl(const flp_csr *A, int k0, uint64_t seed, double *lmin, double *lmax, hipStream_t s,
                         const flp_csr *spmv_A = nullptr);
int orthonormalize_cols(int n, int c, double *&Y, double *&tmp, int ldc, double *sdev, hipStream_t s);
// The same for a block Y whose columns need not be orthonormal (Y itself is
// left as it is): replaces orthonormalising Y and then rayleigh_ritz.
int rayleigh_ritz_gen(const flp_csr *A, int n, int c, const double *Y, double *AY, double *X, double *AX, int ldc,
                      double *sdev, std::vector<double> &lam, std::vector<double> &res, hipStream_t s);
int rayleigh_ritz(const flp_csr *A, int n, int c, const double *Y, double *AY, double *X, double *AX, int ldc,
                  double *sdev, std::vector<double> &lam, std::vector<double> &res, hipStream_t s);

// ---------------------------------------------------------------- solve state
// Device buffers one solve keeps across block steps.
struct SolveBufs {
    Buf Q, W, Vin, U[3], V32, val32, hdev;
    Buf sell_off, sell_col, sell_val;  // sliced ELL copy of A for the filter (FLP_FORMAT_SELL)
    // Ritz blocks of the finish (batched and serving solves: freed with the
    // solve; a single solve uses the calling thread's workspace instead)
    Buf Y, AY, X, AX;
    bool own_ritz = false;
    const double *val32_src = nullptr;
    int64_t val32_nnz = 0;
    // earlier, smaller basis allocations: freed with the rest (a device free
    // waits for all work on the device, so it is kept out of the block steps)
    std::deque<Buf> retired;
};

// One filtered Lanczos solve advanced block step by block step.
// One convergence check of T_k (Section 3.2.2) as a self-contained task:
// a snapshot of T_k and S_k goes in; the Ritz values' candidate set, the
// residual test and the eigen-decomposition's rotation log come out.  It
// runs on a host pool thread while the solve keeps stepping.
struct CheckTask {
    int K = 0, r = 0;
    double tau = 0, tol_p = 0;
    bool fp32 = false;
    // unfiltered Lanczos: candidates are the Ritz values in [lo, hi] plus
    // the nearest one on each side
    bool unfiltered = false;
    double lo = 0, hi = 0;
    std::vector<double> T, Sk;
    int rc = FLP_OK;
    std::string msg;
    bool ok = false;  // every candidate's residual bound met
    std::vector<int> cand, guard;
    EigLog eig;
    double secs = 0.0;
    std::atomic<bool> ready{false};
};
void run_check(CheckTask &c);

// Fixed pool of host threads for work that overlaps the device (the
// convergence checks).  Tasks run in submission order per worker.
void host_pool_submit(std::function<void()> f);

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
    bool unfiltered = false;  // p(Ahat) = Ahat (plain block Lanczos)
    bool sell = false;        // the filter reads A's sliced ELL copy SA (values sval32 in FP32)
    flp_csr SA{};
    const float *sval32 = nullptr;
    std::unique_ptr<flp_filter> filt;
    int check_every = 0, max_steps = 0;
    int check_offset = 0;  // checks fall on steps with (steps + check_offset) % check_every == 0
    int64_t npanels = 0;   // panels the basis may grow to (max_basis)
    int64_t qpanels = 0;   // panels allocated (grown on demand)
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
    std::vector<int> guard;  // FP32 filter: Ritz vectors just outside the candidates, polished with them
    int tile_chunk = 0;       // tile-to-XCD mapping the filter launches use (the polish follows it)
    int tile_win = 0;         // LDS window of the filter launches (the polish follows it)
    flp_stats st{};
    double t_start = 0;
    int code = FLP_OK;  // first error
    // block-step staging: pinned host h1, h2, G, R^{-1} (r x r each) and the
    // device Gram / R^{-1} blocks behind the projection coefficients
    double *pin = nullptr;
    double *gdev = nullptr, *rdev = nullptr;
    std::vector<double> R1;
    bool slow = false;      // this step's block needed the rank repair path
    int checked_step = -1;  // block step whose convergence check was started
    EigLog eig;             // rotation log of the deciding check's T_k
    std::shared_ptr<CheckTask> check;  // check in flight (its T_k may be behind the current step)
    bool check_last = false;           // that check is the final one (no basis room left)
    double t_step0 = 0.0;   // host time the current block step started
    Solve() = default;
    Solve(const Solve &) = delete;
    Solve &operator=(const Solve &) = delete;
    ~Solve();
};

// bounds, filter, buffers, start block (PREPROC and set-up)
int solve_setup(Solve &S);
// Grows the basis allocation (by doubling, on S.s, synchronous) so that it
// holds at least cols columns (capped at max_basis).
int ensure_basis(Solve &S, int64_t cols);
// One block step of a single solve after the filter has produced W, in
// phases separated by a stream synchronisation (the batched engine does the
// first three for all its solves at once with the segmented launches of
// Engine::block_step, then calls step_check per solve):
//   step_orth_launch: CGS2 against the basis, Gram matrix of W (async);
//   step_qr1:         D_j; first Cholesky factor; apply it; second Gram (async);
//   step_qr2:         second Cholesky factor; apply it; S_j;
//   step_check:       applies a finished convergence check; at the cadence
//                     starts the next one on the host pool (the solve keeps
//                     stepping meanwhile: if that check decides convergence,
//                     the result comes from the checked T_k and the extra
//                     steps are dropped); else the new block joins the basis
//                     and becomes the next input.
int step_orth_launch(Solve &S);
int step_qr1(Solve &S);
int step_qr2(Solve &S);
// copy_next = false: the caller has already written the new block into the
// basis and the next filter input
int step_check(Solve &S, bool async = true, bool copy_next = true);
// waits for and applies a check in flight (no-op when there is none)
int wait_check(Solve &S);
// all four phases with synchronisations (single solve)
int solve_after_filter(Solve &S);
// Ritz vectors, Rayleigh-Ritz with A, FP32 polish, result
int solve_finish(Solve &S, flp_result **out);
// Device bytes solve_finish allocates for a solve that has converged (its
// Ritz blocks, the result's eigenvectors, the polish's FP32 blocks); the
// basis the solve already holds is not included.
size_t finish_bytes(const Solve &S);

// ---------------------------------------------------------------- engine
// Segment tables of one block step for the active solves: table t lists
// the solves taking part in filter launch t, in order, with tile offsets.
struct Tables {
    int M = 0, cap = 0, r = 0;
    bool fp32 = false;
    StepShape sh{};  // launch shape of the segmented steps
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
    bool finished = false;  // result handed back (set under the owner's lock)
    std::atomic<bool> cancel{false};  // cancellation requested (serving)
    // serving: recorded on the submitter's stream; the engine's stream waits
    // for it before the request's first launch
    hipEvent_t ready = nullptr;
    Job() = default;
    Job(const Job &) = delete;
    Job &operator=(const Job &) = delete;
    ~Job() {
        if (ready) (void)hipEventDestroy(ready);
    }
};

// Advances a set of active solves in lockstep: per block step, one
// segmented filter launch per Clenshaw step (replayed from a HIP graph while
// the set is unchanged), then one segmented launch sequence for the
// Gram-Schmidt and block QR of all of them, then each solve's convergence
// check; solves that converged go to the finisher threads for their Ritz
// vectors, Rayleigh-Ritz and polish while the others step on.
struct Engine {
    hipStream_t s = nullptr;
    int device = 0;
    int r = 0, prec = 0;
    bool use_graph = true;
    std::vector<Job *> active;
    uint64_t n_added = 0;
    Tables T;
    bool tables_valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    flp_batch_stats stats{};
    // Called once per job when it leaves the engine (result ready, or an
    // error), from the stepping thread or the finisher thread, after the
    // job's device buffers are released.
    std::function<void(Job *)> on_done;
    // Optional gate of the finish phase: before a finisher starts a job it
    // asks for finish_bytes(job) more device memory; `lone` is true when
    // no other job is being finished (such a request must be granted).  A
    // refusal is retried when another job completes.
    std::function<bool(Job *, size_t bytes, bool lone)> reserve_finish;
    Engine() = default;
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;
    ~Engine();
    int init(int r, int prec, bool use_graph);
    void add(Job *j);
    // one block step of every active solve; converged solves leave the
    // active set for the finisher
    int step();
    void graph_reset();
    // blocks until every handed-off solve is finished
    void wait_finisher();
    // engine statistics including the finisher's time
    flp_batch_stats snapshot();
    // waits for the block-step work issued so far
    int sync_steps();

  private:
    // Gram-Schmidt and block QR of every active solve as one segmented
    // launch sequence on s (tables, partial sums, per-solve outputs D_j,
    // S_j and status; pinned staging for the one copy each way per step)
    Buf otab, opart, oout;
    unsigned char *ostage = nullptr;
    size_t ostage_bytes = 0;
    double *oout_pin = nullptr;
    size_t oout_pin_bytes = 0;
    std::vector<OrthSeg> otab_host;
    std::vector<int> opre_host;
    int block_step(double filter_secs);
    // finishers: Ritz vectors, Rayleigh-Ritz and polish of converged solves,
    // each on its own host thread and stream, overlapping later block steps
    static constexpr int kFinishers = 8;
    // The finisher threads share kFinisherStreams streams: HIP maps streams
    // onto a few hardware queues (4 per process by default), and a stream that
    // shares a queue with the stepping stream s would hold the lockstep block
    // steps behind a finisher's Rayleigh-Ritz and polish work.
    static constexpr int kFinisherStreams = 2;
    hipStream_t fs[kFinisherStreams] = {};
    std::thread fin[kFinishers];
    std::mutex fmu;
    std::condition_variable fcv, fdone;
    std::deque<Job *> fq;
    int fbusy = 0;
    uint64_t fdone_count = 0;  // jobs the finishers have completed (wakes gated finishers)
    bool fstop = false;
    double t_finish = 0.0;
    void finisher_main(int w);
    void complete(Job *j);
};

// drivers (solve_impl: the warm start when opts.warm is given, else or on its
// fallback solve_cold, the filtered Lanczos run)
int solve_impl(const flp_csr *A, double alpha, double beta, const flp_opts &o, flp_result **out);
int solve_cold(const flp_csr *A, double alpha, double beta, const flp_opts &o, flp_result **out);
int solve_batch_impl(int count, const flp_csr *const *A, const double *alpha, const double *beta,
                     const flp_opts *opts, int use_graph, flp_result **results, int *codes, flp_batch_stats *bs);
int solve_sliced_impl(const flp_csr *A, double alpha, double beta, int nslices, const flp_opts &o,
                      flp_result **out);
void release_single_bufs();

}  // namespace flp
