// Batched filtered Lanczos: many independent solves advanced in lockstep.
//
// Every block step, the filters of all active solves run as one sequence of
// segmented launches: launch t carries, for each solve, its own Clenshaw
// step (its own matrix, vectors and coefficients), so a batch of small
// problems fills the GPU the way one large problem does.  Filters of
// different degrees are aligned at their last step (a solve of degree m
// joins the sequence at launch M - m).  The launch sequence of a block step
// is captured once into a HIP graph and replayed while the set of active
// solves is unchanged; its segment tables live in device memory and stay
// valid because every solve keeps its buffers for its whole life.  The
// Gram-Schmidt, block QR and convergence checks of each solve follow on the
// same stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "flp_host.h"

namespace flp {

namespace {

struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    void reset() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        x = nullptr;
        g = nullptr;
    }
    ~Graph() { reset(); }
};

struct StreamGuard {
    hipStream_t s = nullptr;
    ~StreamGuard() {
        if (s) (void)hipStreamDestroy(s);
    }
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Segment tables of one block step for the active solves: table t lists
// the solves taking part in launch t, in order, with tile offsets.
struct Tables {
    int M = 0, cap = 0, r = 0;
    bool fp32 = false;
    std::vector<SegEntry> host;    // M x cap
    std::vector<int> nseg, tiles;  // per launch
    Buf dev;
};

int build_tables(const std::vector<Solve *> &act, Tables &T, hipStream_t s) {
    T.M = 0;
    for (Solve *S : act) T.M = std::max(T.M, (int)S->plan.size());
    T.cap = (int)act.size();
    T.host.assign((size_t)T.M * T.cap, SegEntry{});
    T.nseg.assign(T.M, 0);
    T.tiles.assign(T.M, 0);
    const int rpt = seg_rows_per_tile(T.r, T.fp32);
    for (int t = 0; t < T.M; ++t) {
        int ns = 0, tiles = 0;
        for (Solve *S : act) {
            const int m = (int)S->plan.size();
            const int j = t - (T.M - m);
            if (j < 0) continue;
            const ClenshawStep &st = S->plan[j];
            SegEntry e{};
            e.rowptr = S->A->rowptr;
            e.colind = S->A->colind;
            e.val = T.fp32 ? (const void *)S->val32 : (const void *)S->A->val;
            e.X = st.X;
            e.V = st.V;
            e.Y = st.Y;
            e.out = st.out;
            e.n = S->n;
            e.tile0 = tiles;
            e.ldx = st.ldx;
            e.ldv = st.ldv;
            e.ldy = st.ldy;
            e.ldo = st.ldo;
            e.out_f64 = (T.fp32 && st.out_f64) ? 1 : 0;
            e.alpha = st.alpha;
            e.beta = st.beta;
            e.gamma = st.gamma;
            e.delta = st.delta;
            T.host[(size_t)t * T.cap + ns++] = e;
            tiles += (S->n + rpt - 1) / rpt;
        }
        T.nseg[t] = ns;
        T.tiles[t] = tiles;
    }
    CK(ensure(T.dev, sizeof(SegEntry) * std::max<size_t>(T.host.size(), 1)));
    CK(h2d(T.dev.p, T.host.data(), sizeof(SegEntry) * T.host.size(), s));
    return FLP_OK;
}

int launch_tables(const Tables &T, hipStream_t s) {
    const SegEntry *base = (const SegEntry *)T.dev.p;
    for (int t = 0; t < T.M; ++t)
        CK(launch_cheb_seg(T.fp32, T.r, base + (size_t)t * T.cap, T.nseg[t], T.tiles[t], s));
    return FLP_OK;
}

}  // namespace

int solve_batch_impl(int count, const flp_csr *const *A, const double *alpha, const double *beta,
                     const flp_opts *opts, int use_graph, flp_result **results, int *codes, flp_batch_stats *bs) {
    const double t0 = now();
    flp_batch_stats stats{};
    stats.solves = count;
    hipStream_t user = nullptr;
    flp_opts o0;
    flp_opts_default(&o0);
    if (opts) user = (hipStream_t)opts[0].stream;
    for (int i = 0; i < count; ++i) {
        results[i] = nullptr;
        codes[i] = FLP_OK;
    }
    CK(hipStreamSynchronize(user));
    StreamGuard sg;
    CK(hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking));
    hipStream_t s = sg.s;

    std::vector<std::unique_ptr<Solve>> solves(count);
    std::vector<std::unique_ptr<SolveBufs>> bufs(count);
    int r = -1, prec = -1;
    for (int i = 0; i < count; ++i) {
        auto S = std::make_unique<Solve>();
        S->A = A[i];
        S->alpha = alpha[i];
        S->beta = beta[i];
        S->o = opts ? opts[i] : o0;
        S->o.stream = nullptr;
        S->s = s;
        if (r < 0) {
            r = S->o.block;
            prec = S->o.prec;
        }
        if (S->o.block != r || S->o.prec != prec)
            return fail(FLP_E_ARG, "all solves of a batch need the same block size and precision");
        int rc = check_csr(A[i]);
        if (rc == FLP_OK) {
            bufs[i] = std::make_unique<SolveBufs>();
            S->B = bufs[i].get();
            rc = solve_setup(*S);
        }
        codes[i] = rc;
        solves[i] = std::move(S);
    }
    stats.t_setup = now() - t0;

    Tables T;
    T.r = r;
    T.fp32 = prec == FLP_PREC_FP32_FILTER;
    Graph graph;
    bool tables_valid = false;
    EventPair ev;
    CK(hipEventCreate(&ev.a));
    CK(hipEventCreate(&ev.b));
    for (;;) {
        std::vector<Solve *> act;
        for (int i = 0; i < count; ++i)
            if (codes[i] == FLP_OK && !solves[i]->done) act.push_back(solves[i].get());
        if (act.empty()) break;
        if (!tables_valid) {
            graph.reset();
            CKR(build_tables(act, T, s));
            if (use_graph) {
                CK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                int rc = launch_tables(T, s);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(s, &g);
                if (rc != FLP_OK) return rc;
                CK(e);
                graph.g = g;
                CK(hipGraphInstantiate(&graph.x, graph.g, nullptr, nullptr, 0));
                ++stats.graph_captures;
            }
            tables_valid = true;
        }
        // filter phase: one segmented launch per Clenshaw step
        CK(hipEventRecord(ev.a, s));
        if (use_graph) {
            CK(hipGraphLaunch(graph.x, s));
            ++stats.graph_replays;
        } else {
            CKR(launch_tables(T, s));
        }
        CK(hipEventRecord(ev.b, s));
        CK(hipEventSynchronize(ev.b));
        float ms = 0;
        CK(hipEventElapsedTime(&ms, ev.a, ev.b));
        stats.t_filter += ms * 1e-3;
        stats.filter_launches += T.M;
        ++stats.block_steps;
        // per-solve block step; finished solves leave the batch
        const double t1 = now();
        for (Solve *S : act) {
            S->st.t_mv += ms * 1e-3;
            const int i = (int)(std::find_if(solves.begin(), solves.end(),
                                             [&](const std::unique_ptr<Solve> &p) { return p.get() == S; }) -
                                solves.begin());
            int rc = solve_after_filter(*S);
            if (rc != FLP_OK) {
                codes[i] = rc;
                tables_valid = false;
                continue;
            }
            if (S->done) {
                tables_valid = false;
                const double tf = now();
                codes[i] = solve_finish(*S, &results[i]);
                stats.t_finish += now() - tf;
                if (results[i]) results[i]->stats.t_total = now() - t0;  // completion time inside the batch
                stats.filter_bytes += S->st.filter_bytes;
                bufs[i].reset();  // release this solve's device memory
            }
        }
        stats.t_orth_check += now() - t1;
    }
    CK(hipStreamSynchronize(s));
    stats.t_total = now() - t0;
    if (bs) *bs = stats;
    for (int i = 0; i < count; ++i)
        if (codes[i] != FLP_OK && codes[i] != FLP_E_NOCONV) return codes[i];
    return FLP_OK;
}

}  // namespace flp
