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
// Gram-Schmidt and block QR of all active solves follow as one segmented
// launch sequence on the same stream (flp_seg_orth.hip), then each solve's
// convergence check on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <mutex>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "flp_host.h"

namespace flp {

namespace {

int build_tables(const std::vector<Solve *> &act, Tables &T, hipStream_t s) {
    T.M = 0;
    for (Solve *S : act) T.M = std::max(T.M, (int)S->plan.size());
    T.cap = (int)act.size();
    T.host.assign((size_t)T.M * T.cap, SegEntry{});
    T.nseg.assign(T.M, 0);
    T.tiles.assign(T.M, 0);
    const int rpt = seg_rows_per_tile(T.r, T.fp32, T.sh);
    for (int t = 0; t < T.M; ++t) {
        int ns = 0, tiles = 0;
        for (Solve *S : act) {
            const int m = (int)S->plan.size();
            const int j = t - (T.M - m);
            if (j < 0) continue;
            const ClenshawStep &st = S->plan[j];
            SegEntry e{};
            const flp_csr *fa = S->sell ? &S->SA : S->A;  // the filter's copy of A
            e.rowptr = fa->rowptr;
            e.colind = fa->colind;
            e.val = T.fp32 ? (const void *)(S->sell ? S->sval32 : S->val32) : (const void *)fa->val;
            e.sell = S->sell ? 1 : 0;
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
    CK(ensure_grow(T.dev, sizeof(SegEntry) * std::max<size_t>(T.host.size(), 1)));
    CK(h2d(T.dev.p, T.host.data(), sizeof(SegEntry) * T.host.size(), s));
    return FLP_OK;
}

int launch_tables(const Tables &T, hipStream_t s) {
    const SegEntry *base = (const SegEntry *)T.dev.p;
    for (int t = 0; t < T.M; ++t)
        CK(launch_cheb_seg(T.fp32, T.r, base + (size_t)t * T.cap, T.nseg[t], T.tiles[t], s, T.sh));
    return FLP_OK;
}

}  // namespace

// ------------------------------------------------------------------ engine

int Engine::init(int r_, int prec_, bool graph_) {
    r = r_;
    prec = prec_;
    use_graph = graph_;
    T.r = r;
    T.fp32 = prec == FLP_PREC_FP32_FILTER;
    CK(hipGetDevice(&device));
    CK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    for (auto &f : fs) CK(hipStreamCreateWithFlags(&f, hipStreamNonBlocking));
    CK(hipEventCreate(&ev_a));
    CK(hipEventCreate(&ev_b));
    for (int w = 0; w < kFinishers; ++w) fin[w] = std::thread([this, w]() { finisher_main(w); });
    return FLP_OK;
}

Engine::~Engine() {
    {
        std::lock_guard<std::mutex> lk(fmu);
        fstop = true;
    }
    fcv.notify_all();
    for (auto &t : fin)
        if (t.joinable()) t.join();  // the queue is drained first
    graph_reset();
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    for (auto &f : fs)
        if (f) (void)hipStreamDestroy(f);
    if (s) (void)hipStreamSynchronize(s);
    if (ostage) (void)hipHostFree(ostage);
    if (oout_pin) (void)hipHostFree(oout_pin);
    if (s) (void)hipStreamDestroy(s);
}

void Engine::complete(Job *j) {
    if (on_done) on_done(j);
}

void Engine::finisher_main(int w) {
    (void)hipSetDevice(device);
    for (;;) {
        Job *j = nullptr;
        {
            std::unique_lock<std::mutex> lk(fmu);
            for (;;) {
                fcv.wait(lk, [&] { return fstop || !fq.empty(); });
                if (fq.empty()) return;
                Job *cand = fq.front();
                // the finish phase's memory is granted before the job starts
                // (in queue order); a refusal waits for another job to finish
                if (!reserve_finish || reserve_finish(cand, finish_bytes(*cand->S), fbusy == 0)) {
                    j = cand;
                    fq.pop_front();
                    ++fbusy;
                    break;
                }
                // refused only while another job is being finished: its
                // completion wakes this wait
                const uint64_t seen = fdone_count;
                fdone.wait(lk, [&] { return fdone_count != seen; });
            }
        }
        const double t0 = now();
        j->S->s = fs[w % kFinisherStreams];
        if (j->cancel.load()) {
            j->code = FLP_E_CANCELLED;
            j->msg = "request cancelled";
        } else {
            j->code = solve_finish(*j->S, &j->res);
            if (j->code != FLP_OK && j->code != FLP_E_NOCONV) j->msg = last_error_cstr();
        }
        j->t_done = now();
        j->B.reset();  // release this solve's device memory
        {
            std::lock_guard<std::mutex> lk(fmu);
            t_finish += now() - t0;
        }
        complete(j);
        {
            std::lock_guard<std::mutex> lk(fmu);
            --fbusy;
            ++fdone_count;
        }
        fdone.notify_all();
        fcv.notify_all();
    }
}

void Engine::wait_finisher() {
    std::unique_lock<std::mutex> lk(fmu);
    fdone.wait(lk, [&] { return fq.empty() && fbusy == 0; });
}

flp_batch_stats Engine::snapshot() {
    std::lock_guard<std::mutex> lk(fmu);
    flp_batch_stats st = stats;
    st.t_finish = t_finish;
    return st;
}

void Engine::graph_reset() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
}

void Engine::add(Job *j) {
    // the solve's set-up and its block steps run on s
    j->S->s = s;
    // spread the solves' convergence checks over the block steps (solves
    // admitted together would otherwise all hand their checks to the host
    // pool on the same step and wait for them together)
    j->S->check_offset = (int)(n_added++ % (uint64_t)j->S->check_every);
    active.push_back(j);
    tables_valid = false;
}

int Engine::sync_steps() {
    CK(hipStreamSynchronize(s));
    return FLP_OK;
}

namespace {

// Grows a pinned host staging buffer (contents are not kept).
int ensure_pinned(void **p, size_t *have, size_t bytes) {
    if (*have >= bytes && *p) return FLP_OK;
    if (*p) CK(hipHostFree(*p));
    *p = nullptr;
    *have = 0;
    const size_t want = std::max<size_t>({bytes, 4096, *have + *have / 2});
    CK(hipHostMalloc(p, want, hipHostMallocDefault));
    *have = want;
    return FLP_OK;
}

// Row chunk for the partial sums of a K-column projection: 512 rows (one
// basis column per thread walks them on FMA; four waves take 32 rows per
// MFMA step), doubled while the partial sums of one solve exceed 4M
// doubles.
int orth_chunk_rows(int n, int K, int c) {
    int rows = 512;
    while ((size_t)((n + rows - 1) / rows) * K * c > ((size_t)4 << 20)) rows *= 2;
    return rows;
}

}  // namespace

// Full reorthogonalisation and block QR of every active solve (Section
// 3.2.2, eq. lanczos) as one segmented launch sequence, one copy of the
// tables in and one copy of D_j, S_j and the status flags out.
int Engine::block_step(double filter_secs) {
    const double t0 = now();
    const int c = r, ns = (int)active.size();
    const size_t cc = (size_t)c * c, slot = 2 * cc + 2;
    otab_host.assign(ns, OrthSeg{});
    opre_host.assign(kOrthKinds * (size_t)ns, 0);
    int blocks[kOrthKinds] = {};
    std::vector<size_t> poff(ns);
    size_t ptotal = 0;
    CK(ensure_grow(oout, sizeof(double) * slot * ns));
    // room in each basis for this step's projection and the next block
    for (Job *j : active) CKR(ensure_basis(*j->S, (int64_t)(j->S->steps + 2) * c));
    for (int i = 0; i < ns; ++i) {
        Solve &S = *active[i]->S;
        OrthSeg &e = otab_host[i];
        const int n = S.n, k = (S.steps + 1) * c;
        e.n = n;
        e.k = k;
        e.qcap = (int)(S.qpanels << kPanelLog2);
        e.chunk_rows = orth_chunk_rows(n, k, c);
        e.nchunks = (n + e.chunk_rows - 1) / e.chunk_rows;
        e.gchunk_rows = orth_chunk_rows(n, c, c);
        e.gnchunks = (n + e.gchunk_rows - 1) / e.gchunk_rows;
        int add[kOrthKinds] = {};
        add[k > 128 ? kOrthFma : kOrthMfma] = (k > 128 ? (k + 255) / 256 : 1) * e.nchunks;
        add[kOrthGram] = e.gnchunks;
        add[kOrthRed] = (int)((k * (size_t)c + 63) / 64);
        add[kOrthGred] = (int)((cc + 63) / 64);
        add[kOrthRows] = (n + 255) / 256;
        for (int t = 0; t < kOrthKinds; ++t) {
            opre_host[(size_t)t * ns + i] = blocks[t];
            blocks[t] += add[t];
        }
        e.Q = S.Q;
        e.W = S.W;
        e.H = S.hdev;
        e.G = S.gdev;
        e.Ri = S.rdev;
        e.R1 = S.gdev + 2 * cc;
        e.R2 = S.gdev + 3 * cc;
        e.out = (double *)oout.p + (size_t)i * slot;
        e.Vin = S.Vin;
        e.V32 = S.V32;
        poff[i] = ptotal;
        ptotal += std::max((size_t)e.nchunks * k * c, (size_t)e.gnchunks * cc);
        S.t_step0 = t0;
        S.st.filter_bytes += filter_step_bytes(n, S.A->nnz, c, S.o.prec) * S.filt->m;
        S.st.mv += (int64_t)c * S.filt->m;
        S.st.orth_bytes += 4.0 * 8.0 * (double)n * k;
        stats.orth_bytes += 4.0 * 8.0 * (double)n * k;
    }
    CK(ensure_grow(opart, sizeof(double) * std::max<size_t>(ptotal, 1)));
    for (int i = 0; i < ns; ++i) otab_host[i].part = (double *)opart.p + poff[i];
    const size_t tb = sizeof(OrthSeg) * ns, pb = sizeof(int) * opre_host.size();
    CKR(ensure_pinned((void **)&ostage, &ostage_bytes, tb + pb));
    std::memcpy(ostage, otab_host.data(), tb);
    std::memcpy(ostage + tb, opre_host.data(), pb);
    CK(ensure_grow(otab, tb + pb));
    CK(hipMemcpyAsync(otab.p, ostage, tb + pb, hipMemcpyHostToDevice, s));
    OrthPlan plan{(const OrthSeg *)otab.p, (const int *)((const char *)otab.p + tb), ns, {}};
    for (int t = 0; t < kOrthKinds; ++t) plan.blocks[t] = blocks[t];
    CK(launch_seg_orth(plan, c, s));
    CKR(ensure_pinned((void **)&oout_pin, &oout_pin_bytes, sizeof(double) * slot * ns));
    CK(hipMemcpyAsync(oout_pin, oout.p, sizeof(double) * slot * ns, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    const double dt = now() - t0;
    stats.t_orth += dt;
    for (int i = 0; i < ns; ++i) {
        Job *j = active[i];
        Solve &S = *j->S;
        if (j->code != FLP_OK) continue;
        S.st.t_mv += filter_secs;
        const double *o = oout_pin + (size_t)i * slot;
        const double status = o[2 * cc];
        if (status == 2.0) {
            j->code = fail(FLP_E_DEVICE, "block QR: second Cholesky pass broke down");
            j->msg = last_error_cstr();
            continue;
        }
        S.D_all.insert(S.D_all.end(), o, o + cc);
        if (status == 1.0) {
            // numerically dependent columns: the synchronous repair path on
            // the projected block, then the copies the kernels skipped
            const int k = (S.steps + 1) * c;
            int rc = block_qr_impl(S.W, S.n, c, &S.Q, k, S.Sj, S.o.seed, 1000 + S.steps, s, nullptr);
            if (rc == FLP_OK && k + c <= (int)(S.qpanels << kPanelLog2) &&
                launch_copy_block(S.n, c, 1.0, S.W, c, S.Q, k, nullptr, 0, s) != hipSuccess)
                rc = fail(FLP_E_DEVICE, "basis copy failed");
            if (rc == FLP_OK &&
                launch_copy_block(S.n, c, 1.0, S.W, c, plain_mat(S.Vin, c), 0, S.V32, c, s) != hipSuccess)
                rc = fail(FLP_E_DEVICE, "input copy failed");
            if (rc != FLP_OK) {
                j->code = rc;
                j->msg = last_error_cstr();
                continue;
            }
        } else {
            S.Sj.assign(o + cc, o + 2 * cc);
        }
        S.S_all.insert(S.S_all.end(), S.Sj.begin(), S.Sj.end());
        ++S.steps;
        S.st.t_orth += dt;
    }
    return FLP_OK;
}

int Engine::step() {
    if (active.empty()) return FLP_OK;
    // cancelled requests leave at the step boundary
    {
        std::vector<Job *> keep;
        for (Job *j : active) {
            if (!j->cancel.load()) {
                keep.push_back(j);
                continue;
            }
            j->code = FLP_E_CANCELLED;
            j->msg = "request cancelled";
            j->t_done = now();
            j->B.reset();
            complete(j);
            tables_valid = false;
        }
        active.swap(keep);
        if (active.empty()) return FLP_OK;
    }
    std::vector<Solve *> act;
    for (Job *j : active) act.push_back(j->S.get());
    if (!tables_valid) {
        graph_reset();
        // launch shape of the segmented steps, tuned on the largest active
        // matrix (its recurrence buffers are scratch between block steps)
        Solve *big = act[0];
        for (Solve *S : act)
            if (S->A->nnz > big->A->nnz) big = S;
        FilterTune tn;
        void *U[3] = {big->U[0], big->U[1], big->U[2]};
        CKR(tune_filter(big->sell ? &big->SA : big->A, big->sell ? big->sval32 : big->val32, r, T.fp32, false, U,
                        T.fp32 ? (const void *)big->V32 : (const void *)big->Vin, r, s, &tn, big->sell));
        T.sh = tn.sh;
        for (Solve *S : act) {
            S->tile_chunk = tn.sh.win == 2 ? 0 : tn.sh.chunk;
            S->tile_win = tn.sh.win != 0 ? 1 : 0;
        }
        CKR(build_tables(act, T, s));
        if (use_graph) {
            std::shared_lock<std::shared_mutex> cl(capture_mutex());  // no device-wide sync meanwhile
            CK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            const int rc = launch_tables(T, s);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &g);
            if (rc != FLP_OK) return rc;
            CK(e);
            graph = g;
            CK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
            ++stats.graph_captures;
        }
        tables_valid = true;
    }
    // filter phase: one segmented launch per Clenshaw step
    CK(hipEventRecord(ev_a, s));
    if (use_graph) {
        CK(hipGraphLaunch(gexec, s));
        ++stats.graph_replays;
    } else {
        CKR(launch_tables(T, s));
    }
    CK(hipEventRecord(ev_b, s));
    CK(hipEventSynchronize(ev_b));
    float ms = 0;
    CK(hipEventElapsedTime(&ms, ev_a, ev_b));
    stats.t_filter += ms * 1e-3;
    stats.filter_launches += T.M;
    ++stats.block_steps;
    for (Solve *S : act) stats.filter_bytes += filter_step_bytes(S->n, S->A->nnz, S->r, S->o.prec) * S->filt->m;
    // Gram-Schmidt and block QR of every active solve, then their checks
    const double t1 = now();
    auto run_phase = [&](int (*phase)(Solve &)) {
        for (Job *j : active) {
            if (j->code != FLP_OK) continue;
            j->code = phase(*j->S);
            if (j->code != FLP_OK) j->msg = last_error_cstr();
        }
    };
    CKR(block_step(ms * 1e-3));
    // convergence checks: applied when their pool task has finished, started
    // at the cadence (the solves keep stepping meanwhile)
    run_phase([](Solve &S) { return step_check(S, true, false); });
    std::vector<Job *> keep, done;
    for (Job *j : active) {
        if (j->code == FLP_OK && !j->S->done)
            keep.push_back(j);
        else
            done.push_back(j);
    }
    if (!done.empty()) {
        // the finishers read the basis (repair-path copies may be in flight)
        CKR(sync_steps());
        for (Job *j : done) {
            if (j->code == FLP_OK) {
                {
                    std::lock_guard<std::mutex> lk(fmu);
                    fq.push_back(j);
                }
                fcv.notify_one();
            } else {
                j->S->st.t_total = now() - j->S->t_start;
                j->t_done = now();
                j->B.reset();
                complete(j);
            }
        }
        tables_valid = false;
    }
    active.swap(keep);
    stats.t_orth_check += now() - t1;
    return FLP_OK;
}

// ------------------------------------------------------------------ batch

int solve_batch_impl(int count, const flp_csr *const *A, const double *alpha, const double *beta,
                     const flp_opts *opts, int use_graph, flp_result **results, int *codes, flp_batch_stats *bs) {
    const double t0 = now();
    hipStream_t user = opts ? (hipStream_t)opts[0].stream : nullptr;
    flp_opts o0;
    flp_opts_default(&o0);
    for (int i = 0; i < count; ++i) {
        results[i] = nullptr;
        codes[i] = FLP_OK;
    }
    const int r = opts ? opts[0].block : o0.block;
    const int prec = opts ? opts[0].prec : o0.prec;
    for (int i = 0; i < count; ++i) {
        const flp_opts &o = opts ? opts[i] : o0;
        if (o.block != r || o.prec != prec)
            return fail(FLP_E_ARG, "all solves of a batch need the same block size and precision");
        if (o.unfiltered) return fail(FLP_E_ARG, "unfiltered Lanczos runs through flp_solve only");
    }
    CK(hipStreamSynchronize(user));
    Engine E;
    CKR(E.init(r, prec, use_graph != 0));
    E.stats.solves = count;
    std::vector<std::unique_ptr<Job>> jobs(count);
    for (int i = 0; i < count; ++i) {
        auto j = std::make_unique<Job>();
        j->id = (uint64_t)i;
        j->t_submit = t0;
        j->S = std::make_unique<Solve>();
        Solve &S = *j->S;
        S.A = A[i];
        S.alpha = alpha[i];
        S.beta = beta[i];
        S.o = opts ? opts[i] : o0;
        S.o.stream = nullptr;
        jobs[i] = std::move(j);
    }
    // Set-up (bounds estimate, filter, buffers, start block) is a chain of
    // small launches and host round trips per solve: the solves' set-ups run
    // on a few threads at once, each with a stream of its own (the threads'
    // workspaces are released when they join), and join the engine in order.
    {
        const int nt = std::max(1, std::min(count, kSetupThreads));
        const int dev = E.device;
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t)
            th.emplace_back([&jobs, count, nt, t, dev]() {
                hipStream_t st = nullptr;
                const bool ok = hipSetDevice(dev) == hipSuccess &&
                                hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
                for (int i = t; i < count; i += nt) {
                    Job *jp = jobs[i].get();
                    Solve &S = *jp->S;
                    if (!ok) {
                        jp->code = fail(FLP_E_DEVICE, "could not create a set-up stream");
                    } else {
                        S.s = st;
                        jp->code = check_csr(S.A);
                        if (jp->code == FLP_OK) {
                            jp->B = std::make_unique<SolveBufs>();
                            jp->B->own_ritz = true;
                            S.B = jp->B.get();
                            jp->code = solve_setup(S);
                        }
                        if (hipStreamSynchronize(st) != hipSuccess && jp->code == FLP_OK)
                            jp->code = fail(FLP_E_DEVICE, "set-up stream failed");
                        S.s = nullptr;
                    }
                    if (jp->code != FLP_OK) {
                        jp->msg = last_error_cstr();
                        jp->B.reset();
                    }
                }
                if (st) (void)hipStreamDestroy(st);
                ws().release_all();  // this thread's scratch (bounds estimate) goes back now
            });
        for (auto &x : th) x.join();
    }
    for (auto &j : jobs)
        if (j->code == FLP_OK) E.add(j.get());
    E.stats.t_setup = now() - t0;
    int rc = FLP_OK;
    while (!E.active.empty() && rc == FLP_OK) rc = E.step();
    E.wait_finisher();
    CKR(rc);
    CK(hipStreamSynchronize(E.s));
    for (int i = 0; i < count; ++i) {
        results[i] = jobs[i]->res;
        codes[i] = jobs[i]->code;
        if (results[i]) results[i]->stats.t_total = jobs[i]->t_done - t0;  // completion time inside the batch
    }
    const double t_setup = E.stats.t_setup;
    E.stats = E.snapshot();
    E.stats.t_setup = t_setup;
    E.stats.t_total = now() - t0;
    if (bs) *bs = E.stats;
    for (int i = 0; i < count; ++i)
        if (codes[i] != FLP_OK && codes[i] != FLP_E_NOCONV) return fail(codes[i], jobs[i]->msg);
    return FLP_OK;
}

}  // namespace flp
