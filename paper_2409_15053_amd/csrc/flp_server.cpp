// Serving loop: continuous batching of filtered Lanczos solves.
//
// Requests are queued by flp_server_submit and admitted by a worker thread
// while engine slots and device memory allow (each request's footprint --
// Lanczos basis, recurrence vectors, FP32 copies -- is reserved against a
// budget at admission, and its finish phase's Ritz blocks when it has
// converged).  Admitted requests join the engine's active set at the next
// block step boundary and leave it when they converge, so requests that
// arrive while others are on the GPU start without waiting for the batch to
// drain.  Only the worker thread steps the solves; the engine's finisher
// threads run the finish phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "flp_host.h"

using namespace flp;

struct flp_server {
    flp_server_opts o{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job *> pending;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_id = 1;
    bool stop = false;
    size_t mem_in_use = 0, mem_budget = 0, mem_peak = 0;
    int32_t peak_active = 0, admission_waits = 0, finish_waits = 0;
    bool head_waiting = false;  // the queue's head is already counted as waiting
    int device = 0;
    Engine eng;
    flp_batch_stats snapshot{};  // engine statistics, copied under the lock
    int64_t submitted = 0;
    std::thread worker;
    int fatal = FLP_OK;
    std::string fatal_msg;
};

namespace flp {
namespace {

// Device bytes a request holds while active (its SolveBufs).
size_t footprint(const flp_csr &A, const flp_opts &o) {
    const size_t n = (size_t)A.n, r = (size_t)o.block;
    const bool fp32 = o.prec == FLP_PREC_FP32_FILTER;
    const int64_t maxb = std::min<int64_t>(o.max_basis > 0 ? o.max_basis : kDefaultMaxBasis, A.n);
    const size_t steps = std::max<size_t>(1, (size_t)maxb / r);
    const size_t cols = ((steps * r + (1u << kPanelLog2) - 1) >> kPanelLog2) << kPanelLog2;
    size_t b = n * cols * 8;                // basis
    b += n * r * 8 * 2;                     // W, Vin
    b += n * r * (fp32 ? 4 : 8) * 3;        // recurrence vectors
    if (fp32) b += n * r * 4 + (A.val32 ? 0 : (size_t)A.nnz * 4);
    // sliced ELL copy of A (AUTO keeps it within 1.25x the nonzeros)
    if (o.format != FLP_FORMAT_CSR) b += (size_t)(1.25 * (double)A.nnz + 64.0) * (fp32 ? 8 : 12) + n / 16 + 8;
    b += (2 * cols * r + 4 * r * r + 64) * 8;
    return b;
}

void worker_main(flp_server *sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        std::vector<Job *> admit;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // wake for work: active requests to step, or a queued request
            // that fits (or would run alone); a head waiting for memory is
            // woken by the completion that frees it
            sv->cv_work.wait(lk, [&] {
                if (sv->stop || !sv->eng.active.empty()) return true;
                if (sv->pending.empty()) return false;
                return sv->mem_in_use == 0 || sv->mem_in_use + sv->pending.front()->footprint <= sv->mem_budget;
            });
            if (sv->stop && sv->pending.empty() && sv->eng.active.empty()) break;
            // admission: free engine slots and device memory (memory comes
            // back when the finisher releases a solve's buffers)
            while (!sv->pending.empty() &&
                   (int)(sv->eng.active.size() + admit.size()) < sv->o.max_active) {
                Job *j = sv->pending.front();
                if (sv->mem_in_use + j->footprint > sv->mem_budget &&
                    !(sv->eng.active.empty() && admit.empty() && sv->mem_in_use == 0)) {
                    // wait for memory (a lone request is always admitted)
                    if (!sv->head_waiting) ++sv->admission_waits;
                    sv->head_waiting = true;
                    break;
                }
                sv->head_waiting = false;
                sv->pending.pop_front();
                sv->mem_in_use += j->footprint;
                sv->mem_peak = std::max(sv->mem_peak, sv->mem_in_use);
                admit.push_back(j);
            }
            sv->peak_active = std::max<int32_t>(sv->peak_active, (int32_t)(sv->eng.active.size() + admit.size()));
        }
        for (Job *j : admit) {
            Solve &S = *j->S;
            S.s = sv->eng.s;
            if (j->ready) {  // the caller's writes of A come first
                const hipError_t e = hipStreamWaitEvent(S.s, j->ready, 0);
                (void)hipEventDestroy(j->ready);
                j->ready = nullptr;
                if (e != hipSuccess) {
                    j->code = fail(FLP_E_DEVICE, "waiting for the request's event failed");
                    j->msg = last_error_cstr();
                    j->t_done = now();
                    sv->eng.on_done(j);
                    continue;
                }
            }
            j->B = std::make_unique<SolveBufs>();
            j->B->own_ritz = true;  // the finish phase's blocks are this request's (freed with it)
            S.B = j->B.get();
            j->code = solve_setup(S);
            if (j->code == FLP_OK) {
                sv->eng.add(j);
            } else {
                j->msg = last_error_cstr();
                j->B.reset();
                j->t_done = now();
                sv->eng.on_done(j);
            }
        }
        if (!sv->eng.active.empty()) {
            const int rc = sv->eng.step();
            if (rc != FLP_OK) {
                // a device failure ends every active request
                std::string msg = last_error_cstr();
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    sv->fatal = rc;
                    sv->fatal_msg = msg;
                }
                (void)sv->eng.sync_steps();  // nothing may still use the buffers freed below
                std::vector<Job *> act;
                act.swap(sv->eng.active);
                for (Job *j : act) {
                    j->code = rc;
                    j->msg = msg;
                    j->t_done = now();
                    j->B.reset();
                    sv->eng.on_done(j);
                }
            }
        }
        const flp_batch_stats st = sv->eng.snapshot();
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->snapshot = st;
            sv->snapshot.solves = (int32_t)sv->submitted;
            sv->snapshot.peak_active = sv->peak_active;
            sv->snapshot.admission_waits = sv->admission_waits;
            sv->snapshot.finish_waits = sv->finish_waits;
            sv->snapshot.mem_budget = (double)sv->mem_budget;
            sv->snapshot.peak_mem_reserved = (double)sv->mem_peak;
        }
    }
}

// The finish phase's memory of a converged request (finisher thread): granted
// when it fits the budget beside everything reserved, or when no other
// request is being finished.
bool reserve_finish(flp_server *sv, Job *j, size_t bytes, bool lone) {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!lone && sv->mem_in_use + bytes > sv->mem_budget) {
        ++sv->finish_waits;
        return false;
    }
    sv->mem_in_use += bytes;
    j->footprint += bytes;
    sv->mem_peak = std::max(sv->mem_peak, sv->mem_in_use);
    return true;
}

// Completion of a request (stepping or finisher thread): memory returns to
// the admission budget, waiters are woken.
void on_job_done(flp_server *sv, Job *j) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->mem_in_use -= std::min(sv->mem_in_use, j->footprint);
    if (j->res) j->res->stats.t_total = j->t_done - j->t_submit;  // request latency
    j->footprint = 0;
    j->finished = true;
    sv->cv_done.notify_all();
    sv->cv_work.notify_one();
}

int take_result(flp_server *sv, std::map<uint64_t, std::unique_ptr<Job>>::iterator it, flp_result **out) {
    Job *j = it->second.get();
    const int code = j->code;
    if (code != FLP_OK && code != FLP_E_NOCONV) set_error(j->msg);
    *out = j->res;
    j->res = nullptr;
    sv->jobs.erase(it);
    return code;
}

int cancel_request(flp_server *sv, uint64_t ticket) {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) return fail(FLP_E_ARG, "unknown ticket");
    Job *j = it->second.get();
    if (j->finished) return FLP_OK;  // the result is ready: nothing to cancel
    auto q = std::find(sv->pending.begin(), sv->pending.end(), j);
    if (q != sv->pending.end()) {
        // still queued: it never touched the device
        sv->pending.erase(q);
        j->code = FLP_E_CANCELLED;
        j->msg = "request cancelled";
        j->t_done = now();
        j->finished = true;
        sv->cv_done.notify_all();
        sv->cv_work.notify_one();  // the next queued request may fit now
        return FLP_OK;
    }
    j->cancel.store(true);  // the engine or a finisher drops it
    return FLP_OK;
}

}  // namespace
}  // namespace flp

extern "C" {

void flp_server_opts_default(flp_server_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->block = 8;
    o->prec = FLP_PREC_FP32_FILTER;
    o->max_active = 64;
    o->max_basis = 1024;
    o->mem_budget = 0.0;
    o->use_graph = 1;
}

int flp_server_create(const flp_server_opts *opts, flp_server **out) {
    if (!out) return fail(FLP_E_ARG, "out is NULL");
    *out = nullptr;
    flp_server_opts o;
    flp_server_opts_default(&o);
    if (opts) o = *opts;
    if (o.block < 1 || o.block > 16 || o.max_active < 1) return fail(FLP_E_ARG, "bad server options");
    if (o.prec != FLP_PREC_FP64 && o.prec != FLP_PREC_FP32_FILTER) return fail(FLP_E_ARG, "bad precision");
    try {
        auto sv = std::make_unique<flp_server>();
        sv->o = o;
        CK(hipGetDevice(&sv->device));
        if (o.mem_budget > 0) {
            sv->mem_budget = (size_t)o.mem_budget;
        } else {
            size_t fr = 0, tot = 0;
            CK(hipMemGetInfo(&fr, &tot));
            sv->mem_budget = (size_t)(0.7 * (double)fr);
        }
        CKR(sv->eng.init(o.block, o.prec, o.use_graph != 0));
        flp_server *p = sv.get();
        p->eng.on_done = [p](Job *j) { on_job_done(p, j); };
        p->eng.reserve_finish = [p](Job *j, size_t bytes, bool lone) { return reserve_finish(p, j, bytes, lone); };
        p->worker = std::thread(worker_main, p);
        *out = sv.release();
        return FLP_OK;
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(FLP_E_DEVICE, "could not start the server");
    }
}

int flp_server_submit(flp_server *sv, const flp_csr *A, double alpha, double beta, const flp_opts *opts,
                      uint64_t *ticket) {
    if (!sv || !ticket) return fail(FLP_E_ARG, "NULL argument");
    CKR(check_csr(A));
    try {
        auto j = std::make_unique<Job>();
        j->A = *A;
        j->S = std::make_unique<Solve>();
        Solve &S = *j->S;
        S.A = &j->A;
        S.alpha = alpha;
        S.beta = beta;
        flp_opts_default(&S.o);
        if (opts) S.o = *opts;
        if (S.o.unfiltered) return fail(FLP_E_ARG, "unfiltered Lanczos runs through flp_solve only");
        S.o.block = sv->o.block;
        S.o.prec = sv->o.prec;
        if (S.o.max_basis <= 0) S.o.max_basis = sv->o.max_basis;
        S.o.stream = nullptr;
        if (!(std::isfinite(alpha) && std::isfinite(beta)) || !(alpha < beta))
            return fail(FLP_E_ARG, "need finite alpha < beta");
        if (S.o.block > A->n) return fail(FLP_E_ARG, "block size exceeds n");
        j->footprint = footprint(*A, S.o);
        {
            // the engine reads A after what the caller queued on its stream
            hipStream_t cs = opts ? (hipStream_t)opts->stream : nullptr;
            int cur = 0;
            CK(hipGetDevice(&cur));
            if (cur != sv->device) CK(hipSetDevice(sv->device));
            hipError_t e = hipEventCreateWithFlags(&j->ready, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(j->ready, cs);
            if (cur != sv->device) (void)hipSetDevice(cur);
            if (e != hipSuccess) return fail(FLP_E_DEVICE, std::string("recording the request's event: ") + hipGetErrorString(e));
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->fatal != FLP_OK) return fail(sv->fatal, "server stopped after a device error: " + sv->fatal_msg);
        j->id = sv->next_id++;
        j->t_submit = now();
        *ticket = j->id;
        sv->pending.push_back(j.get());
        sv->jobs[j->id] = std::move(j);
        ++sv->submitted;
        sv->cv_work.notify_one();
        return FLP_OK;
    } catch (const std::bad_alloc &) {
        return fail(FLP_E_NOMEM, "host allocation failed");
    }
}

int flp_server_poll(flp_server *sv, uint64_t ticket, flp_result **out) {
    if (!sv || !out) return fail(FLP_E_ARG, "NULL argument");
    *out = nullptr;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) return fail(FLP_E_ARG, "unknown ticket");
    if (!it->second->finished) return FLP_E_PENDING;
    return take_result(sv, it, out);
}

int flp_server_wait(flp_server *sv, uint64_t ticket, flp_result **out) {
    if (!sv || !out) return fail(FLP_E_ARG, "NULL argument");
    *out = nullptr;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) return fail(FLP_E_ARG, "unknown ticket");
    Job *j = it->second.get();
    sv->cv_done.wait(lk, [&] { return j->finished; });
    return take_result(sv, it, out);
}

int flp_server_cancel(flp_server *sv, uint64_t ticket) {
    if (!sv) return fail(FLP_E_ARG, "NULL argument");
    return cancel_request(sv, ticket);
}

int flp_server_footprint(const flp_server *sv, const flp_csr *A, const flp_opts *opts, double *bytes) {
    if (!sv || !bytes) return fail(FLP_E_ARG, "NULL argument");
    CKR(check_csr(A));
    flp_opts o;
    flp_opts_default(&o);
    if (opts) o = *opts;
    o.block = sv->o.block;
    o.prec = sv->o.prec;
    if (o.max_basis <= 0) o.max_basis = sv->o.max_basis;
    *bytes = (double)footprint(*A, o);
    return FLP_OK;
}

int flp_server_stats(flp_server *sv, flp_batch_stats *out) {
    if (!sv || !out) return fail(FLP_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->snapshot;
    return FLP_OK;
}

int flp_server_destroy(flp_server *sv) {
    if (!sv) return FLP_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    sv->eng.wait_finisher();
    for (auto &kv : sv->jobs)
        if (kv.second->res) flp_result_free(kv.second->res);
    const int rc = sv->fatal;
    delete sv;
    return rc;
}

}  // extern "C"
