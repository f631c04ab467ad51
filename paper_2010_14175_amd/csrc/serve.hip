// Serving loop: SPD systems of mixed sizes arrive as requests; each is set up (Sec. 2) and
// solved by PCG (Sec. 5.2) on the device while others are in progress.
//
// Admission: requests wait in arrival order and are admitted while a slot is free and the sum
// of the admitted requests' device footprints (setup temporaries, G and G^T, the SELL copy of
// A, the Krylov vectors) stays within the budget; a finished request frees its slot and its
// memory at once and the waiting requests behind it are admitted (continuous batching, not a
// queue served one at a time).  Heavy requests (many matrix entries) are admitted at most
// max_heavy at a time, in arrival order among themselves; lighter requests behind a heavy one
// that has to wait are admitted past it.  Two heavy solves sharing the device would both finish
// late (the slowest requests set the tail latency), while light ones take little of it.  The
// scheduler enqueues the next chunks of the solving requests lightest first.  Every admitted request owns a HIP stream.  Setup workers (host
// threads) run the setups of newly admitted requests while one scheduler thread advances the
// PCG iterations of all solving requests without blocking: each step enqueues the next chunk of
// a request whose previous chunk has completed, so the kernels of many requests are in flight
// on the device together.  Each request runs exactly the single-system solver of pcg_solve with
// its own data, so its result does not depend on what else is being served.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "handle.hpp"

namespace afsai {

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t ticket = 0;
    afsai_csr A{};
    afsai_params params{};
    const double *b = nullptr;
    double *x = nullptr;
    size_t footprint = 0;
    bool heavy = false;
    double t_submit = 0, t_admit = 0, t_setup = 0, t_done = 0;
    afsai_precond P = nullptr;
    hipStream_t stream = nullptr;
    PcgTask *task = nullptr;
    int status = AFSAI_OK;
    afsai_pcg_info info{};
};

// Device bytes a request holds while admitted (the caller's A, b and x not included): per-row
// setup results and G (CSR, SELL, SELL of G^T with padding), the SELL copy of A and the solver
// vectors.
size_t footprint(const afsai_csr &A, const afsai_params &p) {
    const double n = A.n, nnz = A.nnz;
    const double mmax = 1.0 + (double)p.kmax * (p.kmax > 0 ? p.s : 0);
    const double g = n * mmax * 12.0;
    const double bytes = g * (1.0 + 1.0 + 1.3 + 1.6) + 14.4 * nnz + 160.0 * n + (4 << 20);
    return (size_t)bytes;
}

}  // namespace

}  // namespace afsai

using namespace afsai;

struct afsai_server_s {
    afsai_server_config cfg{};
    int device = 0;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work;   // setup workers
    std::condition_variable cv_sched;  // scheduler
    std::condition_variable cv_done;   // pollers and destroy
    std::deque<Request *> waiting, to_setup, ready;
    std::vector<afsai_request_result> completed;
    std::vector<hipStream_t> streams;  // idle streams
    size_t used = 0;
    int slots = 0;
    int64_t next_ticket = 1;
    int64_t outstanding = 0;  // submitted, not yet completed
    bool stop = false;
    std::vector<std::thread> workers;
    std::thread scheduler;

    double now() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }

    int heavy_in = 0;  // heavy requests admitted

    int heavy_cap() const { return cfg.max_heavy == 0 ? 1 : cfg.max_heavy; }

    // admits waiting requests in arrival order while a slot and the memory are free; a heavy
    // request over the heavy cap waits, and the lighter ones behind it may pass (mu held)
    void admit_locked() {
        for (auto it = waiting.begin(); it != waiting.end() && slots < cfg.max_slots;) {
            Request *r = *it;
            if (used + r->footprint > cfg.hbm_budget) break;  // memory: keep arrival order
            if (r->heavy && heavy_cap() > 0 && heavy_in >= heavy_cap()) {
                ++it;
                continue;
            }
            it = waiting.erase(it);
            used += r->footprint;
            ++slots;
            heavy_in += r->heavy ? 1 : 0;
            r->t_admit = now();
            to_setup.push_back(r);
            cv_work.notify_one();
        }
    }

    // records a finished request and frees what it held (mu not held)
    void complete(Request *r) {
        if (r->stream) (void)hipStreamSynchronize(r->stream);
        if (r->task) pcg_task_free(r->task);
        r->task = nullptr;
        if (r->P) afsai_destroy(r->P);
        r->P = nullptr;
        afsai_request_result res{};
        res.ticket = r->ticket;
        res.status = r->status;
        res.iters = r->info.iters;
        res.converged = r->info.converged;
        res.true_relres = r->info.true_relres;
        res.footprint = (int64_t)r->footprint;
        res.submit_ms = r->t_submit;
        res.admit_ms = r->t_admit;
        res.setup_done_ms = r->t_setup;
        res.done_ms = now();
        std::lock_guard<std::mutex> lk(mu);
        if (r->stream) streams.push_back(r->stream);
        used -= r->footprint;
        --slots;
        heavy_in -= r->heavy ? 1 : 0;
        --outstanding;
        completed.push_back(res);
        delete r;
        admit_locked();
        cv_done.notify_all();
    }

    void worker_main() {
        (void)hipSetDevice(device);
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !to_setup.empty(); });
                if (to_setup.empty()) return;
                r = to_setup.front();
                to_setup.pop_front();
                if (!streams.empty()) {
                    r->stream = streams.back();
                    streams.pop_back();
                }
            }
            int rc = AFSAI_OK;
            if (!r->stream && hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking) != hipSuccess) {
                r->stream = nullptr;
                rc = AFSAI_ERR_HIP;
            }
            if (rc == AFSAI_OK && hipMemsetAsync(r->x, 0, sizeof(double) * (size_t)r->A.n, r->stream) != hipSuccess)
                rc = AFSAI_ERR_HIP;
            if (rc == AFSAI_OK) rc = afsai_setup(&r->A, &r->params, r->stream, &r->P);
            r->t_setup = now();
            if (rc != AFSAI_OK) {
                r->status = rc;
                complete(r);
                continue;
            }
            std::lock_guard<std::mutex> lk(mu);
            ready.push_back(r);
            cv_sched.notify_one();
        }
    }

    void scheduler_main() {
        (void)hipSetDevice(device);
        std::vector<Request *> solving;
        for (;;) {
            std::vector<Request *> fresh;
            {
                std::unique_lock<std::mutex> lk(mu);
                if (solving.empty())
                    cv_sched.wait(lk, [&] { return !ready.empty() || (stop && outstanding == 0); });
                if (solving.empty() && ready.empty() && stop && outstanding == 0) return;
                while (!ready.empty()) {
                    fresh.push_back(ready.front());
                    ready.pop_front();
                }
            }
            for (Request *r : fresh) {
                const int rc = pcg_task_begin(r->A, r->P, r->b, r->x, cfg.rtol, cfg.maxit, r->stream, &r->task);
                if (rc != AFSAI_OK) {
                    r->status = rc;
                    complete(r);
                } else {
                    solving.push_back(r);
                }
            }
            bool progressed = !fresh.empty();
            // lightest first: their next chunks go to the device ahead of the heavy ones'
            std::stable_sort(solving.begin(), solving.end(),
                             [](const Request *a, const Request *b) { return a->A.nnz < b->A.nnz; });
            for (size_t k = 0; k < solving.size();) {
                Request *r = solving[k];
                bool fin = false;
                int rc = pcg_task_advance(r->task, false, &fin);
                if (rc == AFSAI_OK && !fin) {
                    ++k;
                    continue;
                }
                progressed = true;
                if (rc == AFSAI_OK) rc = pcg_task_finish(r->task, &r->info);
                r->status = rc;
                solving.erase(solving.begin() + (std::ptrdiff_t)k);
                complete(r);
            }
            if (!progressed && !solving.empty()) {
                // nothing completed: wait briefly for new work or the device
                std::unique_lock<std::mutex> lk(mu);
                cv_sched.wait_for(lk, std::chrono::microseconds(20), [&] { return !ready.empty(); });
            }
        }
    }
};

static bool params_ok(const afsai_params &p);

extern "C" {

int afsai_server_create(const afsai_server_config *cfg, afsai_server *out) {
    clear_error();
    if (out) *out = nullptr;
    if (!cfg || !out) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_create: null argument");
    if (cfg->max_slots < 1 || cfg->setup_threads < 1 || cfg->setup_threads > 64 || cfg->hbm_budget == 0 ||
        !(cfg->rtol > 0.0) || cfg->maxit < 0)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_create: bad configuration (slots %d, setup threads %d)",
                   cfg->max_slots, cfg->setup_threads);
    if (!params_ok(cfg->params)) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_create: bad setup parameters");
    afsai_server S = new afsai_server_s();
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        AFSAI_FAIL(AFSAI_ERR_HIP, "afsai_server_create: no device");
    }
    S->t0 = Clock::now();
    for (int k = 0; k < cfg->setup_threads; ++k) S->workers.emplace_back([S] { S->worker_main(); });
    S->scheduler = std::thread([S] { S->scheduler_main(); });
    *out = S;
    return AFSAI_OK;
}

static bool params_ok(const afsai_params &p) {
    return !(p.kmax < 0 || (p.kmax > 0 && p.s < 1) || 1 + (int64_t)p.kmax * (p.kmax > 0 ? p.s : 0) > 64 ||
             !(p.eps >= 0.0) || !(p.tie_rtol >= 0.0 && p.tie_rtol < 1.0) ||
             (p.g_prec != AFSAI_F64 && p.g_prec != AFSAI_F32) || (p.flags & ~(AFSAI_VALIDATE | AFSAI_GRAD_F32)));
}

int afsai_server_submit(afsai_server S, const afsai_csr *A, const afsai_params *p, const double *b, double *x,
                        int64_t *ticket) {
    clear_error();
    if (!S || !A || !b || !x || !ticket) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_submit: null argument");
    if (A->n <= 0 || A->nnz < A->n || !A->row_ptr || !A->col_idx || !A->val)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_submit: bad matrix (n = %d, nnz = %d)", A->n, A->nnz);
    if (p && !params_ok(*p)) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_submit: bad setup parameters");
    Request *r = new Request();
    r->A = *A;
    r->params = p ? *p : S->cfg.params;
    r->b = b;
    r->x = x;
    r->footprint = footprint(*A, r->params);
    r->heavy = (int64_t)A->nnz >= (S->cfg.heavy_nnz > 0 ? S->cfg.heavy_nnz : ((int64_t)1 << 22));
    if (r->footprint > S->cfg.hbm_budget) {
        const size_t fp = r->footprint;
        delete r;
        AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_server_submit: request needs %zu bytes, budget %zu", fp,
                   S->cfg.hbm_budget);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        delete r;
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_submit: server is shutting down");
    }
    r->ticket = S->next_ticket++;
    r->t_submit = S->now();
    ++S->outstanding;
    *ticket = r->ticket;
    S->waiting.push_back(r);
    S->admit_locked();
    return AFSAI_OK;
}

int afsai_server_poll(afsai_server S, afsai_request_result *out, int32_t max_results, int32_t *count,
                      int32_t wait_ms) {
    clear_error();
    if (!S || !count || (max_results > 0 && !out) || max_results < 0)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_poll: bad argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->completed.empty() && wait_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->completed.empty(); });
    const int k = std::min<int>(max_results, (int)S->completed.size());
    for (int j = 0; j < k; ++j) out[j] = S->completed[j];
    S->completed.erase(S->completed.begin(), S->completed.begin() + k);
    *count = k;
    return AFSAI_OK;
}

int afsai_server_pending(afsai_server S, int64_t *outstanding, int64_t *bytes_in_use, int32_t *slots_in_use) {
    if (!S) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_server_pending: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (outstanding) *outstanding = S->outstanding;
    if (bytes_in_use) *bytes_in_use = (int64_t)S->used;
    if (slots_in_use) *slots_in_use = S->slots;
    return AFSAI_OK;
}

int afsai_server_destroy(afsai_server S) {
    if (!S) return AFSAI_OK;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->outstanding == 0; });
        S->stop = true;
        S->cv_work.notify_all();
        S->cv_sched.notify_all();
    }
    for (auto &t : S->workers) t.join();
    S->scheduler.join();
    for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
    delete S;
    return AFSAI_OK;
}

}  // extern "C"
