// Serving runtime: TT-SVD requests (Algorithm 2 of arXiv 2102.00104) that
// arrive over time, admitted by their device-memory footprint and executed by
// worker threads, each on its own HIP stream (default priority).
//
// Scheduling (continuous batching): small requests (every TT step of at
// most 128 columns, at most batch_max_elems elements, dense) wait in their own
// FIFO; whenever no batched launch is running, a free worker takes every
// waiting small request that fits the memory budget (up to max_batch) and
// runs them together in one persistent batched launch
// (ttsvd_decompose_batch), so requests that arrive while a batch runs join
// the next one.  Other requests wait in a second FIFO and run alone
// (ttsvd_decompose) on the other workers as their footprint fits the budget
// next to the running work; a large head that does not fit blocks only the
// large FIFO.  Workers that finish return their footprint and wake the
// others, so admitted work starts as soon as memory frees up.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"
#include "driver.h"
#include "tsqr_blk.h"

namespace ttsvd {
namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket;
    ttsvd_tensor X;
    std::vector<int64_t> dims;
    int64_t r_max;
    double tol;
    size_t footprint;
    bool small;
    double t_submit;
    hipEvent_t ready;  // recorded on the producer's stream at submission
};

}  // namespace
}  // namespace ttsvd

struct ttsvd_server {
    ttsvd_server_config cfg;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work;   // workers: new requests or freed memory
    std::condition_variable cv_done;   // pollers: new completions
    std::deque<ttsvd::Request> queue;        // large requests, FIFO
    std::deque<ttsvd::Request> small_queue;  // small requests, FIFO
    bool batch_running = false;
    std::deque<ttsvd_completion> done;
    std::vector<std::thread> workers;
    size_t in_use = 0;
    uint64_t next_ticket = 1;
    int64_t pending = 0;               // submitted, not yet completed
    bool stop = false;
};

namespace ttsvd {
namespace {

bool is_small(const std::vector<int64_t> &dims, int64_t r_max, int64_t max_elems) {
    std::vector<StepShape> steps;
    std::vector<int64_t> rb;
    int64_t nbar;
    if (plan_steps(dims.data(), (int)dims.size(), r_max, steps, rb, nbar) != TTSVD_OK) return false;
    if (nbar > max_elems) return false;
    for (int i = (int)dims.size() - 1; i >= 1; --i)
        if (steps[i].m > 128) return false;
    return true;
}

void worker_main(ttsvd_server *S) {
    (void)hipSetDevice(S->device);
    // several workers share the GPU: keep the TSQR launches non-cooperative
    blk_shared_tiles() = false;
    hipStream_t st = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    std::vector<Request> take;
    for (;;) {
        take.clear();
        size_t claimed = 0;
        bool as_batch = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stop && S->queue.empty() && S->small_queue.empty()) break;
                if (!S->small_queue.empty() && !S->batch_running) {
                    const Request &h = S->small_queue.front();
                    if (S->in_use + h.footprint <= S->cfg.hbm_budget || S->in_use == 0) {
                        as_batch = true;
                        break;
                    }
                }
                if (!S->queue.empty()) {
                    const Request &h = S->queue.front();
                    // a request larger than the whole budget runs alone once nothing else runs
                    if (S->in_use + h.footprint <= S->cfg.hbm_budget || S->in_use == 0) break;
                }
                S->cv_work.wait(lk);
            }
            if (S->queue.empty() && S->small_queue.empty()) break;  // stopping
            if (as_batch) {
                // every waiting small request that fits, in arrival order
                S->batch_running = true;
                for (auto it = S->small_queue.begin();
                     it != S->small_queue.end() && (int)take.size() < S->cfg.max_batch;) {
                    const bool first = take.empty();
                    if (it->X.dtype == S->small_queue.front().X.dtype &&
                        (S->in_use + claimed + it->footprint <= S->cfg.hbm_budget ||
                         (first && S->in_use == 0))) {
                        claimed += it->footprint;
                        take.push_back(*it);
                        it = S->small_queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            } else {
                take.push_back(S->queue.front());
                S->queue.pop_front();
                claimed = take[0].footprint;
            }
            S->in_use += claimed;
        }
        // The work of each request starts after what its producer enqueued
        // before submitting it (the tensor's contents).
        bool waited = have_stream;
        for (const Request &q : take)
            if (waited && hipStreamWaitEvent(st, q.ready, 0) != hipSuccess) waited = false;
        const double t_start = now_s();
        std::vector<ttsvd_completion> comp(take.size());
        for (size_t i = 0; i < take.size(); ++i) {
            memset(&comp[i], 0, sizeof(comp[i]));
            comp[i].ticket = take[i].ticket;
            comp[i].t_submit = take[i].t_submit;
            comp[i].t_start = t_start;
            comp[i].batch_size = (int)take.size();
            comp[i].batched = as_batch;
        }
        if (!waited) {
            for (auto &c : comp) {
                c.status = TTSVD_EHIP;
                snprintf(c.message, sizeof(c.message), "server: worker stream or event wait failed");
            }
        } else if (!as_batch) {
            ttsvd_tensor X = take[0].X;
            X.stream = st;
            comp[0].status = ttsvd_decompose(&X, take[0].dims.data(), (int)take[0].dims.size(),
                                             take[0].r_max, take[0].tol, &comp[0].tt);
            if (comp[0].status != TTSVD_OK)
                snprintf(comp[0].message, sizeof(comp[0].message), "%s", ttsvd_last_error());
        } else {
            const int n = (int)take.size();
            std::vector<ttsvd_tensor> xs(n);
            std::vector<int> d(n);
            std::vector<int64_t> dims, rm(n);
            std::vector<double> tl(n);
            for (int i = 0; i < n; ++i) {
                xs[i] = take[i].X;
                d[i] = (int)take[i].dims.size();
                dims.insert(dims.end(), take[i].dims.begin(), take[i].dims.end());
                rm[i] = take[i].r_max;
                tl[i] = take[i].tol;
            }
            std::vector<ttsvd_tt> outs(n);
            ttsvd_batch_config bc;
            ttsvd_batch_default_config(&bc);
            const int rc = ttsvd_decompose_batch(n, xs.data(), d.data(), dims.data(), rm.data(),
                                                 tl.data(), &bc, st, outs.data());
            for (int i = 0; i < n; ++i) {
                comp[i].status = rc;
                if (rc == TTSVD_OK)
                    comp[i].tt = outs[i];
                else
                    snprintf(comp[i].message, sizeof(comp[i].message), "%s", ttsvd_last_error());
            }
        }
        const double t_done = now_s();
        // the decompositions synchronised st, so the waits on these events are done
        if (have_stream) (void)hipStreamSynchronize(st);
        for (const Request &q : take) (void)hipEventDestroy(q.ready);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->in_use -= claimed;
            if (as_batch) S->batch_running = false;
            for (auto &c : comp) {
                c.t_done = t_done;
                S->done.push_back(c);
            }
            S->pending -= (int64_t)take.size();
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(st);
}

}  // namespace
}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

double ttsvd_server_clock(void) { return now_s(); }

int ttsvd_server_default_config(ttsvd_server_config *cfg) {
    if (!cfg) return TTSVD_EINVAL;
    cfg->hbm_budget = (size_t)64 << 30;
    cfg->workers = 4;
    cfg->max_batch = 512;
    cfg->batch_max_elems = (int64_t)1 << 24;
    return TTSVD_OK;
}

int ttsvd_server_create(const ttsvd_server_config *cfg, ttsvd_server **out) {
    clear_error();
    if (!cfg || !out) return set_error(TTSVD_EINVAL, "server: NULL pointer");
    if (cfg->workers < 1 || cfg->workers > 64 || cfg->max_batch < 1 || cfg->hbm_budget == 0)
        return set_error(TTSVD_EINVAL, "server: bad configuration");
    ttsvd_server *S = new ttsvd_server();
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return set_error(TTSVD_EHIP, "server: hipGetDevice");
    }
    for (int i = 0; i < cfg->workers; ++i) S->workers.emplace_back(worker_main, S);
    *out = S;
    return TTSVD_OK;
}

int ttsvd_server_submit(ttsvd_server *S, const ttsvd_tensor *X, const int64_t *dims, int d,
                        int64_t r_max, double tol, uint64_t *ticket) {
    clear_error();
    if (!S || !X || !X->data || !dims || !ticket) return set_error(TTSVD_EINVAL, "submit: NULL pointer");
    if (d < 1 || d > TTSVD_MAX_D || r_max < 1 || !(tol >= 0.0))
        return set_error(TTSVD_EINVAL, "submit: bad arguments");
    if (!valid_dtype(X->dtype)) return set_error(TTSVD_EUNSUPPORTED, "submit: dtype %d", X->dtype);
    Request r;
    r.X = *X;
    r.dims.assign(dims, dims + d);
    r.r_max = r_max;
    r.tol = tol;
    r.footprint = ttsvd_footprint_bytes(dims, d, r_max, X->dtype);
    if (r.footprint == 0) return set_error(TTSVD_EINVAL, "submit: invalid problem");
    r.small = is_small(r.dims, r_max, S->cfg.batch_max_elems) && X->ld_last == 0;
    r.t_submit = now_s();
    r.ready = nullptr;
    if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
        return set_error(TTSVD_EHIP, "submit: hipEventCreateWithFlags");
    if (hipEventRecord(r.ready, X->stream) != hipSuccess) {
        (void)hipEventDestroy(r.ready);
        return set_error(TTSVD_EHIP, "submit: hipEventRecord on the producer's stream");
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            (void)hipEventDestroy(r.ready);
            return set_error(TTSVD_EINVAL, "submit: server is stopping");
        }
        r.ticket = S->next_ticket++;
        *ticket = r.ticket;
        // small requests go to the batching lane unless batching is off
        if (r.small && S->cfg.max_batch > 1)
            S->small_queue.push_back(std::move(r));
        else
            S->queue.push_back(std::move(r));
        S->pending += 1;
    }
    S->cv_work.notify_one();
    return TTSVD_OK;
}

int ttsvd_server_poll(ttsvd_server *S, ttsvd_completion *out, int max, int wait_ms, int *n) {
    clear_error();
    if (!S || !n || (max > 0 && !out)) return set_error(TTSVD_EINVAL, "poll: NULL pointer");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && wait_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->done.empty(); });
    int k = 0;
    while (k < max && !S->done.empty()) {
        out[k++] = S->done.front();
        S->done.pop_front();
    }
    *n = k;
    return TTSVD_OK;
}

int64_t ttsvd_server_pending(ttsvd_server *S) {
    if (!S) return -1;
    std::lock_guard<std::mutex> lk(S->mu);
    return S->pending;
}

void ttsvd_server_destroy(ttsvd_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &c : S->done)
        if (c.status == TTSVD_OK) ttsvd_tt_free(&c.tt);
    delete S;
}

}  // extern "C"
