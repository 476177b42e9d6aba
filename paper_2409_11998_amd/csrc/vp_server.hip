// Serving loop: continuous admission of potential-evaluation requests.
//
// Plans (a mesh's resident data: tile-sorted nodes, multiplier tables,
// geometry) stay on the device; a request names a plan plus its densities and
// output.  A host worker thread keeps a FIFO of submitted requests and admits
// any of them -- as soon as an in-flight slot and enough HBM are free -- onto
// one of several streams, so requests that arrive while others run start
// without waiting for a batch boundary and their kernels overlap on the GPU.
// Each admitted request gets its own stream-ordered workspace (grids,
// spectra, strengths; hipMallocAsync/hipFreeAsync), whose size is the
// request's HBM footprint; the sum over in-flight requests never exceeds the
// budget.  Requests larger than the whole budget are rejected with
// VP_ERR_OOM; invalid requests complete with their error status.  Latency is
// host time from submission to observed completion of the request's last
// kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vp_internal.hpp"

using namespace vp;
using clk = std::chrono::steady_clock;

namespace {

thread_local std::string s_last_error;

vp_status sfail(vp_status s, const std::string& m)
{
    s_last_error = m;
    return s;
}

struct Req {
    uint64_t id = 0;
    vp_request r{};
    size_t bytes = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    vp_status status = VP_OK;
    bool deferred = false;
    clk::time_point t_submit, t_done;
    Workspace ws;
    hipEvent_t ev = nullptr;
    int stream = -1;
};

}  // namespace

struct vp_server_s {
    vp_server_opts opts{};
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work;   // worker waits for submissions
    std::condition_variable cv_done;   // clients wait for completions
    std::deque<Req*> queue;
    std::vector<Req*> running;
    std::unordered_map<uint64_t, Req*> reqs;
    uint64_t next_id = 1;
    size_t in_flight_bytes = 0;
    bool stop = false;
    // statistics
    uint64_t submitted = 0, completed = 0, rejected = 0, failed = 0, deferred = 0;
    size_t peak_bytes = 0;
    int peak_in_flight = 0;
    std::vector<double> lat;
    double targets_done = 0;
    clk::time_point t_first, t_last;
    bool any = false;
    int device = 0;
    std::vector<hipEvent_t> free_events;  // completion events, reused across requests
};

namespace {

void finish(vp_server_s* S, Req* q, vp_status st)
{
    q->status = st;
    q->state = 2;
    q->t_done = clk::now();
    const double l = std::chrono::duration<double>(q->t_done - q->t_submit).count();
    S->lat.push_back(l);
    S->completed++;
    if (st == VP_OK) S->targets_done += (double)q->r.plan->n_tgt;
    else S->failed++;
    S->t_last = q->t_done;
}

// Worker: poll completions, admit queued requests, launch them.
void worker_main(vp_server_s* S)
{
    hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool progressed = false;
        // completions
        for (size_t i = 0; i < S->running.size();) {
            Req* q = S->running[i];
            const hipError_t e = hipEventQuery(q->ev);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            finish(S, q, e == hipSuccess ? VP_OK : VP_ERR_DEVICE);
            S->in_flight_bytes -= q->bytes;
            S->stream_load[q->stream]--;
            S->free_events.push_back(q->ev);
            q->ev = nullptr;
            S->running[i] = S->running.back();
            S->running.pop_back();
            progressed = true;
        }
        if (progressed) S->cv_done.notify_all();
        // admission (FIFO order; a request that does not fit does not block smaller ones behind it)
        for (auto it = S->queue.begin(); it != S->queue.end();) {
            Req* q = *it;
            if (q->bytes > S->opts.hbm_budget_bytes) {
                finish(S, q, VP_ERR_OOM);
                S->rejected++;
                it = S->queue.erase(it);
                progressed = true;
                S->cv_done.notify_all();
                continue;
            }
            if ((int)S->running.size() >= S->opts.max_in_flight ||
                S->in_flight_bytes + q->bytes > S->opts.hbm_budget_bytes) {
                if (!q->deferred) {
                    q->deferred = true;
                    S->deferred++;
                }
                ++it;
                continue;
            }
            // least-loaded stream
            int si = 0;
            for (int k = 1; k < (int)S->streams.size(); ++k)
                if (S->stream_load[k] < S->stream_load[si]) si = k;
            hipStream_t st = S->streams[si];
            Plan& p = *q->r.plan;
            vp_status vs = VP_OK;
            hipError_t he = workspace_alloc(p, q->ws, st, true);
            if (he != hipSuccess) vs = set_error(VP_ERR_OOM, hipGetErrorString(he));
            if (vs == VP_OK)
                vs = eval_enqueue(p, q->ws, st, q->r.f_src, q->r.jet6, q->r.sigma, q->r.sigma_jet3, q->r.mu,
                                  q->r.mu_jet5, q->r.out, false);
            if (q->ws.block) workspace_free(q->ws, st, true);
            if (vs == VP_OK) {
                if (!S->free_events.empty()) {
                    q->ev = S->free_events.back();
                    S->free_events.pop_back();
                } else if (hipEventCreateWithFlags(&q->ev, hipEventDisableTiming) != hipSuccess) {
                    q->ev = nullptr;
                    vs = VP_ERR_DEVICE;
                }
            }
            if (vs == VP_OK && hipEventRecord(q->ev, st) != hipSuccess) vs = VP_ERR_DEVICE;
            it = S->queue.erase(it);
            progressed = true;
            if (vs != VP_OK) {
                if (q->ev) S->free_events.push_back(q->ev);
                q->ev = nullptr;
                finish(S, q, vs);
                S->cv_done.notify_all();
                continue;
            }
            q->state = 1;
            q->stream = si;
            S->stream_load[si]++;
            S->in_flight_bytes += q->bytes;
            S->running.push_back(q);
            S->peak_bytes = std::max(S->peak_bytes, S->in_flight_bytes);
            S->peak_in_flight = std::max(S->peak_in_flight, (int)S->running.size());
        }
        if (S->stop && S->queue.empty() && S->running.empty()) break;
        if (!progressed) {
            if (S->running.empty()) S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            else {
                // requests on the device: poll again soon (completion latency is what is measured)
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        }
    }
}

}  // namespace

extern "C" {

const char* vp_server_last_error(void) { return s_last_error.c_str(); }

vp_status vp_server_create(vp_server_t* out, const vp_server_opts* opts)
{
    s_last_error.clear();
    if (!out || !opts) return sfail(VP_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (opts->hbm_budget_bytes == 0 || opts->max_in_flight <= 0 || opts->n_streams <= 0 || opts->n_streams > 16)
        return sfail(VP_ERR_ARG, "need hbm_budget_bytes > 0, max_in_flight > 0, 1 <= n_streams <= 16");
    vp_server_s* S = new (std::nothrow) vp_server_s();
    if (!S) return sfail(VP_ERR_OOM, "host allocation");
    S->opts = *opts;
    hipGetDevice(&S->device);
    // Keep freed workspace memory in the device's stream-ordered pool instead of
    // returning it at every synchronization, so admitting a request costs no
    // operating-system allocation once the pool has grown to the working set.
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, S->device) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    for (int i = 0; i < opts->n_streams; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : S->streams) hipStreamDestroy(x);
            delete S;
            return sfail(VP_ERR_DEVICE, "stream creation failed");
        }
        S->streams.push_back(st);
        S->stream_load.push_back(0);
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return VP_OK;
}

vp_status vp_server_submit(vp_server_t S, const vp_request* r, uint64_t* ticket)
{
    s_last_error.clear();
    if (!S || !r || !ticket) return sfail(VP_ERR_ARG, "NULL argument");
    if (!r->plan) return sfail(VP_ERR_ARG, "request without a plan");
    Req* q = new (std::nothrow) Req();
    if (!q) return sfail(VP_ERR_OOM, "host allocation");
    q->r = *r;
    q->bytes = workspace_bytes(*r->plan);
    q->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> g(S->mu);
        q->id = S->next_id++;
        S->reqs[q->id] = q;
        S->queue.push_back(q);
        S->submitted++;
        if (!S->any) {
            S->any = true;
            S->t_first = q->t_submit;
        }
    }
    S->cv_work.notify_one();
    *ticket = q->id;
    return VP_OK;
}

vp_status vp_server_poll(vp_server_t S, uint64_t ticket, int* done, vp_status* result, double* latency_s)
{
    if (!S || !done) return sfail(VP_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return sfail(VP_ERR_ARG, "unknown ticket");
    Req* q = it->second;
    *done = q->state == 2;
    if (*done) {
        if (result) *result = q->status;
        if (latency_s) *latency_s = std::chrono::duration<double>(q->t_done - q->t_submit).count();
    }
    return VP_OK;
}

vp_status vp_server_wait(vp_server_t S, uint64_t ticket, double timeout_s, vp_status* result, double* latency_s)
{
    if (!S) return sfail(VP_ERR_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return sfail(VP_ERR_ARG, "unknown ticket");
    Req* q = it->second;
    const auto deadline = clk::now() + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(timeout_s));
    while (q->state != 2) {
        if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && q->state != 2)
            return sfail(VP_ERR_BUSY, "timed out");
    }
    if (result) *result = q->status;
    if (latency_s) *latency_s = std::chrono::duration<double>(q->t_done - q->t_submit).count();
    return VP_OK;
}

vp_status vp_server_get_stats(vp_server_t S, vp_server_stats* st)
{
    if (!S || !st) return sfail(VP_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->rejected = S->rejected;
    st->failed = S->failed;
    st->deferred = S->deferred;
    st->peak_bytes = S->peak_bytes;
    st->peak_in_flight = S->peak_in_flight;
    std::vector<double> l(S->lat);
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) {
            const size_t k = (size_t)std::min<double>(l.size() - 1, std::ceil(q * l.size()) - 1);
            return l[k];
        };
        st->p50_s = pct(0.50);
        st->p99_s = pct(0.99);
        st->max_s = l.back();
        double sum = 0;
        for (double v : l) sum += v;
        st->mean_s = sum / l.size();
    }
    if (S->any && S->completed) {
        st->span_s = std::chrono::duration<double>(S->t_last - S->t_first).count();
        st->targets_per_s = st->span_s > 0 ? S->targets_done / st->span_s : 0.0;
    }
    return VP_OK;
}

vp_status vp_server_destroy(vp_server_t S)
{
    if (!S) return VP_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto st : S->streams) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
    }
    for (auto e : S->free_events) hipEventDestroy(e);
    for (auto& kv : S->reqs) delete kv.second;
    delete S;
    return VP_OK;
}

}  // extern "C"
