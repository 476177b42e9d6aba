// Serving loop: continuous batching of potential-evaluation requests.
//
// Plans (a mesh's resident data: tile-sorted nodes, multiplier tables,
// geometry) stay on the device; a request names a plan plus its densities and
// output.  A host worker thread keeps a FIFO of submitted requests.  Whenever
// in-flight slots and HBM are free it admits the queued requests that fit --
// in FIFO order, all of one precision (the first admissible request's), a
// request that does not fit never blocking smaller ones behind it -- and runs
// them as one group: the per-stage group kernels of the batched
// execution, one launch per stage for the whole group, on an idle one of
// several streams.  At most one group per stream is in flight: while every
// stream is busy, arrivals wait on the host and the next free stream takes
// them all as one group, so groups grow with the load instead of work queueing
// on the device.  Groups on different streams overlap on the GPU.
//
// Memory.  Every admitted request gets a workspace block (grids, spectra,
// strengths) of its plan's footprint rounded up to a size class (at most
// 1/8 above it).  Blocks come from the server's own cache: a block returns to
// its class's free list when the event of the group that used it has
// completed, so steady-state admission makes no device allocation and no
// stream-ordered pool call.  The server's HBM -- blocks in use plus cached
// blocks -- never exceeds the budget: a miss that would pass it first frees
// cached blocks.  Each group's descriptor image is written to a pinned host
// buffer and copied to a device buffer of a pair that is reused, like the
// blocks, once the group has completed.
//
// Locking.  Clients take the mutex only to queue a request or read state; the
// worker takes it to retire finished groups and to pick the next group, and
// polls events, builds descriptors and launches with the mutex released.
//
// Requests larger than the whole budget are rejected with VP_ERR_OOM; invalid
// requests complete with their error status, alone.  Latency is host time
// from submission to observed completion of the request's group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vp_group.hpp"
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

constexpr int kMaxGroup = 64;  // requests per group

// Workspace size class: bytes rounded up to a multiple of 1/8 of the largest
// power of two not above them (at most 12.5% above the request).
size_t size_class(size_t b)
{
    if (b <= 4096) return 4096;
    const int e = 63 - __builtin_clzll((unsigned long long)b);
    const size_t q = (size_t)1 << (e - 3);
    return (b + q - 1) / q * q;
}

struct Req {
    uint64_t id = 0;
    vp_request r{};
    size_t bytes = 0;  // size class of the plan's workspace
    int state = 0;     // 0 queued, 1 running, 2 done
    vp_status status = VP_OK;
    bool deferred = false;
    clk::time_point t_submit, t_done;
};

// Descriptor buffers of one group: pinned host staging + device copy.
struct TabBuf {
    void* dev = nullptr;
    unsigned char* host = nullptr;
};

struct Group {
    std::vector<Req*> reqs;
    std::vector<void*> blocks;  // workspace block of each request
    TabBuf tab;
    hipEvent_t ev = nullptr;
    int stream = -1;
    size_t bytes = 0;
    hipError_t result = hipSuccess;
};

}  // namespace

struct vp_server_s {
    vp_server_opts opts{};
    int device = 0;
    std::vector<hipStream_t> streams;
    std::thread worker;
    // shared with clients (guarded by mu)
    std::mutex mu;
    std::condition_variable cv_work;  // worker waits for submissions
    std::condition_variable cv_done;  // clients wait for completions
    std::deque<Req*> queue;
    std::unordered_map<uint64_t, Req*> reqs;
    uint64_t next_id = 1;
    size_t in_flight_bytes = 0;
    int in_flight = 0;
    bool stop = false;
    uint64_t submitted = 0, completed = 0, rejected = 0, failed = 0, deferred = 0, groups = 0, grouped = 0;
    size_t peak_bytes = 0, peak_held = 0;
    uint64_t device_allocs = 0;
    int peak_in_flight = 0;
    std::vector<double> lat;
    double targets_done = 0;
    clk::time_point t_first, t_last;
    bool any = false;
    // worker-only state
    std::vector<Group*> running;
    std::vector<int> stream_load;
    std::map<size_t, std::vector<void*>> free_blocks;  // size class -> cached blocks
    size_t held_bytes = 0;                             // blocks in use + cached
    size_t cached_bytes = 0;
    std::vector<TabBuf> free_tabs, all_tabs;
    std::vector<hipEvent_t> free_events, all_events;
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

vp_eval_args args_of(const vp_request& r)
{
    vp_eval_args a;
    a.f_src = r.f_src;
    a.jet6 = r.jet6;
    a.sigma = r.sigma;
    a.sigma_jet3 = r.sigma_jet3;
    a.mu = r.mu;
    a.mu_jet5 = r.mu_jet5;
    a.out = r.out;
    return a;
}

// --- worker-owned memory --------------------------------------------------

void release_block(vp_server_s* S, size_t bytes, void* blk)
{
    S->free_blocks[bytes].push_back(blk);
    S->cached_bytes += bytes;
}

// A block of `bytes` (a size class): cached if possible, else a new device
// allocation after freeing cached blocks while the server would pass its budget.
hipError_t acquire_block(vp_server_s* S, size_t bytes, void** out, bool* allocated)
{
    *allocated = false;
    auto f = S->free_blocks.find(bytes);
    if (f != S->free_blocks.end() && !f->second.empty()) {
        *out = f->second.back();
        f->second.pop_back();
        S->cached_bytes -= bytes;
        return hipSuccess;
    }
    while (S->held_bytes + bytes > S->opts.hbm_budget_bytes && S->cached_bytes > 0) {
        auto big = std::prev(S->free_blocks.end());
        while (big->second.empty()) big = std::prev(big);
        hipFree(big->second.back());
        big->second.pop_back();
        S->cached_bytes -= big->first;
        S->held_bytes -= big->first;
    }
    const hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) return e;
    S->held_bytes += bytes;
    *allocated = true;
    return hipSuccess;
}

hipError_t acquire_tab(vp_server_s* S, TabBuf* t)
{
    if (!S->free_tabs.empty()) {
        *t = S->free_tabs.back();
        S->free_tabs.pop_back();
        return hipSuccess;
    }
    const size_t n = group_bytes_bound(kMaxGroup);
    TabBuf b;
    hipError_t e = hipMalloc(&b.dev, n);
    if (e != hipSuccess) return e;
    e = hipHostMalloc((void**)&b.host, n, hipHostMallocDefault);
    if (e != hipSuccess) {
        hipFree(b.dev);
        return e;
    }
    S->all_tabs.push_back(b);
    *t = b;
    return hipSuccess;
}

hipError_t acquire_event(vp_server_s* S, hipEvent_t* ev)
{
    if (!S->free_events.empty()) {
        *ev = S->free_events.back();
        S->free_events.pop_back();
        return hipSuccess;
    }
    const hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e == hipSuccess) S->all_events.push_back(*ev);
    return e;
}

// Return a group's blocks, descriptor buffers and event to the caches.
void recycle(vp_server_s* S, Group* g)
{
    for (size_t i = 0; i < g->blocks.size(); ++i)
        if (g->blocks[i]) release_block(S, g->reqs[i]->bytes, g->blocks[i]);
    g->blocks.clear();
    if (g->tab.dev) S->free_tabs.push_back(g->tab);
    g->tab = TabBuf{};
    if (g->ev) S->free_events.push_back(g->ev);
    g->ev = nullptr;
}

// --- admission (under the mutex) -----------------------------------------

// Pick the queued requests that run next as one group; rejects oversized and
// invalid requests on the way.  Returns true if any request completed here.
bool select_group(vp_server_s* S, std::vector<Req*>& take, size_t& bytes)
{
    bool finished_any = false;
    int precision = -1;
    bytes = 0;
    // at most one group per stream in flight: while every stream is busy, arrivals
    // wait on the host and join the next group instead of queueing on the device
    const bool room = (int)S->running.size() < S->opts.n_streams;
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        Req* q = *it;
        if (q->bytes > S->opts.hbm_budget_bytes) {
            finish(S, q, VP_ERR_OOM);
            S->rejected++;
            it = S->queue.erase(it);
            finished_any = true;
            continue;
        }
        const Plan& p = *q->r.plan;
        const vp_status vs = eval_validate(p, q->r.f_src, q->r.jet6, q->r.sigma, q->r.sigma_jet3, q->r.mu,
                                           q->r.mu_jet5, q->r.out);
        if (vs != VP_OK) {
            finish(S, q, vs);
            it = S->queue.erase(it);
            finished_any = true;
            continue;
        }
        const bool fits = room && S->in_flight + (int)take.size() < S->opts.max_in_flight &&
                          S->in_flight_bytes + bytes + q->bytes <= S->opts.hbm_budget_bytes &&
                          (int)take.size() < kMaxGroup;
        if (!fits || (precision >= 0 && p.precision != precision)) {
            if (!fits && !q->deferred) {
                q->deferred = true;
                S->deferred++;
            }
            ++it;
            continue;
        }
        precision = p.precision;
        take.push_back(q);
        bytes += q->bytes;
        it = S->queue.erase(it);
    }
    if (!take.empty()) {
        for (Req* q : take) q->state = 1;
        S->in_flight += (int)take.size();
        S->in_flight_bytes += bytes;
        S->groups++;
        S->grouped += take.size();
        S->peak_bytes = std::max(S->peak_bytes, S->in_flight_bytes);
        S->peak_in_flight = std::max(S->peak_in_flight, S->in_flight);
    }
    return finished_any;
}

// --- launch (worker, mutex released) ---------------------------------------

// Allocate, describe and enqueue a selected group.  On failure the group's
// resources are back in the caches and the returned status is the error.
vp_status launch_group(vp_server_s* S, Group* g, uint64_t* allocs)
{
    int si = 0;
    for (int k = 1; k < (int)S->streams.size(); ++k)
        if (S->stream_load[k] < S->stream_load[si]) si = k;
    hipStream_t st = S->streams[si];
    g->stream = si;
    const size_t n = g->reqs.size();
    g->blocks.assign(n, nullptr);
    std::vector<const Plan*> plans(n);
    std::vector<Workspace> wss(n);
    std::vector<vp_eval_args> args(n);
    vp_status vs = VP_OK;
    for (size_t i = 0; i < n; ++i) {
        Req* q = g->reqs[i];
        bool fresh = false;
        const hipError_t he = acquire_block(S, q->bytes, &g->blocks[i], &fresh);
        if (he != hipSuccess) {
            g->blocks[i] = nullptr;
            vs = sfail(VP_ERR_OOM, std::string("workspace: ") + hipGetErrorString(he));
            break;
        }
        *allocs += fresh;
        plans[i] = q->r.plan;
        workspace_bind(*q->r.plan, wss[i], g->blocks[i], q->bytes);
        args[i] = args_of(q->r);
    }
    if (vs == VP_OK && acquire_tab(S, &g->tab) != hipSuccess) vs = sfail(VP_ERR_OOM, "group descriptor buffers");
    if (vs == VP_OK && acquire_event(S, &g->ev) != hipSuccess) vs = sfail(VP_ERR_DEVICE, "event creation");
    bool enqueued = false;
    if (vs == VP_OK)
        vs = group_enqueue(plans, wss, args, g->tab.dev, g->tab.host, group_bytes_bound(kMaxGroup), st, &enqueued);
    if (vs == VP_OK && hipEventRecord(g->ev, st) != hipSuccess) vs = sfail(VP_ERR_DEVICE, "event record");
    if (vs != VP_OK) {
        if (enqueued) hipStreamSynchronize(st);  // the descriptor copy may still read the pinned buffer
        recycle(S, g);
        return vs;
    }
    S->stream_load[si]++;
    S->running.push_back(g);
    return VP_OK;
}

// Worker: retire finished groups, admit and launch the next group.
void worker_main(vp_server_s* S)
{
    hipSetDevice(S->device);
    std::vector<Group*> done;
    std::vector<Req*> take;
    while (true) {
        // 1. poll the running groups
        done.clear();
        for (size_t i = 0; i < S->running.size();) {
            Group* g = S->running[i];
            const hipError_t e = hipEventQuery(g->ev);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            g->result = e;
            done.push_back(g);
            S->stream_load[g->stream]--;
            S->running[i] = S->running.back();
            S->running.pop_back();
        }
        for (Group* g : done) recycle(S, g);
        // 2. retire and select under the mutex
        bool progressed = !done.empty();
        bool hold = false, quit = false;
        clk::time_point deadline{};
        size_t bytes = 0;
        take.clear();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Group* g : done) {
                for (Req* q : g->reqs) finish(S, q, g->result == hipSuccess ? VP_OK : VP_ERR_DEVICE);
                S->in_flight_bytes -= g->bytes;
                S->in_flight -= (int)g->reqs.size();
            }
            // optional admission delay: let the oldest queued request gather a group
            if (!S->queue.empty() && S->opts.max_wait_us > 0 && !S->stop && (int)S->queue.size() < kMaxGroup) {
                deadline = S->queue.front()->t_submit + std::chrono::microseconds(S->opts.max_wait_us);
                hold = clk::now() < deadline;
            }
            if (!S->queue.empty() && !hold && select_group(S, take, bytes)) progressed = true;
            quit = S->stop && S->queue.empty() && S->running.empty() && take.empty();
        }
        for (Group* g : done) delete g;
        if (progressed) S->cv_done.notify_all();
        // 3. launch the selected group
        if (!take.empty()) {
            Group* g = new Group();
            g->reqs = take;
            g->bytes = bytes;
            uint64_t allocs = 0;
            const vp_status vs = launch_group(S, g, &allocs);
            std::lock_guard<std::mutex> lk(S->mu);
            S->device_allocs += allocs;
            S->peak_held = std::max(S->peak_held, S->held_bytes);
            if (vs != VP_OK) {
                for (Req* q : g->reqs) finish(S, q, vs);
                S->in_flight_bytes -= g->bytes;
                S->in_flight -= (int)g->reqs.size();
                delete g;
                S->cv_done.notify_all();
            }
            continue;
        }
        if (quit) break;
        if (progressed) continue;
        // 4. nothing to do right now
        if (S->running.empty()) {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop) continue;
            if (S->queue.empty()) S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            else if (hold) S->cv_work.wait_until(lk, std::min(deadline, clk::now() + std::chrono::milliseconds(5)));
            else S->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        } else {
            std::this_thread::yield();  // groups on the device: completion latency is what is measured
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
    if (opts->hbm_budget_bytes == 0 || opts->max_in_flight <= 0 || opts->n_streams <= 0 || opts->n_streams > 16 ||
        opts->max_wait_us < 0)
        return sfail(VP_ERR_ARG,
                     "need hbm_budget_bytes > 0, max_in_flight > 0, 1 <= n_streams <= 16, max_wait_us >= 0");
    vp_server_s* S = new (std::nothrow) vp_server_s();
    if (!S) return sfail(VP_ERR_OOM, "host allocation");
    S->opts = *opts;
    hipGetDevice(&S->device);
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
    q->bytes = size_class(workspace_bytes(*r->plan));
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
    st->groups = S->groups;
    st->mean_group = S->groups ? (double)S->grouped / (double)S->groups : 0.0;
    st->peak_held_bytes = S->peak_held;
    st->device_allocs = S->device_allocs;
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
    for (auto& kv : S->free_blocks)
        for (void* b : kv.second) hipFree(b);
    for (auto& t : S->all_tabs) {
        hipFree(t.dev);
        hipHostFree(t.host);
    }
    for (auto e : S->all_events) hipEventDestroy(e);
    for (auto& kv : S->reqs) delete kv.second;
    delete S;
    return VP_OK;
}

}  // extern "C"
