// Serving loop: a request queue of embedding jobs, admitted by device-memory footprint and
// run with continuous batching.
//
// Every job is one fixed-step gradient-descent run (the repeat loop of Fig. algo, as in
// gempe_embed) on its own graph, dimension and coordinates.  The server owns one device
// block of the configured budget and a scheduler thread:
//
//  * admission: a released job is admitted when a range of its footprint (graph, X, loss
//    history, workspace) is free in the budget block (first fit, Arena); a job that does
//    not fit waits while later jobs that fit may pass it (backfill), until it has waited
//    kAgingSeconds, after which nothing passes it.  Its graph is uploaded and validated
//    on the transfer stream; an invalid graph fails the job alone.
//  * batched jobs (FP32, d <= 16, at most 65,536 64-tiles, i.e. the jobs gempe_embed runs
//    as one fused launch per iteration): all of them advance together, one iteration per
//    "tick", in ONE launch per padded dimension class (k_iter_batch).  A job admitted while
//    others run joins at the next tick; a finished job leaves the table.  Ticks are
//    enqueued up to kLookahead ahead of the device so the GPU is never idle while the host
//    admits or copies results.
//  * solo jobs (larger n, d > 16, BF16 Gram): their iterations are enqueued in chunks on
//    one of kSoloStreams streams and overlap with the ticks and with each other.
//  * completion: an event after the job's last work; then its coordinates, loss history
//    and status word are copied to the caller's host buffers and its range is released.
//
// Jobs share nothing but launches and the budget block, so a job's result does not depend
// on its companions beyond the order of FP32 atomic additions (the same freedom a single
// gempe_embed has), and a job whose loss turns non-finite fails alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
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

#include "arena.h"
#include "internal.h"

namespace {

constexpr int kDClasses = 6;                      // padded dimensions 1, 2, 3, 4, 8, 16
constexpr int kDValues[kDClasses] = {1, 2, 3, 4, 8, 16};
constexpr int kLookahead = 24;                    // ticks enqueued ahead of the device
constexpr int kTickEvents = 64;                   // ring of tick events (> kLookahead)
constexpr int kTableSlots = 64;                   // pinned staging slots for table uploads
constexpr int kSoloStreams = 3;
constexpr int kSoloChunk = 8;                     // iterations per enqueued solo chunk
constexpr double kAgingSeconds = 2.0;

int dclass_of(int D) {
    for (int c = 0; c < kDClasses; ++c)
        if (kDValues[c] == D) return c;
    return -1;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct JobLayout {
    size_t graph, X, hist, ws, total;
};

struct Job {
    int64_t id = 0;
    // request (host copies)
    int32_t n = 0, d = 0;
    int64_t nnz = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col_idx;
    std::vector<float> X0;
    int32_t iters = 0;
    float eta = 0.0f;
    gempe_params params{};
    double release_s = 0.0;
    float *X_out = nullptr;
    double *hist_out = nullptr;
    // state (guarded by Server::mu)
    int32_t state = GEMPE_JOB_QUEUED;
    gempe_status status = GEMPE_OK;
    std::string error;
    double admit_s = 0.0, done_s = 0.0;
    bool batched = false;
    size_t footprint = 0;
    // device side (scheduler thread only)
    size_t off = gempe::Arena::kNone;
    gempe_graph_s graph;
    SweepPlan plan;
    WsLayout L;
    JobLayout J{};
    unsigned char *base = nullptr;
    int dclass = -1;
    int k0 = 0, K = 0;
    long long finish_tick = 0;
    int stream = 0, next_k = 0;
    std::deque<hipEvent_t> chunk_events;
};

JobLayout job_layout(int32_t n, int64_t nnz, int32_t d, int32_t iters, const WsLayout &L) {
    JobLayout J;
    size_t off = 0;
    J.graph = off;
    off = align256(off + gempe_graph_mem_bytes(n, nnz));
    J.X = off;
    off = align256(off + sizeof(float) * (size_t)n * (size_t)d);
    J.hist = off;
    off = align256(off + sizeof(double) * ((size_t)iters + 1));
    J.ws = off;
    off = align256(off + L.total);
    J.total = off;
    return J;
}

// Plan and workspace layout of a job before its graph exists (they depend on n, nnz, d).
void job_plan(int32_t n, int64_t nnz, int32_t d, const gempe_params &p, SweepPlan &plan, WsLayout &L) {
    gempe_graph_s shape;
    shape.n = n;
    shape.nnz = nnz;
    shape.m = nnz / 2;
    plan = gempe_make_plan(&shape, d, p.precision == GEMPE_BF16_GRAM);
    L = gempe_ws_layout(&shape, d, plan);
}

}  // namespace

struct gempe_server_s {
    // configuration
    int device = 0;
    size_t budget = 0;
    int32_t max_jobs = 0;
    std::chrono::steady_clock::time_point t0;
    // device resources
    unsigned char *block = nullptr;
    gempe::Arena arena;
    hipStream_t batch_stream = nullptr, xfer_stream = nullptr, solo_streams[kSoloStreams] = {};
    void *tables[kDClasses] = {};  // device tables, max_jobs entries each
    unsigned char *pinned = nullptr;  // kTableSlots staging slots of max_jobs entries
    long long slot_tick[kTableSlots] = {};
    int next_slot = 0;
    hipEvent_t tick_ev[kTickEvents] = {};
    long long ev_tick[kTickEvents] = {};
    std::vector<hipEvent_t> event_pool;

    // shared state
    std::mutex mu;
    std::condition_variable cv_submit, cv_done;
    bool stop = false;
    int64_t next_id = 0;
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    std::deque<Job *> incoming;  // submitted, not yet admitted (release order)
    gempe_server_stats stats{};
    std::thread thread;

    // scheduler-thread state
    std::vector<Job *> batch[kDClasses];  // table rows: jobs whose finishing tick is not yet enqueued
    bool table_dirty[kDClasses] = {};
    std::vector<Job *> batch_live;        // batched jobs not yet completed on the host
    std::vector<Job *> solo;
    long long next_tick = 0, done_tick = -1;
    std::deque<long long> pending_ticks;  // enqueued, not yet known complete
    int solo_rr = 0;
    std::string fatal;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    hipEvent_t get_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
    void put_event(hipEvent_t e) { event_pool.push_back(e); }

    void run();
    bool admit_one(Job *j);
    void finish_job(Job *j);
    void fail_job(Job *j, gempe_status st, const std::string &msg);
    void release_job_memory(Job *j);
    bool enqueue_tick();
    void poll_ticks(bool block_one);
    void service_solo();
};

void gempe_server_s::release_job_memory(Job *j) {
    if (j->off != gempe::Arena::kNone) {
        arena.release(j->off);
        j->off = gempe::Arena::kNone;
    }
    std::vector<float>().swap(j->X0);
    std::vector<int64_t>().swap(j->row_ptr);
    std::vector<int32_t>().swap(j->col_idx);
}

void gempe_server_s::fail_job(Job *j, gempe_status st, const std::string &msg) {
    release_job_memory(j);
    std::lock_guard<std::mutex> lk(mu);
    j->state = GEMPE_JOB_FAILED;
    j->status = st;
    j->error = msg;
    j->done_s = now();
    stats.failed++;
    cv_done.notify_all();
}

// Admission: carve the job's range, upload and validate its graph and coordinates.
bool gempe_server_s::admit_one(Job *j) {
    const size_t off = arena.alloc(j->footprint);
    if (off == gempe::Arena::kNone) return false;
    j->off = off;
    j->base = block + off;
    gempe_status st = gempe_graph_build(j->n, j->nnz, j->row_ptr.data(), j->col_idx.data(), hipMemcpyHostToDevice,
                                        j->base + j->J.graph, xfer_stream, &j->graph);
    j->graph.server_owned = true;
    if (st != GEMPE_OK) {
        (void)hipStreamSynchronize(xfer_stream);
        fail_job(j, st, gempe_last_error());
        return true;
    }
    hipError_t e = hipMemcpyAsync(j->base + j->J.X, j->X0.data(), sizeof(float) * j->X0.size(),
                                  hipMemcpyHostToDevice, xfer_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(xfer_stream);
    if (e != hipSuccess) {
        fail_job(j, GEMPE_ERR_HIP, std::string("admission upload: ") + hipGetErrorString(e));
        return true;
    }
    // host copies are no longer needed
    std::vector<float>().swap(j->X0);
    std::vector<int64_t>().swap(j->row_ptr);
    std::vector<int32_t>().swap(j->col_idx);
    {
        std::lock_guard<std::mutex> lk(mu);
        j->state = GEMPE_JOB_RUNNING;
        j->admit_s = now();
        stats.admitted++;
        const size_t used = arena.used();
        if ((int64_t)used > stats.peak_bytes) stats.peak_bytes = (int64_t)used;
    }
    if (j->batched) {
        j->dclass = dclass_of(j->plan.D);
        j->k0 = (int)next_tick;
        j->K = j->iters + 1;
        j->finish_tick = j->k0 + j->K;
        e = gempe_batch_prepare(&j->graph, j->d, j->L, j->base + j->J.ws, batch_stream);
        if (e != hipSuccess) {
            fail_job(j, GEMPE_ERR_HIP, std::string("batch prepare: ") + hipGetErrorString(e));
            return true;
        }
        batch[j->dclass].push_back(j);
        batch_live.push_back(j);
        table_dirty[j->dclass] = true;
    } else {
        j->stream = solo_rr++ % kSoloStreams;
        j->next_k = 0;
        solo.push_back(j);
    }
    return true;
}

void gempe_server_s::finish_job(Job *j) {
    unsigned status_word = 0;
    const size_t nd = (size_t)j->n * (size_t)j->d;
    hipError_t e = hipMemcpyAsync(j->X_out, j->base + j->J.X, sizeof(float) * nd, hipMemcpyDeviceToHost, xfer_stream);
    if (e == hipSuccess && j->hist_out)
        e = hipMemcpyAsync(j->hist_out, j->base + j->J.hist, sizeof(double) * ((size_t)j->iters + 1),
                           hipMemcpyDeviceToHost, xfer_stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&status_word, j->base + j->J.ws + j->L.counters + 8, sizeof(unsigned),
                           hipMemcpyDeviceToHost, xfer_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(xfer_stream);
    if (e != hipSuccess) {
        fail_job(j, GEMPE_ERR_HIP, std::string("result copy: ") + hipGetErrorString(e));
        return;
    }
    if (status_word & kStatusNonFinite) {
        fail_job(j, GEMPE_ERR_NUMERIC, "non-finite loss");
        return;
    }
    release_job_memory(j);
    std::lock_guard<std::mutex> lk(mu);
    j->state = GEMPE_JOB_DONE;
    j->status = GEMPE_OK;
    j->done_s = now();
    stats.done++;
    stats.pairs += (double)j->n * (double)(j->n - 1) * 0.5 * (double)j->iters;
    cv_done.notify_all();
}

// One tick: every batched job advances by one iteration (or finishes).
bool gempe_server_s::enqueue_tick() {
    const long long t = next_tick;
    bool any = false;
    for (int c = 0; c < kDClasses; ++c) {
        auto &v = batch[c];
        // drop jobs whose finishing step was an earlier tick
        size_t w = 0;
        for (size_t r = 0; r < v.size(); ++r) {
            if (v[r]->finish_tick >= t) v[w++] = v[r];
            else table_dirty[c] = true;
        }
        v.resize(w);
        if (v.empty()) continue;
        any = true;
        const size_t eb = gempe_batch_entry_bytes();
        long long blocks = 0;
        if (table_dirty[c]) {
            // stage the table in a pinned slot whose previous upload has executed
            const int slot = next_slot;
            next_slot = (next_slot + 1) % kTableSlots;
            while (slot_tick[slot] > done_tick && !pending_ticks.empty() && fatal.empty()) poll_ticks(true);
            unsigned char *stage = pinned + (size_t)slot * (size_t)max_jobs * eb;
            for (size_t q = 0; q < v.size(); ++q) {
                Job *j = v[q];
                gempe_batch_entry_fill(stage + q * eb, &j->graph, j->d, j->plan,
                                       reinterpret_cast<float *>(j->base + j->J.X), j->iters, j->eta,
                                       reinterpret_cast<double *>(j->base + j->J.hist), j->L, j->base + j->J.ws,
                                       gempe_pair_params(&j->params), blocks, j->k0);
                blocks += j->plan.iter_blocks;
            }
            hipError_t e = hipMemcpyAsync(tables[c], stage, v.size() * eb, hipMemcpyHostToDevice, batch_stream);
            if (e != hipSuccess) {
                fatal = std::string("table upload: ") + hipGetErrorString(e);
                return false;
            }
            slot_tick[slot] = t;
            table_dirty[c] = false;
        } else {
            for (Job *j : v) blocks += j->plan.iter_blocks;
        }
        hipError_t e = gempe_launch_iter_batch(kDValues[c], tables[c], (int)v.size(), blocks, (int)t, batch_stream);
        if (e != hipSuccess) {
            fatal = std::string("tick launch: ") + hipGetErrorString(e);
            return false;
        }
    }
    if (!any) return false;
    const int ei = (int)(t % kTickEvents);
    hipError_t e = hipEventRecord(tick_ev[ei], batch_stream);
    if (e != hipSuccess) {
        fatal = std::string("tick event: ") + hipGetErrorString(e);
        return false;
    }
    ev_tick[ei] = t;
    pending_ticks.push_back(t);
    ++next_tick;
    {
        std::lock_guard<std::mutex> lk(mu);
        stats.ticks++;
    }
    return true;
}

// Retires completed ticks (in order); with block_one, waits for the oldest one.
void gempe_server_s::poll_ticks(bool block_one) {
    while (!pending_ticks.empty()) {
        const long long t = pending_ticks.front();
        hipEvent_t ev = tick_ev[t % kTickEvents];
        hipError_t q = block_one ? hipEventSynchronize(ev) : hipEventQuery(ev);
        block_one = false;
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
            fatal = std::string("tick wait: ") + hipGetErrorString(q);
            break;
        }
        pending_ticks.pop_front();
        done_tick = t;
    }
    // batched jobs whose finishing tick has executed (they may have left the tables already)
    size_t w = 0;
    for (size_t r = 0; r < batch_live.size(); ++r) {
        Job *j = batch_live[r];
        if (j->finish_tick <= done_tick) finish_job(j);
        else batch_live[w++] = j;
    }
    batch_live.resize(w);
}

void gempe_server_s::service_solo() {
    size_t w = 0;
    for (size_t r = 0; r < solo.size(); ++r) {
        Job *j = solo[r];
        // retire executed chunks
        while (!j->chunk_events.empty()) {
            hipError_t q = hipEventQuery(j->chunk_events.front());
            if (q == hipErrorNotReady) break;
            put_event(j->chunk_events.front());
            j->chunk_events.pop_front();
            if (q != hipSuccess) {
                fatal = std::string("solo wait: ") + hipGetErrorString(q);
                break;
            }
        }
        const bool all_enqueued = j->next_k > j->iters;
        if (all_enqueued && j->chunk_events.empty()) {
            finish_job(j);
            continue;  // leaves the solo list
        }
        // keep two chunks in flight
        while (!all_enqueued && j->chunk_events.size() < 2 && j->next_k <= j->iters) {
            const int kb = j->next_k, ke = std::min(j->iters + 1, kb + kSoloChunk);
            hipStream_t s = solo_streams[j->stream];
            hipError_t e = gempe_enqueue_embed_steps(&j->graph, j->d, j->plan, j->L, j->base + j->J.ws,
                                                     reinterpret_cast<float *>(j->base + j->J.X), j->iters, j->eta,
                                                     reinterpret_cast<double *>(j->base + j->J.hist), &j->params, s,
                                                     kb, ke);
            hipEvent_t ev = get_event();
            if (e == hipSuccess && ev) e = hipEventRecord(ev, s);
            if (e != hipSuccess || !ev) {
                fatal = std::string("solo enqueue: ") + (e != hipSuccess ? hipGetErrorString(e) : "no event");
                break;
            }
            j->chunk_events.push_back(ev);
            j->next_k = ke;
        }
        solo[w++] = j;
    }
    solo.resize(w);
}

void gempe_server_s::run() {
    (void)hipSetDevice(device);
    std::deque<Job *> waiting;  // released, not admitted (arrival order)
    while (true) {
        // 1. take submissions whose release time has come
        double next_release = -1.0;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop) break;
            const double tn = now();
            for (auto it = incoming.begin(); it != incoming.end();) {
                if ((*it)->release_s <= tn) {
                    waiting.push_back(*it);
                    it = incoming.erase(it);
                } else {
                    if (next_release < 0 || (*it)->release_s < next_release) next_release = (*it)->release_s;
                    ++it;
                }
            }
        }
        // 2. admission, arrival order with aged backfill
        {
            int running = 0;
            running += (int)batch_live.size();
            running += (int)solo.size();
            bool head_blocked = false;
            for (auto it = waiting.begin(); it != waiting.end();) {
                Job *j = *it;
                if (running >= max_jobs) break;
                if (j->batched && (int)batch[dclass_of(j->plan.D)].size() >= max_jobs) { ++it; continue; }
                if (head_blocked) break;
                if (admit_one(j)) {
                    it = waiting.erase(it);
                    ++running;
                    std::lock_guard<std::mutex> lk(mu);
                    if (running > stats.max_concurrent) stats.max_concurrent = running;
                } else {
                    if (now() - j->release_s > kAgingSeconds) head_blocked = true;
                    ++it;
                }
            }
        }
        // 3. device work
        bool ticked = false;
        bool have_batch = !batch_live.empty();
        if (have_batch) {
            poll_ticks(false);
            if ((long long)pending_ticks.size() >= kLookahead) poll_ticks(true);
            while ((long long)pending_ticks.size() < kLookahead && fatal.empty()) {
                if (!enqueue_tick()) break;
                ticked = true;
            }
            poll_ticks(false);
        }
        service_solo();
        if (!fatal.empty()) {
            // a runtime failure: fail everything that is running and stop scheduling
            (void)hipDeviceSynchronize();
            for (Job *j : batch_live) fail_job(j, GEMPE_ERR_HIP, fatal);
            batch_live.clear();
            for (int c = 0; c < kDClasses; ++c) batch[c].clear();
            for (Job *j : solo) fail_job(j, GEMPE_ERR_HIP, fatal);
            solo.clear();
            for (Job *j : waiting) fail_job(j, GEMPE_ERR_HIP, fatal);
            waiting.clear();
            std::lock_guard<std::mutex> lk(mu);
            for (Job *j : incoming) {
                j->state = GEMPE_JOB_FAILED;
                j->status = GEMPE_ERR_HIP;
                j->error = fatal;
                stats.failed++;
            }
            incoming.clear();
            cv_done.notify_all();
            fatal.clear();
        }
        // 4. idle: sleep until a submission, a release time, or briefly while work is in flight
        bool busy = have_batch || !solo.empty();
        if (!ticked) {
            std::unique_lock<std::mutex> lk(mu);
            if (stop) break;
            double wait_s = busy ? 50e-6 : (waiting.empty() ? 0.05 : 1e-3);
            if (next_release >= 0) wait_s = std::min(wait_s, std::max(0.0, next_release - now()));
            cv_submit.wait_for(lk, std::chrono::duration<double>(wait_s));
        }
    }
    // shutdown: let queued device work finish, then drop everything still pending
    (void)hipStreamSynchronize(batch_stream);
    for (auto &s : solo_streams) (void)hipStreamSynchronize(s);
    for (Job *j : solo)
        for (hipEvent_t e : j->chunk_events) put_event(e);
    std::lock_guard<std::mutex> lk(mu);
    for (auto &kv : jobs) {
        Job *j = kv.second.get();
        if (j->state == GEMPE_JOB_QUEUED || j->state == GEMPE_JOB_RUNNING) {
            j->state = GEMPE_JOB_FAILED;
            j->status = GEMPE_ERR_ARG;
            j->error = "server destroyed before the job finished";
        }
    }
    cv_done.notify_all();
}

// ======================================================================================
// C ABI
// ======================================================================================

extern "C" size_t gempe_job_footprint(int32_t n, int64_t nnz, int32_t d, int32_t iters, const gempe_params *p) {
    if (gempe_check_problem(n, d, p, "job_footprint") != GEMPE_OK) return 0;
    if (nnz < 0 || iters < 0) return 0;
    SweepPlan plan;
    WsLayout L;
    job_plan(n, nnz, d, *p, plan, L);
    if (gempe_check_plan(plan, "job_footprint") != GEMPE_OK) return 0;
    return job_layout(n, nnz, d, iters, L).total;
}

extern "C" gempe_status gempe_server_create(size_t budget_bytes, int32_t max_jobs, gempe_server *out) {
    if (!out) return gempe_fail(GEMPE_ERR_ARG, "server_create: out is NULL");
    *out = nullptr;
    if (budget_bytes < 4096) return gempe_fail(GEMPE_ERR_ARG, "server_create: budget below 4 KiB");
    if (max_jobs < 1 || max_jobs > 4096) return gempe_fail(GEMPE_ERR_ARG, "server_create: max_jobs in [1, 4096]");
    std::unique_ptr<gempe_server_s> s(new gempe_server_s());
    s->budget = budget_bytes & ~size_t(255);
    s->max_jobs = max_jobs;
    GEMPE_HIP_TRY(hipGetDevice(&s->device));
    auto cleanup = [&]() {
        if (s->block) (void)hipFree(s->block);
        for (auto &t : s->tables)
            if (t) (void)hipFree(t);
        if (s->pinned) (void)hipHostFree(s->pinned);
        if (s->batch_stream) (void)hipStreamDestroy(s->batch_stream);
        if (s->xfer_stream) (void)hipStreamDestroy(s->xfer_stream);
        for (auto &st : s->solo_streams)
            if (st) (void)hipStreamDestroy(st);
        for (auto &e : s->tick_ev)
            if (e) (void)hipEventDestroy(e);
    };
    hipError_t e = hipMalloc(&s->block, s->budget);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->block = nullptr;
        cleanup();
        return gempe_fail(GEMPE_ERR_NOMEM, std::string("server_create: budget block: ") + hipGetErrorString(e));
    }
    s->arena.reset(s->budget, 256);
    const size_t eb = gempe_batch_entry_bytes();
    for (auto &t : s->tables) {
        if ((e = hipMalloc(&t, (size_t)max_jobs * eb)) != hipSuccess) break;
    }
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&s->pinned), (size_t)kTableSlots * (size_t)max_jobs * eb,
                          hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->batch_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->xfer_stream, hipStreamNonBlocking);
    for (auto &st : s->solo_streams)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (auto &ev : s->tick_ev)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return gempe_fail(GEMPE_ERR_HIP, std::string("server_create: ") + hipGetErrorString(e));
    }
    for (auto &t : s->slot_tick) t = -1;
    s->t0 = std::chrono::steady_clock::now();
    gempe_server_s *raw = s.get();
    s->thread = std::thread([raw]() { raw->run(); });
    *out = s.release();
    return GEMPE_OK;
}

extern "C" gempe_status gempe_server_submit(gempe_server s, const gempe_job_desc *jd, int64_t *job_id) {
    if (!s || !jd) return gempe_fail(GEMPE_ERR_ARG, "server_submit: null argument");
    gempe_status st = gempe_graph_check_args(jd->n, jd->nnz, jd->row_ptr, jd->col_idx, "server_submit");
    if (st != GEMPE_OK) return st;
    if ((st = gempe_check_problem(jd->n, jd->d, &jd->params, "server_submit")) != GEMPE_OK) return st;
    if (jd->iters < 0) return gempe_fail(GEMPE_ERR_ARG, "server_submit: iters must be >= 0");
    if (!(std::isfinite(jd->eta) && jd->eta > 0.0f))
        return gempe_fail(GEMPE_ERR_ARG, "server_submit: eta must be finite and > 0");
    if (!jd->X0 || !jd->X_out) return gempe_fail(GEMPE_ERR_ARG, "server_submit: X0 and X_out are required");
    if (!std::isfinite(jd->release_s)) return gempe_fail(GEMPE_ERR_ARG, "server_submit: release_s must be finite");
    std::unique_ptr<Job> j(new Job());
    j->n = jd->n;
    j->d = jd->d;
    j->nnz = jd->nnz;
    j->iters = jd->iters;
    j->eta = jd->eta;
    j->params = jd->params;
    j->X_out = jd->X_out;
    j->hist_out = jd->loss_hist;
    job_plan(j->n, j->nnz, j->d, j->params, j->plan, j->L);
    if ((st = gempe_check_plan(j->plan, "server_submit")) != GEMPE_OK) return st;
    j->J = job_layout(j->n, j->nnz, j->d, j->iters, j->L);
    j->footprint = j->J.total;
    j->batched = j->plan.persist && j->params.precision == GEMPE_FP32 && dclass_of(j->plan.D) >= 0;
    if (j->footprint > s->arena.capacity()) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.rejected++;
        return gempe_fail(GEMPE_ERR_NOMEM, "server_submit: job needs " + std::to_string(j->footprint) +
                                               " bytes, the budget is " + std::to_string(s->arena.capacity()));
    }
    j->row_ptr.assign(jd->row_ptr, jd->row_ptr + (size_t)jd->n + 1);
    if (jd->nnz > 0) j->col_idx.assign(jd->col_idx, jd->col_idx + jd->nnz);
    j->X0.assign(jd->X0, jd->X0 + (size_t)jd->n * (size_t)jd->d);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return gempe_fail(GEMPE_ERR_ARG, "server_submit: server is shutting down");
    j->id = s->next_id++;
    j->release_s = std::max(jd->release_s, s->now());  // arrival: never before the submission
    Job *raw = j.get();
    s->jobs[raw->id] = std::move(j);
    s->incoming.push_back(raw);
    s->stats.submitted++;
    if (job_id) *job_id = raw->id;
    s->cv_submit.notify_all();
    return GEMPE_OK;
}

namespace {
void fill_info(const Job *j, gempe_job_info *info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->state = j->state;
    info->status = j->status;
    info->batched = j->batched ? 1 : 0;
    info->release_s = j->release_s;
    info->admit_s = j->admit_s;
    info->done_s = j->done_s;
    info->footprint = j->footprint;
}
}  // namespace

extern "C" gempe_status gempe_server_query(gempe_server s, int64_t job_id, gempe_job_info *info) {
    if (!s || !info) return gempe_fail(GEMPE_ERR_ARG, "server_query: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return gempe_fail(GEMPE_ERR_ARG, "server_query: unknown job id");
    fill_info(it->second.get(), info);
    if (it->second->state == GEMPE_JOB_FAILED) gempe_set_error(it->second->error);
    return GEMPE_OK;
}

extern "C" gempe_status gempe_server_wait(gempe_server s, int64_t job_id, double timeout_s, gempe_job_info *info) {
    if (!s) return gempe_fail(GEMPE_ERR_ARG, "server_wait: null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto finished = [&]() {
        if (job_id >= 0) {
            auto it = s->jobs.find(job_id);
            return it == s->jobs.end() || it->second->state >= GEMPE_JOB_DONE;
        }
        return s->stats.done + s->stats.failed >= s->stats.submitted;
    };
    if (job_id >= 0 && s->jobs.find(job_id) == s->jobs.end())
        return gempe_fail(GEMPE_ERR_ARG, "server_wait: unknown job id");
    bool ok = true;
    if (timeout_s < 0) {
        s->cv_done.wait(lk, finished);
    } else {
        ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished);
    }
    if (!ok) return gempe_fail(GEMPE_ERR_TIMEOUT, "server_wait: timed out");
    if (job_id >= 0) {
        Job *j = s->jobs[job_id].get();
        fill_info(j, info);
        if (j->state == GEMPE_JOB_FAILED) gempe_set_error(j->error);
    }
    return GEMPE_OK;
}

extern "C" gempe_status gempe_server_get_stats(gempe_server s, gempe_server_stats *out) {
    if (!s || !out) return gempe_fail(GEMPE_ERR_ARG, "server_get_stats: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->budget_bytes = (int64_t)s->arena.capacity();
    return GEMPE_OK;
}

extern "C" gempe_status gempe_server_destroy(gempe_server s) {
    if (!s) return gempe_fail(GEMPE_ERR_ARG, "server_destroy: null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_submit.notify_all();
    }
    if (s->thread.joinable()) s->thread.join();
    (void)hipFree(s->block);
    for (auto &t : s->tables) (void)hipFree(t);
    (void)hipHostFree(s->pinned);
    (void)hipStreamDestroy(s->batch_stream);
    (void)hipStreamDestroy(s->xfer_stream);
    for (auto &st : s->solo_streams) (void)hipStreamDestroy(st);
    for (auto &e : s->tick_ev) (void)hipEventDestroy(e);
    for (auto &e : s->event_pool) (void)hipEventDestroy(e);
    delete s;
    return GEMPE_OK;
}
