// Serving loop: continuous batching of PIR queries over resident databases.
//
// The paper's parallelization goal is to cut the servers' online response
// latency under concurrent demand, answering queries in batches over a
// database kept in GPU memory (Section 5.2; Figure 3 reports end-to-end
// delay against the number of users).  This file is the host runtime around
// the Answer kernels that does that on one GPU:
//
// * every registered database owns `slots_per_db` slots: a stream, pinned
//   host staging for queries and answers, device buffers and a workspace
//   sized for the largest batch;
// * a scheduler thread turns each database's queue into batches as soon as
//   one of its slots is free: whatever arrived while earlier batches were on
//   the GPU joins the next batch (continuous batching), up to `max_batch`;
// * admission is by memory: a batch is launched only if its device
//   footprint (queries, answers, workspace) fits in what `mem_budget_bytes`
//   leaves after the batches already in flight; otherwise it waits, and a
//   smaller batch is formed when that fits;
// * batch sizes are rounded up to powers of two; for every (slot, size) the
//   copy-in and kernels were captured once into a HIP graph at start, so a
//   launch is one graph replay (padded queries are ignored), then an event
//   marking the kernels done and the copy-out of the answers;
// * batches for different databases run on different streams and overlap
//   on the device; with max_inflight set, at most that many batches have
//   kernels pending (a batch that only copies its answers out does not
//   count), and each launch goes to the database whose oldest request has
//   waited longest;
// * a poller thread completes batches in any order, copies each answer to
//   its caller's buffer and records the latency from the scheduled arrival
//   time (open-loop: queueing delay is included).
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "qpir_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               Clock::now().time_since_epoch()).count();
}

enum ReqState : int { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct Req {
    uint32_t db = 0;
    const uint32_t* h_q = nullptr;
    uint32_t* h_ans = nullptr;
    uint64_t t_arrival = 0, t_done = 0;
    std::atomic<int> state{kQueued};
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint32_t* h_flag = nullptr;   // pinned word: 1 once a large batch's kernels have run
    uint32_t* d_flag = nullptr;   // the same word as the device addresses it
    uint32_t* h_Q = nullptr;   // pinned, max_batch x C (query-major)
    uint32_t* h_O = nullptr;   // pinned, max_batch x R (answer-major)
    uint32_t* d_Q = nullptr;
    uint32_t* d_O = nullptr;
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<hipGraph_t> graph;
    std::vector<hipGraphExec_t> exec;
    std::vector<Req*> batch;
    uint32_t size = 0;         // padded batch size in flight
    uint64_t cost = 0;         // budget bytes held while in flight
    uint32_t db = 0;           // owning database index
    bool busy = false;
    bool computing = false;    // launched, kernels not yet finished
};

struct DbQueue {
    pir_db_t* db = nullptr;
    uint64_t R = 0, C = 0;
    std::deque<Req*> queue;
    std::vector<Slot> slots;
    bool paused = false;
    uint32_t inflight = 0;
};

// One word to host memory, visible to the host once the kernels before it
// on the stream have finished.
__global__ void k_raise_flag(uint32_t* flag) {
    if (threadIdx.x == 0) __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

uint32_t log2_floor(uint32_t x) {
    uint32_t k = 0;
    while ((2u << k) <= x) ++k;
    return k;
}

uint32_t pow2_ceil(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

struct pir_server {
    pir_server_config cfg{};
    int device = -1;
    std::vector<DbQueue> dbs;
    std::deque<Req> reqs;               // index = ticket
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::thread sched, poller;
    std::vector<Slot*> inflight;
    bool started = false, stopping = false;
    pir_status fault = PIR_OK;
    uint64_t used = 0, peak = 0;
    uint64_t alloc_bytes = 0;           // device memory of the slots (buffers, workspaces)
    uint64_t n_batches = 0, n_batched = 0, n_done = 0, n_failed = 0, n_rejected = 0;
    uint32_t n_computing = 0;           // batches whose kernels have not finished

    uint64_t batch_cost(const DbQueue& d, uint32_t size) const {
        const size_t ws = size == 1 ? pir_workspace_bytes(d.db, 0) : pir_workspace_bytes(d.db, size);
        return (uint64_t)size * (d.R + d.C) * 4u + ws;
    }

    // Batches of at least kDirectCopies queries move their queries in and
    // answers out with plain stream copies around the graph of kernels
    // (the DMA engines then overlap them with other batches' kernels);
    // smaller ones keep both copies inside the graph, one launch in all.
    static constexpr uint32_t kDirectCopies = 8;

    pir_status copy_in(DbQueue& d, Slot& s, uint32_t size) {
        return hipMemcpyAsync(s.d_Q, s.h_Q, (size_t)size * d.C * 4, hipMemcpyHostToDevice,
                              s.stream) == hipSuccess ? PIR_OK : PIR_ERR_DEVICE;
    }

    pir_status copy_out(DbQueue& d, Slot& s, uint32_t size) {
        return hipMemcpyAsync(s.h_O, s.d_O, (size_t)size * d.R * 4, hipMemcpyDeviceToHost,
                              s.stream) == hipSuccess ? PIR_OK : PIR_ERR_DEVICE;
    }

    // The work captured per (slot, size); with `copies`, the two copies too.
    pir_status enqueue(DbQueue& d, Slot& s, uint32_t size, bool copies) {
        hipStream_t st = s.stream;
        pir_status r = copies ? copy_in(d, s, size) : PIR_OK;
        if (r != PIR_OK) return r;
        r = size == 1 ? pir_answer(d.db, s.d_Q, s.d_O, s.d_ws, s.ws_bytes, st)
                      : pir_answer_batch_qmajor(d.db, s.d_Q, size, s.d_O, s.d_ws, s.ws_bytes, st);
        if (r != PIR_OK) return r;
        if (copies) return copy_out(d, s, size);
        // Kernels done, answers not yet copied out: raise the slot's host
        // flag, so the scheduler stops counting the batch against
        // max_inflight.  (A batch with its copies in the graph counts until
        // it completes; it is small, and skipping this launch keeps its
        // latency down.)
        k_raise_flag<<<1, 64, 0, st>>>(s.d_flag);
        return hipGetLastError() == hipSuccess ? PIR_OK : PIR_ERR_DEVICE;
    }

    // One batch: its copies and kernels (a graph replay or direct launches),
    // then the event the poller waits for.
    pir_status launch(DbQueue& d, Slot& s, uint32_t size) {
        const bool direct = size >= kDirectCopies;
        pir_status r = PIR_OK;
        if (cfg.use_graphs) {
            if (direct && (r = copy_in(d, s, size)) != PIR_OK) return r;
            if (hipGraphLaunch(s.exec[log2_floor(size)], s.stream) != hipSuccess)
                return PIR_ERR_DEVICE;
            if (direct && (r = copy_out(d, s, size)) != PIR_OK) return r;
        } else if ((r = enqueue(d, s, size, true)) != PIR_OK) {
            return r;
        }
        return hipEventRecord(s.done, s.stream) == hipSuccess ? PIR_OK : PIR_ERR_DEVICE;
    }

    pir_status setup_slot(DbQueue& d, Slot& s) {
        const uint32_t mb = cfg.max_batch;
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
            return PIR_ERR_DEVICE;
        if (hipHostMalloc((void**)&s.h_Q, (size_t)mb * d.C * 4, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&s.h_O, (size_t)mb * d.R * 4, hipHostMallocDefault) != hipSuccess)
            return PIR_ERR_NO_MEMORY;
        if (hipHostMalloc((void**)&s.h_flag, 64, hipHostMallocDefault) != hipSuccess)
            return PIR_ERR_NO_MEMORY;
        __atomic_store_n(s.h_flag, 0u, __ATOMIC_RELAXED);
        if (hipHostGetDevicePointer((void**)&s.d_flag, s.h_flag, 0) != hipSuccess)
            return PIR_ERR_DEVICE;
        memset(s.h_Q, 0, (size_t)mb * d.C * 4);
        // Every power-of-two size the slot launches (small batches take a
        // different kernel path with its own workspace need).
        s.ws_bytes = pir_workspace_bytes(d.db, 0);
        for (uint32_t b = 2; b <= mb; b *= 2) s.ws_bytes = std::max(s.ws_bytes, pir_workspace_bytes(d.db, b));
        if (hipMalloc((void**)&s.d_Q, (size_t)mb * d.C * 4) != hipSuccess ||
            hipMalloc((void**)&s.d_O, (size_t)mb * d.R * 4) != hipSuccess ||
            (s.ws_bytes && hipMalloc(&s.d_ws, s.ws_bytes) != hipSuccess))
            return PIR_ERR_NO_MEMORY;
        alloc_bytes += (uint64_t)mb * (d.C + d.R) * 4 + s.ws_bytes;
        if (hipMemset(s.d_Q, 0, (size_t)mb * d.C * 4) != hipSuccess) return PIR_ERR_DEVICE;
        const uint32_t nb = log2_floor(mb) + 1;
        s.graph.assign(nb, nullptr);
        s.exec.assign(nb, nullptr);
        if (!cfg.use_graphs) return PIR_OK;
        for (uint32_t k = 0; k < nb; ++k) {
            if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return PIR_ERR_DEVICE;
            pir_status r = enqueue(d, s, 1u << k, (1u << k) < kDirectCopies);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(s.stream, &g);
            if (r != PIR_OK) return r;
            if (e != hipSuccess || !g) return PIR_ERR_DEVICE;
            s.graph[k] = g;
            if (hipGraphInstantiate(&s.exec[k], g, nullptr, nullptr, 0) != hipSuccess)
                return PIR_ERR_DEVICE;
            // One replay now, so first requests do not pay for lazy setup.
            if (hipGraphLaunch(s.exec[k], s.stream) != hipSuccess) return PIR_ERR_DEVICE;
        }
        // Likewise one round of the stream copies of large batches.
        if (mb >= kDirectCopies) {
            pir_status r = copy_in(d, s, mb);
            if (r == PIR_OK) r = copy_out(d, s, mb);
            if (r != PIR_OK) return r;
        }
        return hipStreamSynchronize(s.stream) == hipSuccess ? PIR_OK : PIR_ERR_DEVICE;
    }

    void release_slot(Slot& s) {
        for (auto e : s.exec) if (e) (void)hipGraphExecDestroy(e);
        for (auto g : s.graph) if (g) (void)hipGraphDestroy(g);
        s.exec.clear();
        s.graph.clear();
        if (s.d_ws) (void)hipFree(s.d_ws);
        if (s.d_Q) (void)hipFree(s.d_Q);
        if (s.d_O) (void)hipFree(s.d_O);
        if (s.h_Q) (void)hipHostFree(s.h_Q);
        if (s.h_O) (void)hipHostFree(s.h_O);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.h_flag) (void)hipHostFree(s.h_flag);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        s = Slot();
    }

    // Fail every request of a batch (device error); caller holds the lock.
    void fail_batch(Slot& s) {
        for (Req* r : s.batch) {
            r->state.store(kFailed, std::memory_order_release);
            ++n_failed;
        }
        s.batch.clear();
    }

    // Free slot of a database, or null.
    static Slot* free_slot(DbQueue& d) {
        for (auto& x : d.slots)
            if (!x.busy) return &x;
        return nullptr;
    }

    void scheduler_loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        std::vector<char> blocked;
        for (;;) {
            bool launched = false;
            const size_t nd = dbs.size();
            blocked.assign(nd, 0);
            // Launch while the device takes more batches: each time, the
            // database whose oldest request has waited longest, with
            // everything it has queued (up to max_batch and the budget).
            while (fault == PIR_OK && (cfg.max_inflight == 0 || n_computing < cfg.max_inflight)) {
                size_t pick = nd;
                for (size_t i = 0; i < nd; ++i) {
                    DbQueue& c = dbs[i];
                    if (c.queue.empty() || c.paused || blocked[i] || !free_slot(c)) continue;
                    if (pick == nd || c.queue.front()->t_arrival < dbs[pick].queue.front()->t_arrival)
                        pick = i;
                }
                if (pick == nd) break;
                DbQueue& d = dbs[pick];
                Slot* s = free_slot(d);
                uint32_t n = (uint32_t)std::min<size_t>(d.queue.size(), cfg.max_batch);
                uint32_t size = pow2_ceil(n);
                while (size > 1 && used + batch_cost(d, size) > cfg.mem_budget_bytes) size >>= 1;
                if (used + batch_cost(d, size) > cfg.mem_budget_bytes) {   // wait for memory
                    blocked[pick] = 1;
                    continue;
                }
                n = std::min(n, size);
                s->batch.assign(d.queue.begin(), d.queue.begin() + n);
                d.queue.erase(d.queue.begin(), d.queue.begin() + n);
                s->busy = true;
                s->size = size;
                s->cost = batch_cost(d, size);
                used += s->cost;
                peak = std::max(peak, used);
                ++d.inflight;
                ++n_batches;
                n_batched += n;
                for (Req* r : s->batch) r->state.store(kRunning, std::memory_order_relaxed);
                lk.unlock();
                // Pack the queries (query-major rows of C words) and launch.
                for (uint32_t b = 0; b < n; ++b)
                    memcpy(s->h_Q + (size_t)b * d.C, s->batch[b]->h_q, d.C * 4);
                __atomic_store_n(s->h_flag, 0u, __ATOMIC_RELAXED);   // raised by this launch
                const pir_status st = launch(d, *s, size);
                lk.lock();
                if (st != PIR_OK) {
                    fault = st;
                    fail_batch(*s);
                    s->busy = false;
                    used -= s->cost;
                    --d.inflight;
                    cv_done.notify_all();
                    break;
                }
                s->computing = true;
                ++n_computing;
                inflight.push_back(s);
                launched = true;
                cv_done.notify_all();
            }
            if (fault != PIR_OK) {   // fail whatever is queued
                for (auto& d : dbs) {
                    for (Req* r : d.queue) {
                        r->state.store(kFailed, std::memory_order_release);
                        ++n_failed;
                    }
                    d.queue.clear();
                }
                cv_done.notify_all();
            }
            if (stopping && inflight.empty()) {
                bool empty = true;
                for (auto& d : dbs) empty = empty && d.queue.empty();
                if (empty || fault != PIR_OK) break;
            }
            if (!launched) cv_sched.wait(lk);
        }
    }

    // The batch's kernels have finished (its answers may still be copying
    // out): it no longer counts against max_inflight.  Caller holds the lock.
    void kernels_done(Slot& s) {
        if (!s.computing) return;
        s.computing = false;
        --n_computing;
        cv_sched.notify_all();
    }

    void complete(Slot* s) {
        DbQueue* d = &dbs[s->db];
        const uint64_t t = now_ns();
        for (size_t b = 0; b < s->batch.size(); ++b) {
            Req* r = s->batch[b];
            if (r->h_ans) memcpy(r->h_ans, s->h_O + b * d->R, d->R * 4);
            r->t_done = t;
            r->state.store(kDone, std::memory_order_release);
        }
        std::lock_guard<std::mutex> lk(mu);
        n_done += s->batch.size();
        s->batch.clear();
        kernels_done(*s);
        s->busy = false;
        used -= s->cost;
        --d->inflight;
        inflight.erase(std::find(inflight.begin(), inflight.end(), s));
        cv_sched.notify_all();
        cv_done.notify_all();
    }

    void poller_loop() {
        (void)hipSetDevice(device);
        std::vector<Slot*> watch;
        uint64_t idle_since = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_done.wait(lk, [&] { return !inflight.empty() || (stopping && sched_done); });
                if (inflight.empty() && stopping && sched_done) break;
                watch = inflight;
            }
            bool any = false;
            for (Slot* s : watch) {
                // Only this thread clears `computing` once the slot is in flight.
                if (s->computing && __atomic_load_n(s->h_flag, __ATOMIC_ACQUIRE) == 1u) {
                    std::lock_guard<std::mutex> lk(mu);
                    kernels_done(*s);
                    any = true;
                }
                const hipError_t e = hipEventQuery(s->done);
                if (e == hipSuccess) {
                    complete(s);
                    any = true;
                } else if (e != hipErrorNotReady) {
                    std::lock_guard<std::mutex> lk(mu);
                    fault = PIR_ERR_DEVICE;
                    fail_batch(*s);
                    kernels_done(*s);
                    s->busy = false;
                    used -= s->cost;
                    --dbs[s->db].inflight;
                    inflight.erase(std::find(inflight.begin(), inflight.end(), s));
                    cv_sched.notify_all();
                    cv_done.notify_all();
                }
            }
            // Batches are in flight: yield-spin for low completion latency
            // for up to 2 ms after the last completion, longer than one
            // query's scan of a 2 GiB database (about 0.33 ms), then back
            // off to 20 us sleeps, which overshoot by tens of microseconds.
            // (2000 q/s on the eight regional databases: p99 0.44-0.45 ms
            // with a 0.2 ms spin, 0.42 ms with 2 ms.)
            if (any) {
                idle_since = 0;
            } else {
                const uint64_t t = now_ns();
                if (!idle_since) idle_since = t;
                if (t - idle_since < 2000000) std::this_thread::yield();
                else std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        }
    }

    bool sched_done = false;
};

extern "C" {

pir_status pir_server_create(const pir_server_config* cfg, pir_server_t** out) {
    if (!cfg || !out) return PIR_ERR_INVALID_ARG;
    if (cfg->max_batch == 0 || cfg->max_batch > 1024 || (cfg->max_batch & (cfg->max_batch - 1)) ||
        cfg->slots_per_db == 0 || cfg->slots_per_db > 16 || cfg->mem_budget_bytes == 0)
        return PIR_ERR_SHAPE;
    pir_server_t* s = new (std::nothrow) pir_server_t();
    if (!s) return PIR_ERR_NO_MEMORY;
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return PIR_ERR_DEVICE;
    }
    *out = s;
    return PIR_OK;
}

pir_status pir_server_add_db(pir_server_t* s, pir_db_t* db, uint32_t* db_index) {
    if (!s || !db_ok(db) || !db_index) return PIR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started) return PIR_ERR_INVALID_ARG;
    if (db->device != s->device) return PIR_ERR_INVALID_ARG;
    DbQueue d;
    d.db = db;
    d.R = db->rows;
    d.C = db->cols;
    s->dbs.push_back(std::move(d));
    *db_index = (uint32_t)(s->dbs.size() - 1);
    return PIR_OK;
}

pir_status pir_server_start(pir_server_t* s) {
    if (!s) return PIR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started || s->dbs.empty()) return PIR_ERR_INVALID_ARG;
    for (auto& d : s->dbs) {
        if (s->batch_cost(d, 1) > s->cfg.mem_budget_bytes) return PIR_ERR_NO_MEMORY;
        d.slots.resize(s->cfg.slots_per_db);
        for (auto& sl : d.slots) {
            sl.db = (uint32_t)(&d - &s->dbs[0]);
            pir_status st = s->setup_slot(d, sl);
            if (st != PIR_OK) {
                for (auto& dd : s->dbs)
                    for (auto& x : dd.slots) s->release_slot(x);
                return st;
            }
        }
    }
    s->started = true;
    s->sched = std::thread([s] { s->scheduler_loop(); });
    s->poller = std::thread([s] { s->poller_loop(); });
    return PIR_OK;
}

pir_status pir_server_submit(pir_server_t* s, uint32_t db_index, const uint32_t* h_q,
                             uint32_t* h_answer, uint64_t t_arrival_ns, uint64_t* ticket) {
    if (!s || !h_q || !ticket) return PIR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->started || s->stopping) return PIR_ERR_INVALID_ARG;
    if (db_index >= s->dbs.size()) return PIR_ERR_INVALID_ARG;
    if (s->fault != PIR_OK) return s->fault;
    DbQueue& d = s->dbs[db_index];
    if (s->cfg.max_queue && d.queue.size() >= s->cfg.max_queue) {
        ++s->n_rejected;
        return PIR_ERR_BUSY;
    }
    s->reqs.emplace_back();
    Req& r = s->reqs.back();
    r.db = db_index;
    r.h_q = h_q;
    r.h_ans = h_answer;
    r.t_arrival = t_arrival_ns ? t_arrival_ns : now_ns();
    *ticket = s->reqs.size() - 1;
    d.queue.push_back(&r);
    s->cv_sched.notify_all();
    return PIR_OK;
}

uint64_t pir_server_now_ns(void) { return now_ns(); }

pir_status pir_server_wait(pir_server_t* s, uint64_t ticket, uint64_t timeout_ns) {
    if (!s) return PIR_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket >= s->reqs.size()) return PIR_ERR_INVALID_ARG;
    Req& r = s->reqs[ticket];
    auto done = [&] { return r.state.load(std::memory_order_acquire) >= kDone; };
    if (timeout_ns == UINT64_MAX) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
        return PIR_ERR_TIMEOUT;
    }
    return r.state.load(std::memory_order_acquire) == kDone ? PIR_OK : PIR_ERR_DEVICE;
}

pir_status pir_server_drain(pir_server_t* s) {
    if (!s) return PIR_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    // Requests held by a paused database finish only after its resume, so
    // waiting for them here would block until another thread resumes it.
    auto held = [&] {
        for (auto& d : s->dbs)
            if (d.paused && !d.queue.empty()) return true;
        return false;
    };
    s->cv_done.wait(lk, [&] { return s->n_done + s->n_failed >= s->reqs.size() || held(); });
    if (s->n_done + s->n_failed < s->reqs.size()) return PIR_ERR_BUSY;
    return s->n_failed ? PIR_ERR_DEVICE : PIR_OK;
}

pir_status pir_server_pause_db(pir_server_t* s, uint32_t db_index) {
    if (!s) return PIR_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (db_index >= s->dbs.size()) return PIR_ERR_INVALID_ARG;
    DbQueue& d = s->dbs[db_index];
    d.paused = true;
    s->cv_done.notify_all();   // a drain in progress stops waiting on this queue
    s->cv_done.wait(lk, [&] { return d.inflight == 0; });
    return PIR_OK;
}

pir_status pir_server_resume_db(pir_server_t* s, uint32_t db_index) {
    if (!s) return PIR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (db_index >= s->dbs.size()) return PIR_ERR_INVALID_ARG;
    s->dbs[db_index].paused = false;
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
    return PIR_OK;
}

pir_status pir_server_stats_get(pir_server_t* s, pir_server_stats* out) {
    if (!s || !out) return PIR_ERR_INVALID_ARG;
    std::vector<uint64_t> lat;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        memset(out, 0, sizeof(*out));
        out->submitted = s->reqs.size();
        out->completed = s->n_done;
        out->failed = s->n_failed;
        out->rejected = s->n_rejected;
        out->batches = s->n_batches;
        out->batched_queries = s->n_batched;
        out->budget_bytes = s->cfg.mem_budget_bytes;
        out->peak_inflight_bytes = s->peak;
        out->device_bytes = s->alloc_bytes;
        lat.reserve(s->n_done);
        for (auto& r : s->reqs)
            if (r.state.load(std::memory_order_acquire) == kDone) lat.push_back(r.t_done - r.t_arrival);
    }
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto q = [&](double f) { return lat[std::min(lat.size() - 1, (size_t)(f * lat.size()))]; };
        out->p50_ns = q(0.50);
        out->p99_ns = q(0.99);
        out->max_ns = lat.back();
    }
    return PIR_OK;
}

pir_status pir_server_latencies(pir_server_t* s, uint64_t first, uint64_t count, uint64_t* out_ns) {
    if (!s || (!out_ns && count)) return PIR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (first + count > s->reqs.size()) return PIR_ERR_SHAPE;
    for (uint64_t i = 0; i < count; ++i) {
        const Req& r = s->reqs[first + i];
        out_ns[i] = r.state.load(std::memory_order_acquire) == kDone ? r.t_done - r.t_arrival : 0;
    }
    return PIR_OK;
}

pir_status pir_server_replay(pir_server_t* s, uint64_t n, const uint64_t* offsets_ns,
                             const uint32_t* db_index, const uint32_t* const* h_q,
                             uint32_t* const* h_answer, uint64_t* first_ticket) {
    if (!s || !offsets_ns || !db_index || !h_q || !first_ticket) return PIR_ERR_INVALID_ARG;
    const uint64_t t0 = now_ns();
    bool first = true;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t due = t0 + offsets_ns[i];
        for (;;) {   // sleep until ~100 us before the arrival, then spin
            const uint64_t t = now_ns();
            if (t >= due) break;
            if (due - t > 150000) std::this_thread::sleep_for(std::chrono::nanoseconds(due - t - 100000));
        }
        uint64_t tk = 0;
        pir_status st = pir_server_submit(s, db_index[i], h_q[i], h_answer ? h_answer[i] : nullptr,
                                          due, &tk);
        if (st == PIR_ERR_BUSY) continue;   // counted as rejected
        if (st != PIR_OK) return st;
        if (first) {
            *first_ticket = tk;
            first = false;
        }
    }
    if (first) *first_ticket = UINT64_MAX;
    return PIR_OK;
}

pir_status pir_server_destroy(pir_server_t* s) {
    if (!s) return PIR_OK;
    pir_status st = PIR_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (auto& d : s->dbs) d.paused = false;   // held requests finish too
        s->cv_sched.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->sched_done = true;
        s->cv_done.notify_all();
    }
    if (s->poller.joinable()) s->poller.join();
    if (s->fault != PIR_OK) st = s->fault;
    for (auto& d : s->dbs)
        for (auto& x : d.slots) {
            if (x.stream) (void)hipStreamSynchronize(x.stream);
            s->release_slot(x);
        }
    delete s;
    return st;
}

}  // extern "C"
