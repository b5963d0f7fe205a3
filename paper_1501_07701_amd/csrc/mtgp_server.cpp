// mtgp_server.cpp -- continuous-batching request loop over resident streams.
//
// All stream states stay in device memory (the paper keeps each block's
// generator state in global memory between launches, Sec. 2).  Requests
// (stream, count, dtype) are
//   1. queued (thread-safe submit),
//   2. admitted in submission order while their output bytes fit the
//      caller's device pool; at most one request per stream is in flight,
//      and consecutive queued requests of one stream are fused into one
//      work item over one contiguous pool range, so per-stream order is the
//      submission order,
//   3. launched as a batch through the persistent kernel on one of several
//      HIP streams, so batches admitted later overlap batches still running,
//   4. completed item by item: the kernel raises a per-item flag in pinned
//      host memory as soon as the item's outputs and state are stored, so a
//      short request is not held behind a long one in the same batch.
// Results stay in the pool until the client releases them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mtgp.h"
#include "mtgp_host.hpp"
#include "mtgp_internal.hpp"

namespace mtgp {

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { R_QUEUED, R_ADMITTED, R_LAUNCHED, R_DONE, R_FAILED, R_CANCELED };

struct Req {
    uint64_t ticket = 0;
    int32_t stream = 0;
    uint64_t count = 0;
    int dtype = 0;
    uint64_t off = 0;       // byte offset in the pool
    uint64_t bytes = 0;
    ReqState state = R_QUEUED;
    uint64_t t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    int slot = -1;
    int item = -1;          // index in the slot's launched item list
};

// First-fit allocator over [0, size): ranges start 256-byte aligned;
// frees are exact, so one allocation may be returned in several pieces.
class Pool {
   public:
    explicit Pool(uint64_t size) : size_(size) { free_[0] = size; }
    bool alloc(uint64_t bytes, uint64_t *off) {
        if (bytes == 0) bytes = 1;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const uint64_t start = it->first, len = it->second;
            const uint64_t al = (start + 255) / 256 * 256;
            if (al + bytes > start + len) continue;
            free_.erase(it);
            if (al > start) free_[start] = al - start;
            if (al + bytes < start + len) free_[al + bytes] = start + len - (al + bytes);
            used_ += bytes;
            *off = al;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        if (bytes == 0) return;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }

   private:
    uint64_t size_, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Slot {
    hipStream_t hs = nullptr;
    hipEvent_t done = nullptr;
    void *d_ws = nullptr;          // work list + counter, carved from the pool
    uint32_t *flags = nullptr;     // pinned, host-mapped, one per item
    uint32_t *h_err = nullptr;     // pinned: the batch's repair count and log
    std::unique_ptr<WsState> wst;
    bool busy = false;
    std::vector<std::vector<uint64_t>> item_tickets;  // tickets fused into each item
    std::vector<uint8_t> item_done;
    int n_items = 0;
    int n_done = 0;
};

}  // namespace

struct Server {
    const void *d_params = nullptr;
    uint32_t *d_states = nullptr;
    int stride = 0, n_streams = 0;
    char *d_pool = nullptr;   // output region (after the slot workspaces)
    size_t ws_bytes = 0;      // workspace per slot
    std::shared_ptr<ParamSet> ps;
    mtgp_server_opts opts{};
    int device = 0;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work;   // wakes the loop
    std::condition_variable cv_done;   // wakes waiters
    std::unordered_map<uint64_t, Req> reqs;
    std::list<uint64_t> pending;       // tickets in submission order
    // set by whatever can make a queued request admissible (a submission,
    // released pool bytes, a stream leaving the GPU); admission passes run
    // only when it is set
    bool admit_dirty = true;
    std::vector<uint8_t> blocked_mark;  // per stream, within one admission pass
    std::unordered_map<int32_t, std::deque<uint64_t>> per_stream;
    std::vector<uint8_t> stream_busy;
    std::unique_ptr<Pool> pool;
    uint64_t next_ticket = 1;
    size_t queued = 0;
    uint64_t repaired = 0;  // requests regenerated after a failed segment check
    int waiters = 0;        // threads inside mtgp_wait (destroy waits for them)
    bool stop = false;
    std::vector<Slot> slots;
    std::thread thr;

    uint64_t now() const {
        return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0)
            .count();
    }

    // Requests of admitted-but-not-launched groups: each entry is one fused
    // item (tickets of one stream, contiguous in the pool).
    std::vector<std::vector<uint64_t>> ready;

    void admit_locked() {
        if (pending.empty() || !admit_dirty) return;
        admit_dirty = false;
        const int cap = opts.max_batch_items;
        std::vector<int32_t> touched;
        auto is_blocked = [&](int32_t s) { return blocked_mark[(size_t)s] != 0; };
        auto it = pending.begin();
        for (; it != pending.end() && (int)ready.size() < cap;) {
            auto rit = reqs.find(*it);
            if (rit == reqs.end() || rit->second.state != R_QUEUED) {
                it = pending.erase(it);
                continue;
            }
            const int32_t s = rit->second.stream;
            if (stream_busy[s] || is_blocked(s)) {
                ++it;
                continue;
            }
            // fuse this stream's consecutive queued requests of one dtype
            auto &q = per_stream[s];
            uint64_t bytes = 0;
            std::vector<uint64_t> group;
            const int dt = reqs[q.front()].dtype;
            for (uint64_t tk : q) {
                if (reqs[tk].dtype != dt) break;
                group.push_back(tk);
                bytes += reqs[tk].count * 4;
            }
            uint64_t off = 0;
            if (!pool->alloc(bytes, &off)) {
                blocked_mark[(size_t)s] = 1;  // keep this stream's order: try later
                touched.push_back(s);
                ++it;
                continue;
            }
            const uint64_t t = now();
            uint64_t cur = off;
            for (uint64_t tk : group) {
                Req &r = reqs[tk];
                r.state = R_ADMITTED;
                r.t_admit = t;
                r.off = cur;
                r.bytes = r.count * 4;
                cur += r.bytes;
                --queued;
            }
            q.erase(q.begin(), q.begin() + (long)group.size());
            if (q.empty()) per_stream.erase(s);
            stream_busy[s] = 1;
            ready.push_back(std::move(group));
            it = pending.erase(it);
        }
        if (it != pending.end()) admit_dirty = true;  // stopped at a full batch
        for (int32_t s : touched) blocked_mark[(size_t)s] = 0;
    }

    // Called with `lk` held; releases it while the batch is planned and
    // launched (only this thread touches the slot and the launched items'
    // records meanwhile), so submissions and polls do not wait on planning.
    int launch_locked(int si, std::unique_lock<std::mutex> &lk) {
        Slot &sl = slots[si];
        const int n = (int)ready.size();
        std::vector<mtgp::Request> work((size_t)n);
        for (int i = 0; i < n; ++i) {
            const Req &r0 = reqs[ready[i].front()];
            uint64_t total = 0;
            for (uint64_t tk : ready[i]) total += reqs[tk].count;
            sl.flags[i] = 0u;
            work[i] = mtgp::Request{r0.stream, (uint32_t)r0.dtype, total, d_pool + r0.off,
                                    (uint64_t)(uintptr_t)&sl.flags[i]};
        }
        sl.item_tickets.assign((size_t)n, {});
        sl.item_done.assign((size_t)n, 0);
        const uint64_t t = now();
        for (int i = 0; i < n; ++i) {
            sl.item_tickets[i] = ready[i];
            for (uint64_t tk : sl.item_tickets[i]) {
                Req &r = reqs[tk];
                r.state = R_LAUNCHED;
                r.t_launch = t;
                r.slot = si;
                r.item = i;
            }
        }
        ready.clear();
        sl.n_items = n;
        sl.n_done = 0;
        sl.busy = true;
        int rc;
        lk.unlock();
        {
            std::lock_guard<std::mutex> sg(sl.wst->mu);
            rc = run_batch(ps, d_params, d_states, stride, work, sl.d_ws, ws_bytes, sl.hs,
                           tuning_for(ps->N), false, *sl.wst, true);
            if (rc == MTGP_OK) {
                // the batch's repair count and log come back with the slot
                hipError_t e = hipMemcpyAsync(sl.h_err, (uint32_t *)sl.d_ws + HDR_ERR,
                                              HDR_ERR_WORDS * sizeof(uint32_t),
                                              hipMemcpyDeviceToHost, sl.hs);
                if (e == hipSuccess) e = hipEventRecord(sl.done, sl.hs);
                if (e != hipSuccess) rc = hip_fail(e, "slot completion record");
            }
        }
        lk.lock();
        if (rc != MTGP_OK) {
            for (auto &g : sl.item_tickets)
                for (uint64_t tk : g) finish_locked(reqs[tk], R_FAILED);
            sl.busy = false;
        }
        return rc;
    }

    void finish_locked(Req &r, ReqState st) {
        r.state = st;
        r.t_done = now();
        stream_busy[r.stream] = 0;
        admit_dirty = true;
    }

    // Scan flags of in-flight items; retire finished slots.
    bool reap_locked() {
        bool any = false;
        for (Slot &sl : slots) {
            if (!sl.busy) continue;
            for (int j = 0; j < sl.n_items; ++j) {
                if (sl.item_done[j]) continue;
                if (__atomic_load_n(&sl.flags[j], __ATOMIC_ACQUIRE) != 0u) {
                    sl.item_done[j] = 1;
                    ++sl.n_done;
                    for (uint64_t tk : sl.item_tickets[j]) {
                        auto it = reqs.find(tk);
                        if (it != reqs.end()) finish_locked(it->second, R_DONE);
                    }
                    any = true;
                }
            }
            if (sl.n_done == sl.n_items) {
                hipError_t e = hipEventQuery(sl.done);
                if (e == hipSuccess) {
                    if (sl.h_err[0] != 0) {
                        // results are exact (the device regenerated them);
                        // rebuild those streams' polynomials from their states
                        repaired += sl.h_err[0];
                        note_repairs(*ps, sl.h_err, sl.wst->split_streams);
                    }
                    sl.busy = false;
                    any = true;
                } else if (e != hipErrorNotReady) {
                    // device error: fail whatever the slot still held
                    for (int j = 0; j < sl.n_items; ++j)
                        if (!sl.item_done[j])
                            for (uint64_t tk : sl.item_tickets[j])
                                finish_locked(reqs[tk], R_FAILED);
                    sl.busy = false;
                    any = true;
                }
            } else {
                hipError_t e = hipEventQuery(sl.done);
                if (e != hipSuccess && e != hipErrorNotReady) {
                    for (int j = 0; j < sl.n_items; ++j)
                        if (!sl.item_done[j]) {
                            sl.item_done[j] = 1;
                            for (uint64_t tk : sl.item_tickets[j])
                                finish_locked(reqs[tk], R_FAILED);
                        }
                    sl.busy = false;
                    any = true;
                }
            }
        }
        return any;
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        uint64_t ready_since = 0;
        while (true) {
            bool progressed = reap_locked();
            if (progressed) cv_done.notify_all();
            if (stop) break;
            admit_locked();
            int free_slot = -1, busy_slots = 0;
            for (size_t i = 0; i < slots.size(); ++i) {
                if (!slots[i].busy) {
                    if (free_slot < 0) free_slot = (int)i;
                } else {
                    ++busy_slots;
                }
            }
            if (!ready.empty()) {
                if (ready_since == 0) ready_since = now();
                // Launch at once when the GPU is idle or the batch is full;
                // otherwise give late arrivals a short window to join.
                const bool full = (int)ready.size() >= opts.max_batch_items;
                const bool waited = now() - ready_since >= opts.batch_window_ns;
                if (free_slot >= 0 && (busy_slots == 0 || full || waited)) {
                    (void)launch_locked(free_slot, lk);
                    ready_since = 0;
                    cv_done.notify_all();
                    continue;
                }
            }
            const bool inflight = busy_slots > 0;
            if (!inflight && ready.empty() && (pending.empty() || queued == 0)) {
                cv_work.wait(lk);
            } else {
                cv_work.wait_for(lk, std::chrono::microseconds(inflight ? 5 : 20));
            }
        }
        // shutdown: wait for in-flight batches, cancel the rest
        for (Slot &sl : slots)
            if (sl.busy) (void)hipStreamSynchronize(sl.hs);
        reap_locked();
        for (auto &kv : reqs) {
            Req &r = kv.second;
            if (r.state == R_QUEUED || r.state == R_ADMITTED) finish_locked(r, R_CANCELED);
            if (r.state == R_LAUNCHED) finish_locked(r, R_FAILED);
        }
        cv_done.notify_all();
    }
};

}  // namespace mtgp

using namespace mtgp;

struct mtgp_server {
    Server s;
};

extern "C" {

int mtgp_server_create(const void *d_params, uint32_t *d_states, int state_stride, int n_streams,
                       void *d_pool, uint64_t pool_bytes, const mtgp_server_opts *opts,
                       mtgp_server **out) {
    if (!out) return fail(MTGP_EINVAL, "out is NULL");
    *out = nullptr;
    auto ps = lookup_params(d_params, n_streams);
    if (!ps) return MTGP_EINVAL;
    if (n_streams <= 0 || !d_states || state_stride < ps->N)
        return fail(MTGP_EINVAL, "bad streams/states (n=%d, stride=%d, N=%d)", n_streams,
                    state_stride, ps->N);
    if (!d_pool || ((uintptr_t)d_pool & 255u))
        return fail(MTGP_EINVAL, "d_pool must be non-NULL and 256-byte aligned");
    mtgp_server_opts o{4, 256, 1 << 20, 20000, 64ull << 20};
    if (opts) o = *opts;
    if (o.max_inflight_batches < 1 || o.max_inflight_batches > 16 || o.max_batch_items < 1 ||
        o.max_queue < 1)
        return fail(MTGP_EINVAL, "bad server options");
    size_t ws = std::max<size_t>(batch_min_ws_bytes(o.max_batch_items),
                                 (size_t)o.workspace_bytes_per_batch);
    ws = (ws + 255) / 256 * 256;
    const uint64_t reserved = (uint64_t)ws * (uint64_t)o.max_inflight_batches;
    if (pool_bytes <= reserved + 256)
        return fail(MTGP_EINVAL, "pool of %llu bytes is too small (workspaces need %llu)",
                    (unsigned long long)pool_bytes, (unsigned long long)reserved);
    auto *h = new (std::nothrow) mtgp_server();
    if (!h) return fail(MTGP_ENOMEM, "server allocation");
    Server &S = h->s;
    S.d_params = d_params;
    S.d_states = d_states;
    S.stride = state_stride;
    S.n_streams = n_streams;
    S.ps = ps;
    S.opts = o;
    S.t0 = Clock::now();
    (void)hipGetDevice(&S.device);
    S.stream_busy.assign((size_t)n_streams, 0);
    S.blocked_mark.assign((size_t)n_streams, 0);
    S.slots.resize((size_t)o.max_inflight_batches);
    int rc = MTGP_OK;
    for (int i = 0; i < o.max_inflight_batches && rc == MTGP_OK; ++i) {
        Slot &sl = S.slots[i];
        sl.wst = std::make_unique<WsState>();
        sl.d_ws = (char *)d_pool + (size_t)i * ws;
        hipError_t e = hipStreamCreateWithFlags(&sl.hs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&sl.flags, sizeof(uint32_t) * (size_t)o.max_batch_items,
                              hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&sl.h_err, sizeof(uint32_t) * HDR_ERR_WORDS,
                              hipHostMallocDefault);
        if (e == hipSuccess) std::memset(sl.h_err, 0, sizeof(uint32_t) * HDR_ERR_WORDS);
        if (e != hipSuccess) rc = hip_fail(e, "server slot setup");
    }
    S.d_pool = (char *)d_pool + reserved;
    S.ws_bytes = ws;
    S.pool = std::make_unique<Pool>(pool_bytes - reserved);
    if (rc != MTGP_OK) {
        for (Slot &sl : S.slots) {
            if (sl.flags) (void)hipHostFree(sl.flags);
            if (sl.h_err) (void)hipHostFree(sl.h_err);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.hs) (void)hipStreamDestroy(sl.hs);
        }
        delete h;
        return rc;
    }
    S.thr = std::thread([&S] { S.loop(); });
    *out = h;
    return MTGP_OK;
}

int mtgp_submit(mtgp_server *srv, int32_t stream_id, uint64_t count, int dtype,
                uint64_t *ticket) {
    if (!srv || !ticket) return fail(MTGP_EINVAL, "NULL server or ticket");
    Server &S = srv->s;
    if (stream_id < 0 || stream_id >= S.n_streams)
        return fail(MTGP_EINVAL, "stream %d outside [0, %d)", stream_id, S.n_streams);
    if (dtype != MTGP_U32 && dtype != MTGP_F32) return fail(MTGP_EINVAL, "dtype %d", dtype);
    if (count == 0) return fail(MTGP_EINVAL, "count must be > 0");
    std::lock_guard<std::mutex> lk(S.mu);
    if (count * 4 > S.pool->size())
        return fail(MTGP_ETOOBIG, "request of %llu bytes exceeds the %llu-byte pool",
                    (unsigned long long)(count * 4), (unsigned long long)S.pool->size());
    if (S.stop) return fail(MTGP_ECANCELED, "server is shutting down");
    if ((int)S.queued >= S.opts.max_queue) return fail(MTGP_EAGAIN, "queue full");
    Req r;
    r.ticket = S.next_ticket++;
    r.stream = stream_id;
    r.count = count;
    r.dtype = dtype;
    r.t_submit = S.now();
    auto &q = S.per_stream[stream_id];
    q.push_back(r.ticket);
    S.pending.push_back(r.ticket);
    S.admit_dirty = true;
    S.reqs.emplace(r.ticket, r);
    ++S.queued;
    *ticket = r.ticket;
    S.cv_work.notify_one();
    return MTGP_OK;
}

int mtgp_submit_many(mtgp_server *srv, const int32_t *stream_ids, const uint64_t *counts,
                     const int *dtypes, int n, uint64_t *tickets) {
    if (!srv || n < 0 || (n > 0 && (!stream_ids || !counts || !dtypes || !tickets)))
        return fail(MTGP_EINVAL, "NULL argument or n=%d", n);
    Server &S = srv->s;
    for (int i = 0; i < n; ++i) {
        if (stream_ids[i] < 0 || stream_ids[i] >= S.n_streams)
            return fail(MTGP_EINVAL, "request %d: stream %d outside [0, %d)", i, stream_ids[i],
                        S.n_streams);
        if (dtypes[i] != MTGP_U32 && dtypes[i] != MTGP_F32)
            return fail(MTGP_EINVAL, "request %d: dtype %d", i, dtypes[i]);
        if (counts[i] == 0) return fail(MTGP_EINVAL, "request %d: count must be > 0", i);
    }
    std::lock_guard<std::mutex> lk(S.mu);
    for (int i = 0; i < n; ++i)
        if (counts[i] * 4 > S.pool->size())
            return fail(MTGP_ETOOBIG, "request %d of %llu bytes exceeds the %llu-byte pool", i,
                        (unsigned long long)(counts[i] * 4),
                        (unsigned long long)S.pool->size());
    if (S.stop) return fail(MTGP_ECANCELED, "server is shutting down");
    if ((int)S.queued + n > S.opts.max_queue) return fail(MTGP_EAGAIN, "queue full");
    const uint64_t t = S.now();
    for (int i = 0; i < n; ++i) {
        Req r;
        r.ticket = S.next_ticket++;
        r.stream = stream_ids[i];
        r.count = counts[i];
        r.dtype = dtypes[i];
        r.t_submit = t;
        S.per_stream[r.stream].push_back(r.ticket);
        S.pending.push_back(r.ticket);
        S.admit_dirty = true;
        tickets[i] = r.ticket;
        S.reqs.emplace(r.ticket, r);
        ++S.queued;
    }
    S.cv_work.notify_one();
    return MTGP_OK;
}

int mtgp_poll(mtgp_server *srv, uint64_t ticket, int *state, const void **d_result) {
    if (!srv || !state) return fail(MTGP_EINVAL, "NULL server or state");
    Server &S = srv->s;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket);
    const Req &r = it->second;
    if (d_result) *d_result = nullptr;
    switch (r.state) {
        case R_DONE:
            *state = MTGP_DONE;
            if (d_result) *d_result = S.d_pool + r.off;
            return MTGP_OK;
        case R_FAILED:
            *state = MTGP_FAILED;
            return MTGP_OK;
        case R_CANCELED:
            *state = MTGP_FAILED;
            return fail(MTGP_ECANCELED, "ticket %llu cancelled", (unsigned long long)ticket);
        default:
            *state = MTGP_PENDING;
            return MTGP_OK;
    }
}

int mtgp_server_replay(mtgp_server *srv, const uint64_t *t_arrival_ns, const int32_t *stream_ids,
                       const uint64_t *counts, const int *dtypes, int n, uint64_t *h_latency_ns,
                       uint64_t *h_stages_ns, void *const *d_keep) {
    if (!srv || n < 0 || (n > 0 && (!t_arrival_ns || !stream_ids || !counts || !dtypes ||
                                    !h_latency_ns)))
        return fail(MTGP_EINVAL, "NULL argument or n=%d", n);
    Server &S = srv->s;
    for (int i = 0; i < n; ++i) {
        if (i > 0 && t_arrival_ns[i] < t_arrival_ns[i - 1])
            return fail(MTGP_EINVAL, "arrival %d before arrival %d", i, i - 1);
        if (stream_ids[i] < 0 || stream_ids[i] >= S.n_streams || counts[i] == 0 ||
            (dtypes[i] != MTGP_U32 && dtypes[i] != MTGP_F32) || counts[i] * 4 > S.pool->size())
            return fail(MTGP_EINVAL, "request %d: bad stream, count or dtype", i);
    }
    hipStream_t cs = nullptr;  // copies of kept results
    if (d_keep) {
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate(replay copies)");
    }
    struct Kept {
        int i;
        uint64_t ticket, off, bytes;
    };
    int rc = MTGP_OK;
    const uint64_t start = S.now();
    std::vector<uint64_t> tickets((size_t)n, 0);
    std::vector<int> open;  // submitted, not yet finished
    int next = 0, finished = 0;
    while (finished < n && rc == MTGP_OK) {
        std::vector<Kept> kept;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            if (S.stop) {
                rc = fail(MTGP_ECANCELED, "server is shutting down");
                break;
            }
            const uint64_t t = S.now();
            bool queued_any = false;
            while (next < n && start + t_arrival_ns[next] <= t &&
                   (int)S.queued < S.opts.max_queue) {
                Req r;
                r.ticket = S.next_ticket++;
                r.stream = stream_ids[next];
                r.count = counts[next];
                r.dtype = dtypes[next];
                r.t_submit = t;
                S.per_stream[r.stream].push_back(r.ticket);
                S.pending.push_back(r.ticket);
                S.admit_dirty = true;
                tickets[(size_t)next] = r.ticket;
                S.reqs.emplace(r.ticket, r);
                ++S.queued;
                open.push_back(next++);
                queued_any = true;
            }
            if (queued_any) S.cv_work.notify_one();
            // collect what finished; its pool bytes go back at once (after
            // the copy for kept results)
            size_t w = 0;
            for (size_t k = 0; k < open.size(); ++k) {
                const int i = open[k];
                auto it = S.reqs.find(tickets[(size_t)i]);
                if (it == S.reqs.end()) {
                    rc = fail(MTGP_EDEVICE, "replayed request vanished");
                    break;
                }
                Req &r = it->second;
                if (r.state == R_DONE) {
                    h_latency_ns[i] = r.t_done - (start + t_arrival_ns[i]);
                    if (h_stages_ns) {
                        h_stages_ns[3 * (size_t)i + 0] = r.t_admit - r.t_submit;
                        h_stages_ns[3 * (size_t)i + 1] = r.t_launch - r.t_admit;
                        h_stages_ns[3 * (size_t)i + 2] = r.t_done - r.t_launch;
                    }
                    if (d_keep && d_keep[i]) {
                        kept.push_back(Kept{i, r.ticket, r.off, r.bytes});
                        continue;
                    }
                    if (r.bytes) S.pool->release(r.off, r.bytes);
                    S.admit_dirty = true;
                    S.reqs.erase(it);
                    ++finished;
                    S.cv_work.notify_one();
                } else if (r.state == R_FAILED || r.state == R_CANCELED) {
                    rc = fail(MTGP_EDEVICE, "replayed request %d failed", i);
                    break;
                } else {
                    open[w++] = i;
                }
            }
            open.resize(w);
        }
        if (rc != MTGP_OK) break;
        if (!kept.empty()) {
            // outside the lock: the server keeps launching meanwhile
            for (const Kept &kp : kept) {
                hipError_t e = hipMemcpyAsync(d_keep[kp.i], S.d_pool + kp.off, kp.bytes,
                                              hipMemcpyDeviceToDevice, cs);
                if (e != hipSuccess) rc = hip_fail(e, "hipMemcpyAsync(kept result)");
            }
            hipError_t e = hipStreamSynchronize(cs);
            if (e != hipSuccess && rc == MTGP_OK) rc = hip_fail(e, "hipStreamSynchronize(kept)");
            std::lock_guard<std::mutex> lk(S.mu);
            for (const Kept &kp : kept) {
                if (kp.bytes) S.pool->release(kp.off, kp.bytes);
                S.reqs.erase(kp.ticket);
                ++finished;
            }
            S.admit_dirty = true;
            S.cv_work.notify_one();
            continue;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
    if (cs) (void)hipStreamDestroy(cs);
    return rc;
}

int mtgp_server_repaired(mtgp_server *srv, uint64_t *n) {
    if (!srv || !n) return fail(MTGP_EINVAL, "NULL server or n");
    Server &S = srv->s;
    std::lock_guard<std::mutex> lk(S.mu);
    *n = S.repaired;
    return MTGP_OK;
}

int mtgp_wait(mtgp_server *srv, uint64_t ticket, uint64_t timeout_ns) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    Server &S = srv->s;
    std::unique_lock<std::mutex> lk(S.mu);
    ++S.waiters;
    auto leave = [&](int rc) {
        --S.waiters;
        S.cv_done.notify_all();  // mtgp_server_destroy may be waiting for us
        return rc;
    };
    auto done = [&] {
        auto it = S.reqs.find(ticket);
        return it == S.reqs.end() || it->second.state >= R_DONE;
    };
    if (timeout_ns == 0) {
        S.cv_done.wait(lk, done);
    } else if (!S.cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
        return leave(fail(MTGP_ETIMEDOUT, "ticket %llu not done after %llu ns",
                          (unsigned long long)ticket, (unsigned long long)timeout_ns));
    }
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end())
        return leave(fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket));
    if (it->second.state == R_CANCELED) return leave(fail(MTGP_ECANCELED, "ticket cancelled"));
    if (it->second.state == R_FAILED)
        return leave(fail(MTGP_EDEVICE, "request failed on the device"));
    return leave(MTGP_OK);
}

int mtgp_release(mtgp_server *srv, uint64_t ticket) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    Server &S = srv->s;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket);
    Req &r = it->second;
    if (r.state == R_ADMITTED || r.state == R_LAUNCHED)
        return fail(MTGP_EAGAIN, "ticket %llu is still being generated", (unsigned long long)ticket);
    if (r.state == R_QUEUED) {
        // cancel before admission: drop it from its stream's queue
        auto &q = S.per_stream[r.stream];
        q.erase(std::remove(q.begin(), q.end(), ticket), q.end());
        if (q.empty()) S.per_stream.erase(r.stream);
        --S.queued;
    } else if (r.state == R_DONE || r.state == R_FAILED) {
        if (r.bytes) S.pool->release(r.off, r.bytes);
    }
    S.admit_dirty = true;
    S.reqs.erase(it);
    S.cv_work.notify_one();
    return MTGP_OK;
}

int mtgp_request_times(mtgp_server *srv, uint64_t ticket, uint64_t *t_submit, uint64_t *t_admit,
                       uint64_t *t_launch, uint64_t *t_done) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    Server &S = srv->s;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket);
    const Req &r = it->second;
    if (t_submit) *t_submit = r.t_submit;
    if (t_admit) *t_admit = r.t_admit;
    if (t_launch) *t_launch = r.t_launch;
    if (t_done) *t_done = r.t_done;
    return MTGP_OK;
}

int mtgp_server_destroy(mtgp_server *srv) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    Server &S = srv->s;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
    }
    S.cv_work.notify_all();
    if (S.thr.joinable()) S.thr.join();
    {
        // threads blocked in mtgp_wait have been woken (their requests are
        // finished or cancelled): let them leave before the server goes
        std::unique_lock<std::mutex> lk(S.mu);
        S.cv_done.wait(lk, [&] { return S.waiters == 0; });
    }
    int rc = MTGP_OK;
    for (Slot &sl : S.slots) {
        if (sl.flags) (void)hipHostFree(sl.flags);
        if (sl.h_err) (void)hipHostFree(sl.h_err);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.hs) (void)hipStreamDestroy(sl.hs);
    }
    delete srv;  // slot staging buffers are released by their destructors
    return rc;
}

}  // extern "C"
