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
// Results stay in the pool until the client releases them.  Steps 1, 2 and
// the bookkeeping of 3 and 4 are the HIP-free Scheduler (mtgp_sched.cpp);
// this file is its device backend and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "mtgp.h"
#include "mtgp_host.hpp"
#include "mtgp_internal.hpp"
#include "mtgp_sched.hpp"

namespace mtgp {

namespace {

struct Slot {
    hipStream_t hs = nullptr;
    hipEvent_t done = nullptr;
    void *d_ws = nullptr;          // work list + counter, carved from the pool
    uint32_t *flags = nullptr;     // pinned, host-mapped, one per item
    uint32_t *h_err = nullptr;     // pinned: the batch's repair count and log
    std::unique_ptr<WsState> wst;
};

// The device side of the scheduler: plans and launches batches through the
// batch planner on per-slot HIP streams, reads completion flags and the
// repair words, copies kept results.
class HipBackend final : public SchedBackend {
   public:
    const void *d_params = nullptr;
    uint32_t *d_states = nullptr;
    int stride = 0;
    char *d_pool = nullptr;  // output region (after the slot workspaces)
    size_t ws_bytes = 0;     // workspace per slot
    std::shared_ptr<ParamSet> ps;
    int device = 0;
    std::vector<Slot> slots;

    ~HipBackend() override {
        for (Slot &sl : slots) {
            if (sl.flags) (void)hipHostFree(sl.flags);
            if (sl.h_err) (void)hipHostFree(sl.h_err);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.hs) (void)hipStreamDestroy(sl.hs);
        }
        if (copy_stream_) (void)hipStreamDestroy(copy_stream_);
    }

    void thread_start() override { (void)hipSetDevice(device); }

    int launch(int si, const std::vector<SchedItem> &items) override {
        Slot &sl = slots[(size_t)si];
        const int n = (int)items.size();
        std::vector<Request> work((size_t)n);
        for (int i = 0; i < n; ++i) {
            const SchedItem &it = items[(size_t)i];
            sl.flags[i] = 0u;
            work[(size_t)i] = Request{it.stream, (uint32_t)it.dtype, it.count, d_pool + it.off,
                                      (uint64_t)(uintptr_t)&sl.flags[i]};
        }
        std::lock_guard<std::mutex> sg(sl.wst->mu);
        int rc = run_batch(ps, d_params, d_states, stride, work, sl.d_ws, ws_bytes, sl.hs,
                           tuning_for(ps->N), false, *sl.wst, true, false);
        if (rc == MTGP_OK) {
            // the batch's repair count and log come back with the slot
            hipError_t e = hipMemcpyAsync(sl.h_err, (uint32_t *)sl.d_ws + HDR_ERR,
                                          HDR_ERR_WORDS * sizeof(uint32_t),
                                          hipMemcpyDeviceToHost, sl.hs);
            if (e == hipSuccess) e = hipEventRecord(sl.done, sl.hs);
            if (e != hipSuccess) rc = hip_fail(e, "slot completion record");
        }
        return rc;
    }

    bool item_done(int si, int j) override {
        return __atomic_load_n(&slots[(size_t)si].flags[j], __ATOMIC_ACQUIRE) != 0u;
    }

    int slot_poll(int si) override {
        const hipError_t e = hipEventQuery(slots[(size_t)si].done);
        if (e == hipSuccess) return 0;
        return e == hipErrorNotReady ? 1 : -1;
    }

    uint64_t slot_retire(int si) override {
        Slot &sl = slots[(size_t)si];
        if (sl.h_err[0] == 0) return 0;
        // results are exact (the device regenerated them); rebuild those
        // streams' polynomials from their states
        note_repairs(*ps, sl.h_err, sl.wst->split_streams);
        return sl.h_err[0];
    }

    void slot_wait(int si) override { (void)hipStreamSynchronize(slots[(size_t)si].hs); }

    int copy_out(const std::vector<Copy> &copies) override {
        std::lock_guard<std::mutex> lk(copy_mu_);
        if (!copy_stream_) {
            hipError_t e = hipStreamCreateWithFlags(&copy_stream_, hipStreamNonBlocking);
            if (e != hipSuccess) {
                copy_stream_ = nullptr;
                return hip_fail(e, "hipStreamCreate(result copies)");
            }
        }
        int rc = MTGP_OK;
        for (const Copy &c : copies) {
            hipError_t e = hipMemcpyAsync(c.dst, d_pool + c.off, c.bytes, hipMemcpyDeviceToDevice,
                                          copy_stream_);
            if (e != hipSuccess && rc == MTGP_OK) rc = hip_fail(e, "hipMemcpyAsync(kept result)");
        }
        hipError_t e = hipStreamSynchronize(copy_stream_);
        if (e != hipSuccess && rc == MTGP_OK) rc = hip_fail(e, "hipStreamSynchronize(kept)");
        return rc;
    }

   private:
    std::mutex copy_mu_;
    hipStream_t copy_stream_ = nullptr;
};

}  // namespace

}  // namespace mtgp

using namespace mtgp;

struct mtgp_server {
    HipBackend be;
    std::unique_ptr<Scheduler> sched;
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
    std::unique_ptr<mtgp_server> h(new (std::nothrow) mtgp_server());
    if (!h) return fail(MTGP_ENOMEM, "server allocation");
    HipBackend &B = h->be;
    B.d_params = d_params;
    B.d_states = d_states;
    B.stride = state_stride;
    B.ps = ps;
    B.d_pool = (char *)d_pool + reserved;
    B.ws_bytes = ws;
    (void)hipGetDevice(&B.device);
    B.slots.resize((size_t)o.max_inflight_batches);
    for (int i = 0; i < o.max_inflight_batches; ++i) {
        Slot &sl = B.slots[(size_t)i];
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
        if (e != hipSuccess) return hip_fail(e, "server slot setup");  // ~HipBackend frees
    }
    SchedOpts so;
    so.max_inflight = o.max_inflight_batches;
    so.max_batch_items = o.max_batch_items;
    so.max_queue = o.max_queue;
    so.batch_window_ns = o.batch_window_ns;
    h->sched = std::make_unique<Scheduler>(&B, n_streams, pool_bytes - reserved, so);
    h->sched->start();
    *out = h.release();
    return MTGP_OK;
}

int mtgp_submit(mtgp_server *srv, int32_t stream_id, uint64_t count, int dtype,
                uint64_t *ticket) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    return srv->sched->submit(stream_id, count, dtype, ticket);
}

int mtgp_submit_many(mtgp_server *srv, const int32_t *stream_ids, const uint64_t *counts,
                     const int *dtypes, int n, uint64_t *tickets) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    return srv->sched->submit_many(stream_ids, counts, dtypes, n, tickets);
}

int mtgp_poll(mtgp_server *srv, uint64_t ticket, int *state, const void **d_result) {
    if (!srv || !state) return fail(MTGP_EINVAL, "NULL server or state");
    if (d_result) *d_result = nullptr;
    uint64_t off = 0;
    int st = MTGP_PENDING;
    const int rc = srv->sched->poll(ticket, &st, &off);
    *state = st;
    if (rc == MTGP_OK && st == MTGP_DONE && d_result) *d_result = srv->be.d_pool + off;
    return rc;
}

int mtgp_server_replay(mtgp_server *srv, const uint64_t *t_arrival_ns, const int32_t *stream_ids,
                       const uint64_t *counts, const int *dtypes, int n, uint64_t *h_latency_ns,
                       uint64_t *h_stages_ns, void *const *d_keep) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    return srv->sched->replay(t_arrival_ns, stream_ids, counts, dtypes, n, h_latency_ns,
                              h_stages_ns, d_keep);
}

int mtgp_server_repaired(mtgp_server *srv, uint64_t *n) {
    if (!srv || !n) return fail(MTGP_EINVAL, "NULL server or n");
    *n = srv->sched->repaired();
    return MTGP_OK;
}

int mtgp_wait(mtgp_server *srv, uint64_t ticket, uint64_t timeout_ns) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    return srv->sched->wait(ticket, timeout_ns);
}

int mtgp_release(mtgp_server *srv, uint64_t ticket) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    return srv->sched->release(ticket);
}

int mtgp_request_times(mtgp_server *srv, uint64_t ticket, uint64_t *t_submit, uint64_t *t_admit,
                       uint64_t *t_launch, uint64_t *t_done) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    return srv->sched->times(ticket, t_submit, t_admit, t_launch, t_done);
}

int mtgp_server_destroy(mtgp_server *srv) {
    if (!srv) return fail(MTGP_EINVAL, "NULL server");
    // stops the loop, waits for in-flight batches and for threads inside
    // mtgp_wait / mtgp_server_replay; then the slots' HIP objects go
    srv->sched->shutdown();
    srv->sched.reset();
    delete srv;
    return MTGP_OK;
}

}  // extern "C"
