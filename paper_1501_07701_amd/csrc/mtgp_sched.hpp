// mtgp_sched.hpp -- the serving runtime's request scheduler, free of HIP.
//
// It owns everything about requests that is not device work: the queue in
// submission order, admission while output bytes fit the pool, fusion of a
// stream's consecutive same-dtype requests into one item over one contiguous
// pool range, at most one item per stream in flight (so each stream's
// results follow its submission order, as the paper's per-block state in
// global memory requires between calls, Sec. 2), the in-flight launch slots,
// completion, release, cancellation at shutdown and trace replay.  The
// device side (planning and launching a batch, completion flags, copies)
// sits behind SchedBackend, so the same code runs against a fake device in
// the CPU tests.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mtgp.h"

namespace mtgp {

int fail(int code, const char *fmt, ...);

// First-fit allocator over [0, size): ranges start 256-byte aligned; frees
// are exact, so one allocation may be returned in several pieces.
class Pool {
   public:
    explicit Pool(uint64_t size) : size_(size) { free_[0] = size; }
    bool alloc(uint64_t bytes, uint64_t *off);
    void release(uint64_t off, uint64_t bytes);
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    // free ranges (offset -> length), for the tests' consistency checks
    const std::map<uint64_t, uint64_t> &free_ranges() const { return free_; }

   private:
    uint64_t size_, used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

// One work item of a launch: `count` outputs of `stream` (dtype MTGP_U32 or
// MTGP_F32) written at byte offset `off` of the output pool.
struct SchedItem {
    int32_t stream;
    int dtype;
    uint64_t count;
    uint64_t off;
};

// What the scheduler needs from the device.  launch() is called from the
// scheduler's thread without the scheduler's lock; the queries are called
// from that thread with the lock held; copy_out() from replaying threads.
class SchedBackend {
   public:
    virtual ~SchedBackend() = default;
    // first thing the scheduler's thread does (e.g. select the device)
    virtual void thread_start() {}
    // Plans and enqueues one batch on launch slot `slot`; the slot's
    // previous batch has been retired.  MTGP_OK or an error code.
    virtual int launch(int slot, const std::vector<SchedItem> &items) = 0;
    // true once item `item` of the slot's batch has stored outputs and state
    virtual bool item_done(int slot, int item) = 0;
    // 1 while the slot's batch runs, 0 once it finished, < 0 on a device error
    virtual int slot_poll(int slot) = 0;
    // called once when a finished batch is retired: the number of requests
    // the device regenerated after a failed segment check
    virtual uint64_t slot_retire(int slot) = 0;
    // blocks until the slot's batch finished (shutdown)
    virtual void slot_wait(int slot) = 0;
    struct Copy {
        uint64_t off, bytes;
        void *dst;
    };
    // copies pool bytes out and waits for the copies
    virtual int copy_out(const std::vector<Copy> &copies) = 0;
};

struct SchedOpts {
    int max_inflight = 4;       // launch slots
    int max_batch_items = 256;  // items per launch
    int max_queue = 1 << 20;    // queued (not yet admitted) requests
    uint64_t batch_window_ns = 20000;
};

class Scheduler {
   public:
    Scheduler(SchedBackend *backend, int n_streams, uint64_t pool_bytes, const SchedOpts &opts);
    ~Scheduler();  // shutdown()
    Scheduler(const Scheduler &) = delete;
    Scheduler &operator=(const Scheduler &) = delete;

    void start();  // starts the scheduler's thread
    // Stops the thread: in-flight batches are waited for, what never
    // launched ends cancelled, and threads inside wait() have left when it
    // returns.  Idempotent.
    void shutdown();

    int submit(int32_t stream, uint64_t count, int dtype, uint64_t *ticket);
    int submit_many(const int32_t *streams, const uint64_t *counts, const int *dtypes, int n,
                    uint64_t *tickets);
    // *state = MTGP_PENDING / MTGP_DONE / MTGP_FAILED; *off = pool offset of
    // the result once done
    int poll(uint64_t ticket, int *state, uint64_t *off);
    int wait(uint64_t ticket, uint64_t timeout_ns);
    int release(uint64_t ticket);
    int times(uint64_t ticket, uint64_t *t_submit, uint64_t *t_admit, uint64_t *t_launch,
              uint64_t *t_done);
    int replay(const uint64_t *t_arrival_ns, const int32_t *streams, const uint64_t *counts,
               const int *dtypes, int n, uint64_t *h_latency_ns, uint64_t *h_stages_ns,
               void *const *keep);
    uint64_t repaired();
    uint64_t pool_size() const { return pool_.size(); }
    uint64_t pool_used();
    int n_streams() const { return n_streams_; }

   private:
    enum State { R_QUEUED, R_ADMITTED, R_LAUNCHED, R_DONE, R_FAILED, R_CANCELED };
    struct Req {
        uint64_t ticket = 0;
        int32_t stream = 0;
        uint64_t count = 0;
        int dtype = 0;
        uint64_t off = 0;  // byte offset in the pool
        uint64_t bytes = 0;
        State state = R_QUEUED;
        uint64_t t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    };
    struct Slot {
        bool busy = false;
        std::vector<std::vector<uint64_t>> item_tickets;  // tickets fused into each item
        std::vector<uint8_t> item_done;
        int n_items = 0, n_done = 0;
    };
    using Clock = std::chrono::steady_clock;

    uint64_t now() const;
    int check_request(int32_t stream, uint64_t count, int dtype, int index) const;
    void enqueue_locked(int32_t stream, uint64_t count, int dtype, uint64_t t, uint64_t *ticket);
    void admit_locked();
    int launch_locked(int si, std::unique_lock<std::mutex> &lk);
    void finish_locked(Req &r, State st);
    bool reap_locked();
    void loop();

    SchedBackend *be_;
    const int n_streams_;
    const SchedOpts opts_;
    const Clock::time_point t0_;

    std::mutex mu_;
    std::condition_variable cv_work_;  // wakes the loop
    std::condition_variable cv_done_;  // wakes waiters
    std::unordered_map<uint64_t, Req> reqs_;
    std::list<uint64_t> pending_;  // tickets in submission order
    // set by whatever can make a queued request admissible (a submission,
    // released pool bytes, a stream leaving the device); admission passes
    // run only when it is set
    bool admit_dirty_ = true;
    std::vector<uint8_t> blocked_mark_;  // per stream, within one admission pass
    std::unordered_map<int32_t, std::deque<uint64_t>> per_stream_;
    std::vector<uint8_t> stream_busy_;
    // admitted, not yet launched: each entry one fused item (tickets of one
    // stream, contiguous in the pool)
    std::vector<std::vector<uint64_t>> ready_;
    Pool pool_;
    uint64_t next_ticket_ = 1;
    size_t queued_ = 0;
    uint64_t repaired_ = 0;
    int waiters_ = 0;  // threads inside wait()
    bool stop_ = false;
    bool joined_ = false;
    std::vector<Slot> slots_;
    std::thread thr_;
};

}  // namespace mtgp
