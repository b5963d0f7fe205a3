// mtgp_sched.cpp -- the serving runtime's request scheduler (no HIP here;
// the device side is a SchedBackend).
#include "mtgp_sched.hpp"

#include <algorithm>
#include <iterator>

namespace mtgp {

// ------------------------------------------------------------------ pool --

bool Pool::alloc(uint64_t bytes, uint64_t *off) {
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

void Pool::release(uint64_t off, uint64_t bytes) {
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

// ------------------------------------------------------------- scheduler --

Scheduler::Scheduler(SchedBackend *backend, int n_streams, uint64_t pool_bytes,
                     const SchedOpts &opts)
    : be_(backend),
      n_streams_(n_streams),
      opts_(opts),
      t0_(Clock::now()),
      blocked_mark_((size_t)n_streams, 0),
      stream_busy_((size_t)n_streams, 0),
      pool_(pool_bytes),
      slots_((size_t)opts.max_inflight) {}

Scheduler::~Scheduler() { shutdown(); }

void Scheduler::start() { thr_ = std::thread([this] { loop(); }); }

void Scheduler::shutdown() {
    bool started;
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (joined_) return;
        stop_ = true;
        started = thr_.joinable();
    }
    cv_work_.notify_all();
    if (started) thr_.join();
    std::unique_lock<std::mutex> lk(mu_);
    if (!started) {
        // no thread ever ran: nothing was admitted, cancel what is queued
        for (auto &kv : reqs_)
            if (kv.second.state < R_DONE) finish_locked(kv.second, R_CANCELED);
        cv_done_.notify_all();
    }
    joined_ = true;
    // threads in wait() or replay() have been woken: let them leave
    cv_done_.wait(lk, [&] { return waiters_ == 0; });
}

uint64_t Scheduler::now() const {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0_)
        .count();
}

int Scheduler::check_request(int32_t stream, uint64_t count, int dtype, int index) const {
    if (stream < 0 || stream >= n_streams_)
        return fail(MTGP_EINVAL, "request %d: stream %d outside [0, %d)", index, stream,
                    n_streams_);
    if (dtype != MTGP_U32 && dtype != MTGP_F32)
        return fail(MTGP_EINVAL, "request %d: dtype %d", index, dtype);
    if (count == 0) return fail(MTGP_EINVAL, "request %d: count must be > 0", index);
    if (count > pool_.size() / 4)
        return fail(MTGP_ETOOBIG, "request %d of %llu outputs exceeds the %llu-byte pool", index,
                    (unsigned long long)count, (unsigned long long)pool_.size());
    return MTGP_OK;
}

void Scheduler::enqueue_locked(int32_t stream, uint64_t count, int dtype, uint64_t t,
                               uint64_t *ticket) {
    Req r;
    r.ticket = next_ticket_++;
    r.stream = stream;
    r.count = count;
    r.dtype = dtype;
    r.t_submit = t;
    per_stream_[stream].push_back(r.ticket);
    pending_.push_back(r.ticket);
    admit_dirty_ = true;
    reqs_.emplace(r.ticket, r);
    ++queued_;
    *ticket = r.ticket;
}

int Scheduler::submit(int32_t stream, uint64_t count, int dtype, uint64_t *ticket) {
    if (!ticket) return fail(MTGP_EINVAL, "NULL ticket");
    int rc = check_request(stream, count, dtype, 0);
    if (rc != MTGP_OK) return rc;
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return fail(MTGP_ECANCELED, "server is shutting down");
    if ((int64_t)queued_ >= (int64_t)opts_.max_queue) return fail(MTGP_EAGAIN, "queue full");
    enqueue_locked(stream, count, dtype, now(), ticket);
    cv_work_.notify_one();
    return MTGP_OK;
}

int Scheduler::submit_many(const int32_t *streams, const uint64_t *counts, const int *dtypes,
                           int n, uint64_t *tickets) {
    if (n < 0 || (n > 0 && (!streams || !counts || !dtypes || !tickets)))
        return fail(MTGP_EINVAL, "NULL argument or n=%d", n);
    for (int i = 0; i < n; ++i) {
        int rc = check_request(streams[i], counts[i], dtypes[i], i);
        if (rc != MTGP_OK) return rc;
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return fail(MTGP_ECANCELED, "server is shutting down");
    if ((int64_t)queued_ + n > (int64_t)opts_.max_queue) return fail(MTGP_EAGAIN, "queue full");
    const uint64_t t = now();
    for (int i = 0; i < n; ++i) enqueue_locked(streams[i], counts[i], dtypes[i], t, &tickets[i]);
    if (n > 0) cv_work_.notify_one();
    return MTGP_OK;
}

void Scheduler::admit_locked() {
    if (pending_.empty() || !admit_dirty_) return;
    admit_dirty_ = false;
    const int cap = opts_.max_batch_items;
    std::vector<int32_t> touched;
    auto it = pending_.begin();
    for (; it != pending_.end() && (int)ready_.size() < cap;) {
        auto rit = reqs_.find(*it);
        if (rit == reqs_.end() || rit->second.state != R_QUEUED) {
            it = pending_.erase(it);
            continue;
        }
        const int32_t s = rit->second.stream;
        if (stream_busy_[(size_t)s] || blocked_mark_[(size_t)s]) {
            ++it;
            continue;
        }
        // fuse this stream's consecutive queued requests of one dtype; the
        // stream's queue starts with this request (it is the oldest queued
        // one of the stream, and the stream has nothing in flight)
        auto &q = per_stream_[s];
        uint64_t bytes = 0;
        std::vector<uint64_t> group;
        const int dt = rit->second.dtype;
        // (a group never exceeds the pool, or it could never be admitted)
        for (uint64_t tk : q) {
            const Req &r = reqs_.at(tk);
            if (r.dtype != dt || (!group.empty() && bytes + r.count * 4 > pool_.size())) break;
            group.push_back(tk);
            bytes += r.count * 4;
        }
        uint64_t off = 0;
        bool got = pool_.alloc(bytes, &off);
        if (!got && group.size() > 1) {
            // the whole group does not fit now: admit its first request alone
            group.resize(1);
            bytes = rit->second.count * 4;
            got = pool_.alloc(bytes, &off);
        }
        if (!got) {
            blocked_mark_[(size_t)s] = 1;  // keep this stream's order: try later
            touched.push_back(s);
            ++it;
            continue;
        }
        const uint64_t t = now();
        uint64_t cur = off;
        for (uint64_t tk : group) {
            Req &r = reqs_.at(tk);
            r.state = R_ADMITTED;
            r.t_admit = t;
            r.off = cur;
            r.bytes = r.count * 4;
            cur += r.bytes;
            --queued_;
        }
        q.erase(q.begin(), q.begin() + (long)group.size());
        if (q.empty()) per_stream_.erase(s);
        stream_busy_[(size_t)s] = 1;
        ready_.push_back(std::move(group));
        it = pending_.erase(it);
    }
    if (it != pending_.end()) admit_dirty_ = true;  // stopped at a full batch
    for (int32_t s : touched) blocked_mark_[(size_t)s] = 0;
}

// Called with `lk` held; releases it while the backend plans and launches
// (only this thread touches the slot and the launched requests' records
// meanwhile), so submissions and polls do not wait on planning.
int Scheduler::launch_locked(int si, std::unique_lock<std::mutex> &lk) {
    Slot &sl = slots_[(size_t)si];
    const int n = (int)ready_.size();
    std::vector<SchedItem> items((size_t)n);
    const uint64_t t = now();
    sl.item_tickets.assign((size_t)n, {});
    sl.item_done.assign((size_t)n, 0);
    for (int i = 0; i < n; ++i) {
        const Req &r0 = reqs_.at(ready_[(size_t)i].front());
        uint64_t total = 0;
        for (uint64_t tk : ready_[(size_t)i]) {
            Req &r = reqs_.at(tk);
            total += r.count;
            r.state = R_LAUNCHED;
            r.t_launch = t;
        }
        items[(size_t)i] = SchedItem{r0.stream, r0.dtype, total, r0.off};
        sl.item_tickets[(size_t)i] = std::move(ready_[(size_t)i]);
    }
    ready_.clear();
    sl.n_items = n;
    sl.n_done = 0;
    sl.busy = true;
    lk.unlock();
    int rc = be_->launch(si, items);
    if (rc != MTGP_OK) be_->slot_wait(si);  // nothing of it may still write the pool
    lk.lock();
    if (rc != MTGP_OK) {
        for (auto &g : sl.item_tickets)
            for (uint64_t tk : g) {
                auto it = reqs_.find(tk);
                if (it != reqs_.end()) finish_locked(it->second, R_FAILED);
            }
        sl.busy = false;
    }
    return rc;
}

void Scheduler::finish_locked(Req &r, State st) {
    const bool held = r.state == R_ADMITTED || r.state == R_LAUNCHED;
    r.state = st;
    r.t_done = now();
    if (held) stream_busy_[(size_t)r.stream] = 0;
    admit_dirty_ = true;
}

// Scans completion flags of in-flight items; retires finished slots.
bool Scheduler::reap_locked() {
    bool any = false;
    for (size_t si = 0; si < slots_.size(); ++si) {
        Slot &sl = slots_[si];
        if (!sl.busy) continue;
        for (int j = 0; j < sl.n_items; ++j) {
            if (sl.item_done[(size_t)j] || !be_->item_done((int)si, j)) continue;
            sl.item_done[(size_t)j] = 1;
            ++sl.n_done;
            for (uint64_t tk : sl.item_tickets[(size_t)j]) {
                auto it = reqs_.find(tk);
                if (it != reqs_.end()) finish_locked(it->second, R_DONE);
            }
            any = true;
        }
        const int st = be_->slot_poll((int)si);
        if (st > 0) continue;
        if (st == 0 && sl.n_done < sl.n_items) continue;  // flags not yet seen
        if (st == 0) {
            repaired_ += be_->slot_retire((int)si);
        } else {
            // device error: fail whatever the slot still held
            for (int j = 0; j < sl.n_items; ++j) {
                if (sl.item_done[(size_t)j]) continue;
                sl.item_done[(size_t)j] = 1;
                for (uint64_t tk : sl.item_tickets[(size_t)j]) {
                    auto it = reqs_.find(tk);
                    if (it != reqs_.end()) finish_locked(it->second, R_FAILED);
                }
            }
        }
        sl.busy = false;
        any = true;
    }
    return any;
}

void Scheduler::loop() {
    be_->thread_start();
    std::unique_lock<std::mutex> lk(mu_);
    uint64_t ready_since = 0;
    while (true) {
        if (reap_locked()) cv_done_.notify_all();
        if (stop_) break;
        admit_locked();
        int free_slot = -1, busy_slots = 0;
        for (size_t i = 0; i < slots_.size(); ++i) {
            if (!slots_[i].busy) {
                if (free_slot < 0) free_slot = (int)i;
            } else {
                ++busy_slots;
            }
        }
        if (!ready_.empty()) {
            if (ready_since == 0) ready_since = now() | 1;
            // Launch at once when the device is idle or the batch is full;
            // otherwise give late arrivals a short window to join.
            const bool full = (int)ready_.size() >= opts_.max_batch_items;
            const bool waited = now() - ready_since >= opts_.batch_window_ns;
            if (free_slot >= 0 && (busy_slots == 0 || full || waited)) {
                (void)launch_locked(free_slot, lk);
                ready_since = 0;
                cv_done_.notify_all();
                continue;
            }
        }
        const bool inflight = busy_slots > 0;
        if (!inflight && ready_.empty() && (!admit_dirty_ || queued_ == 0)) {
            cv_work_.wait(lk);
        } else {
            cv_work_.wait_for(lk, std::chrono::microseconds(inflight ? 5 : 20));
        }
    }
    // shutdown: wait for in-flight batches, cancel the rest
    for (size_t i = 0; i < slots_.size(); ++i)
        if (slots_[i].busy) be_->slot_wait((int)i);
    reap_locked();
    for (auto &kv : reqs_) {
        Req &r = kv.second;
        if (r.state == R_QUEUED || r.state == R_ADMITTED) finish_locked(r, R_CANCELED);
        if (r.state == R_LAUNCHED) finish_locked(r, R_FAILED);
    }
    ready_.clear();
    cv_done_.notify_all();
}

int Scheduler::poll(uint64_t ticket, int *state, uint64_t *off) {
    if (!state) return fail(MTGP_EINVAL, "NULL state");
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end())
        return fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket);
    const Req &r = it->second;
    switch (r.state) {
        case R_DONE:
            *state = MTGP_DONE;
            if (off) *off = r.off;
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

int Scheduler::wait(uint64_t ticket, uint64_t timeout_ns) {
    std::unique_lock<std::mutex> lk(mu_);
    ++waiters_;
    auto leave = [&](int rc) {
        --waiters_;
        cv_done_.notify_all();  // shutdown() may be waiting for us
        return rc;
    };
    auto done = [&] {
        auto it = reqs_.find(ticket);
        return it == reqs_.end() || it->second.state >= R_DONE;
    };
    if (timeout_ns == 0) {
        cv_done_.wait(lk, done);
    } else if (!cv_done_.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done)) {
        return leave(fail(MTGP_ETIMEDOUT, "ticket %llu not done after %llu ns",
                          (unsigned long long)ticket, (unsigned long long)timeout_ns));
    }
    auto it = reqs_.find(ticket);
    if (it == reqs_.end())
        return leave(fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket));
    if (it->second.state == R_CANCELED) return leave(fail(MTGP_ECANCELED, "ticket cancelled"));
    if (it->second.state == R_FAILED)
        return leave(fail(MTGP_EDEVICE, "request failed on the device"));
    return leave(MTGP_OK);
}

int Scheduler::release(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end())
        return fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket);
    Req &r = it->second;
    if (r.state == R_ADMITTED || r.state == R_LAUNCHED)
        return fail(MTGP_EAGAIN, "ticket %llu is still being generated",
                    (unsigned long long)ticket);
    if (r.state == R_QUEUED) {
        // cancel before admission: drop it from its stream's queue
        auto qit = per_stream_.find(r.stream);
        if (qit != per_stream_.end()) {
            auto &q = qit->second;
            q.erase(std::remove(q.begin(), q.end(), ticket), q.end());
            if (q.empty()) per_stream_.erase(qit);
        }
        --queued_;
    } else if (r.bytes) {
        pool_.release(r.off, r.bytes);  // done, failed or cancelled after admission
    }
    admit_dirty_ = true;
    reqs_.erase(it);
    cv_work_.notify_one();
    return MTGP_OK;
}

int Scheduler::times(uint64_t ticket, uint64_t *t_submit, uint64_t *t_admit, uint64_t *t_launch,
                     uint64_t *t_done) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end())
        return fail(MTGP_ENOENT, "ticket %llu unknown", (unsigned long long)ticket);
    const Req &r = it->second;
    if (t_submit) *t_submit = r.t_submit;
    if (t_admit) *t_admit = r.t_admit;
    if (t_launch) *t_launch = r.t_launch;
    if (t_done) *t_done = r.t_done;
    return MTGP_OK;
}

uint64_t Scheduler::repaired() {
    std::lock_guard<std::mutex> lk(mu_);
    return repaired_;
}

uint64_t Scheduler::pool_used() {
    std::lock_guard<std::mutex> lk(mu_);
    return pool_.used();
}

int Scheduler::replay(const uint64_t *t_arrival_ns, const int32_t *streams,
                      const uint64_t *counts, const int *dtypes, int n, uint64_t *h_latency_ns,
                      uint64_t *h_stages_ns, void *const *keep) {
    if (n < 0 || (n > 0 && (!t_arrival_ns || !streams || !counts || !dtypes || !h_latency_ns)))
        return fail(MTGP_EINVAL, "NULL argument or n=%d", n);
    for (int i = 0; i < n; ++i) {
        if (i > 0 && t_arrival_ns[i] < t_arrival_ns[i - 1])
            return fail(MTGP_EINVAL, "arrival %d before arrival %d", i, i - 1);
        int rc = check_request(streams[i], counts[i], dtypes[i], i);
        if (rc != MTGP_OK) return rc == MTGP_ETOOBIG ? fail(MTGP_EINVAL, "request %d too big", i)
                                                     : rc;
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) return fail(MTGP_ECANCELED, "server is shutting down");
        ++waiters_;  // shutdown() waits for this call to leave
    }
    struct Kept {
        int i;
        uint64_t ticket, off, bytes;
    };
    int rc = MTGP_OK;
    const uint64_t start = now();
    std::vector<uint64_t> tickets((size_t)n, 0);
    std::vector<int> open;  // submitted, not yet finished
    int next = 0, finished = 0;
    while (finished < n && rc == MTGP_OK) {
        std::vector<Kept> kept;
        {
            std::unique_lock<std::mutex> lk(mu_);
            if (stop_) {
                rc = fail(MTGP_ECANCELED, "server is shutting down");
                break;
            }
            const uint64_t t = now();
            bool queued_any = false;
            while (next < n && start + t_arrival_ns[next] <= t &&
                   (int64_t)queued_ < (int64_t)opts_.max_queue) {
                enqueue_locked(streams[next], counts[next], dtypes[next], t,
                               &tickets[(size_t)next]);
                open.push_back(next++);
                queued_any = true;
            }
            if (queued_any) cv_work_.notify_one();
            // collect what finished; its pool bytes go back at once (after
            // the copy for kept results)
            size_t w = 0, k = 0;
            for (; k < open.size(); ++k) {
                const int i = open[k];
                auto it = reqs_.find(tickets[(size_t)i]);
                if (it == reqs_.end()) {
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
                    if (keep && keep[i]) {
                        kept.push_back(Kept{i, r.ticket, r.off, r.bytes});
                        continue;
                    }
                    pool_.release(r.off, r.bytes);
                    admit_dirty_ = true;
                    reqs_.erase(it);
                    ++finished;
                    cv_work_.notify_one();
                } else if (r.state == R_FAILED || r.state == R_CANCELED) {
                    rc = fail(MTGP_EDEVICE, "replayed request %d failed", i);
                    break;
                } else {
                    open[w++] = i;
                }
            }
            if (rc != MTGP_OK) {
                // keep in `open` every request still held: those kept
                // open before k, the unexamined ones from k, and the kept
                // results whose copies will not be made
                open.erase(open.begin() + (long)w, open.begin() + (long)k);
                for (const Kept &kp : kept) open.push_back(kp.i);
                kept.clear();
                break;
            }
            open.resize(w);
        }
        if (!kept.empty()) {
            // outside the lock: the scheduler keeps launching meanwhile
            std::vector<SchedBackend::Copy> copies;
            copies.reserve(kept.size());
            for (const Kept &kp : kept) copies.push_back({kp.off, kp.bytes, keep[kp.i]});
            rc = be_->copy_out(copies);
            std::lock_guard<std::mutex> lk(mu_);
            for (const Kept &kp : kept) {
                pool_.release(kp.off, kp.bytes);
                reqs_.erase(kp.ticket);
                ++finished;
            }
            admit_dirty_ = true;
            cv_work_.notify_one();
            continue;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
    std::unique_lock<std::mutex> lk(mu_);
    if (rc != MTGP_OK) {
        // give back what this call still holds: queued requests are dropped,
        // finished ones released; requests still on the device are waited
        // for unless the loop has stopped
        for (int i : open) {
            const uint64_t tk = tickets[(size_t)i];
            for (;;) {
                auto it = reqs_.find(tk);
                if (it == reqs_.end()) break;
                const State st = it->second.state;
                if (st == R_ADMITTED || st == R_LAUNCHED) {
                    if (stop_ && joined_) break;
                    cv_done_.wait_for(lk, std::chrono::milliseconds(1));
                    continue;
                }
                if (st == R_QUEUED) {
                    auto qit = per_stream_.find(it->second.stream);
                    if (qit != per_stream_.end()) {
                        auto &q = qit->second;
                        q.erase(std::remove(q.begin(), q.end(), tk), q.end());
                        if (q.empty()) per_stream_.erase(qit);
                    }
                    --queued_;
                } else if (it->second.bytes) {
                    pool_.release(it->second.off, it->second.bytes);
                }
                reqs_.erase(it);
                break;
            }
        }
        admit_dirty_ = true;
        cv_work_.notify_one();
    }
    --waiters_;
    cv_done_.notify_all();
    return rc;
}

}  // namespace mtgp
