// sched_driver.cpp -- CPU tests of the serving scheduler (mtgp_sched.cpp)
// against a fake device.  Built with the address/undefined-behaviour and the
// thread sanitizers by the CPU test suite.
//
// The fake device keeps one position per stream (how many outputs the
// stream has produced, standing in for its state in device memory) and
// fills an item's pool range with words that encode (stream, position,
// dtype).  A result is then right exactly when its words continue its
// stream from where the stream's previous completed request stopped, in
// ticket (submission) order -- which is what the real server promises: each
// result is the next `count` outputs of its stream.
//
// Usage: sched_driver [scenario ...]   (no argument: every scenario)
//
// Schedulers and fake devices live on the heap: the thread sanitizer forgets
// a mutex when its memory is freed, not when a stack frame that held it ends.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "mtgp_sched.hpp"

namespace mtgp {
static thread_local std::string g_detail;
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_detail = buf;
    return code;
}
}  // namespace mtgp

using namespace mtgp;
using Clock = std::chrono::steady_clock;

static std::atomic<int> g_fail{0};
#define CHECK(cond, ...)                                                                  \
    do {                                                                                  \
        if (!(cond)) {                                                                    \
            std::fprintf(stderr, "CHECK failed at line %d: %s -- ", __LINE__, #cond);     \
            std::fprintf(stderr, __VA_ARGS__);                                            \
            std::fprintf(stderr, " (detail: %s)\n", mtgp::g_detail.c_str());              \
            g_fail.fetch_add(1);                                                          \
        }                                                                                 \
    } while (0)

// ---------------------------------------------------------------- encoding --

static const uint32_t K1 = 0x9E3779B1u, K2 = 0x85EBCA77u, KF = 0x5BD1E995u;
static uint32_t inv_k1() {
    uint32_t x = K1;  // Newton: x <- x (2 - a x) doubles the correct low bits
    for (int i = 0; i < 5; ++i) x *= 2u - K1 * x;
    return x;
}
static const uint32_t K1INV = inv_k1();
static uint32_t enc(int32_t s, uint64_t pos, int dtype) {
    uint32_t w = (uint32_t)pos * K1 ^ (uint32_t)s * K2;
    return dtype == MTGP_F32 ? w ^ KF : w;
}
static uint64_t dec(int32_t s, uint32_t w, int dtype) {
    if (dtype == MTGP_F32) w ^= KF;
    return (uint32_t)((w ^ (uint32_t)s * K2) * K1INV);
}

// ------------------------------------------------------------- fake device --

class FakeBackend final : public SchedBackend {
   public:
    FakeBackend(int n_streams, uint64_t pool_bytes, int slots, int max_items)
        : mem_((size_t)(pool_bytes / 4) + 1, 0u),
          pool_bytes_(pool_bytes),
          max_items_(max_items),
          pos_((size_t)n_streams, 0),
          slots_((size_t)slots) {}

    // knobs (set before the scheduler starts, or through the atomics)
    std::set<int> fail_launch;       // launch indices that fail at once
    std::set<int> device_error;      // launch indices whose batch ends in a device error
    int base_ns = 2000;              // per item
    double ns_per_output = 0.25;
    std::atomic<int> hold_us{0};     // added to the next launches' run time
    uint64_t repairs_per_batch = 0;
    bool fail_copies = false;

    // observations
    std::atomic<int> launches{0}, retires{0}, thread_starts{0}, max_seen_items{0};
    std::mutex log_mu;
    std::vector<std::vector<SchedItem>> log;

    const uint32_t *words(uint64_t off) const { return mem_.data() + off / 4; }
    uint64_t position(int32_t s) const { return pos_[(size_t)s]; }

    void thread_start() override { thread_starts.fetch_add(1); }

    int launch(int si, const std::vector<SchedItem> &items) override {
        const int k = launches.fetch_add(1);
        const auto now = Clock::now();
        Rec &sl = slots_[(size_t)si];
        CHECK(now >= sl.done_t, "slot %d relaunched before its batch finished", si);
        CHECK(!items.empty() && (int)items.size() <= max_items_, "batch of %zu items",
              items.size());
        int m = max_seen_items.load();
        while ((int)items.size() > m && !max_seen_items.compare_exchange_weak(m, (int)items.size())) {
        }
        std::set<int32_t> seen;
        for (const SchedItem &it : items) {
            CHECK(seen.insert(it.stream).second, "stream %d twice in one batch", it.stream);
            CHECK(it.off % 256 == 0, "item offset %llu not 256-aligned",
                  (unsigned long long)it.off);
            CHECK(it.count > 0 && it.off + it.count * 4 <= pool_bytes_, "item outside the pool");
            CHECK(it.dtype == MTGP_U32 || it.dtype == MTGP_F32, "dtype %d", it.dtype);
            // the stream must not still run in another slot
            for (size_t o = 0; o < slots_.size(); ++o) {
                if ((int)o == si) continue;
                const Rec &r = slots_[o];
                for (size_t j = 0; j < r.items.size(); ++j) {
                    const bool running = r.dev_err ? now < r.done_t : now < r.item_t[j];
                    CHECK(!(running && r.items[j].stream == it.stream),
                          "stream %d launched while running in slot %zu", it.stream, o);
                }
            }
        }
        if (fail_launch.count(k)) {
            sl.items.clear();
            sl.item_t.clear();
            sl.done_t = now;
            sl.dev_err = false;
            return fail(MTGP_EDEVICE, "injected launch failure %d", k);
        }
        sl.dev_err = device_error.count(k) != 0;
        sl.items = items;
        sl.item_t.resize(items.size());
        const auto t0 = now + std::chrono::microseconds(hold_us.load());
        auto done = t0;
        for (size_t j = 0; j < items.size(); ++j) {
            const SchedItem &it = items[j];
            if (!sl.dev_err) {
                uint64_t &p = pos_[(size_t)it.stream];
                uint32_t *w = mem_.data() + it.off / 4;
                for (uint64_t q = 0; q < it.count; ++q) w[q] = enc(it.stream, p + q, it.dtype);
                p += it.count;
            }
            sl.item_t[j] = t0 + std::chrono::nanoseconds(
                                    base_ns + (int64_t)(ns_per_output * (double)it.count));
            done = std::max(done, sl.item_t[j]);
        }
        sl.done_t = done + std::chrono::microseconds(1);
        std::lock_guard<std::mutex> lk(log_mu);
        log.push_back(items);
        return MTGP_OK;
    }

    bool item_done(int si, int j) override {
        const Rec &sl = slots_[(size_t)si];
        return !sl.dev_err && Clock::now() >= sl.item_t[(size_t)j];
    }

    int slot_poll(int si) override {
        const Rec &sl = slots_[(size_t)si];
        if (Clock::now() < sl.done_t) return 1;
        return sl.dev_err ? -1 : 0;
    }

    uint64_t slot_retire(int) override {
        retires.fetch_add(1);
        return repairs_per_batch;
    }

    void slot_wait(int si) override { std::this_thread::sleep_until(slots_[(size_t)si].done_t); }

    int copy_out(const std::vector<Copy> &copies) override {
        if (fail_copies) return fail(MTGP_EDEVICE, "injected copy failure");
        for (const Copy &c : copies) std::memcpy(c.dst, (const char *)mem_.data() + c.off, c.bytes);
        return MTGP_OK;
    }

   private:
    struct Rec {
        std::vector<SchedItem> items;
        std::vector<Clock::time_point> item_t;
        Clock::time_point done_t{};
        bool dev_err = false;
    };
    std::vector<uint32_t> mem_;
    uint64_t pool_bytes_;
    int max_items_;
    std::vector<uint64_t> pos_;
    std::vector<Rec> slots_;
};

// ------------------------------------------------------------------ helpers --

struct Done {
    uint64_t ticket;
    int32_t stream;
    uint64_t count;
    uint64_t p0;  // position of the first output
};

// Reads a finished request's words; they must continue one position of the
// stream, in the request's dtype.
static bool check_result(Scheduler &S, FakeBackend &B, uint64_t tk, int32_t s, uint64_t count,
                         int dtype, std::vector<Done> *out) {
    int st = -1;
    uint64_t off = ~0ull;
    int rc = S.poll(tk, &st, &off);
    CHECK(rc == MTGP_OK && st == MTGP_DONE, "ticket %llu: rc %d state %d", (unsigned long long)tk,
          rc, st);
    if (rc != MTGP_OK || st != MTGP_DONE) return false;
    const uint32_t *w = B.words(off);
    const uint64_t p0 = dec(s, w[0], dtype);
    for (uint64_t q = 0; q < count; ++q)
        if (w[q] != enc(s, p0 + q, dtype)) {
            CHECK(false, "ticket %llu word %llu: not stream %d position %llu dtype %d",
                  (unsigned long long)tk, (unsigned long long)q, s,
                  (unsigned long long)(p0 + q), dtype);
            return false;
        }
    if (out) out->push_back(Done{tk, s, count, p0});
    return true;
}

// Every stream's completed requests, in ticket order, must tile its
// positions from 0 without gaps; the device's final position closes it.
static void check_chains(std::vector<Done> done, FakeBackend &B, int n_streams) {
    std::sort(done.begin(), done.end(),
              [](const Done &a, const Done &b) { return a.ticket < b.ticket; });
    std::vector<uint64_t> next((size_t)n_streams, 0);
    for (const Done &d : done) {
        CHECK(d.p0 == next[(size_t)d.stream],
              "stream %d ticket %llu starts at %llu, expected %llu", d.stream,
              (unsigned long long)d.ticket, (unsigned long long)d.p0,
              (unsigned long long)next[(size_t)d.stream]);
        next[(size_t)d.stream] = d.p0 + d.count;
    }
    for (int s = 0; s < n_streams; ++s)
        CHECK(next[(size_t)s] == B.position(s), "stream %d: results end at %llu, device at %llu",
              s, (unsigned long long)next[(size_t)s], (unsigned long long)B.position(s));
}

static SchedOpts opts(int inflight, int items, int queue, uint64_t window_ns) {
    SchedOpts o;
    o.max_inflight = inflight;
    o.max_batch_items = items;
    o.max_queue = queue;
    o.batch_window_ns = window_ns;
    return o;
}

static bool wait_until(const std::function<bool()> &pred, int ms) {
    const auto end = Clock::now() + std::chrono::milliseconds(ms);
    while (!pred()) {
        if (Clock::now() > end) return false;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return true;
}

// --------------------------------------------------------------- scenarios --

// Random allocations and releases against a byte map: ranges are aligned,
// in bounds and disjoint, free ranges coalesce, and `used` adds up.
static void pool_consistency() {
    std::mt19937_64 rng(7);
    const uint64_t size = 1 << 20;
    Pool P(size);
    std::vector<uint8_t> owner(size, 0);
    struct A {
        uint64_t off, bytes;
    };
    std::vector<A> live;
    uint64_t used = 0;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3 != 0) {
            const uint64_t bytes = 1 + rng() % (rng() % 4 == 0 ? 65536 : 2048);
            uint64_t off = 0;
            if (!P.alloc(bytes, &off)) continue;
            CHECK(off % 256 == 0 && off + bytes <= size, "range %llu+%llu",
                  (unsigned long long)off, (unsigned long long)bytes);
            for (uint64_t b = off; b < off + bytes && b < size; ++b) {
                if (owner[b]) {
                    CHECK(false, "byte %llu handed out twice", (unsigned long long)b);
                    break;
                }
                owner[b] = 1;
            }
            live.push_back(A{off, bytes});
            used += bytes;
        } else {
            const size_t k = rng() % live.size();
            A a = live[k];
            live[k] = live.back();
            live.pop_back();
            // return it in one or two pieces (fused requests are released one by one)
            const uint64_t cut = a.bytes > 1 && rng() % 2 ? 1 + rng() % (a.bytes - 1) : a.bytes;
            P.release(a.off, cut);
            if (cut < a.bytes) P.release(a.off + cut, a.bytes - cut);
            std::fill(owner.begin() + (long)a.off, owner.begin() + (long)(a.off + a.bytes), 0);
            used -= a.bytes;
        }
        CHECK(P.used() == used, "used %llu vs %llu", (unsigned long long)P.used(),
              (unsigned long long)used);
    }
    uint64_t prev_end = ~0ull, free_bytes = 0;
    for (const auto &kv : P.free_ranges()) {
        CHECK(kv.first != prev_end, "adjacent free ranges at %llu not merged",
              (unsigned long long)kv.first);
        for (uint64_t b = kv.first; b < kv.first + kv.second; ++b)
            if (owner[b]) {
                CHECK(false, "free range covers live byte %llu", (unsigned long long)b);
                break;
            }
        prev_end = kv.first + kv.second;
        free_bytes += kv.second;
    }
    CHECK(free_bytes + used == size, "free %llu + used %llu != %llu",
          (unsigned long long)free_bytes, (unsigned long long)used, (unsigned long long)size);
    for (const A &a : live) P.release(a.off, a.bytes);
    CHECK(P.used() == 0 && P.free_ranges().size() == 1, "pool not whole after releasing all");
}

// Several client threads submit to shared streams under pool pressure,
// wait, check and release; every stream's results tile its positions.
static void threads_fifo_pool_pressure() {
    const int n_streams = 24, n_threads = 6, per_thread = 400;
    const uint64_t pool = 256 << 10;
    auto Bp = std::make_unique<FakeBackend>(n_streams, pool, 3, 16);
    FakeBackend &B = *Bp;
    auto Sp = std::make_unique<Scheduler>(&B, n_streams, pool, opts(3, 16, 1 << 20, 2000));
    Scheduler &S = *Sp;
    S.start();
    std::mutex mu;
    std::vector<Done> all;
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; ++t)
        th.emplace_back([&, t] {
            std::mt19937_64 rng(100 + t);
            std::vector<Done> mine;
            struct Out {
                uint64_t tk;
                int32_t s;
                uint64_t count;
                int dtype;
            };
            std::vector<Out> window;
            // results are checked and released as they complete (a client
            // that holds finished results can starve the pool)
            auto drain = [&](size_t keep) {
                while (window.size() > keep) {
                    bool any = false;
                    for (size_t k = 0; k < window.size();) {
                        int st = -1;
                        CHECK(S.poll(window[k].tk, &st, nullptr) == MTGP_OK, "poll");
                        if (st == MTGP_PENDING) {
                            ++k;
                            continue;
                        }
                        const Out o = window[k];
                        window.erase(window.begin() + (long)k);
                        CHECK(S.wait(o.tk, 0) == MTGP_OK, "wait %llu", (unsigned long long)o.tk);
                        check_result(S, B, o.tk, o.s, o.count, o.dtype, &mine);
                        CHECK(S.release(o.tk) == MTGP_OK, "release");
                        any = true;
                    }
                    if (!any) std::this_thread::sleep_for(std::chrono::microseconds(20));
                }
            };
            for (int i = 0; i < per_thread; ++i) {
                Out o;
                o.s = (int32_t)(rng() % n_streams);
                o.count = 1 + rng() % (rng() % 8 == 0 ? 16384 : 700);
                o.dtype = rng() % 4 == 0 ? MTGP_F32 : MTGP_U32;
                CHECK(S.submit(o.s, o.count, o.dtype, &o.tk) == MTGP_OK, "submit");
                window.push_back(o);
                drain(6);
            }
            drain(0);
            std::lock_guard<std::mutex> lk(mu);
            all.insert(all.end(), mine.begin(), mine.end());
        });
    for (auto &x : th) x.join();
    CHECK((int)all.size() == n_threads * per_thread, "%zu results", all.size());
    check_chains(all, B, n_streams);
    CHECK(S.pool_used() == 0, "pool still holds %llu bytes", (unsigned long long)S.pool_used());
    S.shutdown();
    CHECK(B.thread_starts.load() == 1, "thread_start ran %d times", B.thread_starts.load());
    CHECK(B.max_seen_items.load() <= 16, "batch of %d items", B.max_seen_items.load());
}

// While the device is busy, a stream's consecutive same-dtype requests are
// fused into one item over one contiguous range; a dtype change ends the run.
static void fusion_and_order() {
    const uint64_t pool = 1 << 20;
    auto Bp = std::make_unique<FakeBackend>(4, pool, 1, 64);
    FakeBackend &B = *Bp;
    auto Sp = std::make_unique<Scheduler>(&B, 4, pool, opts(1, 64, 1024, 0));
    Scheduler &S = *Sp;
    S.start();
    B.hold_us = 200000;  // the first batch runs 0.2 s
    uint64_t t0, t[6];
    CHECK(S.submit(1, 100, MTGP_U32, &t0) == MTGP_OK, "submit");
    CHECK(wait_until([&] { return B.launches.load() == 1; }, 5000), "first launch");
    B.hold_us = 0;
    const int dt[6] = {MTGP_U32, MTGP_U32, MTGP_U32, MTGP_F32, MTGP_F32, MTGP_U32};
    const uint64_t cnt[6] = {10, 20, 30, 40, 50, 60};
    // one submission, so that admission sees all six queued (requests that
    // arrive one by one may be admitted one by one: admission does not wait
    // for a free launch slot)
    const int32_t st0[6] = {0, 0, 0, 0, 0, 0};
    CHECK(S.submit_many(st0, cnt, dt, 6, t) == MTGP_OK, "submit_many");
    for (int i = 0; i < 6; ++i) CHECK(S.wait(t[i], 0) == MTGP_OK, "wait %d", i);
    CHECK(S.wait(t0, 0) == MTGP_OK, "wait first");
    std::vector<Done> done;
    for (int i = 0; i < 6; ++i) check_result(S, B, t[i], 0, cnt[i], dt[i], &done);
    check_result(S, B, t0, 1, 100, MTGP_U32, &done);
    // runs: {10,20,30} u32, {40,50} f32, {60} u32 -> three items of stream 0
    std::vector<uint64_t> counts0;
    {
        std::lock_guard<std::mutex> lk(B.log_mu);
        for (auto &batch : B.log)
            for (auto &it : batch)
                if (it.stream == 0) counts0.push_back(it.count);
    }
    CHECK(counts0 == std::vector<uint64_t>({60, 90, 60}), "stream 0 items: %zu", counts0.size());
    uint64_t off[6];
    for (int i = 0; i < 6; ++i) {
        int st;
        S.poll(t[i], &st, &off[i]);
    }
    CHECK(off[1] == off[0] + 40 && off[2] == off[1] + 80, "fused u32 run not contiguous");
    CHECK(off[4] == off[3] + 160, "fused f32 run not contiguous");
    uint64_t ts, ta, tl, td;
    CHECK(S.times(t[2], &ts, &ta, &tl, &td) == MTGP_OK && ts <= ta && ta <= tl && tl <= td,
          "timestamps out of order");
    check_chains(done, B, 4);
    for (int i = 0; i < 6; ++i) S.release(t[i]);
    S.release(t0);
    CHECK(S.pool_used() == 0, "pool not empty");
}

// A fused run longer than the pool is cut so that it can be admitted.
static void fusion_capped_by_pool() {
    const uint64_t pool = 64 << 10;
    auto Bp = std::make_unique<FakeBackend>(2, pool, 1, 8);
    FakeBackend &B = *Bp;
    auto Sp = std::make_unique<Scheduler>(&B, 2, pool, opts(1, 8, 1024, 0));
    Scheduler &S = *Sp;
    S.start();
    B.hold_us = 100000;
    uint64_t tb;
    CHECK(S.submit(1, 16, MTGP_U32, &tb) == MTGP_OK, "submit");
    CHECK(wait_until([&] { return B.launches.load() == 1; }, 5000), "first launch");
    B.hold_us = 0;
    // three requests of 0.4 pool each: two fused would fit, three would not
    const uint64_t c = (pool / 4) * 4 / 10;
    uint64_t t[3];
    for (int i = 0; i < 3; ++i) CHECK(S.submit(0, c, MTGP_U32, &t[i]) == MTGP_OK, "submit");
    std::vector<Done> done;
    for (int i = 0; i < 3; ++i) {
        CHECK(S.wait(t[i], 2000000000ull) == MTGP_OK, "wait %d (a run longer than the pool)", i);
        check_result(S, B, t[i], 0, c, MTGP_U32, &done);
        S.release(t[i]);
    }
    CHECK(S.wait(tb, 0) == MTGP_OK, "wait");
    check_result(S, B, tb, 1, 16, MTGP_U32, &done);
    S.release(tb);
    check_chains(done, B, 2);
}

// Argument checks, a full queue, all-or-nothing submit_many, unknown
// tickets, release while running, and a wait that times out.
static void admission_errors() {
    const uint64_t pool = 4096;
    auto Bp = std::make_unique<FakeBackend>(3, pool, 1, 4);
    FakeBackend &B = *Bp;
    auto Sp = std::make_unique<Scheduler>(&B, 3, pool, opts(1, 4, 5, 0));
    Scheduler &S = *Sp;
    uint64_t tk;
    CHECK(S.submit(3, 1, MTGP_U32, &tk) == MTGP_EINVAL, "stream out of range");
    CHECK(S.submit(-1, 1, MTGP_U32, &tk) == MTGP_EINVAL, "negative stream");
    CHECK(S.submit(0, 0, MTGP_U32, &tk) == MTGP_EINVAL, "count 0");
    CHECK(S.submit(0, 1, 7, &tk) == MTGP_EINVAL, "dtype");
    CHECK(S.submit(0, pool / 4 + 1, MTGP_U32, &tk) == MTGP_ETOOBIG, "larger than the pool");
    CHECK(S.submit(0, ~0ull / 2, MTGP_U32, &tk) == MTGP_ETOOBIG, "count*4 overflows");
    CHECK(S.submit(0, 1, MTGP_U32, nullptr) == MTGP_EINVAL, "NULL ticket");
    // the thread is not started yet: requests stay queued
    uint64_t q[5];
    for (int i = 0; i < 5; ++i) CHECK(S.submit(i % 3, 8, MTGP_U32, &q[i]) == MTGP_OK, "submit");
    CHECK(S.submit(0, 8, MTGP_U32, &tk) == MTGP_EAGAIN, "queue full");
    CHECK(S.release(q[4]) == MTGP_OK, "release a queued request");
    int32_t ss[2] = {0, 1};
    uint64_t cc[2] = {8, 8}, tt[2] = {0, 0};
    int dd[2] = {MTGP_U32, MTGP_U32};
    CHECK(S.submit_many(ss, cc, dd, 2, tt) == MTGP_EAGAIN, "submit_many beyond the queue");
    CHECK(S.submit_many(ss, cc, dd, 1, tt) == MTGP_OK, "submit_many into the last place");
    dd[1] = 9;
    CHECK(S.submit_many(ss, cc, dd, 2, tt) == MTGP_EINVAL, "submit_many with a bad dtype");
    CHECK(S.submit_many(ss, cc, dd, -1, tt) == MTGP_EINVAL, "submit_many n < 0");
    int st;
    CHECK(S.poll(12345, &st, nullptr) == MTGP_ENOENT, "unknown ticket");
    CHECK(S.release(12345) == MTGP_ENOENT, "release unknown");
    CHECK(S.poll(q[0], &st, nullptr) == MTGP_OK && st == MTGP_PENDING, "queued is pending");
    CHECK(S.poll(q[4], &st, nullptr) == MTGP_ENOENT, "released ticket is gone");
    B.hold_us = 300000;
    S.start();
    CHECK(wait_until([&] { return B.launches.load() >= 1; }, 5000), "launch");
    CHECK(S.release(q[0]) == MTGP_EAGAIN, "release while generating");
    CHECK(S.wait(q[0], 1000000) == MTGP_ETIMEDOUT, "wait 1 ms on a 0.3 s batch");
    B.hold_us = 0;
    std::vector<Done> done;
    for (int i = 0; i < 4; ++i) {
        CHECK(S.wait(q[i], 0) == MTGP_OK, "wait %d", i);
        check_result(S, B, q[i], i % 3, 8, MTGP_U32, &done);
        S.release(q[i]);
    }
    CHECK(S.wait(tt[0], 0) == MTGP_OK, "wait");
    check_result(S, B, tt[0], 0, 8, MTGP_U32, &done);
    S.release(tt[0]);
    check_chains(done, B, 3);
    CHECK(S.wait(q[0], 0) == MTGP_ENOENT, "wait on a released ticket");
}

// A launch that fails and a batch that ends in a device error fail their
// requests (and nothing else); the streams go on from where they were.
static void launch_and_device_failures() {
    const uint64_t pool = 1 << 20;
    auto Bp = std::make_unique<FakeBackend>(4, pool, 2, 8);
    FakeBackend &B = *Bp;
    B.fail_launch = {2, 5};
    B.device_error = {3};
    B.repairs_per_batch = 2;
    auto Sp = std::make_unique<Scheduler>(&B, 4, pool, opts(2, 8, 1024, 0));
    Scheduler &S = *Sp;
    S.start();
    std::vector<Done> done;
    int failed = 0;
    for (int i = 0; i < 40; ++i) {
        uint64_t tk;
        const int32_t s = i % 4;
        const uint64_t c = 50 + (uint64_t)i;
        CHECK(S.submit(s, c, MTGP_U32, &tk) == MTGP_OK, "submit");
        const int rc = S.wait(tk, 0);
        CHECK(rc == MTGP_OK || rc == MTGP_EDEVICE, "wait rc %d", rc);
        int st;
        CHECK(S.poll(tk, &st, nullptr) == MTGP_OK, "poll");
        if (rc == MTGP_OK) {
            check_result(S, B, tk, s, c, MTGP_U32, &done);
        } else {
            CHECK(st == MTGP_FAILED, "failed request polls as %d", st);
            ++failed;
        }
        CHECK(S.release(tk) == MTGP_OK, "release");
    }
    CHECK(failed == 3, "%d failed requests (launches 2, 3, 5 fail)", failed);
    check_chains(done, B, 4);
    CHECK(S.pool_used() == 0, "pool holds %llu bytes", (unsigned long long)S.pool_used());
    S.shutdown();
    CHECK(S.repaired() == 2 * (uint64_t)B.retires.load() && B.retires.load() == 37,
          "repaired %llu after %d retired batches", (unsigned long long)S.repaired(),
          B.retires.load());
}

// Shutdown with a batch running, requests queued and threads waiting: the
// running ones finish, the queued ones end cancelled, every waiter returns
// before shutdown does, and nothing is accepted afterwards.
static void shutdown_with_waiters() {
    const uint64_t pool = 1 << 20;
    auto Bp = std::make_unique<FakeBackend>(4, pool, 1, 4);
    FakeBackend &B = *Bp;
    auto Sp = std::make_unique<Scheduler>(&B, 4, pool, opts(1, 4, 1024, 0));
    Scheduler &S = *Sp;
    S.start();
    B.hold_us = 150000;
    uint64_t run[2];
    {
        // one submission, so that both are admitted into the first batch
        int32_t ss[2] = {0, 1};
        uint64_t cc[2] = {64, 64};
        int dd[2] = {MTGP_U32, MTGP_U32};
        CHECK(S.submit_many(ss, cc, dd, 2, run) == MTGP_OK, "submit_many");
    }
    CHECK(wait_until([&] { return B.launches.load() == 1; }, 5000), "launch");
    uint64_t queued[3];
    for (int i = 0; i < 3; ++i) CHECK(S.submit(0, 64, MTGP_U32, &queued[i]) == MTGP_OK, "submit");
    std::atomic<int> ok{0}, canceled{0}, other{0};
    std::vector<std::thread> th;
    for (uint64_t tk : {run[0], run[1], queued[0], queued[1], queued[2]})
        th.emplace_back([&, tk] {
            const int rc = S.wait(tk, 0);
            (rc == MTGP_OK ? ok : rc == MTGP_ECANCELED ? canceled : other).fetch_add(1);
        });
    std::this_thread::sleep_for(std::chrono::milliseconds(20));
    S.shutdown();
    for (auto &x : th) x.join();
    CHECK(ok.load() == 2 && canceled.load() == 3 && other.load() == 0,
          "waiters: %d ok, %d cancelled, %d other", ok.load(), canceled.load(), other.load());
    uint64_t tk;
    CHECK(S.submit(2, 8, MTGP_U32, &tk) == MTGP_ECANCELED, "submit after shutdown");
    int st;
    CHECK(S.poll(queued[0], &st, nullptr) == MTGP_ECANCELED && st == MTGP_FAILED,
          "cancelled request polls as failed");
    CHECK(S.poll(run[0], &st, nullptr) == MTGP_OK && st == MTGP_DONE, "finished one is done");
}

// Trace replay keeps chosen results and returns every pool byte; its
// latencies and stages are filled in.
static void replay_keeps_results() {
    const int n_streams = 16, n = 3000;
    const uint64_t pool = 512 << 10;
    auto Bp = std::make_unique<FakeBackend>(n_streams, pool, 4, 32);
    FakeBackend &B = *Bp;
    auto Sp = std::make_unique<Scheduler>(&B, n_streams, pool, opts(4, 32, 1 << 20, 1000));
    Scheduler &S = *Sp;
    S.start();
    std::mt19937_64 rng(11);
    std::vector<uint64_t> arr(n), cnt(n), lat(n, ~0ull), stages(3 * (size_t)n, ~0ull);
    std::vector<int32_t> str(n);
    std::vector<int> dt(n);
    std::vector<std::vector<uint32_t>> kept(n);
    std::vector<void *> keep(n, nullptr);
    uint64_t t = 0;
    for (int i = 0; i < n; ++i) {
        t += rng() % 3000;
        arr[i] = t;
        str[i] = (int32_t)(rng() % n_streams);
        cnt[i] = 1 + rng() % 3000;
        dt[i] = rng() % 3 == 0 ? MTGP_F32 : MTGP_U32;
        if (i % 7 == 0) {
            kept[i].assign(cnt[i], 0u);
            keep[i] = kept[i].data();
        }
    }
    const int rc = S.replay(arr.data(), str.data(), cnt.data(), dt.data(), n, lat.data(),
                            stages.data(), keep.data());
    CHECK(rc == MTGP_OK, "replay rc %d", rc);
    CHECK(S.pool_used() == 0, "replay left %llu pool bytes", (unsigned long long)S.pool_used());
    for (int i = 0; i < n; ++i) {
        CHECK(lat[i] != ~0ull, "latency %d not set", i);
        // submitted at or after its arrival: the stages fit in the latency
        CHECK(stages[3 * (size_t)i] + stages[3 * (size_t)i + 1] + stages[3 * (size_t)i + 2] <=
                  lat[i],
              "stages of %d", i);
        if (!keep[i]) continue;
        const uint64_t p0 = dec(str[i], kept[i][0], dt[i]);
        for (uint64_t q = 0; q < cnt[i]; ++q)
            if (kept[i][q] != enc(str[i], p0 + q, dt[i])) {
                CHECK(false, "kept result %d word %llu", i, (unsigned long long)q);
                break;
            }
    }
    // the kept results lie where their stream's earlier requests stopped
    std::vector<uint64_t> next((size_t)n_streams, 0);
    for (int i = 0; i < n; ++i) {
        if (keep[i])
            CHECK(dec(str[i], kept[i][0], dt[i]) == next[(size_t)str[i]],
                  "kept result %d starts at the wrong position", i);
        next[(size_t)str[i]] += cnt[i];
    }
    for (int s = 0; s < n_streams; ++s)
        CHECK(next[(size_t)s] == B.position(s), "stream %d ends at %llu", s,
              (unsigned long long)B.position(s));
    CHECK(S.replay(arr.data(), str.data(), cnt.data(), dt.data(), 0, lat.data(), nullptr,
                   nullptr) == MTGP_OK,
          "empty replay");
    std::swap(arr[0], arr[1]);
    arr[1] = arr[0] + 1;
    arr[0] = arr[1] + 5;
    CHECK(S.replay(arr.data(), str.data(), cnt.data(), dt.data(), 2, lat.data(), nullptr,
                   nullptr) == MTGP_EINVAL,
          "arrivals out of order");
}

// A replay that meets a failed launch returns an error and gives back every
// pool byte it held once the device is done; the scheduler serves on.
static void replay_failure_cleanup() {
    const int n_streams = 8, n = 400;
    const uint64_t pool = 256 << 10;
    auto Bp = std::make_unique<FakeBackend>(n_streams, pool, 2, 8);
    FakeBackend &B = *Bp;
    B.fail_launch = {2};
    auto Sp = std::make_unique<Scheduler>(&B, n_streams, pool, opts(2, 8, 1 << 20, 0));
    Scheduler &S = *Sp;
    S.start();
    std::vector<uint64_t> arr(n, 0), cnt(n), lat(n);
    std::vector<int32_t> str(n);
    std::vector<int> dt(n, MTGP_U32);
    for (int i = 0; i < n; ++i) {
        arr[i] = (uint64_t)i * 5000;  // spread out, so that there are many launches
        str[i] = i % n_streams;
        cnt[i] = 100 + (uint64_t)i;
    }
    const int rc = S.replay(arr.data(), str.data(), cnt.data(), dt.data(), n, lat.data(), nullptr,
                            nullptr);
    CHECK(rc == MTGP_EDEVICE && B.launches.load() > 2, "replay rc %d after %d launches", rc,
          B.launches.load());
    CHECK(wait_until([&] { return S.pool_used() == 0; }, 5000), "replay left %llu pool bytes",
          (unsigned long long)S.pool_used());
    uint64_t tk;
    CHECK(S.submit(0, 10, MTGP_U32, &tk) == MTGP_OK && S.wait(tk, 0) == MTGP_OK,
          "serving after a failed replay");
    check_result(S, B, tk, 0, 10, MTGP_U32, nullptr);
    S.release(tk);
    B.fail_copies = true;
    std::vector<uint32_t> buf(200);
    void *keep[1] = {buf.data()};
    CHECK(S.replay(arr.data(), str.data(), cnt.data(), dt.data(), 1, lat.data(), nullptr, keep) ==
              MTGP_EDEVICE,
          "failed copy");
    CHECK(wait_until([&] { return S.pool_used() == 0; }, 5000), "copy failure left pool bytes");
}

// Shutdown while another thread replays: the replay returns (cancelled)
// before shutdown does.
static void shutdown_during_replay() {
    const int n_streams = 4, n = 2000;
    const uint64_t pool = 64 << 10;
    auto Bp = std::make_unique<FakeBackend>(n_streams, pool, 2, 8);
    FakeBackend &B = *Bp;
    B.base_ns = 50000;
    auto Sp = std::make_unique<Scheduler>(&B, n_streams, pool, opts(2, 8, 1 << 20, 0));
    Scheduler &S = *Sp;
    S.start();
    std::vector<uint64_t> arr(n), cnt(n, 500), lat(n);
    std::vector<int32_t> str(n);
    std::vector<int> dt(n, MTGP_U32);
    for (int i = 0; i < n; ++i) {
        arr[i] = (uint64_t)i * 20000;
        str[i] = i % n_streams;
    }
    std::atomic<int> rc{1};
    std::thread r([&] {
        rc = S.replay(arr.data(), str.data(), cnt.data(), dt.data(), n, lat.data(), nullptr,
                      nullptr);
    });
    std::this_thread::sleep_for(std::chrono::milliseconds(30));
    S.shutdown();
    r.join();
    CHECK(rc.load() == MTGP_ECANCELED, "replay rc %d after shutdown", rc.load());
}

// With a long batch window and a free slot, ready items wait for the batch
// to fill while the device is busy, and at most max_batch_items go together.
static void batch_cap_and_window() {
    const uint64_t pool = 1 << 20;
    auto Bp = std::make_unique<FakeBackend>(64, pool, 2, 5);
    FakeBackend &B = *Bp;
    auto Sp = std::make_unique<Scheduler>(&B, 64, pool, opts(2, 5, 1024, 50000000));
    Scheduler &S = *Sp;
    S.start();
    std::vector<uint64_t> tk(23);
    for (int i = 0; i < 23; ++i) CHECK(S.submit(i, 10, MTGP_U32, &tk[(size_t)i]) == MTGP_OK, "submit");
    std::vector<Done> done;
    for (int i = 0; i < 23; ++i) {
        CHECK(S.wait(tk[(size_t)i], 0) == MTGP_OK, "wait");
        check_result(S, B, tk[(size_t)i], i, 10, MTGP_U32, &done);
        S.release(tk[(size_t)i]);
    }
    CHECK(B.max_seen_items.load() <= 5, "batch of %d items", B.max_seen_items.load());
    CHECK(B.launches.load() >= 5, "%d launches for 23 items at 5 per batch", B.launches.load());
    check_chains(done, B, 64);
}

int main(int argc, char **argv) {
    const std::vector<std::pair<const char *, void (*)()>> all = {
        {"pool_consistency", pool_consistency},
        {"threads_fifo_pool_pressure", threads_fifo_pool_pressure},
        {"fusion_and_order", fusion_and_order},
        {"fusion_capped_by_pool", fusion_capped_by_pool},
        {"admission_errors", admission_errors},
        {"launch_and_device_failures", launch_and_device_failures},
        {"shutdown_with_waiters", shutdown_with_waiters},
        {"replay_keeps_results", replay_keeps_results},
        {"replay_failure_cleanup", replay_failure_cleanup},
        {"shutdown_during_replay", shutdown_during_replay},
        {"batch_cap_and_window", batch_cap_and_window},
    };
    int ran = 0;
    for (const auto &sc : all) {
        bool pick = argc < 2;
        for (int i = 1; i < argc; ++i) pick |= std::strcmp(argv[i], sc.first) == 0;
        if (!pick) continue;
        const int before = g_fail.load();
        const auto t0 = Clock::now();
        sc.second();
        const double ms =
            std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        std::printf("%s %s (%.0f ms)\n", g_fail.load() == before ? "PASS" : "FAIL", sc.first, ms);
        std::fflush(stdout);
        ++ran;
    }
    std::printf("%d scenarios, %d failed checks\n", ran, g_fail.load());
    return g_fail.load() == 0 && ran > 0 ? 0 : 1;
}
