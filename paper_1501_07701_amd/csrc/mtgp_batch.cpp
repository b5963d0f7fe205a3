// mtgp_batch.cpp -- batched generation: jump-ahead data per stream,
// segment planning, workspace layout, uploads, hipGraph replay, autotuner.
//
// Jump-ahead.  For a stream with words x_0, x_1, ... (x_0..x_{N-1} its state
// at the start of a call), the sequence x_1, x_2, ... lies in the orbit of
// the GF(2)-linear state transition, so a polynomial p of degree D <= mexp
// annihilates it: sum_i p_i x_{t+i} = 0 for all t >= 1 (word-wise XOR).
// Then for g = x^J mod p, x_{t+J} = XOR_i g_i x_{t+i} for t >= 1, and the
// state J+1 outputs ahead, x_{J+1} .. x_{J+N}, needs only x_1 .. x_{D+N}.
// A split request therefore runs as
//   A: a prefix item: the first P = D+1 outputs, also dumping x_0..x_{N+D};
//   B: one jump per later segment, which starts at output c*lseg
//      (c >= c0 = ceil((P+1)/lseg)): its state from g_c = x^(c*lseg-1) mod p,
//      evaluated as one item per 512 state words;
//   C: every segment (the first one continues after the prefix up to
//      c0*lseg), each checking its end state against the next segment's
//      start state.
// p is built per stream from one orbit: Berlekamp-Massey on two linear
// functionals of 2*mexp+127 words (lcm of the two), checked on the device
// over mexp further positions, all 32 bit functionals if the check fails.
// The orbit is the stream's seed status's while its state was last set by
// seeding (the seed orbit holds every later state of the stream), else the
// orbit of its current state (after mtgp_state_import or
// mtgp_load_params); a stream whose state moved to a new orbit gets the lcm
// of the old and the new polynomial.
//
// The segment checks make every split request exact whatever p is: if all
// checks pass, each segment started from the true state (by induction from
// the prefix); if one fails, the batch's last launch (one check item per
// split request, after every segment has finished) regenerates the request
// in order from its start state (kept by the prefix) and logs the stream,
// which the host then rebuilds from its current state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "mtgp.h"
#include "mtgp_host.hpp"
#include "mtgp_internal.hpp"
#include "mtgp_poly.hpp"

namespace mtgp {

struct StreamJump {
    int status = 0;  // 1 usable, -1 never split this stream
    int D = 0;       // degree of the annihilating polynomial p
    bool has_seed_orbit = false;  // p annihilates the seed status's orbit
    std::unique_ptr<poly::Modulus> mod;
    uint64_t lseg = 0;                       // segment length g is built for
    poly::Poly xl;                           // x^lseg mod p
    std::vector<std::vector<uint32_t>> g;    // g[c-1] = x^(c*lseg-1) mod p, packed
    std::mutex mu;
};

Staging::~Staging() {
    if (pending && done) (void)hipEventSynchronize(done);  // a copy may still read host
    if (host) (void)hipHostFree(host);
    if (done) (void)hipEventDestroy(done);
}

static void size_tracking(ParamSet &ps) {
    if (ps.jumps.size() != (size_t)ps.n) ps.jumps.resize((size_t)ps.n);
    if (ps.seeded.size() != (size_t)ps.n) ps.seeded.resize((size_t)ps.n, 1);
    if (ps.dirty.size() != (size_t)ps.n) ps.dirty.resize((size_t)ps.n, 0);
}

void note_states_seeded(ParamSet &ps, int n) {
    std::lock_guard<std::mutex> lk(ps.jump_mu);
    size_tracking(ps);
    for (int k = 0; k < n && k < ps.n; ++k) {
        ps.seeded[(size_t)k] = 1;
        const StreamJump *sj = ps.jumps[(size_t)k].get();
        if (sj && !(sj->status == 1 && sj->has_seed_orbit)) ps.dirty[(size_t)k] = 1;
    }
}

void note_states_foreign(ParamSet &ps, const int32_t *streams, int n) {
    std::lock_guard<std::mutex> lk(ps.jump_mu);
    size_tracking(ps);
    for (int i = 0; i < n; ++i) {
        const int k = streams ? streams[i] : i;
        if (k < 0 || k >= ps.n) continue;
        ps.seeded[(size_t)k] = 0;
        ps.dirty[(size_t)k] = 1;
    }
}

void note_repairs(ParamSet &ps, const uint32_t *err_words, const std::vector<int32_t> &split) {
    const uint32_t n = err_words[0], logged = err_words[1];
    if (n == 0) return;
    if (logged <= (uint32_t)HDR_LOG_MAX) {
        std::vector<int32_t> ks;
        for (uint32_t i = 0; i < logged; ++i) ks.push_back((int32_t)err_words[2 + i]);
        note_states_foreign(ps, ks.data(), (int)ks.size());
    } else {
        note_states_foreign(ps, split.data(), (int)split.size());
    }
}

template <class F>
static void parallel_for(int n, F f) {
    int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    nt = std::min(nt, n);
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&] {
            for (int i; (i = next.fetch_add(1)) < n;) f(i);
        });
    for (auto &x : th) x.join();
}

// Cost model: outputs a stream yields per dependent step of the wide path
// (one LDS round trip).  Narrow streams with a linear rec_tbl run the
// windowed scan instead, which measures at about 60 + W outputs per
// wide-step time.
uint64_t step_outputs(const ParamSet &ps, int stream, const mtgp_tuning &t) {
    const uint32_t W = ps.W[(size_t)stream];
    const uint64_t smax = (uint64_t)t.threads_per_stream * (uint64_t)t.outputs_per_lane;
    uint64_t s;
    if (W >= 64) s = W & ~31u;
    else if (t.threads_per_stream == 64 && ps.lin[(size_t)stream] &&
             W < (uint32_t)t.window_below_w)
        s = 60 + W;
    else s = W;
    return std::max<uint64_t>(1, std::min(s, smax));
}

static std::vector<uint32_t> pack32(const poly::Poly &p, int nbits) {
    std::vector<uint32_t> w((size_t)(nbits + 31) / 32, 0u);
    for (size_t i = 0; i < w.size(); ++i) {
        const uint64_t v = (i / 2 < p.size()) ? p[i / 2] : 0;
        w[i] = (uint32_t)(v >> (32 * (i & 1)));
    }
    if (nbits & 31) w.back() &= (1u << (nbits & 31)) - 1u;
    return w;
}

// lcm of the annihilators of the bit sequences parity(x_t & r), t >= 1.
static poly::Poly annihilator(const uint32_t *x, int R, const std::vector<uint32_t> &funcs) {
    std::vector<uint8_t> bits((size_t)R - 1);
    poly::Poly acc;
    for (uint32_t r : funcs) {
        for (int t = 1; t < R; ++t) bits[(size_t)t - 1] = (uint8_t)__builtin_parity(x[t] & r);
        poly::Poly p;
        poly::berlekamp_massey(bits.data(), R - 1, &p);
        acc = acc.empty() ? p : poly::lcm(acc, p);
    }
    return acc;
}

namespace {
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc(&p, std::max<size_t>(n, 256)); }
};
}  // namespace

// Builds the annihilating polynomial of every listed stream that has none
// or whose state may have left the orbits its polynomial was built from:
// from the seed status while the stream's state was last set by seeding,
// else from its current state row (d_states; streams needing one are
// skipped when d_states is NULL).  A rebuilt stream keeps the lcm of its
// old and new polynomial.
static int ensure_jumps(const std::shared_ptr<ParamSet> &ps, const void *d_params,
                        const uint32_t *d_states, int stride, const std::vector<int> &streams,
                        const mtgp_tuning &tun, hipStream_t s) {
    std::lock_guard<std::mutex> lk(ps->jump_mu);
    size_tracking(*ps);
    std::vector<int> cand = streams;
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    std::vector<int> todo;
    std::vector<uint8_t> from_seed;
    for (int k : cand) {
        if (k < 0 || k >= ps->n) continue;
        if (ps->jumps[(size_t)k] && !ps->dirty[(size_t)k]) continue;
        const bool seedy = ps->seeded[(size_t)k] != 0;
        if (!seedy && !d_states) continue;
        todo.push_back(k);
        from_seed.push_back(seedy ? 1 : 0);
    }
    if (todo.empty()) return MTGP_OK;

    const int N = ps->N;
    const int mexp = (int)ps->mexp;
    const int R = 2 * mexp + 128;            // raw words per stream (x_0 .. x_{R-1})
    const int V = mexp + 64;                 // verification outputs per stream
    const int PW = (mexp + 2 + 31) / 32 + 1; // packed words of p
    const int chunk = 512;
    hipError_t e;
    DevBuf d_seeded;
    if (std::find(from_seed.begin(), from_seed.end(), 1) != from_seed.end()) {
        if ((e = d_seeded.alloc((size_t)ps->n * N * 4)) != hipSuccess)
            return hip_fail(e, "hipMalloc");
        if ((e = launch_seed((const uint32_t *)d_params, (uint32_t *)d_seeded.p, (uint32_t)N,
                             (uint32_t)ps->n, s)) != hipSuccess)
            return hip_fail(e, "seed kernel");
    }
    const int cn = std::min<int>(chunk, (int)todo.size());
    DevBuf d_raw, d_out, d_items, d_counter, d_jitems, d_poly, d_vout;
    if ((e = d_raw.alloc((size_t)cn * R * 4)) != hipSuccess ||
        (e = d_out.alloc((size_t)cn * (R - N) * 4)) != hipSuccess ||
        (e = d_items.alloc((size_t)cn * sizeof(BatchItem))) != hipSuccess ||
        (e = d_counter.alloc(256)) != hipSuccess ||
        (e = d_jitems.alloc((size_t)cn * JUMP_BLOCK * sizeof(JumpItem))) != hipSuccess ||
        (e = d_poly.alloc((size_t)cn * PW * 4)) != hipSuccess ||
        (e = d_vout.alloc((size_t)cn * V * 4)) != hipSuccess)
        return hip_fail(e, "hipMalloc(jump planning)");
    std::vector<uint32_t> raw((size_t)cn * R), vout((size_t)cn * V);

    for (size_t c0 = 0; c0 < todo.size(); c0 += chunk) {
        const int m = (int)std::min<size_t>(chunk, todo.size() - c0);
        std::vector<BatchItem> items((size_t)m);
        for (int j = 0; j < m; ++j) {
            const int k = todo[c0 + j];
            BatchItem &b = items[j];
            std::memset(&b, 0, sizeof b);
            b.stream = (uint32_t)k;
            b.mode = MODE_RAW;
            b.count = (uint64_t)(R - N);
            b.out = (uint64_t)(uintptr_t)((uint32_t *)d_out.p + (size_t)j * (R - N));
            b.state_in = from_seed[c0 + j]
                             ? (uint64_t)(uintptr_t)((uint32_t *)d_seeded.p + (size_t)k * N)
                             : (uint64_t)(uintptr_t)(d_states + (size_t)k * stride);
            b.raw = (uint64_t)(uintptr_t)((uint32_t *)d_raw.p + (size_t)j * R);
        }
        if ((e = hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(BatchItem),
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(plan items)");
        LaunchArgs a{};
        a.params = (const uint32_t *)d_params;
        a.items = (const BatchItem *)d_items.p;
        a.n_items = (uint32_t)m;
        a.counter = (uint32_t *)d_counter.p;
        a.err = (uint32_t *)d_counter.p + 1;
        a.persistent = true;
        a.num_cus = device_cus();
        a.stream = s;
        a.win_below = (uint32_t)tun.window_below_w;
        if ((e = launch_reset((uint32_t *)d_counter.p, s)) != hipSuccess)
            return hip_fail(e, "reset kernel");
        if ((e = launch_prefix(N, a)) != hipSuccess) return hip_fail(e, "prefix kernel");
        if ((e = hipMemcpyAsync(raw.data(), d_raw.p, (size_t)m * R * 4, hipMemcpyDeviceToHost,
                                s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(e, "raw words to host");

        std::vector<poly::Poly> P((size_t)m);
        std::vector<uint8_t> ok((size_t)m, 0);
        const std::vector<uint32_t> quick = {0xFFFFFFFFu, 0x6A09E667u};
        std::vector<uint32_t> all = quick;
        for (int b = 0; b < 32; ++b) all.push_back(1u << b);
        for (int pass = 0; pass < 2; ++pass) {
            parallel_for(m, [&](int j) {
                if (ok[j]) return;
                P[j] = annihilator(&raw[(size_t)j * R], R, pass == 0 ? quick : all);
            });
            // device check: y_t = sum_i p_i x_{t+i} must vanish for t = 1..D
            // one item per block: each stream's check runs on its own
            std::vector<JumpItem> jit((size_t)m * JUMP_BLOCK);
            std::memset(jit.data(), 0, jit.size() * sizeof(JumpItem));
            std::vector<uint32_t> pw((size_t)m * PW, 0u);
            int nj = 0;
            std::vector<int> which;
            for (int j = 0; j < m; ++j) {
                if (ok[j]) continue;
                const int D = poly::degree(P[j]);
                if (D < 1 || D > mexp) continue;
                const std::vector<uint32_t> w = pack32(P[j], D + 1);
                std::memcpy(&pw[(size_t)nj * PW], w.data(), w.size() * 4);
                JumpItem &ji = jit[(size_t)nj * JUMP_BLOCK];
                ji.raw = (uint64_t)(uintptr_t)((uint32_t *)d_raw.p + (size_t)j * R);
                ji.poly = (uint64_t)(uintptr_t)((uint32_t *)d_poly.p + (size_t)nj * PW);
                ji.out = (uint64_t)(uintptr_t)((uint32_t *)d_vout.p + (size_t)nj * V);
                ji.nbits = (uint32_t)(D + 1);
                ji.m = (uint32_t)mexp;
                which.push_back(j);
                ++nj;
            }
            if (nj == 0) break;
            if ((e = hipMemcpyAsync(d_poly.p, pw.data(), (size_t)nj * PW * 4,
                                    hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipMemcpyAsync(d_jitems.p, jit.data(),
                                    (size_t)nj * JUMP_BLOCK * sizeof(JumpItem),
                                    hipMemcpyHostToDevice, s)) != hipSuccess)
                return hip_fail(e, "hipMemcpyAsync(check items)");
            if ((e = launch_jump((const JumpItem *)d_jitems.p, (uint32_t)nj * JUMP_BLOCK,
                                 device_cus(), s)) !=
                hipSuccess)
                return hip_fail(e, "jump kernel (check)");
            if ((e = hipMemcpyAsync(vout.data(), d_vout.p, (size_t)nj * V * 4,
                                    hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return hip_fail(e, "check results to host");
            // y has order <= mexp (it lies in the same orbit), so mexp
            // consecutive zeros mean y vanishes for every t >= 1
            for (int q = 0; q < nj; ++q) {
                const int j = which[q];
                bool zero = true;
                for (int t = 0; t < mexp && zero; ++t) zero = vout[(size_t)q * V + t] == 0u;
                ok[j] = zero ? 1 : 0;
            }
        }
        std::vector<std::shared_ptr<StreamJump>> built((size_t)m);
        parallel_for(m, [&](int j) {
            const int k = todo[c0 + j];
            const StreamJump *old = ps->jumps[(size_t)k].get();
            const bool old_ok = old && old->status == 1;
            auto sj = std::make_shared<StreamJump>();
            sj->status = -1;
            if (ok[j]) {
                // every polynomial here divides the minimal polynomial of the
                // transition on its image (dimension mexp), so the lcm keeps
                // degree <= mexp
                poly::Poly p = old_ok ? poly::lcm(old->mod->p, P[j]) : P[j];
                const int D = poly::degree(p);
                if (D >= 1 && D <= mexp) {
                    sj->status = 1;
                    sj->D = D;
                    sj->mod = std::make_unique<poly::Modulus>(p);
                    sj->has_seed_orbit = from_seed[c0 + j] || (old_ok && old->has_seed_orbit);
                }
            }
            built[j] = sj;
        });
        for (int j = 0; j < m; ++j) {
            const int k = todo[c0 + j];
            ps->jumps[(size_t)k] = built[j];
            ps->dirty[(size_t)k] = 0;
        }
    }
    return MTGP_OK;
}

// True when the stream's cached powers already serve segment length lseg
// up to cmax.
static bool g_ready(StreamJump &sj, uint64_t lseg, int cmax) {
    std::lock_guard<std::mutex> lk(sj.mu);
    return sj.lseg == lseg && (int)sj.g.size() >= cmax - 1;
}

// g[c-1] = x^(c*lseg-1) mod p for c = 1 .. cmax-1.
static void ensure_g(StreamJump &sj, uint64_t lseg, int cmax) {
    std::lock_guard<std::mutex> lk(sj.mu);
    if (sj.lseg != lseg) {
        sj.lseg = lseg;
        sj.g.clear();
        sj.xl = sj.mod->powx(lseg);
    }
    if ((int)sj.g.size() >= cmax - 1) return;
    poly::Poly cur;
    if (sj.g.empty()) {
        cur = sj.mod->powx(lseg - 1);
        sj.g.push_back(pack32(cur, sj.D));
    } else {
        // unpack the last one
        const std::vector<uint32_t> &w = sj.g.back();
        cur.assign((w.size() + 1) / 2, 0);
        for (size_t i = 0; i < w.size(); ++i) cur[i / 2] |= (uint64_t)w[i] << (32 * (i & 1));
        poly::trim(cur);
    }
    while ((int)sj.g.size() < cmax - 1) {
        cur = sj.mod->mulmod(cur, sj.xl);
        sj.g.push_back(pack32(cur, sj.D));
    }
}

// ---------------------------------------------------------------- plan ----

namespace {
// A request split into C segments: segment 0 covers outputs [0, c0*lseg)
// (the prefix [0, P) with P = D+1, then the rest), segment k >= 1 covers
// [(c0+k-1)*lseg, (c0+k)*lseg) clipped to the request.
struct Seg {
    int req;
    int C = 1;           // segments (1 = not split)
    uint64_t lseg = 0;
    uint64_t c0 = 0;
    int D = 0;           // degree of the stream's polynomial
    int Dsize = 0;       // degree the workspace is sized for (>= D)
    std::shared_ptr<StreamJump> sj;
};

struct Layout {
    size_t off_A = 0, off_B = 0, off_C = 0, off_F = 0, off_rec = 0, off_jdep = 0, off_pflag = 0;
    size_t off_poly = 0, up_end = 0;
    size_t off_raw = 0, off_js = 0, total = 0;
};

size_t al256(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

size_t batch_min_ws_bytes(int n_items) {
    // header + one item per request (no split: no prefix, jump or check
    // items, no request records)
    return HDR_BYTES + al256((size_t)std::max(n_items, 0) * sizeof(BatchItem));
}

// The dependent-step target of a batch: the tuning's jump_target_steps is
// a floor (0 disables splitting); above it the target follows the batch's
// balanced makespan, total steps over the streams the device runs at once,
// so that only streams on the critical path are cut and each segment is
// short against the whole launch.
static uint64_t effective_target(const ParamSet &ps, const std::vector<Request> &reqs,
                                 const mtgp_tuning &t) {
    if (t.jump_target_steps <= 0) return 0;
    uint64_t total = 0;
    for (const Request &r : reqs) {
        const uint64_t so = step_outputs(ps, r.stream, t);
        total += (r.count + so - 1) / so;
    }
    const int wpb = t.threads_per_stream == 64 ? t.workgroup_size / 64 : 1;
    const int per_cu = variant_slots_per_cu(ps.N, t.threads_per_stream, t.outputs_per_lane, wpb);
    const uint64_t slots = (uint64_t)std::max(1, per_cu) * (uint64_t)std::max(1, device_cus());
    // a multiple of the balanced share of steps per resident stream: more,
    // shorter segments shorten the tail of the segment phase but every
    // segment costs a jump (D N / 4 word operations); measured optimum about
    // 0.75 at mexp 11213 and 1.25 at 23209 and 44497 (jumps 4-16x dearer)
    const uint64_t share = total / slots;
    const uint64_t adaptive = ps.N <= 400 ? share * 3 / 4 : share * 5 / 4;
    return std::max<uint64_t>((uint64_t)t.jump_target_steps, adaptive);
}

// Segment length for a target of v outputs: v rounded down to m * 2^e with
// m in {4, 5, 6, 7} (at most 20% short), at least 256.  The coarse grid
// keeps a stream's segment length, and so its cached jump polynomials, the
// same from batch to batch when the target moves a little; whole 256-word
// multiples keep every segment's stores line-aligned.
static uint64_t segment_length(uint64_t v) {
    if (v < 1024) return std::max<uint64_t>(256, v / 256 * 256);
    const int e = 63 - __builtin_clzll(v) - 2;  // v / 2^e in [4, 8), e >= 8
    return (v >> e) << e;
}

// Splits a request when it needs more than T dependent steps, for a stream
// polynomial of degree D (D < 1: never).
static void decide(const ParamSet &ps, const Request &r, int D, uint64_t T, const mtgp_tuning &t,
                   Seg &g) {
    g.C = 1;
    g.D = g.Dsize = 0;
    if (!T || D < 1) return;
    const uint64_t so = step_outputs(ps, r.stream, t);
    if ((r.count + so - 1) / so <= T) return;
    const uint64_t P = (uint64_t)D + 1;
    const uint64_t lseg = segment_length(T * so);
    const uint64_t c0 = (P + 1 + lseg - 1) / lseg;   // segment 0 keeps >= 1 output past P
    const uint64_t cend = (r.count + lseg - 1) / lseg;
    if (cend <= c0) return;
    g.C = (int)(1 + cend - c0);
    g.lseg = lseg;
    g.c0 = c0;
    g.D = g.Dsize = D;
}

static bool wants_split(const ParamSet &ps, const Request &r, uint64_t T, const mtgp_tuning &t) {
    if (!T) return false;
    const uint64_t so = step_outputs(ps, r.stream, t);
    return (r.count + so - 1) / so > T && r.count > (uint64_t)ps.mexp + 128;
}

// Jump items per jump: one per JUMP_OUT_WORDS words of the N-word state.
static size_t jump_passes(int N) {
    return ((size_t)N + JUMP_OUT_WORDS - 1) / JUMP_OUT_WORDS;
}

static Layout layout_for(const ParamSet &ps, const std::vector<Seg> &segs) {
    size_t nA = 0, nB = 0, nC = 0, poly_words = 0, raw_words = 0, js_words = 0;
    for (const Seg &g : segs) {
        if (g.C <= 1) {
            ++nC;
            continue;
        }
        ++nA;
        nB += ((size_t)g.C - 1 + JUMP_BLOCK - 1) / JUMP_BLOCK * JUMP_BLOCK * jump_passes(ps.N);
        nC += (size_t)g.C;
        poly_words += ((size_t)g.C - 1) * (((size_t)g.Dsize + 31) / 32);
        raw_words += ((size_t)ps.N + (size_t)g.Dsize + 1 + 63) / 64 * 64;
        js_words += (size_t)g.C * (size_t)ps.N;
    }
    Layout L;
    L.off_A = HDR_BYTES;
    L.off_B = L.off_A + al256(nA * sizeof(BatchItem));
    L.off_C = L.off_B + al256(nB * sizeof(JumpItem));
    L.off_F = L.off_C + al256(nC * sizeof(BatchItem));
    L.off_rec = L.off_F + al256(nA * sizeof(BatchItem));
    L.off_jdep = L.off_rec + al256(nA * sizeof(ReqRec));
    L.off_pflag = L.off_jdep + al256(nB / JUMP_BLOCK * 4);
    L.off_poly = L.off_pflag + al256(nA * 4);
    L.up_end = L.off_poly + al256(poly_words * 4);
    L.off_raw = L.up_end;
    L.off_js = L.off_raw + al256(raw_words * 4);
    L.total = L.off_js + al256(js_words * 4);
    return L;
}

WsState::~WsState() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
}

// Pinned staging for the uploaded plan: acquire waits until every upload
// from this buffer has been consumed, then hands out at least n bytes; the
// plan is written in place and stage_copy uploads a byte range of it.
static int stage_acquire(Staging &st, size_t n, uint8_t **out) {
    if (st.pending) {
        hipError_t e = hipEventSynchronize(st.done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(staging)");
        st.pending = false;
    }
    if (n > st.cap) {
        if (st.host) (void)hipHostFree(st.host);
        st.host = nullptr;
        const size_t cap = std::max<size_t>(n, 1 << 16);
        hipError_t e = hipHostMalloc((void **)&st.host, cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            st.cap = 0;
            return hip_fail(e, "hipHostMalloc(staging)");
        }
        st.cap = cap;
    }
    if (!st.done) {
        hipError_t e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    *out = st.host;
    return MTGP_OK;
}

static int stage_copy(WsState &w, size_t lo, size_t hi, char *d_base, hipStream_t s) {
    if (hi <= lo) return MTGP_OK;
    if (w.no_alloc) {
        hipError_t e = hipMemcpyAsync(d_base + lo, w.image.data() + lo, hi - lo,
                                      hipMemcpyHostToDevice, s);
        return e == hipSuccess ? MTGP_OK : hip_fail(e, "hipMemcpyAsync(work list)");
    }
    Staging &st = w.stage;
    hipError_t e = hipMemcpyAsync(d_base + lo, st.host + lo, hi - lo, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(work list)");
    e = hipEventRecord(st.done, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    st.pending = true;
    return MTGP_OK;
}

namespace {
uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

// Workspaces the library has planned for, most recently used first; an
// evicted entry lives on until its last call returns.
std::mutex g_ws_mu;
std::list<std::pair<const void *, std::shared_ptr<WsState>>> g_ws;
constexpr size_t kMaxWorkspaces = 64;

std::shared_ptr<WsState> ws_state(const void *d_ws, bool create) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto it = g_ws.begin(); it != g_ws.end(); ++it) {
        if (it->first == d_ws) {
            g_ws.splice(g_ws.begin(), g_ws, it);
            return g_ws.front().second;
        }
    }
    if (!create) return nullptr;
    g_ws.emplace_front(d_ws, std::make_shared<WsState>());
    if (g_ws.size() > kMaxWorkspaces) g_ws.pop_back();
    return g_ws.front().second;
}

struct GraphKey {
    const void *ws;
    uint32_t nA, nB, nC;
    const void *params;
    int N, tps, k, wg, win, device;
    bool stamps, errs;
    bool operator<(const GraphKey &o) const {
        return std::tie(ws, nA, nB, nC, params, N, tps, k, wg, win, device, stamps, errs) <
               std::tie(o.ws, o.nA, o.nB, o.nC, o.params, o.N, o.tps, o.k, o.wg, o.win,
                        o.device, o.stamps, o.errs);
    }
};
std::atomic<bool> g_stamps{false};  // phase timestamps in every batch call
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;
std::map<int, hipStream_t> g_capture_streams;

bool graphs_enabled() {
    const char *v = getenv("MTGP_GRAPH");
    return !(v && v[0] == '0');
}
}  // namespace

// Tag of a workspace header: derived from its address and a per-process
// salt, so reused memory at the same address is recognised as fresh unless
// it still holds a header this process wrote there.
static uint64_t header_tag(const void *d_ws) {
    static const uint64_t salt = mix((uint64_t)(uintptr_t)&salt,
                                     (uint64_t)std::chrono::steady_clock::now()
                                         .time_since_epoch()
                                         .count());
    uint64_t t = mix(salt, (uint64_t)(uintptr_t)d_ws);
    return t ? t : 1;
}

// Launches the phases of the workspace's planned batch on `s`: header,
// prefix items and jump evaluation (one launch), segments, request checks.
// With w.overlap the whole (unsplit) requests, which need nothing from the
// prefix and jump launch, run beside it and the segments: a launch on w.aux,
// capped at w.overlap_groups workgroups per CU so that the prefix and jump
// workgroups keep most of the chip, takes them; the segment launch follows
// the prefix and jump launch on `s` at the CUs' full occupancy (its
// workgroups beyond what is free start as the whole-request launch ends).
// No launch waits for another's results, so the streams may run in any
// order.
static int launch_phases(const ParamSet &ps, const void *d_params, char *ws, const WsState &w,
                         const mtgp_tuning &t, hipStream_t s, bool stamps, bool clear_errors) {
    uint32_t *hdr = (uint32_t *)ws;
    uint64_t *ts = (uint64_t *)(ws + HDR_STAMP_BYTE);
    auto stamp = [&](int i) -> int {
        if (!stamps) return MTGP_OK;
        const hipError_t e = launch_stamp(ts + i, s);
        return e == hipSuccess ? MTGP_OK : hip_fail(e, "stamp kernel");
    };
    hipError_t e;
    if ((e = launch_header(hdr, header_tag(ws), clear_errors, s)) != hipSuccess)
        return hip_fail(e, "header kernel");
    int rc = stamp(0);
    if (rc) return rc;
    LaunchArgs a{};
    a.params = (const uint32_t *)d_params;
    a.err = hdr + HDR_ERR;
    a.persistent = true;
    a.num_cus = device_cus();
    a.stream = s;
    const BatchItem *C = (const BatchItem *)(ws + w.off_C);
    const bool fork = w.overlap && (w.nA || w.nB) && w.nCs < w.nC && w.aux;
    if (fork) {
        if ((e = hipEventRecord(w.ev_fork, s)) != hipSuccess)
            return hip_fail(e, "hipEventRecord(fork)");
        if ((e = hipStreamWaitEvent(w.aux, w.ev_fork, 0)) != hipSuccess)
            return hip_fail(e, "hipStreamWaitEvent(fork)");
        LaunchArgs a1 = a;
        a1.stream = w.aux;
        a1.items = C + w.nCs;
        a1.n_items = w.nC - w.nCs;
        a1.counter = hdr + HDR_W_CLAIM;
        a1.groups_per_cu = w.overlap_groups;
        if ((rc = launch_tuned(ps.N, t, a1))) return rc;
        if ((e = hipEventRecord(w.ev_join, w.aux)) != hipSuccess) {
            (void)hipStreamSynchronize(w.aux);  // nothing to order s after: wait here
            return hip_fail(e, "hipEventRecord(join)");
        }
    }
    // Once the whole requests run on w.aux, an error return still orders s
    // after them, so that a caller who sees the error can free the buffers.
    auto bail = [&](int code) {
        if (fork) (void)hipStreamWaitEvent(s, w.ev_join, 0);
        return code;
    };
    if (w.nA || w.nB) {  // prefix items and jump blocks, one launch
        if ((e = launch_prefix_jumps(ps.N, (const BatchItem *)(ws + w.off_A), w.nA,
                                     (const JumpItem *)(ws + w.off_B), w.nB,
                                     (const uint32_t *)(ws + w.off_jdep),
                                     (uint32_t *)(ws + w.off_pflag), (const uint32_t *)d_params,
                                     hdr, (uint32_t)t.window_below_w, device_cus(), s)) !=
            hipSuccess)
            return bail(hip_fail(e, "prefix and jump kernel"));
    }
    if ((rc = stamp(1))) return bail(rc);
    a.items = C;
    a.counter = hdr + 1;
    a.n_items = fork ? w.nCs : w.nC;
    if ((rc = launch_tuned(ps.N, t, a))) return bail(rc);
    if (fork && (e = hipStreamWaitEvent(s, w.ev_join, 0)) != hipSuccess) {
        (void)hipStreamSynchronize(w.aux);
        return hip_fail(e, "hipStreamWaitEvent(join)");
    }
    if ((rc = stamp(2))) return rc;
    if (w.nF) {  // request checks of the split requests
        a.items = (const BatchItem *)(ws + w.off_F);
        a.n_items = w.nF;
        a.counter = hdr + HDR_FIX_CLAIM;
        a.win_below = (uint32_t)t.window_below_w;
        if ((e = launch_check(ps.N, a)) != hipSuccess) return hip_fail(e, "check kernel");
    }
    return stamp(3);
}

// Writes the plan of `reqs` into the pinned image of w (byte offsets as in
// the workspace) and records where its parts lie.
static int build_plan(const std::shared_ptr<ParamSet> &ps, const void *d_params,
                      uint32_t *d_states, int stride, const std::vector<Request> &reqs,
                      char *ws, size_t ws_bytes, hipStream_t s, const mtgp_tuning &t,
                      WsState &w, bool overlap) {
    const int N = ps->N;
    std::vector<Seg> segs(reqs.size());
    std::vector<int> want;
    uint64_t T = effective_target(*ps, reqs, t);
    for (size_t i = 0; i < reqs.size(); ++i) {
        segs[i].req = (int)i;
        if (wants_split(*ps, reqs[i], T, t)) want.push_back(reqs[i].stream);
    }
    if (!want.empty() && !w.no_alloc) {
        int rc = ensure_jumps(ps, d_params, d_states, stride, want, t, s);
        if (rc) return rc;
    }
    // snapshot of the streams' jump data (an entry may be replaced by a
    // rebuild meanwhile; the snapshot keeps this plan's alive); without
    // building, a stream due for a rebuild is not split
    std::vector<std::shared_ptr<StreamJump>> sjs(reqs.size());
    {
        std::lock_guard<std::mutex> lk(ps->jump_mu);
        if (ps->jumps.size() == (size_t)ps->n && ps->dirty.size() == (size_t)ps->n)
            for (size_t i = 0; i < reqs.size(); ++i)
                if (!(w.no_alloc && ps->dirty[(size_t)reqs[i].stream]))
                    sjs[i] = ps->jumps[reqs[i].stream];
    }
    // plan, doubling the target until the workspace fits
    Layout L;
    while (true) {
        for (size_t i = 0; i < reqs.size(); ++i) {
            const int D = (sjs[i] && sjs[i]->status == 1) ? sjs[i]->D : 0;
            decide(*ps, reqs[i], D, T, t, segs[i]);
            segs[i].sj = segs[i].C > 1 ? sjs[i] : nullptr;
        }
        L = layout_for(*ps, segs);
        if (L.total <= ws_bytes || !T) break;
        T *= 2;
        if (T > (1ull << 40)) T = 0;
    }
    if (L.total > ws_bytes)
        return fail(MTGP_EINVAL, "workspace of %zu bytes too small (need %zu)", ws_bytes,
                    L.total);
    // polynomials: only streams whose cache lacks them (a thread per
    // stream costs more than a batch of cached lookups)
    std::vector<Seg *> split;
    for (Seg &g : segs)
        if (g.C > 1 && !g_ready(*g.sj, g.lseg, (int)(g.c0 + (uint64_t)g.C - 1)))
            split.push_back(&g);
    parallel_for((int)split.size(), [&](int i) {
        const Seg &g = *split[i];
        ensure_g(*g.sj, g.lseg, (int)(g.c0 + (uint64_t)g.C - 1));
    });

    // the image of [HDR_BYTES, up_end): item tables, request records,
    // polynomials (every byte that is read is written; the alignment gaps
    // between tables are never read).  The header is never uploaded.
    uint8_t *img = nullptr;
    if (w.no_alloc) {
        w.image.resize(L.up_end);
        img = w.image.data();
    } else if (int rc = stage_acquire(w.stage, L.up_end, &img)) {
        return rc;
    }
    auto at = [&](size_t off) { return img + off; };
    // segment list entries: steps, item, and whether the item is a segment
    // of a split request (else a whole request)
    struct CItem {
        uint64_t steps;
        BatchItem b;
        bool segment;
    };
    std::vector<CItem> C;
    std::vector<std::tuple<uint64_t, BatchItem, size_t>> A;  // steps, item, split index
    std::vector<std::vector<JumpItem>> Bs;                   // per split request, padded
    std::vector<BatchItem> F;
    std::vector<int32_t> split_streams;
    size_t raw_off = L.off_raw, js_off = L.off_js, poly_off = L.off_poly;
    for (size_t i = 0; i < reqs.size(); ++i) {
        const Request &r = reqs[i];
        const Seg &g = segs[i];
        const uint32_t mode = r.dtype == MTGP_F32 ? MODE_F32 : 0u;
        uint32_t *row = d_states + (size_t)r.stream * stride;
        const uint64_t so = step_outputs(*ps, r.stream, t);
        auto base_item = [&](uint64_t count, uint64_t out_off) {
            BatchItem b;
            std::memset(&b, 0, sizeof b);
            b.stream = (uint32_t)r.stream;
            b.mode = mode;
            b.count = count;
            b.out = (uint64_t)(uintptr_t)((char *)r.d_out + out_off * 4);
            return b;
        };
        if (g.C <= 1) {
            BatchItem b = base_item(r.count, 0);
            b.state_in = b.state_out = (uint64_t)(uintptr_t)row;
            b.flag = r.flag;
            C.push_back(CItem{(r.count + so - 1) / so, b, false});
            continue;
        }
        // request record and check item of a split request
        const size_t ri = F.size();
        ReqRec *rc = (ReqRec *)at(L.off_rec) + ri;
        const uint64_t rec_dev = (uint64_t)(uintptr_t)(ws + L.off_rec + ri * sizeof(ReqRec));
        split_streams.push_back(r.stream);
        const int D = g.D;
        const uint64_t P = (uint64_t)D + 1;
        uint32_t *raw = (uint32_t *)(ws + raw_off);
        raw_off += ((size_t)N + (size_t)g.Dsize + 1 + 63) / 64 * 64 * 4;
        uint32_t *js = (uint32_t *)(ws + js_off);  // C states of N words
        js_off += (size_t)g.C * N * 4;
        std::memset(rc, 0, sizeof *rc);
        rc->stream = (uint32_t)r.stream;
        rc->mode = mode;
        rc->count = r.count;
        rc->out = (uint64_t)(uintptr_t)r.d_out;
        rc->orig = (uint64_t)(uintptr_t)raw;  // x_0 .. x_{N-1}: the start state
        rc->row = (uint64_t)(uintptr_t)row;
        BatchItem f = base_item(0, 0);
        f.mode = MODE_FIXUP | mode;
        f.rec = rec_dev;
        f.flag = r.flag;
        F.push_back(f);
        // A: prefix
        BatchItem a = base_item(P, 0);
        a.mode |= MODE_RAW;
        a.state_in = (uint64_t)(uintptr_t)row;
        a.state_out = (uint64_t)(uintptr_t)js;
        a.raw = (uint64_t)(uintptr_t)raw;
        A.emplace_back((P + so - 1) / so, a, ri);
        // B: jumps, segment k >= 1 starts at output (c0+k-1)*lseg and
        // its state is x^((c0+k-1)*lseg - 1) mod p applied to the words;
        // each jump is evaluated in passes of JUMP_OUT_WORDS state words
        // (blocks of JUMP_BLOCK jumps per pass), word m0 onwards reading the
        // raw words from m0 on
        const size_t pw = ((size_t)D + 31) / 32;
        Bs.emplace_back();
        std::vector<JumpItem> &B = Bs.back();
        std::vector<uint64_t> polys((size_t)g.C);
        for (int k = 1; k < g.C; ++k) {
            const uint64_t c = g.c0 + (uint64_t)k - 1;
            polys[(size_t)k] = (uint64_t)(uintptr_t)(ws + poly_off);
            std::memcpy(at(poly_off), g.sj->g[(size_t)c - 1].data(), pw * 4);
            poly_off += pw * 4;
        }
        for (int m0 = 0; m0 < N; m0 += JUMP_OUT_WORDS) {
            for (int k = 1; k < g.C; ++k) {
                JumpItem j;
                j.raw = (uint64_t)(uintptr_t)(raw + m0);
                j.poly = polys[(size_t)k];
                j.out = (uint64_t)(uintptr_t)(js + (size_t)k * N + (size_t)m0);
                j.nbits = (uint32_t)D;
                j.m = (uint32_t)std::min(JUMP_OUT_WORDS, N - m0);
                B.push_back(j);
            }
            while (B.size() % JUMP_BLOCK) {  // pad this pass's last block
                JumpItem z;
                std::memset(&z, 0, sizeof z);
                B.push_back(z);
            }
        }
        // C: segments; every one but the last checks its end state against
        // the next one's jumped start
        for (int k = 0; k < g.C; ++k) {
            const uint64_t c = k == 0 ? 0 : g.c0 + (uint64_t)k - 1;
            const uint64_t start = k == 0 ? P : c * g.lseg;
            const uint64_t end = std::min<uint64_t>(r.count, k == 0 ? g.c0 * g.lseg
                                                                    : (c + 1) * g.lseg);
            BatchItem b = base_item(end - start, start);
            b.state_in = (uint64_t)(uintptr_t)(js + (size_t)k * N);
            if (k + 1 < g.C) {
                b.mode |= MODE_VERIFY;
                b.verify = (uint64_t)(uintptr_t)(js + (size_t)(k + 1) * N);
                b.rec = rec_dev;
            } else {
                b.state_out = (uint64_t)(uintptr_t)row;
            }
            C.push_back(CItem{(end - start + so - 1) / so, b, true});
        }
    }
    std::stable_sort(A.begin(), A.end(),
                     [](const auto &x, const auto &y) { return std::get<0>(x) > std::get<0>(y); });
    // prefixes longest first; jump blocks of the streams with the shortest
    // prefixes first (their words are ready soonest), each block naming its
    // stream's prefix item
    for (size_t i = 0; i < A.size(); ++i)
        std::memcpy(at(L.off_A) + i * sizeof(BatchItem), &std::get<1>(A[i]), sizeof(BatchItem));
    std::memset(at(L.off_pflag), 0, A.size() * 4);
    size_t nb = 0;
    for (size_t i = A.size(); i-- > 0;) {
        const std::vector<JumpItem> &B = Bs[std::get<2>(A[i])];
        for (size_t j = 0; j < B.size(); j += JUMP_BLOCK, ++nb) {
            std::memcpy(at(L.off_B) + nb * JUMP_BLOCK * sizeof(JumpItem), &B[j],
                        JUMP_BLOCK * sizeof(JumpItem));
            ((uint32_t *)at(L.off_jdep))[nb] = (uint32_t)i;
        }
    }
    // Segment list, longest first.  Overlapped (whole requests beside the
    // prefix and jump launch): the segments of split requests first, then
    // the whole requests, each part longest first.  Only where the whole
    // requests are at most half the segments' steps, so that their launch,
    // capped below the chip's occupancy, does not outlast the segments.
    uint64_t whole_steps = 0, seg_steps = 0;
    for (const CItem &c : C) (c.segment ? seg_steps : whole_steps) += c.steps;
    const bool split_lists =
        overlap && !A.empty() && whole_steps > 0 && 2 * whole_steps <= seg_steps;
    std::stable_sort(C.begin(), C.end(), [&](const CItem &x, const CItem &y) {
        if (split_lists && x.segment != y.segment) return x.segment;
        return x.steps > y.steps;
    });
    size_t n_seg = 0;
    for (size_t i = 0; i < C.size(); ++i) {
        std::memcpy(at(L.off_C) + i * sizeof(BatchItem), &C[i].b, sizeof(BatchItem));
        if (C[i].segment) ++n_seg;
    }
    if (!F.empty()) std::memcpy(at(L.off_F), F.data(), F.size() * sizeof(BatchItem));
    w.nA = (uint32_t)A.size();
    w.nB = (uint32_t)(nb * JUMP_BLOCK);
    w.nC = (uint32_t)C.size();
    w.nF = (uint32_t)F.size();
    w.off_A = L.off_A;
    w.off_B = L.off_B;
    w.off_C = L.off_C;
    w.off_F = L.off_F;
    w.off_jdep = L.off_jdep;
    w.off_pflag = L.off_pflag;
    w.nCs = (uint32_t)(split_lists ? n_seg : C.size());
    w.overlap = split_lists;
    w.tables_end = L.off_poly;
    w.up_end = L.up_end;
    w.ps = ps;
    w.split_streams = std::move(split_streams);
    return MTGP_OK;
}

// Workgroups per CU of the first (concurrent) segment launch in overlapped
// mode, 0 = do not overlap.  At most half the launch variant's occupancy,
// and only where that leaves LDS for a prefix-and-jump workgroup on every
// CU.  MTGP_OVERLAP=0 turns overlapping off; MTGP_OVERLAP=k asks for k.
static int overlap_groups(const ParamSet &ps, const mtgp_tuning &t) {
    const char *v = getenv("MTGP_OVERLAP");
    if (v && v[0] == '0') return 0;
    const int wpb = t.threads_per_stream == 64 ? t.workgroup_size / 64 : 1;
    const int slots = variant_slots_per_cu(ps.N, t.threads_per_stream, t.outputs_per_lane, wpb);
    const int per_cu = t.threads_per_stream == 64 ? slots / wpb : slots;
    if (per_cu < 2) return 0;
    int g = per_cu / 2;
    if (v && v[0] >= '1' && v[0] <= '9') g = std::min(per_cu - 1, atoi(v));
    size_t wg_lds = 0;
    VariantInfo vi[64];
    const int nv = variant_count(ps.N, vi, 64);
    for (int i = 0; i < nv; ++i)
        if (vi[i].tps == t.threads_per_stream && vi[i].k == t.outputs_per_lane &&
            vi[i].wpb == wpb)
            wg_lds = vi[i].lds_bytes;
    int dev = 0, lds_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
            hipSuccess)
        return 0;
    if (!wg_lds || (size_t)g * wg_lds + prefix_jump_lds_bytes() > (size_t)lds_cu) return 0;
    return g;
}

int run_batch(const std::shared_ptr<ParamSet> &ps, const void *d_params, uint32_t *d_states,
              int stride, const std::vector<Request> &reqs, void *d_ws, size_t ws_bytes,
              hipStream_t s, const mtgp_tuning &t, bool use_graph, WsState &w,
              bool per_call_errors, bool allow_overlap) {
    if (reqs.empty()) return MTGP_OK;
    char *ws = (char *)d_ws;
    hipError_t e;
    const bool stamps = g_stamps.load();
    int ov = 0;
    if (allow_overlap && !w.no_alloc && !stamps) {
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cst) == hipSuccess && cst == hipStreamCaptureStatusNone)
            ov = overlap_groups(*ps, t);
    }
    if (ov) {
        // only a batch with both split and whole requests overlaps; for the
        // others the plan is the same either way, and phase-timed calls keep
        // using the cached one
        const uint64_t T = effective_target(*ps, reqs, t);
        bool any_split = false, any_whole = false;
        for (const Request &r : reqs) (wants_split(*ps, r, T, t) ? any_split : any_whole) = true;
        if (!(any_split && any_whole)) ov = 0;
    }
    if (ov && !w.aux) {
        // the second stream and its events, all or none; without them the
        // batch runs unoverlapped
        hipStream_t aux = nullptr;
        hipEvent_t f = nullptr, j = nullptr;
        if (hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
            if (j) (void)hipEventDestroy(j);
            if (f) (void)hipEventDestroy(f);
            if (aux) (void)hipStreamDestroy(aux);
            (void)hipGetLastError();
            ov = 0;
        } else {
            w.aux = aux;
            w.ev_fork = f;
            w.ev_join = j;
        }
    }
    w.overlap_groups = ov;
    uint64_t sig = mix(0x51ull, (uint64_t)(uintptr_t)d_params);
    sig = mix(sig, ps->generation);
    sig = mix(sig, (uint64_t)(uintptr_t)d_states);
    sig = mix(sig, (uint64_t)stride);
    sig = mix(sig, ws_bytes);
    sig = mix(sig, ((uint64_t)t.threads_per_stream << 48) ^ ((uint64_t)t.outputs_per_lane << 32) ^
                       ((uint64_t)t.workgroup_size << 16) ^ (uint64_t)(uint32_t)t.jump_target_steps);
    sig = mix(sig, (uint64_t)(uint32_t)t.window_below_w);
    sig = mix(sig, ov ? 2u : 1u);  // overlapped plans order their segment list differently
    for (const Request &r : reqs) {
        sig = mix(sig, ((uint64_t)(uint32_t)r.stream << 32) | r.dtype);
        sig = mix(sig, r.count);
        sig = mix(sig, (uint64_t)(uintptr_t)r.d_out);
        sig = mix(sig, r.flag);
    }
    if (sig == 0) sig = 1;  // 0 marks "no plan"
    // a request on a stream whose polynomial is to be rebuilt replans
    bool dirty = false;
    {
        std::lock_guard<std::mutex> lk(ps->jump_mu);
        if (ps->dirty.size() == (size_t)ps->n)
            for (const Request &r : reqs)
                if (ps->dirty[(size_t)r.stream]) {
                    dirty = true;
                    break;
                }
    }
    if (w.sig == sig && !dirty && w.ps.lock() == ps) {
        // same plan: the polynomials are in place; the item tables,
        // request records and prefix flags go up every call
        int rc = stage_copy(w, HDR_BYTES, w.tables_end, ws, s);
        if (rc) return rc;
    } else {
        w.sig = 0;
        int rc = build_plan(ps, d_params, d_states, stride, reqs, ws, ws_bytes, s, t, w, ov > 0);
        if (rc) return rc;
        rc = stage_copy(w, HDR_BYTES, w.up_end, ws, s);
        if (rc) return rc;
        w.sig = sig;
    }

    // overlapped calls launch directly (two streams, not a captured graph)
    if (!use_graph || !graphs_enabled() || w.overlap)
        return launch_phases(*ps, d_params, ws, w, t, s, stamps, per_call_errors);

    int dev = 0;
    (void)hipGetDevice(&dev);
    GraphKey key{d_ws, w.nA, w.nB, w.nC, d_params, ps->N, t.threads_per_stream,
                 t.outputs_per_lane, t.workgroup_size, t.window_below_w, dev, stamps,
                 per_call_errors};
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        hipStream_t cs;
        auto cit = g_capture_streams.find(dev);
        if (cit == g_capture_streams.end()) {
            e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
            g_capture_streams[dev] = cs;
        } else {
            cs = cit->second;
        }
        if (g_graphs.size() >= 256) {
            for (auto &kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
            g_graphs.clear();
        }
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        int rc = launch_phases(*ps, d_params, ws, w, t, cs, stamps, per_call_errors);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(cs, &gr);
        if (rc) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        it = g_graphs.emplace(key, ge).first;
    }
    e = hipGraphLaunch(it->second, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return MTGP_OK;
}

int validate_requests(const ParamSet &ps, const mtgp_work *items, int n) {
    if (n < 0 || (n > 0 && !items)) return fail(MTGP_EINVAL, "bad item list (n=%d)", n);
    std::vector<uint8_t> seen((size_t)ps.n, 0);
    for (int i = 0; i < n; ++i) {
        const mtgp_work &w = items[i];
        if (w.stream_id < 0 || w.stream_id >= ps.n)
            return fail(MTGP_EINVAL, "item %d: stream %d outside [0, %d)", i, w.stream_id, ps.n);
        if (seen[w.stream_id]++)
            return fail(MTGP_EINVAL, "item %d: stream %d appears twice in one batch", i,
                        w.stream_id);
        if (w.dtype != MTGP_U32 && w.dtype != MTGP_F32)
            return fail(MTGP_EINVAL, "item %d: dtype %u", i, w.dtype);
        if (w.count > 0 && !w.d_out) return fail(MTGP_EINVAL, "item %d: d_out is NULL", i);
        if (((uintptr_t)w.d_out & 3u) != 0)
            return fail(MTGP_EINVAL, "item %d: d_out not 4-byte aligned", i);
    }
    return MTGP_OK;
}

static std::vector<Request> to_requests(const mtgp_work *items, int n) {
    std::vector<Request> r;
    r.reserve((size_t)n);
    for (int i = 0; i < n; ++i)
        if (items[i].count > 0)
            r.push_back(Request{items[i].stream_id, items[i].dtype, items[i].count,
                                items[i].d_out, 0});
    return r;
}

static int batch_common(const void *d_params, uint32_t *d_states, int stride,
                        const mtgp_work *h_items, int n_items, void *d_ws, size_t ws_bytes,
                        hipStream_t s, const mtgp_tuning *force, bool use_graph,
                        WsState *own) {
    auto ps = lookup_params(d_params, 0);
    if (!ps) return MTGP_EINVAL;
    if (!d_states || stride < ps->N)
        return fail(MTGP_EINVAL, "state_stride %d < N=%d or NULL states", stride, ps->N);
    if (!d_ws || ((uintptr_t)d_ws & 255u))
        return fail(MTGP_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    int rc = validate_requests(*ps, h_items, n_items);
    if (rc) return rc;
    if (ws_bytes < batch_min_ws_bytes(n_items))
        return fail(MTGP_EINVAL, "workspace of %zu bytes below the minimum %zu", ws_bytes,
                    batch_min_ws_bytes(n_items));
    const mtgp_tuning t = force ? *force : tuning_for(ps->N);
    std::shared_ptr<WsState> held = own ? nullptr : ws_state(d_ws, true);
    WsState &w = own ? *own : *held;
    std::lock_guard<std::mutex> lk(w.mu);
    return run_batch(ps, d_params, d_states, stride, to_requests(h_items, n_items), d_ws,
                     ws_bytes, s, t, use_graph, w, false, true);
}

}  // namespace mtgp

using namespace mtgp;

extern "C" {

size_t mtgp_batch_workspace_bytes(int n_items) { return batch_min_ws_bytes(n_items); }

int mtgp_stream_polynomials(const void *d_params, int n_streams, uint32_t *h_coeffs,
                            int words_per_stream, int *h_degrees, void *stream) {
    auto ps = lookup_params(d_params, n_streams);
    if (!ps) return MTGP_EINVAL;
    if (n_streams <= 0 || n_streams > ps->n)
        return fail(MTGP_EINVAL, "n_streams %d outside [1, %d]", n_streams, ps->n);
    if (!h_coeffs || !h_degrees) return fail(MTGP_EINVAL, "NULL output array");
    const int need = (int)ps->mexp / 32 + 1;
    if (words_per_stream < need)
        return fail(MTGP_EINVAL, "words_per_stream %d < %d", words_per_stream, need);
    std::vector<int> all((size_t)n_streams);
    for (int k = 0; k < n_streams; ++k) all[(size_t)k] = k;
    int rc = ensure_jumps(ps, d_params, nullptr, 0, all, tuning_for(ps->N), (hipStream_t)stream);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ps->jump_mu);
    for (int k = 0; k < n_streams; ++k) {
        uint32_t *dst = h_coeffs + (size_t)k * (size_t)words_per_stream;
        std::memset(dst, 0, (size_t)words_per_stream * 4);
        const StreamJump *sj = ps->jumps[(size_t)k].get();
        if (!sj || sj->status != 1) {
            h_degrees[k] = -1;
            continue;
        }
        h_degrees[k] = sj->D;
        const std::vector<uint32_t> w = pack32(sj->mod->p, sj->D + 1);
        std::memcpy(dst, w.data(), std::min(w.size(), (size_t)words_per_stream) * 4);
    }
    return MTGP_OK;
}

int mtgp_batch_workspace_query(const void *d_params, const mtgp_work *h_items, int n_items,
                               size_t *bytes) {
    if (!bytes) return fail(MTGP_EINVAL, "bytes is NULL");
    auto ps = lookup_params(d_params, 0);
    if (!ps) return MTGP_EINVAL;
    int rc = validate_requests(*ps, h_items, n_items);
    if (rc) return rc;
    const mtgp_tuning t = tuning_for(ps->N);
    std::vector<int> want;
    std::vector<Request> reqs = to_requests(h_items, n_items);
    const uint64_t T = effective_target(*ps, reqs, t);
    for (const Request &r : reqs)
        if (wants_split(*ps, r, T, t)) want.push_back(r.stream);
    if (!want.empty()) {
        rc = ensure_jumps(ps, d_params, nullptr, 0, want, t, nullptr);
        if (rc) return rc;
    }
    std::vector<Seg> segs(reqs.size());
    {
        std::lock_guard<std::mutex> lk(ps->jump_mu);
        size_tracking(*ps);
        for (size_t i = 0; i < reqs.size(); ++i) {
            const int k = reqs[i].stream;
            const StreamJump *sj = ps->jumps[(size_t)k].get();
            segs[i].req = (int)i;
            if (sj && sj->status == 1 && !ps->dirty[(size_t)k]) {
                decide(*ps, reqs[i], sj->D, T, t, segs[i]);
            } else if (!sj || ps->dirty[(size_t)k]) {
                // the polynomial will be built from the stream's state at
                // generation time: size for the most segments (D = 1) and
                // the largest degree (mexp)
                decide(*ps, reqs[i], 1, T, t, segs[i]);
                if (segs[i].C > 1) segs[i].Dsize = (int)ps->mexp;
            }
        }
    }
    *bytes = std::max(layout_for(*ps, segs).total, batch_min_ws_bytes(n_items));
    return MTGP_OK;
}

int mtgp_generate_batch(const void *d_params, uint32_t *d_states, int state_stride,
                        const mtgp_work *h_items, int n_items, void *d_workspace,
                        size_t workspace_bytes, void *stream) {
    return batch_common(d_params, d_states, state_stride, h_items, n_items, d_workspace,
                        workspace_bytes, (hipStream_t)stream, nullptr, true, nullptr);
}

int mtgp_generate_batch_noalloc(const void *d_params, uint32_t *d_states, int state_stride,
                                const mtgp_work *h_items, int n_items, void *stream) {
    if (n_items < 0) return fail(MTGP_EINVAL, "n_items=%d", n_items);
    const size_t need = batch_min_ws_bytes(n_items);
    if (need > (size_t)MTGP_NOALLOC_SCRATCH_BYTES)
        return fail(MTGP_ETOOBIG,
                    "a batch of %d items needs %zu bytes of workspace; the static scratch "
                    "holds %u",
                    n_items, need, (unsigned)MTGP_NOALLOC_SCRATCH_BYTES);
    auto ps = lookup_params(d_params, 0);
    if (!ps) return MTGP_EINVAL;
    if (!d_states || state_stride < ps->N)
        return fail(MTGP_EINVAL, "state_stride %d < N=%d or NULL states", state_stride,
                    ps->N);
    int rc = validate_requests(*ps, h_items, n_items);
    if (rc) return rc;
    void *scr = nullptr;
    hipError_t e = scratch_address(&scr);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    // one plan state per GPU's scratch
    static std::mutex mu;
    static std::map<int, std::unique_ptr<WsState>> states;
    int dev = 0;
    (void)hipGetDevice(&dev);
    WsState *w;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto &slot = states[dev];
        if (!slot) {
            slot = std::make_unique<WsState>();
            slot->no_alloc = true;
        }
        w = slot.get();
    }
    std::lock_guard<std::mutex> lk(w->mu);
    return run_batch(ps, d_params, d_states, state_stride, to_requests(h_items, n_items), scr,
                     (size_t)MTGP_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream,
                     tuning_for(ps->N), false, *w, false, false);
}

int mtgp_set_phase_timing(int enable) {
    g_stamps.store(enable != 0);
    return MTGP_OK;
}

int mtgp_batch_phase_times(void *d_workspace, void *stream, double *h_us) {
    if (!d_workspace || !h_us) return fail(MTGP_EINVAL, "NULL workspace or h_us");
    hipStream_t s = (hipStream_t)stream;
    uint64_t ts[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(ts, (char *)d_workspace + HDR_STAMP_BYTE, sizeof ts,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "read phase timestamps");
    if (!ts[0] || ts[1] < ts[0] || ts[2] < ts[1] || ts[3] < ts[2])
        return fail(MTGP_EINVAL, "no phase timestamps in this workspace (timing disabled?)");
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess || khz <= 0) return hip_fail(e, "wall clock rate");
    for (int i = 0; i < 3; ++i) h_us[i] = (double)(ts[i + 1] - ts[i]) * 1e3 / (double)khz;
    return MTGP_OK;
}

int mtgp_batch_errors(void *d_workspace, void *stream, uint32_t *n) {
    if (!d_workspace || !n) return fail(MTGP_EINVAL, "NULL workspace or n");
    hipStream_t s = (hipStream_t)stream;
    uint32_t v[HDR_TAG + 2 - HDR_ERR] = {};
    uint32_t *hw = (uint32_t *)d_workspace + HDR_ERR;
    hipError_t e = hipMemcpyAsync(v, hw, sizeof v, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = launch_clear(hw, HDR_ERR_WORDS, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "read and reset the repair count");
    // a header without this workspace's tag holds no count of ours
    const uint64_t tag = header_tag(d_workspace);
    const bool ours = v[HDR_TAG - HDR_ERR] == (uint32_t)tag &&
                      v[HDR_TAG + 1 - HDR_ERR] == (uint32_t)(tag >> 32);
    *n = ours ? v[0] : 0u;
    if (*n != 0) {
        // rebuild the logged streams' polynomials from their current states
        // and re-upload the whole plan next time (the cached polynomials
        // in the workspace may have been overwritten)
        if (auto w = ws_state(d_workspace, false)) {
            std::lock_guard<std::mutex> lk(w->mu);
            if (auto ps = w->ps.lock()) note_repairs(*ps, v, w->split_streams);
            w->sig = 0;
        }
    }
    return MTGP_OK;
}

int mtgp_autotune(const void *d_params, const uint32_t *d_states, int state_stride,
                  const mtgp_work *h_items, int n_items, void *d_scratch, size_t scratch_bytes,
                  int reps, void *stream, mtgp_tuning *best, float *h_ms, int max_out) {
    auto ps = lookup_params(d_params, 0);
    if (!ps) return MTGP_EINVAL;
    if (!d_scratch || ((uintptr_t)d_scratch & 255u))
        return fail(MTGP_EINVAL, "scratch must be non-NULL and 256-byte aligned");
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    const size_t state_bytes = (size_t)ps->n * (size_t)state_stride * 4;
    const size_t state_al = (state_bytes + 255) / 256 * 256;
    if (scratch_bytes < state_al + batch_min_ws_bytes(n_items))
        return fail(MTGP_EINVAL, "scratch of %zu bytes too small", scratch_bytes);
    uint32_t *scratch_states = (uint32_t *)d_scratch;
    void *ws = (char *)d_scratch + state_al;
    const size_t ws_bytes = scratch_bytes - state_al;
    hipError_t e = hipMemcpyAsync(scratch_states, d_states, state_bytes,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(scratch states)");
    mtgp_tuning cands[64];
    const int nc = std::min(64, mtgp_tuning_candidates(ps->mexp, cands, 64));
    const mtgp_tuning cur = tuning_for(ps->N);
    hipEvent_t ev0, ev1;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&ev1)) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        return hip_fail(e, "hipEventCreate");
    }
    WsState wst;  // the scratch workspace's own plan state
    auto time_one = [&](const mtgp_tuning &t, float *ms) -> int {
        int rc = batch_common(d_params, scratch_states, state_stride, h_items, n_items, ws,
                              ws_bytes, s, &t, false, &wst);  // warm-up + planning
        if (rc) return rc;
        float total = 0.f;
        for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(ev0, s);
            rc = batch_common(d_params, scratch_states, state_stride, h_items, n_items, ws,
                              ws_bytes, s, &t, false, &wst);
            (void)hipEventRecord(ev1, s);
            if (rc) return rc;
            hipError_t e2 = hipEventSynchronize(ev1);
            if (e2 != hipSuccess) return hip_fail(e2, "hipEventSynchronize(autotune)");
            float m = 0.f;
            (void)hipEventElapsedTime(&m, ev0, ev1);
            total += m;
        }
        *ms = total / (float)reps;
        return MTGP_OK;
    };
    float best_ms = 1e30f;
    mtgp_tuning bt = cur;
    int rc = MTGP_OK;
    for (int i = 0; i < nc && rc == MTGP_OK; ++i) {
        cands[i].jump_target_steps = cur.jump_target_steps;
        cands[i].window_below_w = cur.window_below_w;
        float ms = 0.f;
        rc = time_one(cands[i], &ms);
        if (rc) break;
        if (h_ms && i < max_out) h_ms[i] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            bt = cands[i];
        }
    }
    const int targets[] = {0, 1024, 2048, 4096, 8192, 16384, 65536};
    for (int T : targets) {
        if (rc) break;
        if (T == bt.jump_target_steps) continue;
        mtgp_tuning t = bt;
        t.jump_target_steps = T;
        float ms = 0.f;
        rc = time_one(t, &ms);
        if (rc == MTGP_OK && ms < best_ms) {
            best_ms = ms;
            bt = t;
        }
    }
    // the window threshold matters only for one-wave tunings and streams
    // with a linear rec_tbl and W < 64
    bool narrow = false;
    for (int i = 0; i < n_items && !narrow; ++i) {
        const int k = h_items[i].stream_id;
        narrow = k >= 0 && k < ps->n && ps->lin[(size_t)k] && ps->W[(size_t)k] < 64u;
    }
    const int thresholds[] = {0, 16, 24, 32, 48, 64};
    for (int wb : thresholds) {
        if (rc || !narrow || bt.threads_per_stream != 64) break;
        if (wb == bt.window_below_w) continue;
        mtgp_tuning t = bt;
        t.window_below_w = wb;
        float ms = 0.f;
        rc = time_one(t, &ms);
        if (rc == MTGP_OK && ms < best_ms) {
            best_ms = ms;
            bt = t;
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (rc) return rc;
    rc = mtgp_set_tuning(ps->mexp, &bt);
    if (rc) return rc;
    if (best) *best = bt;
    return MTGP_OK;
}

}  // extern "C"
