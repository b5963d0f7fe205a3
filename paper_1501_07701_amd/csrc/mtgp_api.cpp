// mtgp_api.cpp -- host side of the C ABI (include/mtgp.h): validation,
// parameter packing, plain launches, tuning tables, checkpoint copies.
// Batched generation lives in mtgp_batch.cpp, serving in mtgp_server.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "mtgp.h"
#include "mtgp_host.hpp"
#include "mtgp_internal.hpp"

namespace mtgp {

// ----------------------------------------------------------------- errors --

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

int hip_fail(hipError_t e, const char *what) {
    return fail(MTGP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// --------------------------------------------------------------- devices --

int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    cache[dev] = cus;
    return cus;
}

// ------------------------------------------------------------- params ------

int words_for_mexp(uint32_t mexp) {
    switch (mexp) {
        case 3217: case 11213: case 23209: case 44497:
            return (int)(mexp / 32 + 1);
        default:
            return -1;
    }
}

static int check_one(const mtgp_params &p, int k, uint32_t mexp0) {
    const int n = words_for_mexp(p.mexp);
    if (n < 0) return fail(MTGP_EINVAL, "stream %d: unsupported mexp %u", k, p.mexp);
    if (p.mexp != mexp0)
        return fail(MTGP_EINVAL, "stream %d: mexp %u differs from stream 0's %u", k, p.mexp, mexp0);
    const uint32_t r = 32u * (uint32_t)n - p.mexp;
    const uint32_t want = 0xFFFFFFFFu << r;
    if (p.mask != want)
        return fail(MTGP_EINVAL, "stream %d: mask 0x%08x, expected 0x%08x", k, p.mask, want);
    if (p.pos < 1 || p.pos > (uint32_t)n - 2)
        return fail(MTGP_EINVAL, "stream %d: pos=%u outside [1, %d]", k, p.pos, n - 2);
    if (p.sh1 > 31) return fail(MTGP_EINVAL, "stream %d: sh1=%u > 31", k, p.sh1);
    if (p.sh2 > 31) return fail(MTGP_EINVAL, "stream %d: sh2=%u > 31", k, p.sh2);
    for (int i = 0; i < 16; ++i)
        if ((p.flt_tbl[i] >> 23) != 0x7Fu)
            return fail(MTGP_EINVAL, "stream %d: flt_tbl[%d]=0x%08x lacks exponent 0x7F",
                        k, i, p.flt_tbl[i]);
    return MTGP_OK;
}

int check_params(const mtgp_params *h, int n) {
    if (!h || n <= 0) return fail(MTGP_EINVAL, "no parameter sets (n=%d)", n);
    for (int k = 0; k < n; ++k) {
        int rc = check_one(h[k], k, h[0].mexp);
        if (rc) return rc;
    }
    return MTGP_OK;
}

static std::mutex g_reg_mu;
static std::unordered_map<const void *, std::shared_ptr<ParamSet>> g_reg;

std::shared_ptr<ParamSet> lookup_params(const void *d_params, int n_streams) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_reg.find(d_params);
    if (it == g_reg.end()) {
        fail(MTGP_EINVAL, "d_params %p was not written by mtgp_init_states/mtgp_load_params",
             d_params);
        return nullptr;
    }
    if (n_streams > it->second->n) {
        fail(MTGP_EINVAL, "n_streams=%d exceeds the %d streams of d_params", n_streams,
             it->second->n);
        return nullptr;
    }
    return it->second;
}

// 32x32 matrices over GF(2) as column words: m[j] = M e_j.
using Mat32 = std::array<uint32_t, 32>;

static uint32_t mat_vec(const Mat32 &m, uint32_t v) {
    uint32_t r = 0;
    for (int j = 0; j < 32; ++j)
        if ((v >> j) & 1u) r ^= m[j];
    return r;
}

static Mat32 mat_mul(const Mat32 &a, const Mat32 &b) {
    Mat32 c;
    for (int j = 0; j < 32; ++j) c[j] = mat_vec(a, b[j]);
    return c;
}

static Mat32 mat_pow(Mat32 m, uint64_t e) {
    Mat32 r;
    for (int j = 0; j < 32; ++j) r[j] = 1u << j;
    while (e) {
        if (e & 1u) r = mat_mul(r, m);
        m = mat_mul(m, m);
        e >>= 1;
    }
    return r;
}

// Windowed small-step data for a linear recursion table and W < 64: the
// tap chain x_n = G(X_n) ^ M x_{n-W}, with G(y) = y ^ rec[y & 15] and
// M y = G(y >> sh2), is split across q = 64/W lanes per residue class with
// E elements per lane; lanes are stitched by a scan with M^(E*2^r).
static void window_data(const mtgp_params &p, int N, uint32_t *b) {
    const uint32_t W = (uint32_t)N - p.pos;
    const uint32_t q = 64u / W;
    const uint32_t wn = std::min<uint32_t>((uint32_t)N - 1, W * q * (uint32_t)WIN_EMAX);
    const uint32_t per_class = (wn + W - 1) / W;
    const uint32_t E = (per_class + q - 1) / q;
    uint32_t rounds = 0;
    while ((1u << rounds) < q) ++rounds;
    b[P_WIN_WN] = wn;
    b[P_WIN_E] = E;
    b[P_WIN_Q] = q;
    b[P_WIN_ROUNDS] = rounds;
    Mat32 M;
    for (int j = 0; j < 32; ++j) {
        if ((uint32_t)j < p.sh2) {
            M[j] = 0;
            continue;
        }
        const uint32_t y = 1u << (j - p.sh2);
        M[j] = y ^ p.rec_tbl[y & 15u];
    }
    Mat32 P = mat_pow(M, E);
    for (uint32_t r = 0; r < rounds; ++r) {
        uint32_t *t = b + P_WIN_MAT + r * WIN_MAT_WORDS;
        for (int k = 0; k < 8; ++k)
            for (uint32_t v = 0; v < 16; ++v) t[k * 16 + v] = mat_vec(P, v << (4 * k));
        P = mat_mul(P, P);
    }
}

static int upload_params(const mtgp_params *h, const uint32_t *seeds, int n, void *d_params,
                         hipStream_t s) {
    int rc = check_params(h, n);
    if (rc) return rc;
    if (!d_params) return fail(MTGP_EINVAL, "d_params is NULL");
    const int N = words_for_mexp(h[0].mexp);
    std::vector<uint32_t> blob((size_t)n * P_WORDS, 0u);
    auto set = std::make_shared<ParamSet>();
    set->n = n;
    set->N = N;
    set->mexp = h[0].mexp;
    set->W.resize(n);
    set->lin.resize(n);
    // seeded streams' jump-ahead polynomials come from their seed orbits;
    // after a parameter reload the states come from elsewhere
    set->seeded.assign((size_t)n, seeds ? 1 : 0);
    set->dirty.assign((size_t)n, seeds ? 0 : 1);
    for (int k = 0; k < n; ++k) {
        uint32_t *b = &blob[(size_t)k * P_WORDS];
        b[P_MEXP] = h[k].mexp;
        b[P_N] = (uint32_t)N;
        b[P_POS] = h[k].pos;
        b[P_SH1] = h[k].sh1;
        b[P_SH2] = h[k].sh2;
        b[P_MASK] = h[k].mask;
        b[P_W] = (uint32_t)N - h[k].pos;
        b[P_SEED] = seeds ? seeds[k] : 0u;
        // a linear recursion table is a span of four basis words; the
        // latency-bound small-step path then forms rec[Y & 15] in registers
        bool lin = h[k].rec_tbl[0] == 0u;
        for (int i = 1; i < 16 && lin; ++i) {
            uint32_t v = 0;
            for (int bit = 0; bit < 4; ++bit)
                if ((i >> bit) & 1) v ^= h[k].rec_tbl[1 << bit];
            lin = v == h[k].rec_tbl[i];
        }
        b[P_LIN] = lin ? 1u : 0u;
        for (int bit = 0; bit < 4; ++bit) b[P_RB + bit] = h[k].rec_tbl[1 << bit];
        if (lin && (uint32_t)N - h[k].pos < 64u) window_data(h[k], N, b);
        std::memcpy(b + P_REC, h[k].rec_tbl, 64);
        std::memcpy(b + P_TMP, h[k].tmp_tbl, 64);
        std::memcpy(b + P_FLT, h[k].flt_tbl, 64);
        set->W[k] = (uint32_t)N - h[k].pos;
        set->lin[k] = lin ? 1 : 0;
    }
    hipError_t e = hipMemcpyAsync(d_params, blob.data(), blob.size() * 4,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(params)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    static std::atomic<uint64_t> generation{1};
    set->generation = generation.fetch_add(1);
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_reg[d_params] = set;
    return MTGP_OK;
}

// ----------------------------------------------------------------- tuning --

static std::mutex g_tune_mu;
static std::map<int, mtgp_tuning> g_tune;  // keyed by N

static mtgp_tuning default_tuning(int N) {
    // One wave per stream, 4 waves per workgroup; K trades step width
    // against LDS per wave (occupancy); jump-ahead splits streams on a
    // batch's critical path, with segments of at least 1024 dependent steps;
    // narrow streams take the windowed scan below W = 56 (it is ahead of
    // W-word steps up to about there), below 64 at N <= 128, where every
    // window is short and the wide path's steps are at most 96 words
    // (measured on 10000 mexp-3217 streams of 2^20 outputs: 22.1 ms against
    // 23.3 ms with 56 and 29.5 ms with K = 1), and below 48 at N = 351
    // (128 mexp-11213 streams of 2^24 outputs: 2.81 ms against 2.84 ms with
    // 56, 2.93 with 64 and 2.96 with 40; at N = 726 and 1391 48 and 56
    // time alike).
    mtgp_tuning t;
    t.threads_per_stream = 64;
    t.workgroup_size = 256;
    t.outputs_per_lane = N <= 400 ? 4 : 8;
    t.jump_target_steps = 1024;
    t.window_below_w = N <= 128 ? 64 : N <= 400 ? 48 : 56;
    return t;
}

mtgp_tuning tuning_for(int N) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(N);
    return it == g_tune.end() ? default_tuning(N) : it->second;
}

static int wpb_of(const mtgp_tuning &t) {
    return t.threads_per_stream == 64 ? t.workgroup_size / 64 : 1;
}

int launch_tuned(int N, const mtgp_tuning &t, const LaunchArgs &a) {
    bool found = false;
    LaunchArgs la = a;
    la.win_below = t.threads_per_stream == 64 ? (uint32_t)t.window_below_w : 0u;
    hipError_t e = launch_variant(N, t.threads_per_stream, t.outputs_per_lane, wpb_of(t), la,
                                  &found);
    if (!found)
        return fail(MTGP_EINVAL, "no kernel compiled for N=%d tps=%d k=%d wg=%d", N,
                    t.threads_per_stream, t.outputs_per_lane, t.workgroup_size);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return MTGP_OK;
}

static int generate_plain(const void *d_params, uint32_t *d_states, int stride, int n_streams,
                          uint64_t count, uint32_t *d_out, uint32_t f32, hipStream_t s) {
    auto ps = lookup_params(d_params, n_streams);
    if (!ps) return MTGP_EINVAL;
    if (n_streams <= 0) return fail(MTGP_EINVAL, "n_streams=%d", n_streams);
    if (!d_states || stride < ps->N)
        return fail(MTGP_EINVAL, "state_stride %d < N=%d or NULL states", stride, ps->N);
    if (count == 0) return MTGP_OK;
    if (!d_out) return fail(MTGP_EINVAL, "d_out is NULL");
    const mtgp_tuning t = tuning_for(ps->N);
    LaunchArgs a{};
    a.params = (const uint32_t *)d_params;
    a.items = nullptr;
    a.n_items = (uint32_t)n_streams;
    a.plain_states = d_states;
    a.plain_stride = (uint32_t)stride;
    a.plain_out = d_out;
    a.plain_count = count;
    a.plain_mode = f32 ? MODE_F32 : 0u;
    a.persistent = false;
    a.num_cus = device_cus();
    a.stream = s;
    return launch_tuned(ps->N, t, a);
}

}  // namespace mtgp

using namespace mtgp;

// ================================================================ C ABI ===

extern "C" {

int mtgp_state_words(uint32_t mexp) {
    int n = words_for_mexp(mexp);
    return n < 0 ? fail(MTGP_EINVAL, "unsupported mexp %u", mexp) : n;
}

int mtgp_check_params(const mtgp_params *h_params, int n_streams) {
    return check_params(h_params, n_streams);
}

int mtgp_init_states(const mtgp_params *h_params, const uint32_t *h_seeds, int n_streams,
                     void *d_params, uint32_t *d_states, int state_stride, void *stream) {
    if (!h_seeds) return fail(MTGP_EINVAL, "h_seeds is NULL");
    if (!d_states) return fail(MTGP_EINVAL, "d_states is NULL");
    if (n_streams > 0 && h_params) {
        int n = words_for_mexp(h_params[0].mexp);
        if (n > 0 && state_stride < n)
            return fail(MTGP_EINVAL, "state_stride %d < N=%d", state_stride, n);
    }
    hipStream_t s = (hipStream_t)stream;
    int rc = upload_params(h_params, h_seeds, n_streams, d_params, s);
    if (rc) return rc;
    hipError_t e = launch_seed((const uint32_t *)d_params, d_states, (uint32_t)state_stride,
                               (uint32_t)n_streams, s);
    if (e != hipSuccess) return hip_fail(e, "seed kernel");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(seed)");
    return MTGP_OK;
}

int mtgp_seed_states(const void *d_params, uint32_t *d_states, int state_stride, int n_streams,
                     void *stream) {
    auto ps = lookup_params(d_params, n_streams);
    if (!ps) return MTGP_EINVAL;
    if (n_streams <= 0 || !d_states || state_stride < ps->N)
        return fail(MTGP_EINVAL, "bad states (n=%d, stride=%d, N=%d)", n_streams, state_stride,
                    ps->N);
    hipError_t e = launch_seed((const uint32_t *)d_params, d_states, (uint32_t)state_stride,
                               (uint32_t)n_streams, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "seed kernel");
    note_states_seeded(*ps, n_streams);
    return MTGP_OK;
}

int mtgp_load_params(const mtgp_params *h_params, int n_streams, void *d_params, void *stream) {
    return upload_params(h_params, nullptr, n_streams, d_params, (hipStream_t)stream);
}

int mtgp_release_params(const void *d_params) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    if (g_reg.erase(d_params) == 0) return fail(MTGP_ENOENT, "d_params %p unknown", d_params);
    return MTGP_OK;
}

int mtgp_generate_u32(const void *d_params, uint32_t *d_states, int state_stride, int n_streams,
                      uint64_t count_per_stream, uint32_t *d_out, void *stream) {
    return generate_plain(d_params, d_states, state_stride, n_streams, count_per_stream, d_out, 0,
                          (hipStream_t)stream);
}

int mtgp_generate_f32(const void *d_params, uint32_t *d_states, int state_stride, int n_streams,
                      uint64_t count_per_stream, float *d_out, void *stream) {
    return generate_plain(d_params, d_states, state_stride, n_streams, count_per_stream,
                          (uint32_t *)d_out, 1, (hipStream_t)stream);
}

int mtgp_get_tuning(uint32_t mexp, mtgp_tuning *out) {
    int n = words_for_mexp(mexp);
    if (n < 0 || !out) return fail(MTGP_EINVAL, "unsupported mexp %u or NULL out", mexp);
    *out = tuning_for(n);
    return MTGP_OK;
}

int mtgp_set_tuning(uint32_t mexp, const mtgp_tuning *t) {
    int n = words_for_mexp(mexp);
    if (n < 0 || !t) return fail(MTGP_EINVAL, "unsupported mexp %u or NULL tuning", mexp);
    VariantInfo v[64];
    int c = variant_count(n, v, 64);
    for (int i = 0; i < c && i < 64; ++i) {
        const int wg = v[i].tps == 64 ? 64 * v[i].wpb : v[i].tps;
        if (v[i].tps == t->threads_per_stream && v[i].k == t->outputs_per_lane &&
            wg == t->workgroup_size) {
            if (t->jump_target_steps < 0)
                return fail(MTGP_EINVAL, "jump_target_steps %d < 0", t->jump_target_steps);
            if (t->window_below_w < 0 || t->window_below_w > 64)
                return fail(MTGP_EINVAL, "window_below_w %d outside [0, 64]",
                            t->window_below_w);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[n] = *t;
            return MTGP_OK;
        }
    }
    return fail(MTGP_EINVAL, "tuning tps=%d k=%d wg=%d not compiled for mexp %u",
                t->threads_per_stream, t->outputs_per_lane, t->workgroup_size, mexp);
}

int mtgp_tuning_candidates(uint32_t mexp, mtgp_tuning *out, int max_out) {
    int n = words_for_mexp(mexp);
    if (n < 0) return fail(MTGP_EINVAL, "unsupported mexp %u", mexp);
    VariantInfo v[64];
    int c = variant_count(n, v, 64);
    for (int i = 0; out && i < c && i < max_out && i < 64; ++i) {
        out[i].threads_per_stream = v[i].tps;
        out[i].outputs_per_lane = v[i].k;
        out[i].workgroup_size = v[i].tps == 64 ? 64 * v[i].wpb : v[i].tps;
        out[i].jump_target_steps = default_tuning(n).jump_target_steps;
        out[i].window_below_w = default_tuning(n).window_below_w;
    }
    return c;
}

int mtgp_state_export(const void *d_params, const uint32_t *d_states, int state_stride,
                      int n_streams, uint32_t *h_out, void *stream) {
    auto ps = lookup_params(d_params, n_streams);
    if (!ps) return MTGP_EINVAL;
    if (!h_out || !d_states || state_stride < ps->N || n_streams < 0)
        return fail(MTGP_EINVAL, "bad export arguments");
    hipError_t e = hipMemcpy2DAsync(h_out, (size_t)ps->N * 4, d_states, (size_t)state_stride * 4,
                                    (size_t)ps->N * 4, (size_t)n_streams, hipMemcpyDeviceToHost,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync(export)");
    e = hipStreamSynchronize((hipStream_t)stream);
    return e == hipSuccess ? MTGP_OK : hip_fail(e, "hipStreamSynchronize(export)");
}

int mtgp_state_import(const void *d_params, uint32_t *d_states, int state_stride, int n_streams,
                      const uint32_t *h_in, void *stream) {
    auto ps = lookup_params(d_params, n_streams);
    if (!ps) return MTGP_EINVAL;
    if (!h_in || !d_states || state_stride < ps->N || n_streams < 0)
        return fail(MTGP_EINVAL, "bad import arguments");
    hipError_t e = hipMemcpy2DAsync(d_states, (size_t)state_stride * 4, h_in, (size_t)ps->N * 4,
                                    (size_t)ps->N * 4, (size_t)n_streams, hipMemcpyHostToDevice,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync(import)");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(import)");
    // the imported states may lie outside the orbits the streams' jump-ahead
    // polynomials annihilate: rebuild those from the states themselves
    note_states_foreign(*ps, nullptr, n_streams);
    return MTGP_OK;
}

int mtgp_generate_workgroup(const void *d_params, uint32_t *d_states, int state_stride,
                            int n_streams, uint64_t count_per_stream, int dtype, int threads,
                            void *d_out, void *stream) {
    auto ps = lookup_params(d_params, n_streams);
    if (!ps) return MTGP_EINVAL;
    if (n_streams <= 0) return fail(MTGP_EINVAL, "n_streams=%d", n_streams);
    if (!d_states || state_stride < ps->N)
        return fail(MTGP_EINVAL, "state_stride %d < N=%d or NULL states", state_stride, ps->N);
    if (dtype != MTGP_U32 && dtype != MTGP_F32) return fail(MTGP_EINVAL, "dtype %d", dtype);
    if (threads < 64 || threads > 1024 || (threads & 63))
        return fail(MTGP_EINVAL, "threads %d: a multiple of 64 in [64, 1024]", threads);
    if (count_per_stream == 0) return MTGP_OK;
    if (!d_out) return fail(MTGP_EINVAL, "d_out is NULL");
    hipError_t e = launch_workgroup((const uint32_t *)d_params, d_states, (uint32_t)state_stride,
                                    (uint32_t)n_streams, count_per_stream, (uint32_t *)d_out,
                                    dtype == MTGP_F32 ? 1u : 0u, (uint32_t)threads,
                                    (uint32_t)ps->N, (hipStream_t)stream);
    return e == hipSuccess ? MTGP_OK : hip_fail(e, "workgroup kernel");
}

int mtgp_screen(const uint32_t *d_outputs, int n_streams, uint64_t count_per_stream,
                uint32_t gap_lo, uint32_t gap_hi, int gap_bins, uint64_t *d_counts,
                void *stream) {
    if (!d_outputs || !d_counts) return fail(MTGP_EINVAL, "NULL outputs or counts");
    if (n_streams <= 0) return fail(MTGP_EINVAL, "n_streams=%d", n_streams);
    if (count_per_stream < 2 || count_per_stream >= (1ull << 32))
        return fail(MTGP_EINVAL, "count_per_stream %llu outside [2, 2^32)",
                    (unsigned long long)count_per_stream);
    if (gap_lo >= gap_hi) return fail(MTGP_EINVAL, "empty gap interval [%u, %u)", gap_lo, gap_hi);
    if (gap_bins < 2 || gap_bins > 64) return fail(MTGP_EINVAL, "gap_bins %d outside [2, 64]", gap_bins);
    hipError_t e = launch_screen(d_outputs, (uint32_t)n_streams, count_per_stream, gap_lo, gap_hi,
                                 (uint32_t)gap_bins, d_counts, (hipStream_t)stream);
    return e == hipSuccess ? MTGP_OK : hip_fail(e, "screen kernel");
}

int mtgp_fill_u32(uint32_t *d_out, uint64_t n_words, uint32_t value, void *stream) {
    if (!d_out || ((uintptr_t)d_out & 15u)) return fail(MTGP_EINVAL, "d_out must be 16-byte aligned");
    if (n_words == 0) return MTGP_OK;
    hipError_t e = launch_fill(d_out, n_words, value, device_cus(), (hipStream_t)stream);
    return e == hipSuccess ? MTGP_OK : hip_fail(e, "fill kernel");
}

const char *mtgp_strerror(int code) {
    switch (code) {
        case MTGP_OK: return "ok";
        case MTGP_EINVAL: return "invalid argument";
        case MTGP_ENOMEM: return "out of host memory";
        case MTGP_EDEVICE: return "HIP runtime error";
        case MTGP_ETOOBIG: return "request larger than the output pool";
        case MTGP_EAGAIN: return "queue full, try again";
        case MTGP_ENOENT: return "unknown ticket or handle";
        case MTGP_ECANCELED: return "cancelled";
        case MTGP_ETIMEDOUT: return "timed out";
        default: return "unknown error";
    }
}

const char *mtgp_last_error_detail(void) { return g_detail.c_str(); }

}  // extern "C"
