// mtgp_api.cpp -- host side of the C ABI (include/mtgp.h): validation,
// parameter packing, launch planning, batch scheduling with hipGraph replay,
// the autotuner, checkpoint copies.
#include <hip/hip_runtime.h>

#include <algorithm>
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
        std::memcpy(b + P_REC, h[k].rec_tbl, 64);
        std::memcpy(b + P_TMP, h[k].tmp_tbl, 64);
        std::memcpy(b + P_FLT, h[k].flt_tbl, 64);
        set->W[k] = (uint32_t)N - h[k].pos;
    }
    hipError_t e = hipMemcpyAsync(d_params, blob.data(), blob.size() * 4,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(params)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_reg[d_params] = set;
    return MTGP_OK;
}

// ----------------------------------------------------------------- tuning --

static std::mutex g_tune_mu;
static std::map<int, mtgp_tuning> g_tune;  // keyed by N

static mtgp_tuning default_tuning(int N) {
    // One wave per stream, 4 waves per workgroup; K sized so a step can
    // cover the typical step width W (uniform in [2, N-1]).
    mtgp_tuning t;
    t.threads_per_stream = 64;
    t.workgroup_size = 256;
    t.outputs_per_lane = N <= 128 ? 1 : (N <= 400 ? 4 : 8);
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
    hipError_t e = launch_variant(N, t.threads_per_stream, t.outputs_per_lane, wpb_of(t), a, &found);
    if (!found)
        return fail(MTGP_EINVAL, "no kernel compiled for N=%d tps=%d k=%d wg=%d", N,
                    t.threads_per_stream, t.outputs_per_lane, t.workgroup_size);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return MTGP_OK;
}

// ------------------------------------------------------------- batching --

// Orders items longest-critical-path first: a stream needs
// ceil(count / min(W, lanes*K)) dependent steps whatever else runs.
// order[j] is the input index of output item j.  Zero-count items are
// dropped.
void plan_items_indexed(const ParamSet &ps, const mtgp_tuning &t, const mtgp_work *items, int n,
                        std::vector<BatchItem> &out, std::vector<int> &order) {
    const uint64_t smax = (uint64_t)t.threads_per_stream * (uint64_t)t.outputs_per_lane;
    std::vector<std::pair<uint64_t, int>> key;
    key.reserve(n);
    for (int i = 0; i < n; ++i) {
        if (items[i].count == 0) continue;
        const uint64_t w = std::min<uint64_t>(ps.W[items[i].stream_id], smax);
        key.emplace_back((items[i].count + w - 1) / w, i);
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const auto &x, const auto &y) { return x.first > y.first; });
    out.clear();
    order.clear();
    out.reserve(key.size());
    order.reserve(key.size());
    for (auto &kv : key) {
        const mtgp_work &w = items[kv.second];
        BatchItem b;
        b.stream = (uint32_t)w.stream_id;
        b.dtype = w.dtype;
        b.count = w.count;
        b.out = (uint64_t)(uintptr_t)w.d_out;
        b.flag = 0;
        out.push_back(b);
        order.push_back(kv.second);
    }
}

int validate_items(const ParamSet &ps, int n_streams_limit, const mtgp_work *items, int n) {
    if (n < 0 || (n > 0 && !items)) return fail(MTGP_EINVAL, "bad item list (n=%d)", n);
    std::vector<uint8_t> seen((size_t)n_streams_limit, 0);
    for (int i = 0; i < n; ++i) {
        const mtgp_work &w = items[i];
        if (w.stream_id < 0 || w.stream_id >= n_streams_limit)
            return fail(MTGP_EINVAL, "item %d: stream %d outside [0, %d)", i, w.stream_id,
                        n_streams_limit);
        if (seen[w.stream_id]++)
            return fail(MTGP_EINVAL, "item %d: stream %d appears twice in one batch", i,
                        w.stream_id);
        if (w.dtype != MTGP_U32 && w.dtype != MTGP_F32)
            return fail(MTGP_EINVAL, "item %d: dtype %u", i, w.dtype);
        if (w.count > 0 && !w.d_out) return fail(MTGP_EINVAL, "item %d: d_out is NULL", i);
        if (((uintptr_t)w.d_out & 3u) != 0)
            return fail(MTGP_EINVAL, "item %d: d_out not 4-byte aligned", i);
    }
    (void)ps;
    return MTGP_OK;
}

// Graph cache: one instantiated [reset counter -> generate] graph per
// (buffers, item count, tuning); the work list contents change between
// replays, its address does not.
struct GraphKey {
    const void *params;
    void *states;
    uint32_t stride;
    void *ws;
    uint32_t n_items;
    int N, tps, k, wg;
    int device;
    bool operator<(const GraphKey &o) const {
        return std::tie(params, states, stride, ws, n_items, N, tps, k, wg, device) <
               std::tie(o.params, o.states, o.stride, o.ws, o.n_items, o.N, o.tps, o.k, o.wg,
                        o.device);
    }
};

static std::mutex g_graph_mu;
static std::map<GraphKey, hipGraphExec_t> g_graphs;
static std::map<int, hipStream_t> g_capture_streams;

static bool graphs_enabled() {
    const char *v = getenv("MTGP_GRAPH");
    return !(v && v[0] == '0');
}

int run_batch_device(const ParamSet &ps, const void *d_params, uint32_t *d_states,
                     int stride, const BatchItem *d_items, uint32_t n_items, uint32_t *d_counter,
                     const mtgp_tuning &t, hipStream_t s, bool use_graph) {
    LaunchArgs a{};
    a.params = (const uint32_t *)d_params;
    a.states = d_states;
    a.stride = (uint32_t)stride;
    a.items = d_items;
    a.n_items = n_items;
    a.counter = d_counter;
    a.grid = 0;
    a.num_cus = device_cus();
    if (!use_graph || !graphs_enabled()) {
        hipError_t e = launch_reset(d_counter, s);
        if (e != hipSuccess) return hip_fail(e, "reset kernel");
        a.stream = s;
        return launch_tuned(ps.N, t, a);
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    GraphKey key{d_params, d_states, (uint32_t)stride, (void *)d_counter, n_items, ps.N,
                 t.threads_per_stream, t.outputs_per_lane, t.workgroup_size, dev};
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        hipStream_t cs;
        auto cit = g_capture_streams.find(dev);
        if (cit == g_capture_streams.end()) {
            hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
            g_capture_streams[dev] = cs;
        } else {
            cs = cit->second;
        }
        if (g_graphs.size() >= 256) {
            for (auto &kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
            g_graphs.clear();
        }
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t e1 = launch_reset(d_counter, cs);
        a.stream = cs;
        int rc = (e1 == hipSuccess) ? launch_tuned(ps.N, t, a) : hip_fail(e1, "reset kernel");
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        it = g_graphs.emplace(key, ge).first;
    }
    hipError_t e = hipGraphLaunch(it->second, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return MTGP_OK;
}

static Staging g_stage;

int upload_items(Staging &st, const std::vector<BatchItem> &items, void *d_dst, hipStream_t s) {
    if (st.pending) {
        hipError_t e = hipEventSynchronize(st.done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(staging)");
        st.pending = false;
    }
    if (items.size() > st.cap) {
        if (st.host) (void)hipHostFree(st.host);
        size_t cap = std::max<size_t>(items.size(), 1024);
        hipError_t e = hipHostMalloc((void **)&st.host, cap * sizeof(BatchItem), hipHostMallocDefault);
        if (e != hipSuccess) {
            st.host = nullptr;
            st.cap = 0;
            return hip_fail(e, "hipHostMalloc(staging)");
        }
        st.cap = cap;
    }
    if (!st.done) {
        hipError_t e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    if (items.empty()) return MTGP_OK;
    std::memcpy(st.host, items.data(), items.size() * sizeof(BatchItem));
    hipError_t e = hipMemcpyAsync(d_dst, st.host, items.size() * sizeof(BatchItem),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(work list)");
    e = hipEventRecord(st.done, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    st.pending = true;
    return MTGP_OK;
}

size_t batch_ws_bytes(int n_items) { return 256 + (size_t)std::max(n_items, 0) * sizeof(BatchItem); }

int launch_planned(const ParamSet &ps, const void *d_params, uint32_t *d_states, int stride,
                   const std::vector<BatchItem> &planned, void *d_ws, hipStream_t s,
                   const mtgp_tuning &t, bool use_graph, Staging &stage) {
    if (planned.empty()) return MTGP_OK;
    uint32_t *counter = (uint32_t *)d_ws;
    BatchItem *d_items = (BatchItem *)((char *)d_ws + 256);
    int rc = upload_items(stage, planned, d_items, s);
    if (rc) return rc;
    return run_batch_device(ps, d_params, d_states, stride, d_items, (uint32_t)planned.size(),
                            counter, t, s, use_graph);
}

int generate_batch_impl(const void *d_params, uint32_t *d_states, int stride,
                        const mtgp_work *h_items, int n_items, void *d_ws, hipStream_t s,
                        const mtgp_tuning *force, bool use_graph, Staging &stage) {
    auto ps = lookup_params(d_params, 0);
    if (!ps) return MTGP_EINVAL;
    if (!d_states || stride < ps->N)
        return fail(MTGP_EINVAL, "state_stride %d < N=%d or NULL states", stride, ps->N);
    if (!d_ws || ((uintptr_t)d_ws & 255u))
        return fail(MTGP_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    int rc = validate_items(*ps, ps->n, h_items, n_items);
    if (rc) return rc;
    const mtgp_tuning t = force ? *force : tuning_for(ps->N);
    std::vector<BatchItem> planned;
    std::vector<int> order;
    plan_items_indexed(*ps, t, h_items, n_items, planned, order);
    std::lock_guard<std::mutex> lk(stage.mu);
    return launch_planned(*ps, d_params, d_states, stride, planned, d_ws, s, t, use_graph, stage);
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
    const int per_block = wpb_of(t);
    LaunchArgs a{};
    a.params = (const uint32_t *)d_params;
    a.states = d_states;
    a.stride = (uint32_t)stride;
    a.items = nullptr;
    a.n_items = (uint32_t)n_streams;
    a.counter = nullptr;
    a.plain_out = d_out;
    a.plain_count = count;
    a.plain_f32 = f32;
    a.grid = (n_streams + per_block - 1) / per_block;
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
    return e == hipSuccess ? MTGP_OK : hip_fail(e, "seed kernel");
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

size_t mtgp_batch_workspace_bytes(int n_items) { return batch_ws_bytes(n_items); }

int mtgp_generate_batch(const void *d_params, uint32_t *d_states, int state_stride,
                        const mtgp_work *h_items, int n_items, void *d_workspace, void *stream) {
    return generate_batch_impl(d_params, d_states, state_stride, h_items, n_items, d_workspace,
                               (hipStream_t)stream, nullptr, true, g_stage);
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
    }
    return c;
}

int mtgp_autotune(const void *d_params, const uint32_t *d_states, int state_stride,
                  const mtgp_work *h_items, int n_items, void *d_scratch, int reps, void *stream,
                  mtgp_tuning *best, float *h_ms, int max_out) {
    auto ps = lookup_params(d_params, 0);
    if (!ps) return MTGP_EINVAL;
    if (!d_scratch || ((uintptr_t)d_scratch & 255u))
        return fail(MTGP_EINVAL, "scratch must be non-NULL and 256-byte aligned");
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    const size_t state_bytes = (size_t)ps->n * (size_t)state_stride * 4;
    const size_t state_bytes_al = (state_bytes + 255) / 256 * 256;
    uint32_t *scratch_states = (uint32_t *)d_scratch;
    void *ws = (char *)d_scratch + state_bytes_al;
    hipError_t e = hipMemcpyAsync(scratch_states, d_states, state_bytes,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(scratch states)");
    mtgp_tuning cands[64];
    const int nc = std::min(64, mtgp_tuning_candidates(ps->mexp, cands, 64));
    hipEvent_t ev0, ev1;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&ev1)) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        return hip_fail(e, "hipEventCreate");
    }
    float best_ms = 1e30f;
    int best_i = -1, rc = MTGP_OK;
    Staging stage;
    for (int i = 0; i < nc && rc == MTGP_OK; ++i) {
        rc = generate_batch_impl(d_params, scratch_states, state_stride, h_items, n_items, ws, s,
                                 &cands[i], false, stage);  // warm-up
        if (rc) break;
        float total = 0.f;
        for (int r = 0; r < reps && rc == MTGP_OK; ++r) {
            (void)hipEventRecord(ev0, s);
            rc = generate_batch_impl(d_params, scratch_states, state_stride, h_items, n_items, ws,
                                     s, &cands[i], false, stage);
            (void)hipEventRecord(ev1, s);
            if ((e = hipEventSynchronize(ev1)) != hipSuccess) {
                rc = hip_fail(e, "hipEventSynchronize(autotune)");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev0, ev1);
            total += ms;
        }
        if (rc) break;
        const float avg = total / (float)reps;
        if (h_ms && i < max_out) h_ms[i] = avg;
        if (avg < best_ms) {
            best_ms = avg;
            best_i = i;
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (stage.host) (void)hipHostFree(stage.host);
    if (stage.done) (void)hipEventDestroy(stage.done);
    if (rc) return rc;
    if (best_i < 0) return fail(MTGP_EINVAL, "no candidate kernels for mexp %u", ps->mexp);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[ps->N] = cands[best_i];
    }
    if (best) *best = cands[best_i];
    return MTGP_OK;
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
    return e == hipSuccess ? MTGP_OK : hip_fail(e, "hipStreamSynchronize(import)");
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
