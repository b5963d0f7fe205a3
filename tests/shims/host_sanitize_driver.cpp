// host_sanitize_driver.cpp -- runs the library's host code on a GPU in a
// build whose host objects carry AddressSanitizer and UndefinedBehavior-
// Sanitizer (device code is built as usual): argument validation, parameter
// packing, plain launches, batch planning with jump-ahead splits (polynomial
// set-up, workspace sizing, per-call table uploads), the repair bookkeeping,
// checkpoint copies, the allocation-free batch entry, the serving runtime
// (submit / wait / poll / release / replay / destroy) and the remaining
// entry points.  The library's paths are compared with one another bit for
// bit (plain one-launch generation is the reference), so a host-side bug
// that corrupts a plan shows up as a mismatch even where no sanitizer fires.
//
// Exit status 0 and a last line "host sanitize driver: ok" on success.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "mtgp.h"

#define CK(x)                                                                             \
    do {                                                                                  \
        const int rc_ = (x);                                                              \
        if (rc_ != MTGP_OK) {                                                             \
            std::fprintf(stderr, "line %d: %s -> %s (%s)\n", __LINE__, #x,                \
                         mtgp_strerror(rc_), mtgp_last_error_detail());                   \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)
#define EXPECT_RC(x, want)                                                                \
    do {                                                                                  \
        const int rc_ = (x);                                                              \
        if (rc_ != (want)) {                                                              \
            std::fprintf(stderr, "line %d: %s -> %d, expected %d\n", __LINE__, #x, rc_,    \
                         (int)(want));                                                    \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)
#define HK(x)                                                                             \
    do {                                                                                  \
        const hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                           \
            std::fprintf(stderr, "line %d: %s -> %s\n", __LINE__, #x, hipGetErrorString(e_)); \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

static const uint32_t MEXP = 11213;
static const int NS = 32;                  // streams
static const uint64_t C = 1ull << 21;      // outputs per stream in the reference
static int N = 0;                          // state words

static void step(const char *what) {
    std::printf("step: %s\n", what);
    std::fflush(stdout);
}

// Random parameter sets of MTGP's shape: tables are GF(2) spans of four
// random words, the float table derived from the tempering table.
static std::vector<mtgp_params> make_params(uint64_t seed) {
    std::mt19937_64 rng(seed);
    std::vector<mtgp_params> p((size_t)NS);
    const uint32_t mask = 0xFFFFFFFFu << (32 * N - (int)MEXP);
    for (auto &q : p) {
        q.mexp = MEXP;
        q.pos = 1 + (uint32_t)(rng() % (uint64_t)(N - 2));
        q.sh1 = (uint32_t)(rng() % 32);
        q.sh2 = (uint32_t)(rng() % 32);
        q.mask = mask;
        uint32_t rb[4], tb[4];
        for (int b = 0; b < 4; ++b) {
            rb[b] = (uint32_t)rng();
            tb[b] = (uint32_t)rng();
        }
        for (int i = 0; i < 16; ++i) {
            uint32_t r = 0, t = 0;
            for (int b = 0; b < 4; ++b)
                if ((i >> b) & 1) {
                    r ^= rb[b];
                    t ^= tb[b];
                }
            q.rec_tbl[i] = r;
            q.tmp_tbl[i] = t;
            q.flt_tbl[i] = 0x3F800000u | (t >> 9);
        }
    }
    return p;
}

static std::vector<uint32_t> d2h(const void *d, size_t words) {
    std::vector<uint32_t> h(words);
    HK(hipMemcpy(h.data(), d, words * 4, hipMemcpyDeviceToHost));
    return h;
}

static void same(const uint32_t *got, const uint32_t *want, size_t words, const char *what) {
    if (std::memcmp(got, want, words * 4) == 0) return;
    for (size_t i = 0; i < words; ++i)
        if (got[i] != want[i]) {
            std::fprintf(stderr, "%s: word %zu is %08x, expected %08x\n", what, i, got[i],
                         want[i]);
            break;
        }
    std::exit(1);
}

int main() {
    N = mtgp_state_words(MEXP);
    if (N <= 0) return 1;
    hipStream_t s;
    HK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    auto params = make_params(1501);
    std::vector<uint32_t> seeds((size_t)NS);
    for (int k = 0; k < NS; ++k) seeds[(size_t)k] = (uint32_t)(k + 1);

    step("parameter validation");
    {
        auto bad = params;
        bad[3].pos = (uint32_t)N - 1;
        EXPECT_RC(mtgp_check_params(bad.data(), NS), MTGP_EINVAL);
        bad = params;
        bad[5].mask ^= 1u << 31;
        EXPECT_RC(mtgp_check_params(bad.data(), NS), MTGP_EINVAL);
        bad = params;
        bad[7].flt_tbl[2] = 0;
        EXPECT_RC(mtgp_check_params(bad.data(), NS), MTGP_EINVAL);
        CK(mtgp_check_params(params.data(), NS));
    }

    void *d_params;
    uint32_t *d_states;
    uint32_t *d_ref, *d_out;
    const int stride = N + 7;  // rows with a gap
    HK(hipMalloc(&d_params, (size_t)NS * MTGP_DEVICE_PARAM_BYTES));
    HK(hipMalloc((void **)&d_states, (size_t)NS * stride * 4));
    HK(hipMalloc((void **)&d_ref, (size_t)NS * C * 4));
    HK(hipMalloc((void **)&d_out, (size_t)NS * C * 4));

    step("plain reference: u32 then f32");
    CK(mtgp_init_states(params.data(), seeds.data(), NS, d_params, d_states, stride, s));
    std::vector<uint32_t> st0((size_t)NS * N);
    CK(mtgp_state_export(d_params, d_states, stride, NS, st0.data(), s));
    CK(mtgp_generate_u32(d_params, d_states, stride, NS, C, d_ref, s));
    HK(hipStreamSynchronize(s));
    const auto ref = d2h(d_ref, (size_t)NS * C);
    CK(mtgp_generate_f32(d_params, d_states, stride, NS, C / 2, (float *)d_ref, s));
    HK(hipStreamSynchronize(s));
    const auto ref_f = d2h(d_ref, (size_t)NS * C / 2);
    std::vector<uint32_t> st_end((size_t)NS * N);
    CK(mtgp_state_export(d_params, d_states, stride, NS, st_end.data(), s));

    step("batched, split by jump-ahead: u32 then f32");
    CK(mtgp_seed_states(d_params, d_states, stride, NS, s));
    std::vector<mtgp_work> items((size_t)NS);
    for (int k = 0; k < NS; ++k)
        items[(size_t)k] = mtgp_work{k, MTGP_U32, C, d_out + (size_t)k * C};
    size_t ws_bytes = 0;
    CK(mtgp_batch_workspace_query(d_params, items.data(), NS, &ws_bytes));
    if (ws_bytes <= mtgp_batch_workspace_bytes(NS)) {
        std::fprintf(stderr, "no split planned (%zu workspace bytes)\n", ws_bytes);
        return 1;
    }
    void *d_ws;
    HK(hipMalloc(&d_ws, ws_bytes));
    CK(mtgp_generate_batch(d_params, d_states, stride, items.data(), NS, d_ws, ws_bytes, s));
    HK(hipStreamSynchronize(s));
    same(d2h(d_out, (size_t)NS * C).data(), ref.data(), (size_t)NS * C, "batch u32");
    for (int k = 0; k < NS; ++k)
        items[(size_t)k] = mtgp_work{k, MTGP_F32, C / 2, d_out + (size_t)k * C / 2};
    CK(mtgp_generate_batch(d_params, d_states, stride, items.data(), NS, d_ws, ws_bytes, s));
    HK(hipStreamSynchronize(s));
    same(d2h(d_out, (size_t)NS * C / 2).data(), ref_f.data(), (size_t)NS * C / 2, "batch f32");
    {
        std::vector<uint32_t> st((size_t)NS * N);
        CK(mtgp_state_export(d_params, d_states, stride, NS, st.data(), s));
        same(st.data(), st_end.data(), st.size(), "states after the batches");
    }
    uint32_t repairs = 99;
    CK(mtgp_batch_errors(d_ws, s, &repairs));
    if (repairs != 0) return std::fprintf(stderr, "%u repairs\n", repairs), 1;

    step("uneven batch with mixed lengths, twice on one workspace");
    for (int rep = 0; rep < 2; ++rep) {
        CK(mtgp_seed_states(d_params, d_states, stride, NS, s));
        uint64_t off = 0;
        for (int k = 0; k < NS; ++k) {
            const uint64_t c = (uint64_t)(k % 7 + 1) * (C / 8) + (uint64_t)k * 33 + 1;
            items[(size_t)k] = mtgp_work{(k * 13) % NS, MTGP_U32, std::min(c, C), d_out + off};
            off += std::min(c, C);
        }
        CK(mtgp_generate_batch(d_params, d_states, stride, items.data(), NS, d_ws, ws_bytes, s));
        HK(hipStreamSynchronize(s));
        const auto out = d2h(d_out, off);
        uint64_t o = 0;
        for (int k = 0; k < NS; ++k) {
            const auto &it = items[(size_t)k];
            same(out.data() + o, ref.data() + (size_t)it.stream_id * C, it.count, "uneven batch");
            o += it.count;
        }
    }

    step("imported states: batch vs plain generation from them");
    {
        std::vector<uint32_t> mid((size_t)NS * N);
        CK(mtgp_state_export(d_params, d_states, stride, NS, mid.data(), s));
        CK(mtgp_seed_states(d_params, d_states, stride, NS, s));
        CK(mtgp_state_import(d_params, d_states, stride, NS, mid.data(), s));
        CK(mtgp_generate_u32(d_params, d_states, stride, NS, C / 2, d_ref, s));
        HK(hipStreamSynchronize(s));
        const auto plain = d2h(d_ref, (size_t)NS * C / 2);
        CK(mtgp_state_import(d_params, d_states, stride, NS, mid.data(), s));
        for (int k = 0; k < NS; ++k)
            items[(size_t)k] = mtgp_work{k, MTGP_U32, C / 2, d_out + (size_t)k * C / 2};
        size_t need = 0;
        CK(mtgp_batch_workspace_query(d_params, items.data(), NS, &need));
        void *d_ws2;
        HK(hipMalloc(&d_ws2, need));
        CK(mtgp_generate_batch(d_params, d_states, stride, items.data(), NS, d_ws2, need, s));
        HK(hipStreamSynchronize(s));
        same(d2h(d_out, (size_t)NS * C / 2).data(), plain.data(), (size_t)NS * C / 2,
             "batch from imported states");
        CK(mtgp_batch_errors(d_ws2, s, &repairs));
        HK(hipFree(d_ws2));
    }

    step("allocation-free batch entry");
    {
        CK(mtgp_seed_states(d_params, d_states, stride, NS, s));
        std::vector<mtgp_work> few(4);
        for (int k = 0; k < 4; ++k)
            few[(size_t)k] = mtgp_work{k + 3, MTGP_U32, 100000, d_out + (size_t)k * 100000};
        CK(mtgp_generate_batch_noalloc(d_params, d_states, stride, few.data(), 4, s));
        HK(hipStreamSynchronize(s));
        const auto out = d2h(d_out, 400000);
        for (int k = 0; k < 4; ++k)
            same(out.data() + (size_t)k * 100000, ref.data() + (size_t)(k + 3) * C, 100000,
                 "no-alloc batch");
    }

    step("argument errors");
    {
        std::vector<mtgp_work> dup = {mtgp_work{1, MTGP_U32, 10, d_out},
                                      mtgp_work{1, MTGP_U32, 10, d_out + 16}};
        EXPECT_RC(mtgp_generate_batch(d_params, d_states, stride, dup.data(), 2, d_ws, ws_bytes, s),
                  MTGP_EINVAL);
        // below the unsplit minimum: rejected before anything runs
        EXPECT_RC(mtgp_generate_batch(d_params, d_states, stride, items.data(), NS, d_ws, 64, s),
                  MTGP_EINVAL);
        EXPECT_RC(mtgp_generate_u32(d_params, d_states, N - 1, NS, 16, d_out, s), MTGP_EINVAL);
        EXPECT_RC(mtgp_state_words(12345), MTGP_EINVAL);
    }

    step("serving: submit / wait / poll / release, then replay with kept results");
    {
        CK(mtgp_seed_states(d_params, d_states, stride, NS, s));
        HK(hipStreamSynchronize(s));
        void *d_pool;
        const uint64_t pool_bytes = 512ull << 20;
        HK(hipMalloc(&d_pool, pool_bytes));
        mtgp_server_opts o{3, 16, 4096, 20000, 48ull << 20};
        mtgp_server *srv = nullptr;
        CK(mtgp_server_create(d_params, d_states, stride, NS, d_pool, pool_bytes, &o, &srv));
        uint64_t tk_big;
        EXPECT_RC(mtgp_submit(srv, 0, pool_bytes, MTGP_U32, &tk_big), MTGP_ETOOBIG);
        // every stream: C/4, C/4 (submitted together), then C/2
        std::vector<uint64_t> tk((size_t)NS * 3);
        std::vector<int32_t> ids((size_t)NS * 2);
        std::vector<uint64_t> cnt((size_t)NS * 2, C / 4);
        std::vector<int> dts((size_t)NS * 2, MTGP_U32);
        for (int k = 0; k < NS; ++k) ids[2 * (size_t)k] = ids[2 * (size_t)k + 1] = k;
        CK(mtgp_submit_many(srv, ids.data(), cnt.data(), dts.data(), 2 * NS, tk.data()));
        for (int k = 0; k < NS; ++k) CK(mtgp_submit(srv, k, C / 2, MTGP_U32, &tk[2 * NS + (size_t)k]));
        std::vector<uint32_t> h(C);
        for (int k = 0; k < NS; ++k) {
            const uint64_t parts[3] = {tk[2 * (size_t)k], tk[2 * (size_t)k + 1],
                                       tk[2 * NS + (size_t)k]};
            const uint64_t lens[3] = {C / 4, C / 4, C / 2};
            uint64_t at = 0;
            for (int j = 0; j < 3; ++j) {
                CK(mtgp_wait(srv, parts[j], 0));
                int state = -1;
                const void *res = nullptr;
                CK(mtgp_poll(srv, parts[j], &state, &res));
                if (state != MTGP_DONE || !res) return std::fprintf(stderr, "not done\n"), 1;
                HK(hipMemcpy(h.data(), res, lens[j] * 4, hipMemcpyDeviceToHost));
                same(h.data(), ref.data() + (size_t)k * C + at, lens[j], "served result");
                uint64_t ts, ta, tl, td;
                CK(mtgp_request_times(srv, parts[j], &ts, &ta, &tl, &td));
                CK(mtgp_release(srv, parts[j]));
                at += lens[j];
            }
        }
        EXPECT_RC(mtgp_release(srv, tk[0]), MTGP_ENOENT);
        // replay from the seed status again: two requests per stream, kept
        CK(mtgp_seed_states(d_params, d_states, stride, NS, s));
        HK(hipStreamSynchronize(s));
        const int n = 2 * NS;
        std::vector<uint64_t> arr((size_t)n), lat((size_t)n), stages(3 * (size_t)n);
        std::vector<int32_t> rs((size_t)n);
        std::vector<uint64_t> rcount((size_t)n);
        std::vector<int> rd((size_t)n, MTGP_U32);
        std::vector<void *> keep((size_t)n);
        for (int i = 0; i < n; ++i) {
            arr[(size_t)i] = (uint64_t)i * 20000;
            rs[(size_t)i] = i % NS;
            rcount[(size_t)i] = C / 2;
            keep[(size_t)i] = d_out + (size_t)(i % NS) * C + (size_t)(i / NS) * (C / 2);
        }
        CK(mtgp_server_replay(srv, arr.data(), rs.data(), rcount.data(), rd.data(), n, lat.data(),
                              stages.data(), keep.data()));
        same(d2h(d_out, (size_t)NS * C).data(), ref.data(), (size_t)NS * C, "replayed results");
        uint64_t fixed = 99;
        CK(mtgp_server_repaired(srv, &fixed));
        if (fixed != 0) return std::fprintf(stderr, "%llu repaired\n", (unsigned long long)fixed), 1;
        // destroy with requests still queued
        for (int k = 0; k < NS; ++k) CK(mtgp_submit(srv, k, C / 8, MTGP_U32, &tk[(size_t)k]));
        CK(mtgp_server_destroy(srv));
        HK(hipFree(d_pool));
    }

    step("tuning, polynomials, draw API, screening");
    {
        mtgp_tuning t, cands[64];
        CK(mtgp_get_tuning(MEXP, &t));
        const int nc = mtgp_tuning_candidates(MEXP, cands, 64);
        if (nc <= 0) return 1;
        CK(mtgp_set_tuning(MEXP, &cands[nc - 1]));
        CK(mtgp_set_tuning(MEXP, &t));
        std::vector<uint32_t> coeffs((size_t)4 * (MEXP / 32 + 1));
        std::vector<int> degs(4);
        CK(mtgp_stream_polynomials(d_params, 4, coeffs.data(), (int)MEXP / 32 + 1, degs.data(), s));
        CK(mtgp_seed_states(d_params, d_states, stride, NS, s));
        CK(mtgp_generate_workgroup(d_params, d_states, stride, NS, 4096, MTGP_U32, 256, d_out, s));
        HK(hipStreamSynchronize(s));
        const auto wg = d2h(d_out, (size_t)NS * 4096);
        for (int k = 0; k < NS; ++k)
            same(wg.data() + (size_t)k * 4096, ref.data() + (size_t)k * C, 4096, "draw API");
        uint64_t *d_counts;
        HK(hipMalloc((void **)&d_counts, (size_t)NS * (16 + 9) * 8));
        CK(mtgp_screen(d_ref, NS, C / 2, 0, 1u << 28, 16, d_counts, s));
        HK(hipStreamSynchronize(s));
        HK(hipFree(d_counts));
    }

    CK(mtgp_release_params(d_params));
    HK(hipFree(d_ws));
    HK(hipFree(d_out));
    HK(hipFree(d_ref));
    HK(hipFree((void *)d_states));
    HK(hipFree(d_params));
    HK(hipStreamDestroy(s));
    std::printf("host sanitize driver: ok\n");
    return 0;
}
