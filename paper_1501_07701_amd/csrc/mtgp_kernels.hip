// mtgp_kernels.hip -- gfx950 kernels for bulk MTGP32 generation.
//
// One stream per thread group (the paper's per-block generator scope, Sec. 2
// and Sec. 3.2): a group is either one 64-lane wave (several independent
// streams per workgroup, no s_barrier) or a whole workgroup.  The stream's
// N-word state lives in an LDS buffer while it runs (shared memory, Sec. 2)
// and in device memory between launches.
//
// Step structure.  With W = N - pos, the new words x_n .. x_{n+W-1} depend
// only on words older than x_n, so one step produces up to W outputs at once:
// every lane loads its taps for up to K outputs, computes, writes the new
// words to LDS and the tempered outputs to HBM, then the group synchronises
// once.  Steps are rounded down to multiples of 32 words when W >= 64 so that
// the stores of a step cover whole 128-byte lines.  The LDS buffer is linear
// (x_n at a fixed offset from the step's head) so that every tap is an
// immediate offset from one or two per-lane base registers; when the head
// reaches the end of the buffer the last N words are copied to the front.
//
// Jump-ahead.  A work item may start from any state: a long stream is cut
// into segments whose start states jump_kernel computes from the stream's
// first words (the generator is GF(2)-linear, so the state J outputs ahead
// is a fixed XOR-combination of consecutive words, given by x^(J-1) mod p
// for a polynomial p that annihilates the word sequence).  Each segment
// checks that its final state equals the next segment's jumped start state.
//
// Work is bit-level GF(2) arithmetic: no MFMA.  The bound is HBM write
// bandwidth (4 bytes per output), with VALU and LDS close behind.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mtgp_internal.hpp"

namespace mtgp {

// Pointer into global memory (address space 1), so stores are emitted as
// global_store rather than flat_store.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <int TPS>
__device__ __forceinline__ void group_sync() {
    if constexpr (TPS == 64) {
        // One wave: LDS operations issue in order, so only the compiler
        // must be kept from moving loads across the step boundary.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// LDS buffer length (words) for a stream of N words and up to SMAX outputs
// per step: at least 2N + SMAX so the compaction copy never overlaps itself.
__host__ __device__ constexpr int buf_words(int N, int SMAX) {
    return ((2 * N + 4 * SMAX) + 63) / 64 * 64;
}

template <int N, int TPS, int K>
struct Core {
    static constexpr int SMAX = TPS * K;
    static constexpr int BUF = buf_words(N, SMAX);
    static_assert(BUF >= 2 * N + SMAX, "compaction would overlap");
    static constexpr int LDS_WORDS = BUF + 32;  // + recursion and output tables

    // Advance one stream by item.count outputs.
    template <bool F32>
    static __device__ __forceinline__ void run(const uint32_t *__restrict__ prm,
                                               const BatchItem &item,
                                               uint32_t *__restrict__ buf, uint32_t lane,
                                               uint32_t *__restrict__ err) {
        uint32_t *__restrict__ tbl = buf + BUF;
        const uint32_t pos = prm[P_POS];
        const uint32_t sh1 = prm[P_SH1];
        const uint32_t sh2 = prm[P_SH2];
        const uint32_t mask = prm[P_MASK];
        const uint32_t W = N - pos;
        const uint64_t count = item.count;
        const uint32_t *st_in = reinterpret_cast<const uint32_t *>(item.state_in);
        uint32_t *st_out = reinterpret_cast<uint32_t *>(item.state_out);
        gptr<uint32_t> raw = (gptr<uint32_t>)(reinterpret_cast<uint32_t *>(item.raw));
        const bool want_raw = (item.mode & MODE_RAW) != 0;

        group_sync<TPS>();  // previous user of this buffer is done with it
        for (uint32_t i = lane; i < N; i += TPS) {
            const uint32_t v = st_in[i];
            buf[i] = v;
            if (want_raw) raw[i] = v;
        }
        if (lane < 16) {
            tbl[lane] = prm[P_REC + lane];
            tbl[16 + lane] = prm[(F32 ? P_FLT : P_TMP) + lane];
        }
        group_sync<TPS>();

        // Full steps: W rounded down to whole 128-byte lines when wide.
        uint32_t smax = W >= 64 ? (W & ~31u) : W;
        if (smax > (uint32_t)SMAX) smax = SMAX;
        uint32_t h = N;  // buffer index of the next new word
        uint64_t done = 0;
        gptr<uint32_t> gout = (gptr<uint32_t>)(reinterpret_cast<uint32_t *>(item.out));
        while (done < count) {
            const uint64_t rem = count - done;
            const uint32_t S = rem < smax ? (uint32_t)rem : smax;
            const uint32_t keff = (S + TPS - 1) / TPS;
            // Lanes compute every word of their k < keff, so keep h + SMAX
            // inside the buffer: loads and LDS writes of lanes beyond S then
            // stay in bounds (their words are rewritten by the next step
            // before anything reads them).
            if (h + SMAX > (uint32_t)BUF) {
                for (uint32_t i = lane; i < N; i += TPS) buf[i] = buf[h - N + i];
                group_sync<TPS>();
                h = N;
            }
            // q[0] = x_{n-N}, q[1] = x_{n-N+1}, q[pos-1] = helper, q[pos] = tap
            const uint32_t *q = buf + (h + lane - N);
            const uint32_t *qp = q + (pos - 1);
            uint32_t a[K], b[K], hh[K], c[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < (int)keff) {
                    a[k] = q[k * TPS];
                    b[k] = q[k * TPS + 1];
                    hh[k] = qp[k * TPS];
                    c[k] = qp[k * TPS + 1];
                }
            }
            uint32_t x[K], r[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < (int)keff) {
                    uint32_t X = (a[k] & mask) ^ b[k];
                    X ^= X << sh1;
                    const uint32_t Y = X ^ (c[k] >> sh2);
                    x[k] = Y ^ tbl[Y & 15u];
                    uint32_t H = hh[k] ^ (hh[k] >> 16);
                    H ^= H >> 8;
                    const uint32_t tv = tbl[16 + (H & 15u)];
                    if constexpr (F32)
                        r[k] = __float_as_uint(__uint_as_float((x[k] >> 9) ^ tv) - 1.0f);
                    else
                        r[k] = x[k] ^ tv;
                }
            }
            uint32_t *w = buf + (h + lane);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k < (int)keff) w[k * TPS] = x[k];
            gptr<uint32_t> o = gout + done + lane;
            if (S == keff * TPS) {
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k < (int)keff) __builtin_nontemporal_store(r[k], o + k * TPS);
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k < (int)keff && lane + k * TPS < S)
                        __builtin_nontemporal_store(r[k], o + k * TPS);
            }
            if (want_raw) {
                gptr<uint32_t> rw = raw + N + done + lane;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k < (int)keff && lane + k * TPS < S) rw[k * TPS] = x[k];
            }
            group_sync<TPS>();
            h += S;
            done += S;
        }
        if (st_out != nullptr)
            for (uint32_t i = lane; i < N; i += TPS) st_out[i] = buf[h - N + i];
        if (item.mode & MODE_VERIFY) {
            // the end state must equal the next segment's jumped start state
            const uint32_t *ref = reinterpret_cast<const uint32_t *>(item.verify);
            uint32_t bad = 0;
            for (uint32_t i = lane; i < N; i += TPS) bad |= (buf[h - N + i] != ref[i]) ? 1u : 0u;
            if (bad) atomicAdd(err, 1u);
        }
    }
};

// Generation kernel.  Each group (a wave when TPS == 64, else the workgroup)
// takes work items until none are left.
//  persistent != 0 : items are claimed in order through *counter.
//  persistent == 0 : group g takes items g, g + n_groups, ...
// Plain mode (items == nullptr): item i is stream i, advanced in place in
// its state row by plain_count outputs written at plain_out + i*plain_count.
struct PlainArgs {
    uint32_t *states;
    uint32_t stride;
    uint32_t mode;
    uint32_t *out;
    uint64_t count;
};

template <int N, int TPS, int K, int WPB>
__global__ void __launch_bounds__(TPS == 64 ? 64 * WPB : TPS)
gen_kernel(const uint32_t *__restrict__ params, const BatchItem *__restrict__ items,
           uint32_t n_items, uint32_t *__restrict__ counter, uint32_t *__restrict__ err,
           uint32_t persistent, PlainArgs plain) {
    using C = Core<N, TPS, K>;
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t s_claim;
    const uint32_t wave =
        (TPS == 64) ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0u;
    const uint32_t lane = (TPS == 64) ? (threadIdx.x & 63u) : threadIdx.x;
    uint32_t *buf = lds + wave * C::LDS_WORDS;
    const uint32_t n_groups = gridDim.x * (TPS == 64 ? WPB : 1);
    uint32_t it = blockIdx.x * (TPS == 64 ? WPB : 1) + wave;

    while (true) {
        if (persistent) {
            if constexpr (TPS == 64) {
                uint32_t v = 0;
                if (lane == 0) v = atomicAdd(counter, 1u);
                it = __builtin_amdgcn_readfirstlane(v);
            } else {
                __syncthreads();
                if (threadIdx.x == 0) s_claim = atomicAdd(counter, 1u);
                __syncthreads();
                it = s_claim;
            }
        }
        if (it >= n_items) break;
        BatchItem item;
        if (items != nullptr) {
            item = items[it];
        } else {
            uint32_t *row = plain.states + (uint64_t)it * plain.stride;
            item.stream = it;
            item.mode = plain.mode;
            item.count = plain.count;
            item.out = (uint64_t)(uintptr_t)(plain.out + (uint64_t)it * plain.count);
            item.state_in = item.state_out = (uint64_t)(uintptr_t)row;
            item.raw = item.verify = item.flag = item.countdown = 0;
        }
        const uint32_t *prm = params + (uint64_t)item.stream * P_WORDS;
        if (item.count > 0) {
            if (item.mode & MODE_F32)
                C::template run<true>(prm, item, buf, lane, err);
            else
                C::template run<false>(prm, item, buf, lane, err);
        }
        if (item.flag != 0) {
            // Publish completion of the request to the host once its last
            // segment is done: every lane's output and state stores are made
            // visible system-wide first.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            group_sync<TPS>();
            if (lane == 0) {
                bool last = true;
                if (item.countdown != 0)
                    last = __hip_atomic_fetch_add(reinterpret_cast<uint32_t *>(item.countdown),
                                                  0xFFFFFFFFu, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT) == 1u;
                if (last)
                    __hip_atomic_store(reinterpret_cast<uint32_t *>(item.flag), 1u,
                                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        if (!persistent) it += n_groups;
    }
}

// Jump evaluation: out[m] = XOR over the set bits i < D of g of raw[1+i+m],
// for m < M.  One 256-thread workgroup per item; the words are staged
// through LDS in chunks of JUMP_CH coefficients plus the output tail, and
// lane t owns output words m = t + 256 j of the current pass.
constexpr int JUMP_THREADS = 256;
constexpr int JUMP_CH = 4096;   // coefficients per LDS chunk
constexpr int JUMP_MT = 1024;   // output words per pass (4 per lane)

__global__ void __launch_bounds__(JUMP_THREADS)
jump_kernel(const JumpItem *__restrict__ items, uint32_t n_items) {
    __shared__ uint32_t base[JUMP_CH + JUMP_MT];
    const uint32_t t = threadIdx.x;
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const JumpItem jit = items[it];
        const uint32_t *raw = reinterpret_cast<const uint32_t *>(jit.raw) + 1;
        const uint32_t *g = reinterpret_cast<const uint32_t *>(jit.poly);
        uint32_t *out = reinterpret_cast<uint32_t *>(jit.out);
        const uint32_t D = jit.nbits, M = jit.m;
        for (uint32_t m0 = 0; m0 < M; m0 += JUMP_MT) {
            const uint32_t mt = (M - m0) < (uint32_t)JUMP_MT ? (M - m0) : (uint32_t)JUMP_MT;
            uint32_t acc[JUMP_MT / JUMP_THREADS] = {};
            for (uint32_t i0 = 0; i0 < D; i0 += JUMP_CH) {
                const uint32_t ch = (D - i0) < (uint32_t)JUMP_CH ? (D - i0) : (uint32_t)JUMP_CH;
                __syncthreads();
                for (uint32_t j = t; j < ch + mt; j += JUMP_THREADS) base[j] = raw[i0 + m0 + j];
                __syncthreads();
                const uint32_t nw = (ch + 31) / 32;
                for (uint32_t w = 0; w < nw; ++w) {
                    uint32_t bits = g[(i0 >> 5) + w];
                    if (w == nw - 1 && (ch & 31)) bits &= (1u << (ch & 31)) - 1u;
                    while (bits) {
                        const uint32_t i = 32 * w + (uint32_t)__builtin_ctz(bits);
                        bits &= bits - 1u;
#pragma unroll
                        for (int j = 0; j < JUMP_MT / JUMP_THREADS; ++j)
                            acc[j] ^= base[i + t + j * JUMP_THREADS];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < JUMP_MT / JUMP_THREADS; ++j) {
                const uint32_t m = t + j * JUMP_THREADS;
                if (m < mt) out[m0 + m] = acc[j];
            }
        }
    }
}

// Seeding: one lane per stream runs the N-step initialisation recurrence.
__global__ void seed_kernel(const uint32_t *__restrict__ params,
                            uint32_t *__restrict__ states, uint32_t stride,
                            uint32_t n_streams) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_streams) return;
    const uint32_t *p = params + (uint64_t)k * P_WORDS;
    const uint32_t n = p[P_N];
    uint32_t x = p[P_SEED];
    uint32_t *s = states + (uint64_t)k * stride;
    s[0] = x;
    for (uint32_t i = 1; i < n; ++i) {
        x = 1812433253u * (x ^ (x >> 30)) + i;
        s[i] = x;
    }
}

__global__ void reset_counter_kernel(uint32_t *counter) { *counter = 0u; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Store-only fill: the achievable write bandwidth next to the generator.
__global__ void __launch_bounds__(256)
fill_kernel(u32x4 *__restrict__ out, uint64_t n_vec, uint32_t *__restrict__ tail,
            uint32_t n_tail, uint32_t value) {
    const u32x4 v = {value, value, value, value};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vec; i += stride)
        __builtin_nontemporal_store(v, out + i);
    if (blockIdx.x == 0 && threadIdx.x < n_tail) tail[threadIdx.x] = value;
}

// ------------------------------------------------------------- dispatch --

template <int N, int TPS, int K, int WPB>
static hipError_t launch_gen(const LaunchArgs &a) {
    using C = Core<N, TPS, K>;
    auto fn = gen_kernel<N, TPS, K, WPB>;
    const int threads = TPS == 64 ? 64 * WPB : TPS;
    const size_t lds = (size_t)C::LDS_WORDS * 4 * (TPS == 64 ? WPB : 1);
    static bool attr_set = false;  // benign race: idempotent attribute
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)fn,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int per_block = TPS == 64 ? WPB : 1;
    const int need = (int)((a.n_items + per_block - 1) / per_block);
    int grid = need > 0 ? need : 1;
    if (a.persistent) {  // fill every CU to its occupancy, no more groups than items
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        if (per_cu * a.num_cus < grid) grid = per_cu * a.num_cus;
    }
    PlainArgs plain{a.plain_states, a.plain_stride, a.plain_mode, a.plain_out, a.plain_count};
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds, (hipStream_t)a.stream, a.params,
                       a.items, a.n_items, a.counter, a.err, a.persistent ? 1u : 0u, plain);
    return hipGetLastError();
}

template <int N, int TPS, int K, int WPB>
static size_t lds_bytes_of() {
    return (size_t)Core<N, TPS, K>::LDS_WORDS * 4 * (TPS == 64 ? WPB : 1);
}

struct Variant {
    int N, tps, k, wpb;
    hipError_t (*launch)(const LaunchArgs &);
    size_t (*lds)();
};

#define MTGP_V(N, T, K, P) {N, T, K, P, &launch_gen<N, T, K, P>, &lds_bytes_of<N, T, K, P>}
#define MTGP_VARIANTS(N)                                                              \
    MTGP_V(N, 64, 1, 4), MTGP_V(N, 64, 2, 4), MTGP_V(N, 64, 4, 4), MTGP_V(N, 64, 8, 4), \
    MTGP_V(N, 64, 2, 8), MTGP_V(N, 64, 4, 8), MTGP_V(N, 64, 4, 16),                   \
    MTGP_V(N, 256, 1, 1), MTGP_V(N, 256, 2, 1), MTGP_V(N, 512, 1, 1),                 \
    MTGP_V(N, 512, 2, 1), MTGP_V(N, 1024, 1, 1)

static const Variant kVariants[] = {
    MTGP_VARIANTS(101), MTGP_VARIANTS(351), MTGP_VARIANTS(726), MTGP_VARIANTS(1391),
};

// LDS per workgroup on gfx950.
static constexpr size_t kLdsBytes = 160 * 1024;

int variant_count(int n_words, VariantInfo *out, int max_out) {
    int c = 0;
    for (const Variant &v : kVariants) {
        if (v.N != n_words || v.lds() + 64 > kLdsBytes) continue;
        if (out && c < max_out) {
            out[c].tps = v.tps;
            out[c].k = v.k;
            out[c].wpb = v.wpb;
            out[c].lds_bytes = v.lds();
        }
        ++c;
    }
    return c;
}

hipError_t launch_variant(int n_words, int tps, int k, int wpb, const LaunchArgs &a,
                          bool *found) {
    for (const Variant &v : kVariants) {
        if (v.N == n_words && v.tps == tps && v.k == k && v.wpb == wpb &&
            v.lds() + 64 <= kLdsBytes) {
            *found = true;
            return v.launch(a);
        }
    }
    *found = false;
    return hipSuccess;
}

hipError_t launch_jump(const JumpItem *items, uint32_t n_items, int num_cus, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    int grid = (int)n_items;
    const int cap = num_cus * 8;
    if (grid > cap) grid = cap;
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(jump_kernel, dim3(grid), dim3(JUMP_THREADS), 0, s, items, n_items);
    return hipGetLastError();
}

hipError_t launch_seed(const uint32_t *params, uint32_t *states, uint32_t stride,
                       uint32_t n_streams, hipStream_t s) {
    const int threads = 256;
    const int grid = (int)((n_streams + threads - 1) / threads);
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(seed_kernel, dim3(grid), dim3(threads), 0, s, params, states,
                       stride, n_streams);
    return hipGetLastError();
}

hipError_t launch_reset(uint32_t *counter, hipStream_t s) {
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_fill(uint32_t *out, uint64_t n_words, uint32_t value, int num_cus,
                       hipStream_t s) {
    const uint64_t n_vec = n_words / 4;
    const uint32_t n_tail = (uint32_t)(n_words % 4);
    uint64_t want = (n_vec + 255) / 256;
    uint64_t cap = (uint64_t)num_cus * 8;
    int grid = (int)(want < cap ? (want > 0 ? want : 1) : cap);
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, s,
                       reinterpret_cast<u32x4 *>(out), n_vec, out + n_vec * 4, n_tail, value);
    return hipGetLastError();
}

}  // namespace mtgp
