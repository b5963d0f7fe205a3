// mtgp_kernels.hip -- gfx950 kernels for bulk MTGP32 generation.
//
// One stream per thread group (the paper's per-block generator scope, Sec. 2
// and Sec. 3.2): a group is either one 64-lane wave (several independent
// streams per workgroup, no s_barrier) or a whole workgroup.  The stream's
// N-word state lives in an LDS buffer while it runs (shared memory, Sec. 2)
// and in device memory between launches.
//
// Step structure.  With W = N - pos, the new words x_n .. x_{n+W-1} depend
// only on words older than x_n, so one step produces S = min(W, lanes * K)
// outputs at once: every lane loads its taps for K outputs, computes, writes
// the new words to LDS and the tempered outputs to HBM, then the group
// synchronises once.  The LDS buffer is linear (x_n at a fixed offset from
// the step's head) so that every tap is an immediate offset from one or two
// per-lane base registers; when the head reaches the end of the buffer the
// last N words are copied back to the front.
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

    // Advance one stream by `count` outputs written to out[0..count).
    template <bool F32>
    static __device__ __forceinline__ void run(const uint32_t *__restrict__ prm,
                                               uint32_t *__restrict__ st,
                                               uint32_t *__restrict__ out,
                                               uint64_t count,
                                               uint32_t *__restrict__ buf,
                                               uint32_t lane) {
        uint32_t *__restrict__ tbl = buf + BUF;
        const uint32_t pos = prm[P_POS];
        const uint32_t sh1 = prm[P_SH1];
        const uint32_t sh2 = prm[P_SH2];
        const uint32_t mask = prm[P_MASK];
        const uint32_t W = N - pos;

        group_sync<TPS>();  // previous user of this buffer is done with it
        for (uint32_t i = lane; i < N; i += TPS) buf[i] = st[i];
        if (lane < 16) {
            tbl[lane] = prm[P_REC + lane];
            tbl[16 + lane] = prm[(F32 ? P_FLT : P_TMP) + lane];
        }
        group_sync<TPS>();

        const uint32_t smax = W < (uint32_t)SMAX ? W : (uint32_t)SMAX;
        uint32_t h = N;  // buffer index of the next new word
        uint64_t done = 0;
        gptr<uint32_t> gout = (gptr<uint32_t>)(out);
        while (done < count) {
            const uint64_t rem = count - done;
            const uint32_t S = rem < smax ? (uint32_t)rem : smax;
            // Every lane computes all K words of a full-width step, so keep
            // h + SMAX inside the buffer: the loads and LDS writes of lanes
            // beyond S then stay in bounds (their words are rewritten by the
            // next step before anything reads them).
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
                a[k] = q[k * TPS];
                b[k] = q[k * TPS + 1];
                hh[k] = qp[k * TPS];
                c[k] = qp[k * TPS + 1];
            }
            uint32_t x[K], r[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
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
            uint32_t *w = buf + (h + lane);
#pragma unroll
            for (int k = 0; k < K; ++k) w[k * TPS] = x[k];
            gptr<uint32_t> o = gout + done + lane;
            if (S == (uint32_t)SMAX) {
#pragma unroll
                for (int k = 0; k < K; ++k) __builtin_nontemporal_store(r[k], o + k * TPS);
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (lane + k * TPS < S) __builtin_nontemporal_store(r[k], o + k * TPS);
            }
            group_sync<TPS>();
            h += S;
            done += S;
        }
        for (uint32_t i = lane; i < N; i += TPS) st[i] = buf[h - N + i];
    }
};

// Persistent / plain generation kernel.  Each group (a wave when TPS == 64,
// else the workgroup) takes work items until none are left.
//  items != nullptr : batch mode, items claimed through *counter.
//  items == nullptr : plain mode, item i is stream i with `plain_count`
//                     outputs at plain_out + i * plain_count, groups take
//                     items i = group, group + n_groups, ...
template <int N, int TPS, int K, int WPB>
__global__ void __launch_bounds__(TPS == 64 ? 64 * WPB : TPS)
gen_kernel(const uint32_t *__restrict__ params, uint32_t *__restrict__ states,
           uint32_t stride, const BatchItem *__restrict__ items,
           uint32_t n_items, uint32_t *__restrict__ counter,
           uint32_t *__restrict__ plain_out, uint64_t plain_count,
           uint32_t plain_f32) {
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
        if (items != nullptr) {
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
        uint32_t stream;
        uint32_t f32;
        uint64_t count;
        uint32_t *out;
        if (items != nullptr) {
            const BatchItem item = items[it];
            stream = item.stream;
            f32 = item.dtype;
            count = item.count;
            out = reinterpret_cast<uint32_t *>(item.out);
        } else {
            stream = it;
            f32 = plain_f32;
            count = plain_count;
            out = plain_out + (uint64_t)it * plain_count;
        }
        const uint32_t *prm = params + (uint64_t)stream * P_WORDS;
        uint32_t *st = states + (uint64_t)stream * stride;
        if (f32)
            C::template run<true>(prm, st, out, count, buf, lane);
        else
            C::template run<false>(prm, st, out, count, buf, lane);
        if (items == nullptr) {
            it += n_groups;
        } else if (items[it].flag != 0) {
            // Publish completion of this item to the host: every lane's
            // output and state stores are made visible system-wide first.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            group_sync<TPS>();
            if (lane == 0)
                __hip_atomic_store(reinterpret_cast<uint32_t *>(items[it].flag), 1u,
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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

// Store-only fill: the achievable write bandwidth next to the generator.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

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
    int grid = a.grid;
    if (grid <= 0) {  // persistent: fill every CU to its occupancy
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        grid = per_cu * a.num_cus;
        // no more groups than items
        const int per_block = TPS == 64 ? WPB : 1;
        const int need = (int)((a.n_items + per_block - 1) / per_block);
        if (need < grid) grid = need > 0 ? need : 1;
    }
    hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds, (hipStream_t)a.stream,
                       a.params, a.states, a.stride, a.items, a.n_items, a.counter,
                       a.plain_out, a.plain_count, a.plain_f32);
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

hipError_t launch_seed(const uint32_t *params, uint32_t *states, uint32_t stride,
                       uint32_t n_streams, hipStream_t s) {
    const int threads = 256;
    const int grid = (int)((n_streams + threads - 1) / threads);
    hipLaunchKernelGGL(seed_kernel, dim3(grid), dim3(threads), 0, s, params, states,
                       stride, n_streams);
    return hipGetLastError();
}

hipError_t launch_reset(uint32_t *counter, hipStream_t s) {
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
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, s,
                       reinterpret_cast<u32x4 *>(out), n_vec, out + n_vec * 4, n_tail, value);
    return hipGetLastError();
}

}  // namespace mtgp
