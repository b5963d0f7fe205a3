/*
 * mtgp_device.h -- device-side draw API: a workgroup of a user kernel owns
 * one stream and draws from it with its state kept in LDS, without an HBM
 * round trip per number.
 *
 * This is the paper's consumer model made explicit (Sec. 2, Sec. 3.2): the
 * generator belongs to one thread block, its state is manipulated in the
 * block's shared memory, and it persists in device memory between kernel
 * calls.  The numbers are exactly those of mtgp_generate_u32/f32 (the same
 * definition, see mtgp.h), in the same order: a stream advances by the
 * number of outputs drawn, whatever the dtype and however the draws are cut.
 *
 * Use (all threads of the workgroup call every function, uniformly):
 *
 *     extern __shared__ uint32_t lds[];           // MTGP_DEVICE_LDS_WORDS(N, T)
 *     mtgp_device_stream s;
 *     mtgp_device_begin(s, d_params, k, d_states + k * stride, lds, words);
 *     uint32_t r = mtgp_device_draw_u32(s, n);    // thread t < n gets output t
 *     float f = mtgp_device_draw_f32(s, n);
 *     mtgp_device_end(s, d_states + k * stride);
 *
 * d_params is the parameter buffer written by mtgp_init_states (its layout
 * is given below), d_states a state row of N words.  The workgroup is
 * one-dimensional with T = blockDim.x threads (a multiple of 64, at most
 * 1024); a draw produces n <= T outputs in steps of at most W = N - pos
 * words, so streams with a small step width take several steps per draw.
 * Concurrent use of one stream by two workgroups is a race.
 */
#ifndef MTGP_DEVICE_H
#define MTGP_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

/* Word offsets in a stream's device parameter block (MTGP_DP_WORDS words per
 * stream, stream k at d_params + k * MTGP_DP_WORDS). */
enum : uint32_t {
    MTGP_DP_MEXP = 0,
    MTGP_DP_N = 1,     /* state words */
    MTGP_DP_POS = 2,
    MTGP_DP_SH1 = 3,
    MTGP_DP_SH2 = 4,
    MTGP_DP_MASK = 5,
    MTGP_DP_REC = 16,  /* rec_tbl[16], then tmp_tbl[16] at 32, flt_tbl[16] at 48 */
    MTGP_DP_TMP = 32,
    MTGP_DP_FLT = 48,
    MTGP_DP_WORDS = 1024,
};

/* LDS words a workgroup of T threads needs for a stream of N state words:
 * a buffer of 2N + 4T words (compacted, without overlap, when full) and the
 * three tables. */
#define MTGP_DEVICE_LDS_WORDS(n_words, threads) (2u * (n_words) + 4u * (threads) + 48u)

struct mtgp_device_stream {
    uint32_t *buf;  /* LDS: state buffer, then rec, tmp, flt tables */
    uint32_t cap;   /* buffer words */
    uint32_t h;     /* buffer index of the next word */
    uint32_t N, W, sh1, sh2, mask;
};

/* Loads stream `stream_id`'s tables and its state d_state[0..N) into lds
 * (lds_words >= MTGP_DEVICE_LDS_WORDS(N, blockDim.x)). */
__device__ inline void mtgp_device_begin(mtgp_device_stream &s, const uint32_t *d_params,
                                         uint32_t stream_id, const uint32_t *d_state,
                                         uint32_t *lds, uint32_t lds_words) {
    const uint32_t *p = d_params + (uint64_t)stream_id * MTGP_DP_WORDS;
    s.N = p[MTGP_DP_N];
    s.W = s.N - p[MTGP_DP_POS];
    s.sh1 = p[MTGP_DP_SH1];
    s.sh2 = p[MTGP_DP_SH2];
    s.mask = p[MTGP_DP_MASK];
    s.buf = lds;
    s.cap = lds_words - 48u;
    s.h = s.N;
    for (uint32_t i = threadIdx.x; i < s.N; i += blockDim.x) lds[i] = d_state[i];
    for (uint32_t i = threadIdx.x; i < 48u; i += blockDim.x) lds[s.cap + i] = p[MTGP_DP_REC + i];
    __syncthreads();
}

/* Orders the LDS accesses of one wave across a step without a workgroup
 * barrier (a wave's LDS operations complete in issue order). */
__device__ inline void mtgp_device_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

/* Next n (<= blockDim.x) outputs: thread t < n receives output t as raw
 * bits (uint32 output, or the float32 output's bit pattern when F32).
 * The new state words are produced first, in steps of at most W words (a
 * word's recursion reads words at least W older); streams with W < 64 take
 * their steps on the first wave alone, which needs no workgroup barrier
 * between steps and carries each lane's pos tap in a register (the word a
 * lane makes is its own tap W words later).  Every thread then tempers its
 * own word. */
template <bool F32>
__device__ inline uint32_t mtgp_device_draw_bits(mtgp_device_stream &s, uint32_t n) {
    const uint32_t T = blockDim.x, tid = threadIdx.x;
    uint32_t *buf = s.buf;
    const uint32_t *tbl = s.buf + s.cap;
    if (s.h + T > s.cap) {
        // every thread is done with the previous draw's words; cap >= 2N + T,
        // so the last N words never overlap the front
        __syncthreads();
        uint32_t v[4];
        for (uint32_t i0 = 0; i0 < s.N; i0 += 4 * T) {
            for (int j = 0; j < 4; ++j) {
                const uint32_t i = i0 + j * T + tid;
                v[j] = i < s.N ? buf[s.h - s.N + i] : 0u;
            }
            for (int j = 0; j < 4; ++j) {
                const uint32_t i = i0 + j * T + tid;
                if (i < s.N) buf[i] = v[j];
            }
        }
        __syncthreads();
        s.h = s.N;
    }
    const uint32_t h0 = s.h;
    if (s.W < 64u) {
        if (tid < 64u) {
            uint32_t c = tid < s.W ? buf[h0 - s.W + tid] : 0u;  // x_{k-W} of word k = h0 + tid
            for (uint32_t o = 0; o < n; o += s.W) {
                if (tid < s.W && o + tid < n) {
                    const uint32_t k = h0 + o + tid;
                    uint32_t X = (buf[k - s.N] & s.mask) ^ buf[k - s.N + 1];
                    X ^= X << s.sh1;
                    const uint32_t Y = X ^ (c >> s.sh2);
                    c = Y ^ tbl[Y & 15u];
                    buf[k] = c;
                }
                mtgp_device_wave_sync();
            }
        }
    } else {
        const uint32_t smax = s.W < T ? s.W : T;
        for (uint32_t o = 0; o < n; o += smax) {
            const uint32_t S = (n - o) < smax ? (n - o) : smax;
            if (tid >= o && tid < o + S) {
                const uint32_t k = h0 + tid;
                uint32_t X = (buf[k - s.N] & s.mask) ^ buf[k - s.N + 1];
                X ^= X << s.sh1;
                const uint32_t Y = X ^ (buf[k - s.W] >> s.sh2);
                buf[k] = Y ^ tbl[Y & 15u];
            }
            __syncthreads();
        }
    }
    __syncthreads();
    uint32_t result = 0;
    if (tid < n) {
        const uint32_t k = h0 + tid;
        const uint32_t x = buf[k];
        uint32_t H = buf[k - s.W - 1];
        H ^= H >> 16;
        H ^= H >> 8;
        if (F32)
            result = __float_as_uint(__uint_as_float((x >> 9) ^ tbl[32 + (H & 15u)]) - 1.0f);
        else
            result = x ^ tbl[16 + (H & 15u)];
    }
    s.h = h0 + n;
    return result;
}

__device__ inline uint32_t mtgp_device_draw_u32(mtgp_device_stream &s, uint32_t n) {
    return mtgp_device_draw_bits<false>(s, n);
}

__device__ inline float mtgp_device_draw_f32(mtgp_device_stream &s, uint32_t n) {
    return __uint_as_float(mtgp_device_draw_bits<true>(s, n));
}

/* Stores the stream's state (the last N words) to d_state[0..N). */
__device__ inline void mtgp_device_end(mtgp_device_stream &s, uint32_t *d_state) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < s.N; i += blockDim.x) d_state[i] = s.buf[s.h - s.N + i];
}

#endif /* MTGP_DEVICE_H */
