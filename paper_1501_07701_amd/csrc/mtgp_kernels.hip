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

#include <map>
#include <mutex>

#include "mtgp.h"
#include "mtgp_device.h"
#include "mtgp_internal.hpp"

namespace mtgp {

// Batch workspace of mtgp_generate_batch_noalloc: one per GPU, held until
// the process ends.  Host code never passes this name to a kernel (it is a
// host-side stand-in there); it uses the device address that
// scratch_address() looked up on that device.
static __device__ __align__(256) uint8_t scratch[MTGP_NOALLOC_SCRATCH_BYTES];

hipError_t scratch_address(void **out) {
    static std::mutex mu;
    static std::map<int, void *> addr;  // per device
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // with `dev` current
        if (e != hipSuccess) return e;
        it = addr.emplace(dev, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

// Pointer into global memory (address space 1), so stores are emitted as
// global_store rather than flat_store.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

// a ^ b ^ c in one VALU operation (v_bitop3_b32 with truth table 0x96, the
// odd-parity function of its three inputs); hipcc keeps XOR chains as
// two-input operations.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

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
// per step, with room for about four steps between compactions.  Several
// waves need at least 2N + SMAX so the compaction copy never overlaps
// itself; a single wave copies overlapping ranges safely and needs only
// N + SMAX.
__host__ __device__ constexpr int buf_words(int N, int SMAX, int TPS) {
    return ((TPS == 64 ? N : 2 * N) + 4 * SMAX + 63) / 64 * 64;
}

template <int N, int TPS, int K>
struct Core {
    static constexpr int SMAX = TPS * K;
    static constexpr int BUF = buf_words(N, SMAX, TPS);
    static_assert(BUF >= (TPS == 64 ? N : 2 * N) + SMAX, "compaction would overlap");
    static_assert(N > 64, "the small-step path assumes N > 64");
    // Window path (one wave, W < 64, linear table): a buffer of at least
    // N + WNMAX words, then the recursion and output tables, a 64-word
    // exchange area and the scan matrices.  The per-wave LDS block is the
    // larger of the two layouts; the window buffer takes whatever the
    // wide layout leaves.
    static constexpr int WNMAX = (N - 1) < 64 * WIN_EMAX ? (N - 1) : 64 * WIN_EMAX;
    static constexpr int WTAIL = 32 + 64 + WIN_MAXROUNDS * WIN_MAT_WORDS;
    static constexpr int WLDS = (N + WNMAX + 63) / 64 * 64 + WTAIL;
    static constexpr int LDS_WORDS = (BUF + 32) > WLDS ? (BUF + 32) : WLDS;
    static constexpr int WBUF = LDS_WORDS - WTAIL;
    static_assert(WBUF >= N + WNMAX, "window buffer too small");

    struct Step {  // per-item values, uniform across the group
        uint32_t pos, sh1, sh2, mask, W;
        uint32_t rb0, rb1, rb2, rb3;  // basis of a linear recursion table
    };

    // x = Y ^ rec[Y & 15]: from LDS, or for a linear table as the XOR of
    // the basis words selected by the low four bits of Y (no LDS round trip
    // on the dependent chain).
    template <bool LIN>
    static __device__ __forceinline__ uint32_t rec(const Step &p, const uint32_t *tbl,
                                                   uint32_t Y) {
        if constexpr (LIN) {
            uint32_t r = (0u - (Y & 1u)) & p.rb0;
            r ^= (0u - ((Y >> 1) & 1u)) & p.rb1;
            r ^= (0u - ((Y >> 2) & 1u)) & p.rb2;
            r ^= (0u - ((Y >> 3) & 1u)) & p.rb3;
            return Y ^ r;
        } else {
            return Y ^ tbl[Y & 15u];
        }
    }

    template <bool F32>
    static __device__ __forceinline__ uint32_t temper(const uint32_t *tbl, uint32_t x,
                                                      uint32_t hh) {
        uint32_t H = hh ^ (hh >> 16);
        H ^= H >> 8;
        const uint32_t tv = tbl[16 + (H & 15u)];
        if constexpr (F32)
            return __float_as_uint(__uint_as_float((x >> 9) ^ tv) - 1.0f);
        else
            return x ^ tv;
    }

    // Copies the newest N words to the front of the buffer when a step of
    // `reach` words would run past its end (LIM words).  With several waves
    // the source [h-N, h) and destination [0, N) never overlap
    // (h > BUF - SMAX >= 2N); a single wave may copy with overlap, which is
    // safe because its LDS reads and writes execute in instruction order and
    // the copy moves words towards lower addresses.
    // The copy runs in chunks of up to 8 words per lane, all reads of a chunk
    // issued before its writes; a later chunk's sources lie above every
    // earlier chunk's destinations (h > N), so chunking keeps that order.
    template <int LIM = BUF>
    static __device__ __forceinline__ void maybe_compact(uint32_t *buf, uint32_t &h,
                                                         uint32_t reach, uint32_t lane) {
        if (h + reach > (uint32_t)LIM) {
            constexpr int R = (N + TPS - 1) / TPS;
            constexpr int CH = R < 8 ? R : 8;
            const uint32_t *src = buf + (h - N);
#pragma unroll
            for (int j0 = 0; j0 < R; j0 += CH) {
                uint32_t tmp[CH];
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const uint32_t i = lane + (uint32_t)(j0 + j) * TPS;
                    tmp[j] = (j0 + j < R && i < (uint32_t)N) ? src[i] : 0u;
                }
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const uint32_t i = lane + (uint32_t)(j0 + j) * TPS;
                    if (j0 + j < R && i < (uint32_t)N) buf[i] = tmp[j];
                }
            }
            group_sync<TPS>();
            h = N;
        }
    }

    // Steps with W < 64 on one wave: S = W outputs per step, lane l makes
    // x_{h+l}.  Its tap x_{h+l-W} is the word it made in the previous step,
    // so the dependent chain never leaves registers.  The next step's LDS
    // loads are issued right after this step's word is stored, and this
    // step's tempering and output store run while they are in flight.
    template <bool F32, bool LIN>
    static __device__ __forceinline__ void steps_small(const Step &p, uint32_t *__restrict__ buf,
                                                       const uint32_t *__restrict__ tbl,
                                                       gptr<uint32_t> gout, gptr<uint32_t> raw,
                                                       bool want_raw, uint64_t count,
                                                       uint32_t &h, uint64_t &done,
                                                       uint32_t lane) {
        const uint32_t W = p.W;
        maybe_compact(buf, h, 64, lane);
        uint32_t c = buf[h - W + lane];  // in bounds for every lane: h >= N > 64
        uint32_t a = buf[h + lane - N], b = buf[h + lane - N + 1];
        uint32_t hh = buf[h + lane - W - 1];
        while (done < count) {
            const uint64_t rem = count - done;
            const uint32_t S = rem < W ? (uint32_t)rem : W;
            const uint32_t X = (a & p.mask) ^ b;
            const uint32_t x = rec<LIN>(p, tbl, xor3(X, X << p.sh1, c >> p.sh2));
            // lanes >= S write into the next step's slots, which it rewrites
            buf[h + lane] = x;
            const uint32_t hh_cur = hh;
            uint32_t hn = h + S;
            group_sync<TPS>();
            maybe_compact(buf, hn, 64, lane);
            a = buf[hn + lane - N];
            b = buf[hn + lane - N + 1];
            hh = buf[hn + lane - W - 1];
            const uint32_t r = temper<F32>(tbl, x, hh_cur);
            if (lane < S) {
                gout[done + lane] = r;
                if (want_raw) raw[N + done + lane] = x;
            }
            c = x;
            h = hn;
            done += S;
        }
    }

    // y = P v for a 32x32 GF(2) matrix given as 8 nibble tables of 16 words.
    static __device__ __forceinline__ uint32_t mat_apply(const uint32_t *t, uint32_t v) {
        uint32_t y = t[(v & 15u)] ^ t[16 + ((v >> 4) & 15u)];
#pragma unroll
        for (int k = 2; k < 8; k += 2)
            y = xor3(y, t[k * 16 + ((v >> (4 * k)) & 15u)], t[k * 16 + 16 + ((v >> (4 * k + 4)) & 15u)]);
        return y;
    }

    // Windowed steps for W < 64 with a linear recursion table, one wave.
    // A window of wn <= N-1 words only reads words older than its start for
    // x_{n-N} and x_{n-N+1}, so all of them are loaded first.  What remains
    // is the tap chain x_n = G(X_n) ^ M x_{n-W} per residue class n mod W,
    // which is affine: class r is cut into q chunks of E elements (one lane
    // each); every lane runs its chunk from a zero carry, a Hillis-Steele
    // scan with M^(E*2^k) gives each lane its true carry, and the lane
    // reruns its chunk from it.  Tempering and stores then run as one
    // coalesced pass over the window.  E is a compile-time constant so the
    // element loops are straight-line; lanes past the window end compute
    // junk that they write to the exchange area.
    template <bool F32, int E>
    static __device__ __forceinline__ void steps_window_e(const Step &p,
                                                          const uint32_t *__restrict__ prm,
                                                          uint32_t *__restrict__ buf,
                                                          gptr<uint32_t> gout, gptr<uint32_t> raw,
                                                          bool want_raw, uint64_t count,
                                                          uint32_t &h, uint64_t &done,
                                                          uint32_t lane) {
        const uint32_t *tbl = buf + WBUF;
        uint32_t *scr = buf + WBUF + 32;
        uint32_t *mats = scr + 64;
        const uint32_t W = p.W;
        const uint32_t wn = prm[P_WIN_WN], q = prm[P_WIN_Q];
        const uint32_t rounds = prm[P_WIN_ROUNDS];
        for (uint32_t i = lane; i < rounds * WIN_MAT_WORDS; i += 64) mats[i] = prm[P_WIN_MAT + i];
        const uint32_t r = lane / q, sub = lane - (lane / q) * q;
        const bool lane_ok = r < W;
        const uint32_t i0 = sub * (uint32_t)E;
        const uint32_t off0 = r + W * i0;  // the lane's first element in the window
        group_sync<TPS>();
        while (done < count) {
            const uint64_t rem = count - done;
            const uint32_t wc = rem < wn ? (uint32_t)rem : wn;
            maybe_compact<WBUF>(buf, h, wc, lane);
            // this lane's elements: class r, indices i0 .. i0+cnt-1
            const uint32_t lr = (lane_ok && wc > r) ? (wc - 1 - r) / W + 1 : 0u;
            const uint32_t cnt = lr > i0 ? (lr - i0 < (uint32_t)E ? lr - i0 : (uint32_t)E) : 0u;
            uint32_t X[E];
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const uint32_t idx = ((uint32_t)j < cnt) ? h + off0 + W * j - N : h - N;
                const uint32_t a = buf[idx], b = buf[idx + 1];
                const uint32_t x0 = (a & p.mask) ^ b;
                X[j] = x0 ^ (x0 << p.sh1);
            }
            // chunk from a zero carry (the first chunk of a class from its
            // true carry, the class's last word before the window)
            uint32_t c = (sub == 0 && lane_ok) ? buf[h + r - W] : 0u;
            uint32_t v[E];
#pragma unroll
            for (int j = 0; j < E; ++j) {
                c = rec<false>(p, tbl, X[j] ^ (c >> p.sh2));
                v[j] = c;
            }
            if (rounds) {
                // u_s <- u_s ^ M^(E*d) u_{s-d}: true last word of each chunk
                uint32_t u = v[E - 1];
                for (uint32_t k = 0; k < rounds; ++k) {
                    const uint32_t d = 1u << k;
                    scr[lane] = u;
                    group_sync<TPS>();
                    const uint32_t w = scr[sub >= d ? lane - d : lane];
                    group_sync<TPS>();
                    if (sub >= d) u ^= mat_apply(mats + k * WIN_MAT_WORDS, w);
                }
                scr[lane] = u;
                group_sync<TPS>();
                const uint32_t cin = scr[sub > 0 ? lane - 1 : lane];
                group_sync<TPS>();
                if (sub > 0) {
                    c = cin;
#pragma unroll
                    for (int j = 0; j < E; ++j) {
                        c = rec<false>(p, tbl, X[j] ^ (c >> p.sh2));
                        v[j] = c;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const uint32_t dst = ((uint32_t)j < cnt) ? h + off0 + W * j : WBUF + 32 + lane;
                buf[dst] = v[j];
            }
            group_sync<TPS>();
            // tempering and stores, coalesced over the window
            for (uint32_t pp = lane; pp < wc; pp += 64) {
                const uint32_t x = buf[h + pp];
                const uint32_t hh = buf[h + pp - W - 1];
                gout[done + pp] = temper<F32>(tbl, x, hh);
                if (want_raw) raw[N + done + pp] = x;
            }
            group_sync<TPS>();
            h += wc;
            done += wc;
        }
    }

    template <bool F32>
    static __device__ __forceinline__ void steps_window(const Step &p,
                                                        const uint32_t *__restrict__ prm,
                                                        uint32_t *__restrict__ buf,
                                                        gptr<uint32_t> gout, gptr<uint32_t> raw,
                                                        bool want_raw, uint64_t count,
                                                        uint32_t &h, uint64_t &done,
                                                        uint32_t lane) {
        switch (prm[P_WIN_E]) {
#define MTGP_WE(E) \
    case E: steps_window_e<F32, E>(p, prm, buf, gout, raw, want_raw, count, h, done, lane); break;
            MTGP_WE(1) MTGP_WE(2) MTGP_WE(3) MTGP_WE(4)
            MTGP_WE(5) MTGP_WE(6) MTGP_WE(7) MTGP_WE(8)
#undef MTGP_WE
            default: break;
        }
    }

    // One step of KE outputs per lane (KE = ceil(S / TPS)), straight-line.
    template <bool F32, int KE>
    static __device__ __forceinline__ void body(const Step &p, uint32_t *__restrict__ buf,
                                                const uint32_t *__restrict__ tbl,
                                                gptr<uint32_t> o, gptr<uint32_t> rw,
                                                bool want_raw, uint32_t h, uint32_t S,
                                                uint32_t lane) {
        const uint32_t *q = buf + (h + lane - N);
        const uint32_t *qp = q + (p.pos - 1);
        uint32_t a[KE], b[KE], hh[KE], c[KE];
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            a[k] = q[k * TPS];
            b[k] = q[k * TPS + 1];
            hh[k] = qp[k * TPS];
            c[k] = qp[k * TPS + 1];
        }
        uint32_t x[KE], r[KE];
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            const uint32_t X = (a[k] & p.mask) ^ b[k];
            x[k] = rec<false>(p, tbl, xor3(X, X << p.sh1, c[k] >> p.sh2));
            r[k] = temper<F32>(tbl, x[k], hh[k]);
        }
        uint32_t *w = buf + (h + lane);
#pragma unroll
        for (int k = 0; k < KE; ++k) w[k * TPS] = x[k];
        // every k but the last is full (S > (KE-1)*TPS)
#pragma unroll
        for (int k = 0; k < KE - 1; ++k) o[k * TPS] = r[k];
        if (lane + (KE - 1) * TPS < S) o[(KE - 1) * TPS] = r[KE - 1];
        if (want_raw) {
#pragma unroll
            for (int k = 0; k < KE; ++k)
                if (lane + k * TPS < S) rw[k * TPS] = x[k];
        }
    }

    // Whole steps of S = KE rows (the same S every step), then nothing:
    // the caller finishes the partial last step.
    template <bool F32, int KE>
    static __device__ __forceinline__ void full_steps(const Step &p, uint32_t *__restrict__ buf,
                                                      const uint32_t *__restrict__ tbl,
                                                      gptr<uint32_t> gout, gptr<uint32_t> raw,
                                                      bool want_raw, uint64_t n_steps,
                                                      uint32_t S, uint32_t &h, uint64_t &done,
                                                      uint32_t lane) {
        for (uint64_t st = 0; st < n_steps; ++st) {
            maybe_compact(buf, h, SMAX, lane);
            body<F32, KE>(p, buf, tbl, gout + done + lane, raw + N + done + lane, want_raw, h,
                          S, lane);
            group_sync<TPS>();
            h += S;
            done += S;
        }
    }

    template <bool F32>
    static __device__ __forceinline__ void steps_wide(const Step &p, uint32_t *__restrict__ buf,
                                                      const uint32_t *__restrict__ tbl,
                                                      gptr<uint32_t> gout, gptr<uint32_t> raw,
                                                      bool want_raw, uint64_t count,
                                                      uint32_t &h, uint64_t &done,
                                                      uint32_t lane) {
        // full steps: W rounded down to whole 128-byte lines when wide
        uint32_t smax = p.W >= 64 ? (p.W & ~31u) : p.W;
        if (smax > (uint32_t)SMAX) smax = SMAX;
        // lanes compute every word of their rows, so keep h + SMAX inside
        // the buffer (words past S are rewritten before any read)
        const uint64_t n_full = (count - done) / smax;
        switch ((smax + TPS - 1) / TPS) {
#define MTGP_FULL(KE)                                                                       \
    case KE:                                                                                \
        if constexpr (KE <= K)                                                              \
            full_steps<F32, KE>(p, buf, tbl, gout, raw, want_raw, n_full, smax, h, done,   \
                                lane);                                                      \
        break;
            MTGP_FULL(1) MTGP_FULL(2) MTGP_FULL(3) MTGP_FULL(4)
            MTGP_FULL(5) MTGP_FULL(6) MTGP_FULL(7) MTGP_FULL(8)
#undef MTGP_FULL
            default: break;
        }
        if (done < count) {
            const uint32_t S = (uint32_t)(count - done);
            maybe_compact(buf, h, SMAX, lane);
            gptr<uint32_t> o = gout + done + lane;
            gptr<uint32_t> rw = raw + N + done + lane;
            switch ((S + TPS - 1) / TPS) {
#define MTGP_BODY(KE) \
    case KE: if constexpr (KE <= K) body<F32, KE>(p, buf, tbl, o, rw, want_raw, h, S, lane); break;
                MTGP_BODY(1) MTGP_BODY(2) MTGP_BODY(3) MTGP_BODY(4)
                MTGP_BODY(5) MTGP_BODY(6) MTGP_BODY(7) MTGP_BODY(8)
#undef MTGP_BODY
                default: break;
            }
            group_sync<TPS>();
            h += S;
            done += S;
        }
    }

    // Advance one stream by item.count outputs.  A MODE_VERIFY item that
    // ends in a state other than item.verify sets *fail.  RAW: the
    // MODE_RAW word dump is compiled in (prefix kernels only).
    template <bool F32, bool RAW>
    static __device__ __forceinline__ void run(const uint32_t *__restrict__ prm,
                                               const BatchItem &item,
                                               uint32_t *__restrict__ buf, uint32_t lane,
                                               uint32_t *fail, uint32_t win_below) {
        // a stream takes the window path when the host gave it window data
        const bool win = TPS == 64 && prm[P_WIN_E] != 0u && prm[P_W] < win_below;
        uint32_t *__restrict__ tbl = buf + (win ? WBUF : BUF);
        Step p;
        p.pos = prm[P_POS];
        p.sh1 = prm[P_SH1];
        p.sh2 = prm[P_SH2];
        p.mask = prm[P_MASK];
        p.W = N - p.pos;
        p.rb0 = prm[P_RB + 0];
        p.rb1 = prm[P_RB + 1];
        p.rb2 = prm[P_RB + 2];
        p.rb3 = prm[P_RB + 3];
        const uint32_t lin = prm[P_LIN];
        const uint64_t count = item.count;
        const uint32_t *st_in = reinterpret_cast<const uint32_t *>(item.state_in);
        uint32_t *st_out = reinterpret_cast<uint32_t *>(item.state_out);
        gptr<uint32_t> raw = (gptr<uint32_t>)(reinterpret_cast<uint32_t *>(item.raw));
        gptr<uint32_t> gout = (gptr<uint32_t>)(reinterpret_cast<uint32_t *>(item.out));
        const bool want_raw = RAW && (item.mode & MODE_RAW) != 0;

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

        uint32_t h = N;  // buffer index of the next new word
        uint64_t done = 0;
        if (win) {
            steps_window<F32>(p, prm, buf, gout, raw, want_raw, count, h, done, lane);
        } else if (TPS == 64 && p.W < 64) {
            if (lin)
                steps_small<F32, true>(p, buf, tbl, gout, raw, want_raw, count, h, done, lane);
            else
                steps_small<F32, false>(p, buf, tbl, gout, raw, want_raw, count, h, done, lane);
        } else {
            steps_wide<F32>(p, buf, tbl, gout, raw, want_raw, count, h, done, lane);
        }
        group_sync<TPS>();
        if (st_out != nullptr)
            for (uint32_t i = lane; i < N; i += TPS) st_out[i] = buf[h - N + i];
        if ((item.mode & MODE_VERIFY) && fail != nullptr) {
            // the end state must equal the next segment's jumped start state
            const uint32_t *ref = reinterpret_cast<const uint32_t *>(item.verify);
            uint32_t bad = 0;
            for (uint32_t i = lane; i < N; i += TPS) bad |= (buf[h - N + i] != ref[i]) ? 1u : 0u;
            if (bad) atomicOr(fail, 1u);
        }
    }
};

// Plain mode (items == nullptr): item i is stream i, advanced in place in
// its state row by plain_count outputs written at plain_out + i*plain_count.
struct PlainArgs {
    uint32_t *states;
    uint32_t stride;
    uint32_t mode;
    uint32_t *out;
    uint64_t count;
};

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Value of lane 0 (wave) or thread 0 (workgroup) for the whole group.
template <int TPS>
__device__ __forceinline__ uint32_t group_first(uint32_t v, uint32_t *slot) {
    if constexpr (TPS == 64) {
        return __builtin_amdgcn_readfirstlane(v);
    } else {
        __syncthreads();
        if (threadIdx.x == 0) *slot = v;
        __syncthreads();
        return *slot;
    }
}

// The work loop shared by the generation kernels: claim an item (or take
// stream `it` in plain mode), run it, raise its completion flag.
template <int N, int TPS, int K, int WPB, bool RAW>
__device__ __forceinline__ void gen_body(const uint32_t *__restrict__ params,
                                         const BatchItem *__restrict__ items, uint32_t n_items,
                                         uint32_t *__restrict__ counter,
                                         uint32_t *__restrict__ err, uint32_t persistent,
                                         uint32_t win_below, PlainArgs plain) {
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
            uint32_t v = 0;
            if (lane == 0) v = atomicAdd(counter, 1u);
            it = group_first<TPS>(v, &s_claim);
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
            item.raw = item.verify = item.rec = item.flag = 0;
        }
        if (item.mode & MODE_FIXUP) {
            // Request check, after every segment of the request has
            // finished: if a segment started from a wrong jumped state (the
            // stream's state lay outside the orbit its polynomial
            // annihilates), regenerate the whole request in order from its
            // start state and log it.  Record fields are loaded from
            // writable memory, so they are made wave-uniform explicitly.
            const ReqRec *rec = reinterpret_cast<const ReqRec *>(item.rec);
            const uint32_t failed = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(&rec->failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            item.count = 0;
            if (failed) {
                item.stream = __builtin_amdgcn_readfirstlane(rec->stream);
                item.mode = __builtin_amdgcn_readfirstlane(rec->mode);
                item.count = uniform64(rec->count);
                item.out = uniform64(rec->out);
                item.state_in = uniform64(rec->orig);
                item.state_out = uniform64(rec->row);
                item.raw = item.verify = 0;
                if (lane == 0) {
                    atomicAdd(err, 1u);
                    const uint32_t slot = atomicAdd(err + 1, 1u);
                    if (slot < (uint32_t)HDR_LOG_MAX) err[2 + slot] = item.stream;
                }
            }
        }
        if (item.count > 0) {
            const uint32_t *prm = params + (uint64_t)item.stream * P_WORDS;
            uint32_t *fail = (item.mode & MODE_VERIFY)
                                 ? &reinterpret_cast<ReqRec *>(item.rec)->failed
                                 : nullptr;
            if (item.mode & MODE_F32)
                C::template run<true, RAW>(prm, item, buf, lane, fail, win_below);
            else
                C::template run<false, RAW>(prm, item, buf, lane, fail, win_below);
        }
        if (item.flag != 0) {
            // Publish completion of the request to the host: every lane's
            // output and state stores are made visible system-wide first.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            group_sync<TPS>();
            if (lane == 0)
                __hip_atomic_store(reinterpret_cast<uint32_t *>(item.flag), 1u, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
        }
        if (!persistent) it += n_groups;
    }
}

// Segments of a batch, whole unsplit requests and plain calls.
template <int N, int TPS, int K, int WPB>
__global__ void __launch_bounds__(TPS == 64 ? 64 * WPB : TPS)
gen_kernel(const uint32_t *__restrict__ params, const BatchItem *__restrict__ items,
           uint32_t n_items, uint32_t *__restrict__ counter, uint32_t *__restrict__ err,
           uint32_t persistent, uint32_t win_below, PlainArgs plain) {
    gen_body<N, TPS, K, WPB, false>(params, items, n_items, counter, err, persistent, win_below,
                                    plain);
}

// Outputs per lane and step of the prefix kernel (the default tuning's).
__host__ __device__ constexpr int prefix_k(int N) { return N <= 400 ? 4 : 8; }

// Prefix items of split requests (the first D+1 outputs, dumping the raw
// words the jump evaluation reads), and the word runs jump-ahead planning
// takes its polynomials from: one wave per item, four waves per workgroup.
template <int N>
__global__ void __launch_bounds__(256)
prefix_kernel(const uint32_t *__restrict__ params, const BatchItem *__restrict__ items,
              uint32_t n_items, uint32_t *__restrict__ counter, uint32_t *__restrict__ err,
              uint32_t persistent, uint32_t win_below, PlainArgs plain) {
    gen_body<N, 64, prefix_k(N), 4, true>(params, items, n_items, counter, err, persistent,
                                          win_below, plain);
}

// Request checks of split requests (MODE_FIXUP items), after the segments:
// usually no generation at all; a failed request is regenerated here.
template <int N>
__global__ void __launch_bounds__(256)
check_kernel(const uint32_t *__restrict__ params, const BatchItem *__restrict__ items,
             uint32_t n_items, uint32_t *__restrict__ counter, uint32_t *__restrict__ err,
             uint32_t persistent, uint32_t win_below, PlainArgs plain) {
    gen_body<N, 64, 1, 4, false>(params, items, n_items, counter, err, persistent, win_below,
                                 plain);
}

// Jump evaluation: out[m] = XOR over the set bits i < D of g of r[i+m] with
// r[n] = raw[1+n], for m < M.  Items come in blocks of JUMP_WAVES: one
// workgroup per block, one wave per item; the items of a block use the same
// words r (same stream, D and M) and null items (out == 0) only pad a block.
// Coefficients are taken four at a time: for a nibble value v of g at
// coefficients 4c..4c+3 the wave adds Q_v[4c+m], where
// Q_v[n] = XOR over the set bits j of v of r[n+j].  The workgroup builds the
// 15 planes Q_1..Q_15 for a chunk of JUMP_CH coefficients and JUMP_MT outputs
// in LDS once, and every wave of the block reads them: per output word one
// LDS read per nibble instead of one per set bit.  Plane 0 stays zero, so
// the lookups are branch-free and several nibbles' reads are in flight.
// Lane l owns output words 4l..4l+3 (+256 j) of a pass and reads them as one
// 16-byte LDS access per nibble (4c + 4l is a multiple of 4).
constexpr int JUMP_WAVES = JUMP_BLOCK;
constexpr int JUMP_CH = 256;    // coefficients per chunk (multiple of 32)
constexpr int JUMP_JA = 8;      // output words per lane per pass
constexpr int JUMP_MT = 64 * JUMP_JA;
constexpr int JUMP_PL = JUMP_CH + JUMP_MT;  // plane length (words)
static_assert(JUMP_MT == JUMP_OUT_WORDS, "the planner splits jumps into passes of JUMP_MT words");
constexpr int JUMP_LDS_BYTES = 16 * JUMP_PL * 4;

typedef uint32_t jv4 __attribute__((ext_vector_type(4)));

template <int JA>
__device__ __forceinline__ void jump_pass(gptr<const uint32_t> r, gptr<const uint32_t> g,
                                          uint32_t *__restrict__ out, bool active, uint32_t D,
                                          uint32_t rlen, uint32_t m0, uint32_t mt,
                                          uint32_t *__restrict__ planes, uint32_t lane) {
    jv4 acc[JA];
#pragma unroll
    for (int j = 0; j < JA; ++j) acc[j] = jv4{0u, 0u, 0u, 0u};
    for (uint32_t i0 = 0; i0 < D; i0 += JUMP_CH) {
        const uint32_t ch = (D - i0) < (uint32_t)JUMP_CH ? (D - i0) : (uint32_t)JUMP_CH;
        const uint32_t L = ch + mt;
        const uint32_t base = i0 + m0;
        const uint32_t nw = (ch + 31) / 32;
        // this chunk's coefficient words, one per lane, fetched early
        const uint32_t gv = (active && lane < nw) ? g[(i0 >> 5) + lane] : 0u;
        __syncthreads();  // every wave is done with the previous chunk's planes
        for (uint32_t t = threadIdx.x; t < L; t += 64 * JUMP_WAVES) {
            const uint32_t n = base + t;
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) w[j] = (n + j < rlen) ? r[n + j] : 0u;
            uint32_t q[16];
            q[0] = 0;
#pragma unroll
            for (int v = 1; v < 16; ++v) {
                const int low = v & -v;
                const int bit = low == 1 ? 0 : (low == 2 ? 1 : (low == 4 ? 2 : 3));
                q[v] = q[v & (v - 1)] ^ w[bit];
                planes[v * JUMP_PL + t] = q[v];
            }
        }
        __syncthreads();
        if (active) {
            for (uint32_t cw = 0; cw < nw; ++cw) {
                uint32_t bits = __builtin_amdgcn_readlane(gv, cw);
                if (cw == nw - 1 && (ch & 31)) bits &= (1u << (ch & 31)) - 1u;
                const uint32_t *col = planes + 32 * cw + 4 * lane;
                // two nibbles per three-input XOR
#pragma unroll
                for (int k = 0; k < 8; k += 2) {
                    const uint32_t v0 = (bits >> (4 * k)) & 15u;
                    const uint32_t v1 = (bits >> (4 * k + 4)) & 15u;
                    const uint32_t *s0 = col + v0 * JUMP_PL + 4 * k;
                    const uint32_t *s1 = col + v1 * JUMP_PL + 4 * k + 4;
#pragma unroll
                    for (int j = 0; j < JA; ++j) {
                        const jv4 a = *reinterpret_cast<const jv4 *>(s0 + 256 * j);
                        const jv4 b = *reinterpret_cast<const jv4 *>(s1 + 256 * j);
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[j][e] = xor3(acc[j][e], a[e], b[e]);
                    }
                }
            }
        }
    }
    if (active) {
#pragma unroll
        for (int j = 0; j < JA; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t m = 4 * lane + 256 * j + e;
                if (m < mt) out[m0 + m] = acc[j][e];
            }
        }
    }
}

// One block of JUMP_WAVES jump items (one wave each), planes in LDS.
__device__ __forceinline__ void jump_block(const JumpItem *__restrict__ items, uint32_t n_items,
                                           uint32_t blk, uint32_t *__restrict__ planes,
                                           uint32_t wave, uint32_t lane) {
    const JumpItem lead = items[blk * JUMP_WAVES];
    const uint32_t mine = blk * JUMP_WAVES + wave;
    JumpItem jit = lead;
    jit.out = 0;
    if (mine < n_items) jit = items[mine];
    const bool active = jit.out != 0;
    gptr<const uint32_t> r = (gptr<const uint32_t>)(reinterpret_cast<const uint32_t *>(lead.raw)) + 1;
    gptr<const uint32_t> g = (gptr<const uint32_t>)(reinterpret_cast<const uint32_t *>(jit.poly));
    uint32_t *out = reinterpret_cast<uint32_t *>(jit.out);
    const uint32_t D = lead.nbits, M = lead.m, rlen = lead.nbits + lead.m;
    for (uint32_t m0 = 0; m0 < M; m0 += JUMP_MT) {
        const uint32_t mt = (M - m0) < (uint32_t)JUMP_MT ? (M - m0) : (uint32_t)JUMP_MT;
        switch ((mt + 255) / 256) {
#define MTGP_JP(JA) \
    case JA: jump_pass<JA>(r, g, out, active, D, rlen, m0, mt, planes, lane); break;
            MTGP_JP(1) MTGP_JP(2)
#undef MTGP_JP
            default: break;
        }
    }
}

// Jump evaluation alone (the planning checks of jump-ahead polynomials).
__global__ void __launch_bounds__(64 * JUMP_WAVES)
jump_kernel(const JumpItem *__restrict__ items, uint32_t n_items) {
    extern __shared__ uint32_t planes[];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n_blocks = (n_items + JUMP_WAVES - 1) / JUMP_WAVES;
    for (uint32_t t = threadIdx.x; t < (uint32_t)JUMP_PL; t += 64 * JUMP_WAVES) planes[t] = 0u;
    for (uint32_t blk = blockIdx.x; blk < n_blocks; blk += gridDim.x)
        jump_block(items, n_items, blk, planes, wave, lane);
}

// Waits (a whole wave, every lane reading the same flag) until *flag is
// nonzero; gives up after a bound far above any legitimate wait, counting
// the give-up in *timeouts (the repair count: a jump evaluated too early
// fails its segment check, and the request is regenerated).  The flag value
// is made wave-uniform so that the loop exit is uniform.
__device__ __forceinline__ void wait_flag(const uint32_t *flag, uint32_t *timeouts,
                                          uint32_t lane) {
    for (uint32_t spins = 0;; ++spins) {
        const uint32_t f = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (f != 0u) break;
        if (spins > (1u << 24)) {  // seconds of s_sleep
            atomicAdd(timeouts, lane == 0 ? 1u : 0u);
            break;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// Prefix items and jump blocks of a batch in one persistent launch.  Every
// wave first claims prefix items (one wave each, RAW: they dump the words
// the jumps read); once the prefix counter is exhausted (every prefix has
// been claimed by a running wave) the workgroup claims jump blocks, each of
// which waits for its stream's prefix flag.  A jump block waits only on a
// prefix claimed before any block, so every wait ends.
struct PJArgs {
    const uint32_t *params;
    const BatchItem *prefix;  // nP prefix items
    uint32_t nP;
    const JumpItem *jumps;    // nJ jump items in blocks of JUMP_WAVES
    uint32_t nJ;
    const uint32_t *jdep;     // per block: index of its stream's prefix item
    uint32_t *pflag;          // per prefix item: set to 1 when its words are stored
    uint32_t *hdr;            // workspace header (claim counters, timeouts)
    uint32_t win_below;
};

constexpr int PJ_LDS_BYTES = JUMP_LDS_BYTES + 16;  // planes + claim word

template <int N>
__global__ void __launch_bounds__(64 * JUMP_WAVES) pj_kernel(PJArgs a) {
    using C = Core<N, 64, 4>;
    static_assert(JUMP_WAVES * C::LDS_WORDS * 4 <= JUMP_LDS_BYTES, "prefix buffers fit the planes");
    // No static LDS: the planes are read with 16-byte LDS loads, and a
    // static word would move the dynamic region to offset 4.  The claim
    // broadcast word sits right after the planes.
    extern __shared__ uint32_t lds[];
    uint32_t &s_claim = lds[JUMP_LDS_BYTES / 4];
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t *buf = lds + wave * C::LDS_WORDS;
    while (true) {  // prefix items, one per wave
        uint32_t v = 0;
        if (lane == 0) v = atomicAdd(a.hdr + 0, 1u);
        const uint32_t it = __builtin_amdgcn_readfirstlane(v);
        if (it >= a.nP) break;
        const BatchItem item = a.prefix[it];
        const uint32_t *prm = a.params + (uint64_t)item.stream * P_WORDS;
        if (item.mode & MODE_F32)
            C::template run<true, true>(prm, item, buf, lane, nullptr, a.win_below);
        else
            C::template run<false, true>(prm, item, buf, lane, nullptr, a.win_below);
        // every lane stores the flag: a lane-0-only store here lets the
        // compiler split the claim loop by lane
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(a.pflag + it, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t n_blocks = (a.nJ + JUMP_WAVES - 1) / JUMP_WAVES;
    __syncthreads();  // every wave of this workgroup is done with its prefix buffer
    for (uint32_t t = threadIdx.x; t < (uint32_t)JUMP_PL; t += 64 * JUMP_WAVES) lds[t] = 0u;
    while (true) {  // jump blocks, one per workgroup
        __syncthreads();
        if (threadIdx.x == 0) s_claim = atomicAdd(a.hdr + HDR_J_CLAIM, 1u);
        __syncthreads();
        const uint32_t blk = __builtin_amdgcn_readfirstlane(s_claim);
        if (blk >= n_blocks) break;
        if (wave == 0) wait_flag(a.pflag + a.jdep[blk], a.hdr + HDR_ERR, lane);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        jump_block(a.jumps, a.nJ, blk, lds, wave, lane);
    }
}

template <int N>
static hipError_t launch_pj_n(const PJArgs &a, int num_cus, hipStream_t s) {
    static bool attr_set = false;  // benign race: idempotent attribute
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)pj_kernel<N>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           PJ_LDS_BYTES);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const uint32_t work = a.nP + (a.nJ + JUMP_WAVES - 1) / JUMP_WAVES;
    int grid = (int)(work > 0 ? work : 1);
    const int cap = num_cus * 3;  // three workgroups of 48 KB fit a CU's LDS
    if (grid > cap) grid = cap;
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(pj_kernel<N>, dim3(grid), dim3(64 * JUMP_WAVES), PJ_LDS_BYTES, s, a);
    return hipGetLastError();
}

hipError_t launch_prefix_jumps(int n_words, const BatchItem *prefix, uint32_t nP,
                               const JumpItem *jumps, uint32_t nJ, const uint32_t *jdep,
                               uint32_t *pflag, const uint32_t *params, uint32_t *hdr,
                               uint32_t win_below, int num_cus, hipStream_t s) {
    PJArgs a{params, prefix, nP, jumps, nJ, jdep, pflag, hdr, win_below};
    switch (n_words) {
        case 101: return launch_pj_n<101>(a, num_cus, s);
        case 351: return launch_pj_n<351>(a, num_cus, s);
        case 726: return launch_pj_n<726>(a, num_cus, s);
        case 1391: return launch_pj_n<1391>(a, num_cus, s);
        default: return hipErrorInvalidValue;
    }
}

size_t prefix_jump_lds_bytes() { return PJ_LDS_BYTES; }

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

__global__ void clear_kernel(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// One wave; lane i owns header word i (i < 24).  Every lane reads the tag
// before any lane writes it.
__global__ void header_kernel(uint32_t *hdr, uint32_t tag_lo, uint32_t tag_hi,
                              uint32_t clear_errors) {
    const uint32_t i = threadIdx.x;
    const bool fresh = hdr[HDR_TAG] != tag_lo || hdr[HDR_TAG + 1] != tag_hi;
    __builtin_amdgcn_wave_barrier();
    const bool claim = i < (uint32_t)HDR_ERR || i == (uint32_t)HDR_FIX_CLAIM ||
                       i == (uint32_t)HDR_J_CLAIM || i == (uint32_t)HDR_W_CLAIM;
    const bool errw = i >= (uint32_t)HDR_ERR && i < (uint32_t)(HDR_ERR + HDR_ERR_WORDS);
    const bool stamp = i >= HDR_STAMP_BYTE / 4 && i < HDR_STAMP_BYTE / 4 + 8;
    if (claim || (errw && (fresh || clear_errors)) || (stamp && fresh)) hdr[i] = 0u;
    if (i == (uint32_t)HDR_TAG) hdr[i] = tag_lo;
    if (i == (uint32_t)HDR_TAG + 1) hdr[i] = tag_hi;
}

// Device timestamp (the constant-rate wall clock) for phase timing.
__global__ void stamp_kernel(uint64_t *dst) {
    if (threadIdx.x == 0) *dst = wall_clock64();
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Store-only fill: the achievable write bandwidth next to the generator
// (plain stores, as the generator uses; on gfx950 they measured faster than
// non-temporal ones).
__global__ void __launch_bounds__(256)
fill_kernel(u32x4 *__restrict__ out, uint64_t n_vec, uint32_t *__restrict__ tail,
            uint32_t n_tail, uint32_t value) {
    const u32x4 v = {value, value, value, value};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vec; i += stride)
        out[i] = v;
    if (blockIdx.x == 0 && threadIdx.x < n_tail) tail[threadIdx.x] = value;
}

// ------------------------------------------------------------- dispatch --

typedef void (*GenFn)(const uint32_t *, const BatchItem *, uint32_t, uint32_t *, uint32_t *,
                      uint32_t, uint32_t, PlainArgs);

// Launches one of the generation kernels with the LDS of Core<N, TPS, K>
// times the groups per workgroup; persistent launches fill every CU to its
// occupancy with no more groups than items.
template <int N, int TPS, int K, int WPB>
static hipError_t launch_with(GenFn fn, bool *attr_set, const LaunchArgs &a) {
    using C = Core<N, TPS, K>;
    const int threads = TPS == 64 ? 64 * WPB : TPS;
    const size_t lds = (size_t)C::LDS_WORDS * 4 * (TPS == 64 ? WPB : 1);
    if (!*attr_set) {  // benign race: idempotent attribute
        hipError_t e = hipFuncSetAttribute((const void *)fn,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        *attr_set = true;
    }
    const int per_block = TPS == 64 ? WPB : 1;
    const int need = (int)((a.n_items + per_block - 1) / per_block);
    int grid = need > 0 ? need : 1;
    if (a.persistent) {
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
        if (e != hipSuccess) return e;
        if (a.groups_per_cu > 0 && a.groups_per_cu < per_cu) per_cu = a.groups_per_cu;
        if (per_cu < 1) per_cu = 1;
        if (per_cu * a.num_cus < grid) grid = per_cu * a.num_cus;
    }
    PlainArgs plain{a.plain_states, a.plain_stride, a.plain_mode, a.plain_out, a.plain_count};
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds, (hipStream_t)a.stream, a.params,
                       a.items, a.n_items, a.counter, a.err, a.persistent ? 1u : 0u,
                       a.win_below, plain);
    return hipGetLastError();
}

template <int N, int TPS, int K, int WPB>
static hipError_t launch_gen(const LaunchArgs &a) {
    static bool attr_set = false;
    return launch_with<N, TPS, K, WPB>(gen_kernel<N, TPS, K, WPB>, &attr_set, a);
}

template <int N>
static hipError_t launch_prefix_n(const LaunchArgs &a) {
    static bool attr_set = false;
    return launch_with<N, 64, prefix_k(N), 4>(prefix_kernel<N>, &attr_set, a);
}

template <int N>
static hipError_t launch_check_n(const LaunchArgs &a) {
    static bool attr_set = false;
    return launch_with<N, 64, 1, 4>(check_kernel<N>, &attr_set, a);
}

hipError_t launch_prefix(int n_words, const LaunchArgs &a) {
    switch (n_words) {
        case 101: return launch_prefix_n<101>(a);
        case 351: return launch_prefix_n<351>(a);
        case 726: return launch_prefix_n<726>(a);
        case 1391: return launch_prefix_n<1391>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_check(int n_words, const LaunchArgs &a) {
    switch (n_words) {
        case 101: return launch_check_n<101>(a);
        case 351: return launch_check_n<351>(a);
        case 726: return launch_check_n<726>(a);
        case 1391: return launch_check_n<1391>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int N, int TPS, int K, int WPB>
static size_t lds_bytes_of() {
    return (size_t)Core<N, TPS, K>::LDS_WORDS * 4 * (TPS == 64 ? WPB : 1);
}

// Streams a CU runs at once with this variant (waves for TPS = 64, else
// workgroups), from the occupancy the runtime reports; 0 on error.
template <int N, int TPS, int K, int WPB>
static int slots_of() {
    static int cached = -1;  // benign race: idempotent query
    if (cached < 0) {
        int per_cu = 0;
        const int threads = TPS == 64 ? 64 * WPB : TPS;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gen_kernel<N, TPS, K, WPB>,
                                                         threads, lds_bytes_of<N, TPS, K, WPB>()) !=
            hipSuccess)
            return 0;
        cached = per_cu * (TPS == 64 ? WPB : 1);
    }
    return cached;
}

struct Variant {
    int N, tps, k, wpb;
    hipError_t (*launch)(const LaunchArgs &);
    size_t (*lds)();
    int (*slots)();
};

#define MTGP_V(N, T, K, P) \
    {N, T, K, P, &launch_gen<N, T, K, P>, &lds_bytes_of<N, T, K, P>, &slots_of<N, T, K, P>}
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

int variant_slots_per_cu(int n_words, int tps, int k, int wpb) {
    for (const Variant &v : kVariants)
        if (v.N == n_words && v.tps == tps && v.k == k && v.wpb == wpb &&
            v.lds() + 64 <= kLdsBytes)
            return v.slots();
    return 0;
}

hipError_t launch_jump(const JumpItem *items, uint32_t n_items, int num_cus, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    static bool attr_set = false;  // benign race: idempotent attribute
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)jump_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           JUMP_LDS_BYTES);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int grid = (int)((n_items + JUMP_WAVES - 1) / JUMP_WAVES);
    const int cap = num_cus * 3;  // three blocks of 48 KB planes fit a CU's LDS

    if (grid > cap) grid = cap;
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(jump_kernel, dim3(grid), dim3(64 * JUMP_WAVES), JUMP_LDS_BYTES, s, items,
                       n_items);
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

hipError_t launch_clear(uint32_t *p, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_header(uint32_t *hdr, uint64_t tag, bool clear_errors, hipStream_t s) {
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(header_kernel, dim3(1), dim3(64), 0, s, hdr, (uint32_t)tag,
                       (uint32_t)(tag >> 32), clear_errors ? 1u : 0u);
    return hipGetLastError();
}

hipError_t launch_stamp(uint64_t *dst, hipStream_t s) {
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(64), 0, s, dst);
    return hipGetLastError();
}

// The device API reads the same parameter blocks the library writes.
static_assert(MTGP_DP_N == P_N && MTGP_DP_POS == P_POS && MTGP_DP_SH1 == P_SH1 &&
                  MTGP_DP_SH2 == P_SH2 && MTGP_DP_MASK == P_MASK && MTGP_DP_REC == P_REC &&
                  MTGP_DP_TMP == P_TMP && MTGP_DP_FLT == P_FLT && MTGP_DP_WORDS == P_WORDS,
              "device API parameter layout");

// Generation through the device-side draw API: workgroup k owns stream k and
// writes count outputs at out + k*count, drawing blockDim.x at a time.
__global__ void __launch_bounds__(1024)
workgroup_kernel(const uint32_t *__restrict__ params, uint32_t *__restrict__ states,
                 uint32_t stride, uint64_t count, uint32_t *__restrict__ out, uint32_t f32,
                 uint32_t lds_words) {
    extern __shared__ uint32_t lds[];
    mtgp_device_stream s;
    const uint32_t k = blockIdx.x;
    uint32_t *row = states + (uint64_t)k * stride;
    mtgp_device_begin(s, params, k, row, lds, lds_words);
    gptr<uint32_t> o = (gptr<uint32_t>)(out + (uint64_t)k * count);
    for (uint64_t done = 0; done < count; done += blockDim.x) {
        const uint64_t rem = count - done;
        const uint32_t n = rem < blockDim.x ? (uint32_t)rem : blockDim.x;
        const uint32_t r = f32 ? mtgp_device_draw_bits<true>(s, n)
                               : mtgp_device_draw_bits<false>(s, n);
        if (threadIdx.x < n) o[done + threadIdx.x] = r;
    }
    mtgp_device_end(s, row);
}

hipError_t launch_workgroup(const uint32_t *params, uint32_t *states, uint32_t stride,
                            uint32_t n_streams, uint64_t count, uint32_t *out, uint32_t f32,
                            uint32_t threads, uint32_t n_words, hipStream_t s) {
    const uint32_t words = MTGP_DEVICE_LDS_WORDS(n_words, threads);
    static bool attr_set = false;  // benign race: idempotent attribute
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)workgroup_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)MTGP_DEVICE_LDS_WORDS(1391u, 1024u) * 4);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(workgroup_kernel, dim3(n_streams), dim3(threads), (size_t)words * 4, s,
                       params, states, stride, count, out, f32, words);
    return hipGetLastError();
}

// Screening statistics over generated uint32 outputs, one workgroup per
// stream of `count` words at out + k*count:
//  gap test (Knuth, Sec. 3.3.2 D, between consecutive hits): a hit is a word
//    in [lo, hi); the gap between consecutive hits j < j' is j' - j - 1,
//    counted in bin min(gap, bins-1);
//  Hamming-weight dependency: the weight class of a word (popcount <= 14,
//    15..17, >= 18) and of its successor, counted in a 3x3 table.
// counts[k * (bins + 9) ..] = gap bins, then the table row-major.
// Wave w takes the region [w R, (w+1) R) of the stream (R a multiple of 64)
// and reads it 64 consecutive words per load, SCREEN_LOADS loads per pass,
// so the pass streams from HBM.  In a 64-word slice the hit lanes form a
// ballot mask: a hit's previous hit is the highest hit lane below it, else
// the wave's last hit so far.  Each lane counts the weight pair that ends at
// its word (its predecessor's class from the lane below, lane 0's from the
// previous slice's last word) in a register of nine 7-bit fields, added
// into plain counters every 127 slices, so the counting is vector work.
// Gaps and pairs across regions are added at the end, in region order.
constexpr int SCREEN_WAVES = 4;
constexpr int SCREEN_THREADS = 64 * SCREEN_WAVES;
constexpr int SCREEN_LOADS = 8;
constexpr uint32_t SCREEN_NONE = 0xFFFFFFFFu;  // no hit yet (positions < count < 2^32)

__device__ __forceinline__ uint32_t weight_class(uint32_t v) {
    const uint32_t w = (uint32_t)__builtin_popcount(v);
    return w <= 14u ? 0u : (w <= 17u ? 1u : 2u);
}

__global__ void __launch_bounds__(SCREEN_THREADS)
screen_kernel(const uint32_t *__restrict__ out, uint64_t count, uint32_t lo, uint32_t hi,
              uint32_t bins, uint64_t *__restrict__ counts) {
    __shared__ uint32_t hist[64 + 9];
    __shared__ uint32_t first_hit[SCREEN_WAVES], last_hit[SCREEN_WAVES];
    const uint32_t k = blockIdx.x, tid = threadIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63u;
    for (uint32_t i = tid; i < bins + 9; i += SCREEN_THREADS) hist[i] = 0;
    __syncthreads();
    gptr<const uint32_t> x = (gptr<const uint32_t>)(out + (uint64_t)k * count);
    const uint64_t R = (count + 64 * SCREEN_WAVES - 1) / (64 * SCREEN_WAVES) * 64;
    const uint64_t r0 = (uint64_t)wave * R < count ? (uint64_t)wave * R : count;
    const uint64_t r1 = r0 + R < count ? r0 + R : count;
    const uint32_t span = hi - lo;  // a hit: v - lo < span
    const uint64_t lanes_below = lane ? ~0ull >> (64u - lane) : 0ull;
    uint32_t carry = SCREEN_NONE, first = SCREEN_NONE;
    uint32_t prev_cls = 3u;  // class of the previous full slice's last word; 3 = none
    uint32_t hw[9] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};  // this lane's pair counts
    uint64_t packed = 0;     // pair counts of the slices since the last flush, 7 bits each
    uint32_t since = 0;      // slices since the last flush (uniform)
    for (uint64_t b0 = r0; b0 < r1; b0 += 64 * SCREEN_LOADS) {
        uint32_t v[SCREEN_LOADS];
#pragma unroll
        for (int e = 0; e < SCREEN_LOADS; ++e) {
            const uint64_t j = b0 + 64u * e + lane;
            v[e] = j < r1 ? x[j] : 0u;
        }
#pragma unroll
        for (int e = 0; e < SCREEN_LOADS; ++e) {
            const uint64_t base = b0 + 64u * e;
            if (base >= r1) break;  // uniform
            const uint64_t j = base + lane;
            const bool valid = j < r1;
            const bool hit = valid && v[e] - lo < span;
            const uint64_t m = __builtin_amdgcn_ballot_w64(hit);
            if (hit) {
                const uint64_t bm = m & lanes_below;
                const uint32_t prev = bm ? (uint32_t)base + 63u - (uint32_t)__builtin_clzll(bm)
                                         : carry;
                if (prev != SCREEN_NONE) {
                    const uint32_t gap = (uint32_t)j - prev - 1u;
                    atomicAdd(&hist[gap < bins - 1u ? gap : bins - 1u], 1u);
                }
            }
            if (m) {
                if (first == SCREEN_NONE) first = (uint32_t)base + (uint32_t)__builtin_ctzll(m);
                carry = (uint32_t)base + 63u - (uint32_t)__builtin_clzll(m);
            }
            // the pair (j-1, j): j-1's class from the lane below, lane 0's
            // from the previous slice (3 at the region's start: no pair)
            const uint32_t c = weight_class(v[e]);
            const uint32_t below_c = (uint32_t)__shfl_up((int)c, 1, 64);
            const uint32_t pc = lane ? below_c : prev_cls;
            if (valid && pc < 3u) packed += 1ull << (7u * (3u * pc + c));
            // a full slice's last word precedes the next slice's first
            prev_cls = base + 64u <= r1 ? (uint32_t)__shfl((int)c, 63, 64) : 3u;
            if (++since == 127u) {
#pragma unroll
                for (int q = 0; q < 9; ++q) hw[q] += (uint32_t)(packed >> (7 * q)) & 127u;
                packed = 0;
                since = 0;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        hw[q] += (uint32_t)(packed >> (7 * q)) & 127u;
        if (hw[q]) atomicAdd(&hist[bins + q], hw[q]);
    }
    if (lane == 0) {
        first_hit[wave] = first;
        last_hit[wave] = carry;
    }
    __syncthreads();
    if (tid == 0) {
        // gaps across regions, in region order
        uint32_t pl = SCREEN_NONE;
        for (int w = 0; w < SCREEN_WAVES; ++w) {
            if (first_hit[w] == SCREEN_NONE) continue;
            if (pl != SCREEN_NONE) {
                const uint32_t gap = first_hit[w] - pl - 1u;
                hist[gap < bins - 1u ? gap : bins - 1u] += 1u;
            }
            pl = last_hit[w];
        }
        // weight pairs across regions
        for (int w = 0; w + 1 < SCREEN_WAVES; ++w) {
            const uint64_t e = (uint64_t)(w + 1) * R;
            if (e < count) hist[bins + 3u * weight_class(x[e - 1]) + weight_class(x[e])] += 1u;
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < bins + 9; i += SCREEN_THREADS)
        counts[(uint64_t)k * (bins + 9) + i] = hist[i];
}

hipError_t launch_screen(const uint32_t *out, uint32_t n_streams, uint64_t count, uint32_t lo,
                         uint32_t hi, uint32_t bins, uint64_t *counts, hipStream_t s) {
    (void)hipGetLastError();  // report this launch only
    hipLaunchKernelGGL(screen_kernel, dim3(n_streams), dim3(SCREEN_THREADS), 0, s, out, count,
                       lo, hi, bins, counts);
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
