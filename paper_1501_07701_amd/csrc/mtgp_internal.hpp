// mtgp_internal.hpp -- declarations shared by the kernels and the host
// library (never installed; the public interface is include/mtgp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mtgp {

// Device parameter block: 1024 words (4 KB) per stream.
enum : uint32_t {
    P_MEXP = 0,
    P_N = 1,
    P_POS = 2,
    P_SH1 = 3,
    P_SH2 = 4,
    P_MASK = 5,
    P_W = 6,
    P_SEED = 7,
    P_LIN = 8,     // 1 if the recursion table is GF(2)-linear (rec[i^j] = rec[i]^rec[j])
    P_RB = 9,      // its basis: rec[1], rec[2], rec[4], rec[8] (words 9..12)
    P_REC = 16,
    P_TMP = 32,
    P_FLT = 48,
    // windowed small-step path (linear recursion table, W < 64)
    P_WIN_WN = 64,       // window length (<= N-1)
    P_WIN_E = 65,        // elements per lane and window
    P_WIN_Q = 66,        // lanes per residue class (64 / W)
    P_WIN_ROUNDS = 67,   // cross-lane scan rounds, ceil(log2 q)
    P_WIN_MAT = 128,     // nibble tables of M^(E*2^r): [round][nibble][16]
    P_WORDS = 1024,      // 4 KB per stream
};
constexpr int WIN_EMAX = 8;
constexpr int WIN_MAXROUNDS = 5;
constexpr int WIN_MAT_WORDS = 128;   // 8 nibbles x 16 entries

// BatchItem.mode bits
enum : uint32_t {
    MODE_F32 = 1u,     // float32 output (else uint32)
    MODE_RAW = 2u,     // also store the raw words x_0 .. x_{N+count-1} at raw
    MODE_VERIFY = 4u,  // compare the end state with verify[0..N), count mismatches
};

// Device work-list entry (80 bytes): advance a stream from state_in by
// `count` outputs written to `out`, store the end state at state_out.
struct BatchItem {
    uint32_t stream;
    uint32_t mode;
    uint64_t count;
    uint64_t out;        // device address of the outputs
    uint64_t state_in;   // N words
    uint64_t state_out;  // N words, or 0
    uint64_t raw;        // MODE_RAW destination
    uint64_t verify;     // MODE_VERIFY reference state
    uint64_t flag;       // 0, or a host-mapped uint32 set to 1 when the request is done
    uint64_t countdown;  // 0, or a device uint32 of segments still running for
                         // this request: the segment that ends it raises `flag`
    uint64_t reserved;
};
static_assert(sizeof(BatchItem) == 80, "BatchItem layout");

// Jump evaluation item (32 bytes): out[m] = XOR_{i < nbits, g_i = 1}
// raw[1 + i + m] for m < m_count.
// Jump items are launched in blocks of JUMP_BLOCK: the items of a block
// share raw, nbits and m (one stream); null items (out == 0) pad a block and
// the first item of a block is never null.
constexpr int JUMP_BLOCK = 4;
struct JumpItem {
    uint64_t raw;     // words x_0, x_1, ... of a stream (at least nbits + m + 1)
    uint64_t poly;    // coefficients g_0 .. g_{nbits-1}, 32 per uint32 word
    uint64_t out;     // m words; 0 = padding
    uint32_t nbits;
    uint32_t m;
};
static_assert(sizeof(JumpItem) == 32, "JumpItem layout");

struct LaunchArgs {
    const uint32_t *params;
    const BatchItem *items;  // nullptr: plain mode, item i is stream i
    uint32_t n_items;
    uint32_t *plain_states;  // plain mode: state rows, outputs, count, dtype
    uint32_t plain_stride;
    uint32_t *plain_out;
    uint64_t plain_count;
    uint32_t plain_mode;
    uint32_t *counter;
    uint32_t *err;
    uint32_t win_below;      // window path for eligible streams with W below this
    bool persistent;
    int num_cus;
    void *stream;
};

struct VariantInfo {
    int tps, k, wpb;
    size_t lds_bytes;
};

int variant_count(int n_words, VariantInfo *out, int max_out);
hipError_t launch_variant(int n_words, int tps, int k, int wpb, const LaunchArgs &a,
                          bool *found);
hipError_t launch_jump(const JumpItem *items, uint32_t n_items, int num_cus, hipStream_t s);
int variant_slots_per_cu(int n_words, int tps, int k, int wpb);
hipError_t launch_seed(const uint32_t *params, uint32_t *states, uint32_t stride,
                       uint32_t n_streams, hipStream_t s);
hipError_t launch_reset(uint32_t *counter, hipStream_t s);
// Batch workspace header: claim counters (words 0, 1), segment-check errors
// (word 2), phase timestamps (64-bit words from byte HDR_STAMP_BYTE: start,
// after the prefix items, after the jumps, end).
constexpr size_t HDR_STAMP_BYTE = 64;
hipError_t launch_stamp(uint64_t *dst, hipStream_t s);
hipError_t launch_workgroup(const uint32_t *params, uint32_t *states, uint32_t stride,
                            uint32_t n_streams, uint64_t count, uint32_t *out, uint32_t f32,
                            uint32_t threads, uint32_t n_words, hipStream_t s);
hipError_t launch_screen(const uint32_t *out, uint32_t n_streams, uint64_t count, uint32_t lo,
                         uint32_t hi, uint32_t bins, uint64_t *counts, hipStream_t s);
hipError_t launch_fill(uint32_t *out, uint64_t n_words, uint32_t value, int num_cus,
                       hipStream_t s);

}  // namespace mtgp
