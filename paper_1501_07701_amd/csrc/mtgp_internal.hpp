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
    MODE_VERIFY = 4u,  // compare the end state with verify[0..N); a mismatch
                       // marks the item's request record as failed
    MODE_FIXUP = 8u,   // request check (last launch of a batch): regenerate
                       // the request from its record if a segment failed,
                       // then raise `flag`
};

// Request record (64 bytes) of a request split by jump-ahead: its segments
// mark `failed` when a check fails, and the batch's last launch (after
// every segment has finished, so no later store can land on its outputs)
// regenerates such a request in order from `orig`.
struct ReqRec {
    uint32_t failed;     // nonzero once a segment's end state missed the next start
    uint32_t stream;
    uint32_t mode;       // MODE_F32 or 0
    uint32_t reserved0;
    uint64_t count;      // outputs of the whole request
    uint64_t out;        // device address of its first output
    uint64_t orig;       // N words: the stream's state when the request starts
    uint64_t row;        // where the request's final state goes
    uint64_t reserved[2];
};
static_assert(sizeof(ReqRec) == 64, "ReqRec layout");

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
    uint64_t rec;        // the request's ReqRec (MODE_VERIFY, MODE_FIXUP), or 0
    uint64_t flag;       // 0, or a host-mapped uint32 set to 1 when the request is done
    uint64_t reserved;
};
static_assert(sizeof(BatchItem) == 80, "BatchItem layout");

// Batch workspace header (256 bytes, never part of an uploaded plan):
//   word 0, 1   claim counters of the prefix and segment launches
//   word 2      requests regenerated after a failed segment check
//   word 3      entries written to the log (may exceed HDR_LOG_MAX)
//   word 4..11  stream ids of the first HDR_LOG_MAX such requests
//   word 12     claim counter of the request-check launch
//   word 13, 14 tag: a 64-bit value derived from the workspace address; a
//               header without it (fresh or reused memory) is cleared by
//               the first launch of the next call
//   word 15     claim counter of the jump blocks
//   byte 64..95 phase timestamps (64-bit: start, after the prefix and
//               jump launch, after the segments, end)
//   word 24     claim counter of the whole-request list when it runs beside
//               the prefix and jump launch
constexpr int HDR_ERR = 2;
constexpr int HDR_LOG_MAX = 8;
constexpr int HDR_ERR_WORDS = 2 + HDR_LOG_MAX;  // words HDR_ERR .. HDR_ERR + 9
constexpr int HDR_FIX_CLAIM = 12;
constexpr int HDR_TAG = 13;
constexpr int HDR_J_CLAIM = 15;
constexpr int HDR_W_CLAIM = 24;
constexpr size_t HDR_STAMP_BYTE = 64;
constexpr size_t HDR_BYTES = 256;

// Jump evaluation item (32 bytes): out[m] = XOR_{i < nbits, g_i = 1}
// raw[1 + i + m] for m < m_count.
// Jump items are launched in blocks of JUMP_BLOCK: the items of a block
// share raw, nbits and m (one stream); null items (out == 0) pad a block and
// the first item of a block is never null.
constexpr int JUMP_BLOCK = 4;
// Output words one jump item evaluates in a single pass over its
// coefficients; longer states are split into items of at most this many
// words (item p covers words p * JUMP_OUT_WORDS onwards, its raw pointer
// moved by as many words), so the passes of one jump run on different
// workgroups at once.
constexpr int JUMP_OUT_WORDS = 512;
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
    uint32_t *err;           // header word HDR_ERR (repair count, then the log)
    uint32_t win_below;      // window path for eligible streams with W below this
    int groups_per_cu;       // persistent launches: at most this many groups per CU (0 = occupancy)
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
// Persistent launches of the prefix kernel (items may carry MODE_RAW) and
// of the request-check kernel (MODE_FIXUP items) for state length n_words
// (one wave per item; a.win_below applies).
hipError_t launch_prefix(int n_words, const LaunchArgs &a);
// LDS bytes of one prefix-and-jump workgroup.
size_t prefix_jump_lds_bytes();
// Prefix items (nP, one wave each) and jump blocks (nJ items in blocks of
// JUMP_BLOCK; block b waits for pflag[jdep[b]]) in one persistent launch.
hipError_t launch_prefix_jumps(int n_words, const BatchItem *prefix, uint32_t nP,
                               const JumpItem *jumps, uint32_t nJ, const uint32_t *jdep,
                               uint32_t *pflag, const uint32_t *params, uint32_t *hdr,
                               uint32_t win_below, int num_cus, hipStream_t s);
hipError_t launch_check(int n_words, const LaunchArgs &a);
int variant_slots_per_cu(int n_words, int tps, int k, int wpb);
hipError_t launch_seed(const uint32_t *params, uint32_t *states, uint32_t stride,
                       uint32_t n_streams, hipStream_t s);
hipError_t launch_reset(uint32_t *counter, hipStream_t s);
// Zeroes n consecutive words with a small kernel (no memset node, so it is
// safe inside captured graphs).
hipError_t launch_clear(uint32_t *p, uint32_t n, hipStream_t s);
// First launch of every batch call: zeroes the claim counters; zeroes the
// repair count and log when clear_errors is set or the header lacks `tag`
// (then also the timestamps), and writes the tag.
hipError_t launch_header(uint32_t *hdr, uint64_t tag, bool clear_errors, hipStream_t s);
hipError_t launch_stamp(uint64_t *dst, hipStream_t s);
// Device address of the current GPU's static scratch array (looked up once
// per device).
hipError_t scratch_address(void **out);
hipError_t launch_workgroup(const uint32_t *params, uint32_t *states, uint32_t stride,
                            uint32_t n_streams, uint64_t count, uint32_t *out, uint32_t f32,
                            uint32_t threads, uint32_t n_words, hipStream_t s);
hipError_t launch_screen(const uint32_t *out, uint32_t n_streams, uint64_t count, uint32_t lo,
                         uint32_t hi, uint32_t bins, uint64_t *counts, hipStream_t s);
hipError_t launch_fill(uint32_t *out, uint64_t n_words, uint32_t value, int num_cus,
                       hipStream_t s);

}  // namespace mtgp
