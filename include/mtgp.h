/*
 * mtgp.h -- C ABI of the MI355X (gfx950) MTGP32 bulk generator.
 *
 * Model (Passerat-Palmbach et al., ESM 2010):
 *   - A generator is a seed status plus a parameterised status (Sec. 3.1):
 *     here a uint32 seed plus an `mtgp_params` record.
 *   - Every generator is an independent stream owned by one GPU thread group,
 *     its state manipulated in on-chip shared memory (LDS) and kept in device
 *     memory between calls (Sec. 2, Sec. 3.2).
 *   - The CPU and GPU produce the same numbers (Sec. 3.2): every output of
 *     this library is bit-identical to a plain CPU evaluation of the
 *     definition below.
 *
 * Definition computed (the paper leaves the word-level recurrence to Saito's
 * MTGP; this is the published MTGP32 form).  For a stream with N state words
 * x_j .. x_{j+N-1}, N = floor(mexp/32)+1, W = N - pos:
 *     X   = (x_j & mask) ^ x_{j+1};   X ^= X << sh1;
 *     Y   = X ^ (x_{j+pos} >> sh2);   x_{j+N} = Y ^ rec_tbl[Y & 15];
 *     H   = x_{j+pos-1};  H ^= H >> 16;  H ^= H >> 8;  t = H & 15;
 *     u32 output j = x_{j+N} ^ tmp_tbl[t]
 *     f32 output j = as_float((x_{j+N} >> 9) ^ flt_tbl[t]) - 1.0f   (in [0,1))
 * Initial state from a seed (Mersenne Twister initialisation):
 *     x_0 = seed;  x_i = 1812433253 * (x_{i-1} ^ (x_{i-1} >> 30)) + i.
 *
 * Conventions
 *   - Device pointers (prefix d_) are allocated and owned by the caller; the
 *     library borrows them for the duration of the call (and, for the
 *     server, until mtgp_server_destroy).  Host pointers (prefix h_) are
 *     read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls are asynchronous and stream-ordered unless stated otherwise.
 *     The calls that synchronise are set-up and host-transfer calls
 *     (mtgp_init_states, mtgp_load_params, mtgp_batch_workspace_query,
 *     mtgp_stream_polynomials, mtgp_autotune, mtgp_state_export/import,
 *     mtgp_batch_errors, mtgp_batch_phase_times), mtgp_generate_batch when
 *     it first builds a stream's jump-ahead polynomial, and the server's
 *     mtgp_wait, mtgp_server_replay and mtgp_server_destroy.
 *   - Every function returns MTGP_OK (0) or a negative MTGP_E* code; nothing
 *     is launched when validation fails.  mtgp_last_error_detail() gives a
 *     thread-local human-readable reason for the last failure.
 *   - One parameter set (all streams passed to mtgp_init_states together)
 *     shares one mexp in {3217, 11213, 23209, 44497}.
 *   - Each call advances each touched stream by exactly the number of
 *     outputs it produces, whatever the dtype.
 */
#ifndef MTGP_H
#define MTGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameterised status of one generator (Sec. 3.1), 212 bytes, host side.
 * rec_tbl: recursion table; tmp_tbl: uint32 tempering table; flt_tbl: float
 * tempering table, each entry with sign 0 and exponent 0x7F (bits 31..23 ==
 * 0x7F) so that the float lies in [1,2) before the subtraction of 1.0. */
typedef struct mtgp_params {
    uint32_t mexp, pos, sh1, sh2, mask;
    uint32_t rec_tbl[16], tmp_tbl[16], flt_tbl[16];
} mtgp_params;

enum {
    MTGP_OK = 0,
    MTGP_EINVAL = -1,     /* bad argument or parameter set                 */
    MTGP_ENOMEM = -2,     /* host allocation failed                        */
    MTGP_EDEVICE = -3,    /* HIP runtime error                             */
    MTGP_ETOOBIG = -4,    /* request larger than the server's output pool  */
    MTGP_EAGAIN = -5,     /* server queue full / try again                 */
    MTGP_ENOENT = -6,     /* unknown ticket                                */
    MTGP_ECANCELED = -7,  /* request cancelled (server destroyed)          */
    MTGP_ETIMEDOUT = -8   /* wait deadline passed                          */
};

enum { MTGP_U32 = 0, MTGP_F32 = 1 };

/* Bytes of device memory one stream's parameter block takes (4096): the
 * parameters plus derived data (for linear recursion tables with a short
 * step width, the 32x32 GF(2) matrix powers the windowed path uses). */
#define MTGP_DEVICE_PARAM_BYTES 4096

/* N = floor(mexp/32)+1 for a supported mexp, else MTGP_EINVAL. */
int mtgp_state_words(uint32_t mexp);

/* Validates n host parameter sets: supported mexp, one mexp for all, mask ==
 * 0xFFFFFFFF << (32N - mexp), 1 <= pos <= N-2, sh1, sh2 <= 31, float-table
 * exponent bits 0x7F.  MTGP_OK or MTGP_EINVAL (detail names stream + field). */
int mtgp_check_params(const mtgp_params *h_params, int n_streams);

/* Seed status -> initial state for every stream (Sec. 3.1, Sec. 5.1).
 * Like mtgp_load_params, this is a set-up call that synchronises.
 *   h_params   : n_streams parameter sets (validated first).
 *   h_seeds    : n_streams seeds (uint32).
 *   d_params   : device buffer of n_streams * MTGP_DEVICE_PARAM_BYTES bytes,
 *                written with the library's packed parameter layout.
 *   d_states   : device buffer of n_streams * state_stride uint32; row k
 *                receives x_0..x_{N-1} of stream k.
 *   state_stride >= N (words between consecutive rows).
 * Synchronises `stream` before returning (the host staging buffer is freed).
 * The library keeps a host copy of the parameter sets, keyed by d_params,
 * which generate/batch/server calls use for launch planning. */
int mtgp_init_states(const mtgp_params *h_params, const uint32_t *h_seeds,
                     int n_streams, void *d_params, uint32_t *d_states,
                     int state_stride, void *stream);

/* Re-seeds streams 0..n_streams-1 from the seeds stored in d_params by
 * mtgp_init_states (device only, asynchronous): the states return to the
 * streams' seed status (Sec. 3.1). */
int mtgp_seed_states(const void *d_params, uint32_t *d_states, int state_stride,
                     int n_streams, void *stream);

/* Uploads parameter sets without touching states (e.g. before importing
 * checkpointed states).  Same layout and synchronisation as above.  The
 * stored seeds are 0 (mtgp_seed_states then seeds every stream with 0);
 * jump-ahead polynomials are built from the streams' states as found in
 * d_states when they are first split. */
int mtgp_load_params(const mtgp_params *h_params, int n_streams,
                     void *d_params, void *stream);

/* Forgets the host copy kept for d_params (call before freeing it). */
int mtgp_release_params(const void *d_params);

/* Plain bulk generation, one launch, one thread group per stream (Sec. 2):
 * advances streams 0..n_streams-1 of the set by `count_per_stream` outputs
 * each and writes output j of stream k to d_out[k * count_per_stream + j]
 * (stream-major, 64-bit indexing).  d_states rows are updated in place.
 * d_out must hold n_streams * count_per_stream words.  No stream is split
 * and nothing is allocated, so the call lasts as long as its slowest
 * stream (the narrowest step width); mtgp_generate_batch with a workspace
 * sized by mtgp_batch_workspace_query splits long streams by jump-ahead. */
int mtgp_generate_u32(const void *d_params, uint32_t *d_states,
                      int state_stride, int n_streams,
                      uint64_t count_per_stream, uint32_t *d_out, void *stream);
int mtgp_generate_f32(const void *d_params, uint32_t *d_states,
                      int state_stride, int n_streams,
                      uint64_t count_per_stream, float *d_out, void *stream);

/* One request of a batch: advance `stream_id` by `count` outputs of `dtype`
 * and write them contiguously at d_out. */
typedef struct mtgp_work {
    int32_t stream_id;
    uint32_t dtype;       /* MTGP_U32 or MTGP_F32 */
    uint64_t count;
    void *d_out;
} mtgp_work;

/* Smallest workspace mtgp_generate_batch accepts for n_items requests (no
 * stream is split into jump-ahead segments with this much). */
size_t mtgp_batch_workspace_bytes(int n_items);

/* Workspace bytes that let this batch split every long stream into the
 * jump-ahead segments the current tuning asks for.  Builds the seeded
 * streams' jump-ahead polynomials first (device work + host polynomial
 * arithmetic, once per stream; synchronises the device).  Streams whose
 * polynomial must come from their current state (after an import) are
 * sized for the largest polynomial. */
int mtgp_batch_workspace_query(const void *d_params, const mtgp_work *h_items,
                               int n_items, size_t *bytes);

/* Batched generation: one persistent kernel advances many streams with
 * uneven lengths and mixed dtypes in a single launch, replayed from a
 * hipGraph captured once per (buffers, plan, tuning).  Items are scheduled
 * longest-critical-path first.  A stream id may appear at most once per
 * call.  When a batch has both split (see below) and whole requests, the
 * whole requests run beside the jump-ahead evaluation on a second HIP
 * stream the library owns per workspace (joined back into `stream` before
 * the call's last kernel; launched directly, not from a graph, and not
 * while `stream` is being captured).  MTGP_OVERLAP=0 in the environment
 * turns this off.
 *
 * Jump-ahead (not in the paper; the generator's GF(2)-linearity makes it
 * exact): a stream whose request needs more dependent steps than the
 * batch's target (see mtgp_tuning) is cut into segments that run in
 * parallel.  Their start states are XOR-combinations of the stream's first
 * words given by x^(J-1) mod p, p an annihilating polynomial of the
 * stream's word sequence found by Berlekamp-Massey and checked on the
 * device.  p is built once per stream from its seed status's orbit while
 * the stream's state was last set by seeding, and from the orbit of its
 * current state after mtgp_load_params or mtgp_state_import (rebuilt as
 * the lcm with the old one).  Each segment checks its final state against
 * the next segment's start; if any check fails (a state written into
 * d_states behind the library's back, or overwritten workspace contents),
 * the device regenerates the whole request in order from its start state
 * before the call's kernels end, so outputs and final states are always
 * those of unsplit generation.  Such repairs are counted in the workspace
 * (mtgp_batch_errors), which also makes the library rebuild those streams'
 * polynomials from their current states.
 *
 * d_workspace: workspace_bytes (>= mtgp_batch_workspace_bytes(n_items)) of
 * device memory the caller owns, 256-byte aligned; splitting is reduced to
 * fit.  Its first 256 bytes hold claim counters, the repair count and
 * phase timestamps.  Every call uploads the plan's item tables (an async
 * copy from pinned host memory on `stream`, ahead of the kernels); the jump
 * polynomials are uploaded only when the plan changes, so keep the
 * workspace's contents between calls for speed (results do not depend on
 * it).  Calls on one workspace must not overlap.
 *
 * Asynchronous, except that planning a stream's first split (or a split
 * after an import) builds its polynomial: device work on `stream` plus
 * host Berlekamp-Massey, which synchronises `stream` (milliseconds per
 * stream; call mtgp_batch_workspace_query beforehand to do it up front). */
int mtgp_generate_batch(const void *d_params, uint32_t *d_states,
                        int state_stride, const mtgp_work *h_items,
                        int n_items, void *d_workspace, size_t workspace_bytes,
                        void *stream);

/* Bytes of the static device scratch that mtgp_generate_batch_noalloc uses
 * as its batch workspace (64 MiB, one per GPU, held until the process
 * ends). */
#define MTGP_NOALLOC_SCRATCH_BYTES (64u << 20)

/* mtgp_generate_batch for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same generation, results and state advance, with the
 * batch workspace in a static device array of MTGP_NOALLOC_SCRATCH_BYTES
 * per GPU instead of a caller buffer.  It calls no hipMalloc, hipFree,
 * pinned-host or other device-allocating routine (its plan is staged in
 * ordinary host memory and copied with hipMemcpyAsync, kernels are
 * launched directly): streams are split by jump-ahead only where their
 * polynomial already exists (built by an earlier mtgp_generate_batch or
 * mtgp_batch_workspace_query on the same parameter set) and only as far as
 * the scratch holds the plan.  MTGP_ETOOBIG if even the unsplit plan of
 * n_items requests exceeds the scratch (more than about 838,000 items).
 * Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's contents: calls that overlap on one GPU race (issue them on one
 * stream, or synchronise between them).  Repairs after a failed segment
 * check keep results exact but are not reported by this entry point. */
int mtgp_generate_batch_noalloc(const void *d_params, uint32_t *d_states,
                                int state_stride, const mtgp_work *h_items,
                                int n_items, void *stream);

/* Phase timing, for measurement.  While enabled (process-wide; default
 * off), every mtgp_generate_batch call writes four device wall-clock
 * timestamps into its workspace header: at its start, after the launch
 * that runs the prefix items and the jump-ahead evaluation, after the
 * segments and at its end (after the request checks).  Each costs a
 * one-thread kernel launch between the phases, so leave it off for timed
 * runs.  Always MTGP_OK. */
int mtgp_set_phase_timing(int enable);

/* Synchronises `stream` and returns in h_us[0..2] the durations in
 * microseconds of the prefix-and-jump launch, the segment launch and the
 * request checks of the last batch call on d_workspace that ran with phase
 * timing enabled.  MTGP_EINVAL if the workspace holds no timestamps. */
int mtgp_batch_phase_times(void *d_workspace, void *stream, double *h_us);

int mtgp_batch_errors(void *d_workspace, void *stream, uint32_t *n);

/* Launch tuning for one mexp: threads per stream (64 = one wave per stream,
 * several streams per workgroup; 256/512/1024 = one stream per workgroup),
 * outputs per lane per step, and workgroup size. */
typedef struct mtgp_tuning {
    int threads_per_stream;
    int outputs_per_lane;
    int workgroup_size;
    int jump_target_steps;  /* 0 = never split streams by jump-ahead; else the
                               least number of dependent steps per segment:
                               a batch splits the streams that need more
                               steps than max(this, a multiple (0.75 to
                               1.25) of its total steps over the streams
                               the device runs at once) */
    int window_below_w;     /* with threads_per_stream = 64, streams with a
                               linear rec_tbl and step width W = N - pos below
                               this (at most 64) run the windowed scan instead
                               of W-word steps; 0 = never */
} mtgp_tuning;

int mtgp_get_tuning(uint32_t mexp, mtgp_tuning *out);
int mtgp_set_tuning(uint32_t mexp, const mtgp_tuning *t);
/* Number of candidate tunings compiled in for mexp, and candidate i. */
int mtgp_tuning_candidates(uint32_t mexp, mtgp_tuning *out, int max_out);

/* Autotuner: times every compiled launch candidate on the given batch (run
 * on a scratch copy of the states, so the caller's states are untouched),
 * then the jump-ahead target steps in {0, 1024, 2048, 4096, 8192, 16384,
 * 65536} and window_below_w in {0, 16, 24, 32, 48, 64} with the fastest
 * candidate, keeps the fastest combination as the tuning for this
 * mexp and returns it in *best.  d_scratch holds n_streams * state_stride * 4
 * bytes (rounded up to 256) followed by the batch workspace;
 * scratch_bytes is its size.  Output buffers named by the items are
 * overwritten.  Synchronises `stream`.  h_ms (may be NULL) receives up to
 * max_out per-candidate times in ms, in mtgp_tuning_candidates order. */
int mtgp_autotune(const void *d_params, const uint32_t *d_states,
                  int state_stride, const mtgp_work *h_items, int n_items,
                  void *d_scratch, size_t scratch_bytes, int reps, void *stream,
                  mtgp_tuning *best, float *h_ms, int max_out);

/* Checkpoint: copy n_streams state rows device -> host (h_out holds
 * n_streams * N words, densely packed) and back.  Synchronise `stream`.
 * This is the paper's persistence of generator state in global memory
 * between launches (Sec. 2).  Imported streams get their jump-ahead
 * polynomial rebuilt from the imported state when next split. */
int mtgp_state_export(const void *d_params, const uint32_t *d_states,
                      int state_stride, int n_streams, uint32_t *h_out,
                      void *stream);
int mtgp_state_import(const void *d_params, uint32_t *d_states,
                      int state_stride, int n_streams, const uint32_t *h_in,
                      void *stream);

/* Generation through the device-side draw API of mtgp_device.h: one
 * workgroup of `threads` threads (a multiple of 64 in [64, 1024]) per stream
 * keeps the stream's state in LDS and draws `threads` outputs per call
 * (the paper's per-block consumer, Sec. 2 and Sec. 3.2).  Same outputs,
 * layout (out[k * count + j]) and state advance as mtgp_generate_u32/f32
 * for dtype MTGP_U32/MTGP_F32; it also serves as the reference user of that
 * API.  MTGP_EINVAL on a bad argument. */
int mtgp_generate_workgroup(const void *d_params, uint32_t *d_states,
                            int state_stride, int n_streams,
                            uint64_t count_per_stream, int dtype, int threads,
                            void *d_out, void *stream);

/* Minimal polynomial of each stream's output word sequence from its seed
 * status (the polynomial the jump-ahead uses; Berlekamp-Massey on the host,
 * checked on the device to annihilate the word sequence; for a stream
 * whose states were imported it also covers the imported states' orbits,
 * and it is -1 until such a stream was first split).  For parameter
 * sets from the Dynamic Creator it is the characteristic polynomial of the
 * generator, whose uniqueness across a set is what makes the streams
 * distinct (Sec. 3.2): equal polynomials flag duplicate generators.
 * Streams [0, n_streams): h_degrees[k] = degree (<= mexp), or -1 when no
 * polynomial could be verified; h_coeffs[k * words_per_stream ..] holds the
 * coefficients, bit i (word i/32, bit i%32) = coefficient of x^i,
 * words_per_stream >= mexp/32 + 1.  Synchronous (runs device work on
 * `stream`; the result is cached per parameter set). */
int mtgp_stream_polynomials(const void *d_params, int n_streams,
                            uint32_t *h_coeffs, int words_per_stream,
                            int *h_degrees, void *stream);

/* Screening statistics of generated uint32 outputs (informative, not a
 * quality certificate; the paper screens statuses with TestU01's gap and
 * Hamming-weight tests, Sec. 4 and 5).  For stream k, the count_per_stream
 * words at d_outputs + k * count_per_stream:
 *   gap test (Knuth, Sec. 3.3.2 D, gaps between consecutive hits): a hit is
 *     a word in [gap_lo, gap_hi); the gap between consecutive hits j < j' is
 *     j' - j - 1, counted in bin min(gap, gap_bins - 1);
 *   Hamming-weight dependency: the weight class (popcount <= 14, 15..17,
 *     >= 18) of each word and of the next one, counted in a 3x3 table.
 * d_counts[k * (gap_bins + 9) ..] = the gap_bins gap counts, then the table
 * row-major (device memory the caller owns; overwritten).  2 <= gap_bins
 * <= 64, gap_lo < gap_hi, 2 <= count_per_stream < 2^32.  MTGP_EINVAL on a
 * bad argument. */
int mtgp_screen(const uint32_t *d_outputs, int n_streams,
                uint64_t count_per_stream, uint32_t gap_lo, uint32_t gap_hi,
                int gap_bins, uint64_t *d_counts, void *stream);

/* Store-only fill of n words (bandwidth reference for the roofline). */
int mtgp_fill_u32(uint32_t *d_out, uint64_t n_words, uint32_t value,
                  void *stream);

/* ------------------------------------------------------------ serving --
 * A request loop over resident stream states: requests (stream, count,
 * dtype) are admitted while their output bytes fit a caller-owned device
 * pool, served in submission order per stream, batched with whatever else
 * is waiting or running, and launched through the persistent kernel on
 * several HIP streams so that work admitted later overlaps earlier work.
 * Each result is exactly the next `count` outputs of its stream. */
typedef struct mtgp_server mtgp_server;

typedef struct mtgp_server_opts {
    int max_inflight_batches;  /* concurrent launches (HIP streams), >= 1  */
    int max_batch_items;       /* requests per launch                      */
    int max_queue;             /* pending requests before MTGP_EAGAIN      */
    uint64_t batch_window_ns;  /* wait this long for more requests when a
                                  launch slot is free but the queue is short */
    uint64_t workspace_bytes_per_batch;  /* carved from the pool per launch
                                  slot; bounds jump-ahead splitting */
} mtgp_server_opts;

enum { MTGP_PENDING = 0, MTGP_DONE = 1, MTGP_FAILED = 2 };

int mtgp_server_create(const void *d_params, uint32_t *d_states,
                       int state_stride, int n_streams, void *d_pool,
                       uint64_t pool_bytes, const mtgp_server_opts *opts,
                       mtgp_server **out);
/* Queue a request; *ticket identifies it.  MTGP_ETOOBIG if count*4 bytes
 * exceed the pool, MTGP_EAGAIN if the queue is full. Thread-safe. */
int mtgp_submit(mtgp_server *srv, int32_t stream_id, uint64_t count,
                int dtype, uint64_t *ticket);
/* Queue n requests at once (stream_ids[i], counts[i], dtypes[i]; tickets[i]
 * receives each ticket), in order, as n mtgp_submit calls would; all or
 * none: every request is validated first, MTGP_EAGAIN if the queue lacks
 * room for all of them.  Thread-safe. */
int mtgp_submit_many(mtgp_server *srv, const int32_t *stream_ids,
                     const uint64_t *counts, const int *dtypes, int n,
                     uint64_t *tickets);
/* Non-blocking status; *d_result is the device address of the output once
 * MTGP_DONE (valid until mtgp_release). */
int mtgp_poll(mtgp_server *srv, uint64_t ticket, int *state,
              const void **d_result);
/* Block until done or timeout (0 = forever).  MTGP_ETIMEDOUT on deadline. */
int mtgp_wait(mtgp_server *srv, uint64_t ticket, uint64_t timeout_ns);
/* Return the request's output bytes to the pool and forget the ticket. */
int mtgp_release(mtgp_server *srv, uint64_t ticket);
/* Trace replay for serving measurements: submits request i (stream_ids[i],
 * counts[i], dtypes[i]) t_arrival_ns[i] after the call starts (arrivals
 * non-decreasing) from the calling thread, returns each result's pool
 * bytes as soon as it completes, and blocks until all are done.
 * h_latency_ns[i] = completion - scheduled arrival; h_stages_ns (3n, may be
 * NULL) = queued, admitted-to-launch and running time of each request.
 * d_keep (may be NULL): where d_keep[i] is not NULL, request i's result
 * (counts[i] * 4 bytes) is copied there (device memory the caller owns)
 * before its pool bytes are returned; other results are not kept. */
int mtgp_server_replay(mtgp_server *srv, const uint64_t *t_arrival_ns,
                       const int32_t *stream_ids, const uint64_t *counts,
                       const int *dtypes, int n, uint64_t *h_latency_ns,
                       uint64_t *h_stages_ns, void *const *d_keep);
/* Requests the server's batches regenerated on the device after a failed
 * jump-ahead segment check (their results are exact), since creation. */
int mtgp_server_repaired(mtgp_server *srv, uint64_t *n);
/* Per-request timestamps in ns since server creation: submitted, admitted
 * (pool bytes granted), launched, completed (observed by the server). */
int mtgp_request_times(mtgp_server *srv, uint64_t ticket, uint64_t *t_submit,
                       uint64_t *t_admit, uint64_t *t_launch,
                       uint64_t *t_done);
/* Stops the loop; queued requests never admitted end as MTGP_ECANCELED,
 * in-flight launches are waited for, and threads blocked in mtgp_wait
 * return (MTGP_ECANCELED for cancelled requests) before it frees the
 * server.  No call may start on the server once destroy has begun. */
int mtgp_server_destroy(mtgp_server *srv);

const char *mtgp_strerror(int code);
const char *mtgp_last_error_detail(void);

#ifdef __cplusplus
}
#endif
#endif /* MTGP_H */
