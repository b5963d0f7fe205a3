// mtgp_host.hpp -- host-side declarations shared by the C ABI, the batch
// planner and the serving runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <vector>

#include "mtgp.h"
#include "mtgp_internal.hpp"

namespace mtgp {

struct StreamJump;  // jump-ahead data of one stream (mtgp_batch.cpp)

// Host copy of what mtgp_init_states / mtgp_load_params wrote to a d_params
// buffer: enough to plan launches (state length, step widths), plus the
// lazily built jump-ahead data of each stream.
struct ParamSet {
    int n = 0;                 // streams
    int N = 0;                 // state words
    uint32_t mexp = 0;
    std::vector<uint32_t> W;   // step width N - pos per stream
    std::vector<uint8_t> lin;  // 1 where rec_tbl is linear (the windowed path applies)
    uint64_t generation = 0;   // changes whenever the parameter block is rewritten
    // Jump-ahead data per stream (guarded by jump_mu).  A stream's
    // polynomial annihilates the orbits it was built from; `seeded` says
    // whether the stream's state was last set from its seed status (so its
    // orbit is the seed's), `dirty` that the state may lie outside every
    // orbit the current polynomial was built from (after an import, a
    // parameter reload, or an observed segment-check failure).
    std::mutex jump_mu;
    std::vector<std::shared_ptr<StreamJump>> jumps;  // per stream, or null
    std::vector<uint8_t> seeded;
    std::vector<uint8_t> dirty;
};

// Marks streams [0, n) as seeded (mtgp_seed_states) or as holding states
// from elsewhere (mtgp_state_import), for the jump-ahead planner.
void note_states_seeded(ParamSet &ps, int n);
void note_states_foreign(ParamSet &ps, const int32_t *streams, int n);

// Pinned staging buffer for uploads; rewritten only once its last copy
// finished.
struct Staging {
    uint8_t *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    ~Staging();
};

// What the library keeps for one batch workspace: the pinned image of the
// last plan and where its parts lie.  Every call uploads the plan's item
// tables and request records (so a workspace whose memory was reused in
// between is rewritten before any kernel reads it); the jump polynomials
// are uploaded when the plan changes.  The caller holds `mu` for a call.
struct WsState {
    std::mutex mu;
    Staging stage;
    uint64_t sig = 0;          // plan signature, 0 = no plan
    uint32_t nA = 0, nB = 0, nC = 0, nF = 0;  // prefix, jump, segment, check items
    size_t off_A = 0, off_B = 0, off_C = 0, off_F = 0, off_jdep = 0, off_pflag = 0;
    // overlap: the plan's whole requests (after the nCs segments of split
    // requests in the segment list) start on `aux` beside the prefix and
    // jump launch, with at most overlap_groups workgroups per CU
    uint32_t nCs = 0;
    bool overlap = false;
    int overlap_groups = 0;
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    size_t tables_end = 0, up_end = 0;
    std::weak_ptr<ParamSet> ps;         // parameter set of the last plan
    std::vector<int32_t> split_streams;  // streams the last plan split
    // no_alloc: the plan is staged in `image` (ordinary host memory, which
    // hipMemcpyAsync has finished reading when it returns) instead of
    // pinned memory, and no jump-ahead data is built
    bool no_alloc = false;
    std::vector<uint8_t> image;
    ~WsState();
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int device_cus();
int words_for_mexp(uint32_t mexp);
std::shared_ptr<ParamSet> lookup_params(const void *d_params, int n_streams);
mtgp_tuning tuning_for(int N);
int launch_tuned(int N, const mtgp_tuning &t, const LaunchArgs &a);

// Outputs per step the generator achieves for step width W under a tuning.
uint64_t step_outputs(const ParamSet &ps, int stream, const mtgp_tuning &t);

// One request of a batch as the planner sees it.
struct Request {
    int32_t stream;
    uint32_t dtype;
    uint64_t count;
    void *d_out;
    uint64_t flag;       // host-mapped completion flag (server), or 0
};

// Plans, uploads and launches one batch.  Splits long streams into
// jump-ahead segments as far as ws_bytes allows.  The caller holds wst.mu.
// per_call_errors zeroes the workspace's repair count and log at the start
// of the call (else they accumulate until mtgp_batch_errors reads them).
// allow_overlap: whole requests may start beside the prefix and jump launch
// (on a second stream the workspace state owns; not while `s` is being
// captured, with phase timing on, or for no_alloc workspaces).
int run_batch(const std::shared_ptr<ParamSet> &ps, const void *d_params, uint32_t *d_states,
              int stride, const std::vector<Request> &reqs, void *d_ws, size_t ws_bytes,
              hipStream_t s, const mtgp_tuning &t, bool use_graph, WsState &wst,
              bool per_call_errors, bool allow_overlap);
// Streams named in a workspace header's repair log (all streams the plan
// split when the log overflowed) are marked dirty so that their jump-ahead
// polynomial is rebuilt from their current state.
void note_repairs(ParamSet &ps, const uint32_t *err_words, const std::vector<int32_t> &split);
size_t batch_min_ws_bytes(int n_items);
int validate_requests(const ParamSet &ps, const mtgp_work *items, int n);

}  // namespace mtgp
