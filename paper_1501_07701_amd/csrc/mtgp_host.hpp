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
    std::mutex jump_mu;
    std::vector<std::shared_ptr<StreamJump>> jumps;  // per stream, or null
};

// Pinned staging buffer for uploads; reused once its last copy finished.
struct Staging {
    std::mutex mu;
    uint8_t *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    ~Staging();
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
// jump-ahead segments as far as ws_bytes allows.  The caller holds stage.mu.
int run_batch(const std::shared_ptr<ParamSet> &ps, const void *d_params, uint32_t *d_states,
              int stride, const std::vector<Request> &reqs, void *d_ws, size_t ws_bytes,
              hipStream_t s, const mtgp_tuning &t, bool use_graph, Staging &stage);
size_t batch_min_ws_bytes(int n_items);
int validate_requests(const ParamSet &ps, const mtgp_work *items, int n);

}  // namespace mtgp
