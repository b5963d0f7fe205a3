// mtgp_host.hpp -- host-side declarations shared by the C ABI and the
// serving runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <vector>

#include "mtgp.h"
#include "mtgp_internal.hpp"

namespace mtgp {

// Host copy of what mtgp_init_states / mtgp_load_params wrote to a d_params
// buffer: enough to plan launches (state length, step widths).
struct ParamSet {
    int n = 0;                 // streams
    int N = 0;                 // state words
    uint32_t mexp = 0;
    std::vector<uint32_t> W;   // step width N - pos per stream
};

// Pinned staging buffer for work lists; reused once its last copy finished.
struct Staging {
    std::mutex mu;
    BatchItem *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int device_cus();
int words_for_mexp(uint32_t mexp);
std::shared_ptr<ParamSet> lookup_params(const void *d_params, int n_streams);
mtgp_tuning tuning_for(int N);
size_t batch_ws_bytes(int n_items);
int validate_items(const ParamSet &ps, int n_streams_limit, const mtgp_work *items, int n);
void plan_items_indexed(const ParamSet &ps, const mtgp_tuning &t, const mtgp_work *items, int n,
                        std::vector<BatchItem> &out, std::vector<int> &order);
// Uploads an already planned work list and launches it; the caller holds
// stage.mu.
int launch_planned(const ParamSet &ps, const void *d_params, uint32_t *d_states, int stride,
                   const std::vector<BatchItem> &planned, void *d_ws, hipStream_t s,
                   const mtgp_tuning &t, bool use_graph, Staging &stage);
int generate_batch_impl(const void *d_params, uint32_t *d_states, int stride,
                        const mtgp_work *h_items, int n_items, void *d_ws, hipStream_t s,
                        const mtgp_tuning *force, bool use_graph, Staging &stage);

}  // namespace mtgp
