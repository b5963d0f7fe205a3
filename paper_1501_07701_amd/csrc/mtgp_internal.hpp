// mtgp_internal.hpp -- declarations shared by the kernels and the host
// library (never installed; the public interface is include/mtgp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mtgp {

// Device parameter block: 64 words (256 bytes) per stream.
enum : uint32_t {
    P_MEXP = 0,
    P_N = 1,
    P_POS = 2,
    P_SH1 = 3,
    P_SH2 = 4,
    P_MASK = 5,
    P_W = 6,
    P_SEED = 7,
    P_REC = 16,
    P_TMP = 32,
    P_FLT = 48,
    P_WORDS = 64,
};

// Device work-list entry (32 bytes).
struct BatchItem {
    uint32_t stream;
    uint32_t dtype;  // 0 uint32, 1 float32
    uint64_t count;
    uint64_t out;    // device address
    uint64_t flag;   // 0, or a host-mapped uint32 set to 1 when the item is done
};
static_assert(sizeof(BatchItem) == 32, "BatchItem layout");

struct LaunchArgs {
    const uint32_t *params;
    uint32_t *states;
    uint32_t stride;
    const BatchItem *items;  // nullptr: plain mode
    uint32_t n_items;
    uint32_t *counter;
    uint32_t *plain_out;
    uint64_t plain_count;
    uint32_t plain_f32;
    int grid;      // <= 0: persistent (occupancy x CUs)
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
hipError_t launch_seed(const uint32_t *params, uint32_t *states, uint32_t stride,
                       uint32_t n_streams, hipStream_t s);
hipError_t launch_reset(uint32_t *counter, hipStream_t s);
hipError_t launch_fill(uint32_t *out, uint64_t n_words, uint32_t value, int num_cus,
                       hipStream_t s);

}  // namespace mtgp
