// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/paf.h"

namespace paf {

constexpr int kLdsRow = 65;  // uint64 per LDS row: 64 lanes + 1 pad word

// Everything one filter launch needs.  Plain data; passed by value.
struct FilterParams {
    const uint64_t* reads;
    const uint64_t* refs;
    const uint64_t* word_offset;
    uint32_t stride_words;
    const uint16_t* len;
    uint32_t uniform_len;
    const uint8_t* E;
    uint32_t uniform_E;
    const uint32_t* perm;   // slot -> pair id (bucketed order), or NULL
    uint64_t n_pairs;
    uint32_t n_tiles;
    uint32_t wmax;          // words per sequence row in LDS = ceil(max_len / 32)
    uint32_t max_len;
    uint32_t max_E;
    uint32_t filters;
    uint32_t* acc[3];       // accept bit words (plain order); NULL in bucketed order
    uint16_t* cnt[3];
    uint32_t* err;          // sticky range flag
    uint32_t* queue;        // tile counter of the persistent launch, or NULL
    uint32_t grab;          // tiles per queue access
};

// Kernel selection.
enum class Engine { Snake, Whole };

struct LaunchShape {
    uint32_t waves_per_block;
    uint32_t blocks;        // grid size
    size_t lds_bytes;
};

// filter.hip
int emax_bucket(int max_E);  // smallest instantiated EMAX >= max_E, or -1
hipError_t launch_filter(const FilterParams& p, Engine eng, bool general, int emax,
                         const LaunchShape& shape, hipStream_t stream);
hipError_t launch_pack(const uint8_t* codes, uint32_t code_stride, const uint16_t* len,
                       uint32_t uniform_len, const uint64_t* word_offset, uint32_t stride_words,
                       uint64_t n, uint32_t wmax, uint64_t* words, uint32_t* err, hipStream_t s);
hipError_t launch_accept_from_counts(const uint16_t* cnt, const uint16_t* len, uint32_t uniform_len,
                                     const uint8_t* E, uint32_t uniform_E, uint32_t max_len,
                                     uint32_t max_E, uint64_t n, uint32_t* acc, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
const void* filter_kernel_ptr(Engine eng, bool general, int emax);
size_t filter_lds_bytes(uint32_t waves_per_block, uint32_t wmax);

// mlp.hip
hipError_t launch_features(const FilterParams& p, float* feat, hipStream_t s);
struct MlpDev {
    float* master;      // PAF_MLP_NPARAMS fp32 master weights
    uint16_t* w16;      // bf16 working copies of W1, W2, W3 (same offsets as master for W's)
    float* adam_m;
    float* adam_v;
    float* grad;        // PAF_MLP_NPARAMS
    float* act;         // workspace for training activations
    size_t act_cap;     // rows
    int step;
};
hipError_t mlp_round_weights(MlpDev& m, hipStream_t s);
hipError_t mlp_forward(const MlpDev& m, const float* feat, uint64_t n, float* out, hipStream_t s);
hipError_t mlp_train_step(MlpDev& m, const float* feat, const float* tgt, uint64_t n, float lr,
                          float* loss, hipStream_t s);
hipError_t launch_bucket(const FilterParams& p, const float* pred, uint32_t* perm, uint32_t* hist,
                         uint32_t* ws, hipStream_t s);
size_t bucket_ws_words(uint64_t n);

}  // namespace paf

struct paf_ctx {
    int device = 0;
    int num_cus = 256;
    uint32_t* d_err = nullptr;
    uint32_t* d_queue = nullptr;
    std::map<std::tuple<int, int, uint32_t>, paf_layout> tuned;  // (wmax, emax, filters) -> layout
    bool layout_forced = false;
    paf_layout forced{};
    struct GraphKey {
        uint64_t a, b, c, d;
        bool operator<(const GraphKey& o) const {
            return std::tie(a, b, c, d) < std::tie(o.a, o.b, o.c, o.d);
        }
    };
    std::map<GraphKey, hipGraphExec_t> graphs;
    paf::MlpDev mlp{};
    bool mlp_ready = false;
    // bucketed-pipeline workspace
    float* ws_feat = nullptr;
    float* ws_pred = nullptr;
    uint32_t* ws_perm = nullptr;
    uint32_t* ws_hist = nullptr;
    uint32_t* ws_bucket = nullptr;
    uint16_t* ws_cnt[3] = {nullptr, nullptr, nullptr};
    uint64_t ws_cap = 0;
};
