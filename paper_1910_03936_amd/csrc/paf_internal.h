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
    uint32_t chunk;         // tiles per wave-owned chunk (compacting engine)
    uint32_t span0, span;   // compacting engine: windows of the first pass and of later passes
    const uint8_t* order_key;  // compacting engine: per-pair key (original order); each chunk's
                               // pairs enter the first window in ascending key order, or NULL
    uint32_t part;             // compacting engine, partitioned maze: sub-maze width in columns
    uint32_t part_cap;         // ... and the most obstacles one sub-maze counts (~0u: no cap)
};

// Kernel selection.
// Chunk2: the compacting engine with two lanes per pair (whole maze, max_E 9..31).
enum class Engine { Snake, Whole, Chunk, ChunkPart, Chunk2 };

struct LaunchShape {
    uint32_t waves_per_block;
    uint32_t blocks;        // grid size
    size_t lds_bytes;
};

// api.hip: error reporting and batch checks shared by every entry point.
paf_status fail(paf_status st, const std::string& msg);
paf_status hip_fail(hipError_t e, const char* what);
paf_status check_batch(const paf_ctx* ctx, const paf_batch* b, uint32_t filters, FilterParams& p);
inline uint32_t words_for(uint32_t m) { return (m + 31u) / 32u; }

// Calls that use the context's own device memory (the work-queue counter,
// the bucketing workspace, the cost model's weights and training workspace)
// are ordered across streams: a call on another stream than the previous such
// call first waits (on the device) for that call's work.  scratch_begin
// before enqueueing, scratch_end after (outside any graph capture).
paf_status scratch_begin(paf_ctx* ctx, hipStream_t s);
void scratch_end(paf_ctx* ctx, hipStream_t s);
struct ScratchScope {
    paf_ctx* ctx;
    hipStream_t s;
    paf_status st;
    ScratchScope(paf_ctx* c, hipStream_t st_) : ctx(c), s(st_), st(scratch_begin(c, st_)) {}
    ~ScratchScope() {
        if (st == PAF_OK) scratch_end(ctx, s);
    }
};

#define PAF_HIP(call, what)                                        \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::paf::hip_fail(e_, what);    \
    } while (0)

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
const void* filter_kernel_ptr(Engine eng, bool general, int emax, uint32_t filters);
const void* whole_kernel_ptr(bool general, int emax, uint32_t filters);
size_t filter_lds_bytes(uint32_t waves_per_block, uint32_t wmax);
// LDS of a compacting launch (keyed launches sort inside the list itself).
size_t chunk_lds_bytes(uint32_t waves_per_block, bool general, int emax, uint32_t chunk_tiles, uint32_t lpp);

// verify.hip: banded edit distance of the selected pairs (sel: accept-bit
// words, or NULL for every pair).
hipError_t launch_verify(const FilterParams& p, int emax, const uint32_t* sel, uint16_t* dist, hipStream_t s);

// magnet.hip: MAGNET counts into p.cnt[0], then accept bits into p.acc[0];
// flag/counts/order/hist: the bucketing workspace (flag: n_pairs bytes).
hipError_t launch_magnet(const FilterParams& p, int emax, uint8_t* flag, uint32_t* counts, uint32_t* order,
                         uint32_t* hist, int num_cus, hipStream_t s);
// The same on the static workspace of paf_filter_magnet_noalloc (`base` is
// its device address, from magnet_noalloc_address on the current device);
// more pairs than it holds: hipErrorInvalidValue, nothing launched.
hipError_t launch_magnet_noalloc(const FilterParams& p, int emax, uint8_t* base, int num_cus, hipStream_t s);
hipError_t magnet_noalloc_address(uint8_t** ptr);
size_t magnet_noalloc_bytes();

// mlp.hip
struct MlpDev {
    float* master = nullptr;  // PAF_MLP_NPARAMS fp32 master weights (host layout of paf.h)
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* grad = nullptr;    // PAF_MLP_NPARAMS
    // bf16 working copies (stored as raw 16-bit words)
    uint16_t* w1b = nullptr;  // [128][64]   W1[h][f]
    uint16_t* w2b = nullptr;  // [128][128]  W2[o][h]
    uint16_t* w2tb = nullptr; // [128][128]  W2[o][h] stored as [h][o]
    float* w3r = nullptr;     // [128] bf16-rounded W3 values held in fp32
    uint16_t* w1f = nullptr;  // W1 in matrix-core fragment order [8][2][64][8]
    uint16_t* w2f = nullptr;  // W2 in fragment order, K permuted [8][4][64][8]
    // training workspace
    void* ws = nullptr;
    size_t ws_rows = 0;       // padded batch rows the workspace holds
    int step = 0;
};
size_t bucket_count_words(uint64_t n);
hipError_t launch_learned_buckets(const MlpDev& m, const FilterParams& p, int num_cus, float* pred,
                                  uint8_t* bucket, hipStream_t s,
                                  bool chunk_key = false);
hipError_t launch_bucket_from_pred(const FilterParams& p, const float* pred, uint8_t* bucket, hipStream_t s);
hipError_t launch_bucket_sort(const uint8_t* bucket, uint64_t n, uint32_t* counts, uint32_t* perm,
                              uint32_t* hist, hipStream_t s);
hipError_t mlp_alloc(MlpDev& m);
void mlp_free(MlpDev& m);
hipError_t mlp_round_weights(MlpDev& m, hipStream_t s);
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
    // bucketed-pipeline workspace (grows to the largest batch seen)
    float* ws_pred = nullptr;
    uint8_t* ws_bucket = nullptr;
    uint32_t* ws_perm = nullptr;
    uint32_t* ws_counts = nullptr;
    uint32_t* ws_hist = nullptr;
    uint64_t ws_cap = 0;
    // Device address of paf_filter_magnet_noalloc's static workspace on this
    // context's device (NULL if the lookup failed, with its error).
    uint8_t* magnet_scratch = nullptr;
    hipError_t magnet_scratch_err = hipSuccess;
    // Ordering of the calls that use the memory above across streams.
    hipEvent_t scratch_ev = nullptr;
    hipStream_t scratch_stream = nullptr;
    bool scratch_used = false;
};
