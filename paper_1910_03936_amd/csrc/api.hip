// Host side of libpaf: the C ABI declared in include/paf.h.
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "paf_internal.h"

using namespace paf;

namespace {
thread_local std::string g_err;
}  // namespace

namespace paf {
paf_status fail(paf_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

paf_status hip_fail(hipError_t e, const char* what) {
    return fail(PAF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Host-side checks of a batch; fills the launch-invariant part of FilterParams.
paf_status check_batch(const paf_ctx* ctx, const paf_batch* b, uint32_t filters, FilterParams& p) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (!b) return fail(PAF_ERR_ARG, "batch is NULL");
    if (!b->reads || !b->refs) return fail(PAF_ERR_ARG, "batch reads/refs is NULL");
    if (b->n_pairs == 0) return fail(PAF_ERR_ARG, "batch has no pairs");
    if (b->n_pairs > (uint64_t)UINT32_MAX * 64ull)
        return fail(PAF_ERR_RANGE, "batch has too many pairs (max 2^32 tiles of 64)");
    if (filters == 0 || filters > 7u) return fail(PAF_ERR_ARG, "filters must be a nonzero mask of PAF_* bits");
    uint32_t max_len = b->max_len;
    uint32_t max_E = b->max_E;
    if (!b->len) {
        if (b->uniform_len < 1 || b->uniform_len > PAF_MAX_LEN)
            return fail(PAF_ERR_RANGE, "uniform_len outside [1, PAF_MAX_LEN]");
        if (max_len == 0) max_len = b->uniform_len;
        if (b->uniform_len > max_len) return fail(PAF_ERR_RANGE, "uniform_len exceeds max_len");
    }
    if (max_len < 1 || max_len > PAF_MAX_LEN) return fail(PAF_ERR_RANGE, "max_len outside [1, PAF_MAX_LEN]");
    if (!b->E) {
        if (b->uniform_E > PAF_MAX_E) return fail(PAF_ERR_RANGE, "uniform_E exceeds PAF_MAX_E");
        if (b->uniform_E > max_E) max_E = b->uniform_E;
    }
    if (max_E > PAF_MAX_E) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    const uint32_t wmax = words_for(max_len);
    if (!b->word_offset && b->stride_words < wmax)
        return fail(PAF_ERR_ARG, "stride_words is smaller than ceil(max_len / 32)");
    memset(&p, 0, sizeof(p));
    p.reads = b->reads;
    p.refs = b->refs;
    p.word_offset = b->word_offset;
    p.stride_words = b->stride_words;
    p.len = b->len;
    p.uniform_len = b->len ? 0u : b->uniform_len;
    p.E = b->E;
    p.uniform_E = b->E ? 0u : b->uniform_E;
    p.n_pairs = b->n_pairs;
    p.n_tiles = (uint32_t)((b->n_pairs + 63) / 64);
    p.wmax = wmax;
    p.max_len = max_len;
    p.max_E = max_E;
    p.filters = filters;
    p.err = ctx->d_err;
    p.grab = 1;
    p.chunk = 0;
    p.span0 = p.span = 1;
    p.order_key = nullptr;
    return PAF_OK;
}

paf_status scratch_begin(paf_ctx* ctx, hipStream_t s) {
    if (ctx->scratch_used && ctx->scratch_stream != s)
        PAF_HIP(hipStreamWaitEvent(s, ctx->scratch_ev, 0), "hipStreamWaitEvent");
    return PAF_OK;
}

void scratch_end(paf_ctx* ctx, hipStream_t s) {
    if (hipEventRecord(ctx->scratch_ev, s) == hipSuccess) {
        ctx->scratch_stream = s;
        ctx->scratch_used = true;
    }
}

}  // namespace paf

namespace {

paf_status check_out(const paf_out* out, uint32_t filters) {
    if (!out) return fail(PAF_ERR_ARG, "out is NULL");
    for (int f = 0; f < 3; ++f)
        if ((filters >> f) & 1u)
            if (!out->accept_bits[f] || !out->count[f])
                return fail(PAF_ERR_ARG, "a requested filter has a NULL output pointer");
    return PAF_OK;
}

Engine engine_for(uint32_t filters) {
    return filters == PAF_SNEAKYSNAKE ? Engine::Snake : Engine::Whole;
}

// Block-size limit of each engine (its launch bound).
uint32_t max_waves(Engine e) { return e == Engine::Whole ? 4u : 8u; }

hipError_t allow_lds(const void* k, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Default layout of the persistent launch.
paf_layout default_layout() {
    paf_layout l;
    l.lanes_per_pair = 1;
    l.waves_per_block = 4;
    l.blocks_per_cu = 4;
    l.tiles_per_grab = 2;
    l.chunk_tiles = 0;
    return l;
}

// Launch shape of paf_filter's SneakySnake-only launch (measured best on
// 10M pairs of 250 bp, full grid): up to max_E 3, four-wave blocks and
// chunks of 4 tiles; 4 to 6, two-wave blocks and chunks of 4; from 7 on,
// chunks of 6 (the kernel runs five waves per SIMD up to 8, so a wave's LDS
// must stay under 8 KB).  Up to 15 a two-window first pass, then passes of
// three windows (two at 7 and 8).  Above 15 pairs are decided later and a
// pass regroups fewer of them, so the first pass is longer (three windows,
// four at 31) and every later pass regroups after one window: 8.8% / 5.7% /
// 3.7% less time at E = 20 / 25 / 31 than two-window passes, and no slower
// on the partitioned engine, which shares this shape.
paf_layout plain_layout(int emax) {
    if (emax <= 3) return paf_layout{1u, 4u, 0u, 1u, 4u, 2u, 3u};
    if (emax <= 6) return paf_layout{1u, 2u, 0u, 1u, 4u, 2u, 3u};
    if (emax <= 8) return paf_layout{1u, 2u, 0u, 1u, 6u, 2u, 2u};
    if (emax <= 15) return paf_layout{1u, 2u, 0u, 1u, 6u, 2u, 3u};
    if (emax <= 25) return paf_layout{1u, 2u, 0u, 1u, 6u, 3u, 1u};
    return paf_layout{1u, 2u, 0u, 1u, 6u, 4u, 1u};
}

// Launch shape of paf_filter_partitioned: paf_filter's, except at max_E 4 to
// 6, where chunks of 6 tiles and one-window later passes measured 1.3-6.4%
// faster on 10M pairs of 250 bp at E = 5 (t = 5, 10, 25, 50 and the fixed
// tile t = 8, y = 3): a probe stops at its sub-maze's end, so pairs stay
// undecided for more windows and regrouping after each one pays.
paf_layout part_layout(int emax) {
    if (emax >= 4 && emax <= 6) return paf_layout{1u, 2u, 0u, 1u, 6u, 2u, 1u};
    return plain_layout(emax);
}

bool layout_ok(const paf_layout& l) {
    return (l.lanes_per_pair == 1 || l.lanes_per_pair == 2) &&
           (l.waves_per_block == 1 || l.waves_per_block == 2 || l.waves_per_block == 4 ||
            l.waves_per_block == 8) &&
           l.blocks_per_cu <= 64 && l.tiles_per_grab >= 1 &&
           l.tiles_per_grab <= 64 && l.chunk_tiles <= 16 && l.first_pass_windows <= 16 &&
           l.pass_windows <= 16;
}

// Largest resident block count per CU for this kernel and LDS size.
int resident_blocks(const void* k, uint32_t waves, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * waves, lds) != hipSuccess) return 1;
    return std::max(1, nb);
}

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

// The compacting engine of a layout: one lane per pair, or two (the whole
// maze with the diagonals split between the lanes, from max_E 9 on).
Engine compacting_engine(const paf_layout& L, int emax, paf_status& st) {
    if (L.lanes_per_pair != 2) return Engine::Chunk;
    if (emax < 10) st = fail(PAF_ERR_ARG, "two lanes per pair need max_E >= 9");
    return Engine::Chunk2;
}

// Replays the graph cached under `key`, or captures `body` (which must only
// enqueue work on the stream it is given) into a new graph first.
template <typename F>
paf_status run_graph(paf_ctx* ctx, const paf_ctx::GraphKey& key, hipStream_t stream, F&& body) {
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 64) {
            for (auto& kv : ctx->graphs) hipGraphExecDestroy(kv.second);
            ctx->graphs.clear();
        }
        hipStream_t cap;
        PAF_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
        hipGraph_t g = nullptr;
        paf_status st = PAF_OK;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = body(cap);
            e = hipStreamEndCapture(cap, &g);
        }
        hipGraphExec_t ex = nullptr;
        if (e == hipSuccess && st == PAF_OK) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        hipStreamDestroy(cap);
        if (st != PAF_OK) return st;
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        it = ctx->graphs.emplace(key, ex).first;
    }
    PAF_HIP(hipGraphLaunch(it->second, stream), "hipGraphLaunch");
    return PAF_OK;
}

// Launch the persistent filter through a cached HIP graph (queue reset by a
// fill kernel, then the kernel).  The graph is captured on a private stream
// and launched on `stream`.
paf_status run_persistent(paf_ctx* ctx, FilterParams p, Engine eng, int emax, const paf_layout& L,
                          hipStream_t stream, bool use_graph) {
    // Per-pair lengths, thresholds, offsets or an order need the general
    // kernels; a uniform batch in place takes the plain ones.
    const bool general = p.len || p.E || p.word_offset || p.perm;
    // SneakySnake alone with a chunk size: the compacting engine (one or two
    // lanes per pair); its queue and grid count chunks instead of tiles.
    paf_status st = PAF_OK;
    if (eng == Engine::Snake && L.chunk_tiles > 0) eng = compacting_engine(L, emax, st);
    else if (L.lanes_per_pair != 1) st = fail(PAF_ERR_ARG, "two lanes per pair need the compacting engine");
    if (st != PAF_OK) return st;
    const bool compacting = eng == Engine::Chunk || eng == Engine::Chunk2;
    const void* k = filter_kernel_ptr(eng, general, emax, p.filters);
    if (!k) return fail(PAF_ERR_RANGE, "no kernel for this threshold");
    if (L.waves_per_block > max_waves(eng)) return fail(PAF_ERR_ARG, "too many waves per block for this engine");
    LaunchShape sh;
    sh.waves_per_block = L.waves_per_block;
    p.chunk = compacting ? L.chunk_tiles : 0u;
    p.span0 = std::max(1u, L.first_pass_windows);
    p.span = std::max(1u, L.pass_windows);
    sh.lds_bytes = compacting ? chunk_lds_bytes(L.waves_per_block, general, emax, L.chunk_tiles, L.lanes_per_pair)
                              : filter_lds_bytes(L.waves_per_block, p.wmax);
    if (sh.lds_bytes > 160 * 1024) return fail(PAF_ERR_RANGE, "layout needs more LDS than a CU has");
    PAF_HIP(allow_lds(k, sh.lds_bytes), "hipFuncSetAttribute");
    const uint64_t units = compacting ? (p.n_tiles + p.chunk - 1) / p.chunk : p.n_tiles;
    const uint64_t need = (units + L.waves_per_block - 1) / L.waves_per_block;
    if (L.blocks_per_cu == 0) {
        // Full grid, one tile per wave: the hardware dispatcher is the queue.
        sh.blocks = (uint32_t)need;
        p.queue = nullptr;
        p.grab = 1;
        return [&]() -> paf_status {
            PAF_HIP(launch_filter(p, eng, general, emax, sh, stream), "filter launch");
            return PAF_OK;
        }();
    }
    const int nb = std::min<int>((int)L.blocks_per_cu, resident_blocks(k, L.waves_per_block, sh.lds_bytes));
    const uint64_t want = (uint64_t)ctx->num_cus * nb;
    sh.blocks = (uint32_t)std::max<uint64_t>(1, std::min(want, need));
    p.queue = ctx->d_queue;
    p.grab = L.tiles_per_grab;
    if (!use_graph) {
        PAF_HIP(launch_fill_u32(ctx->d_queue, 0u, 1, stream), "queue reset");
        PAF_HIP(launch_filter(p, eng, general, emax, sh, stream), "filter launch");
        return PAF_OK;
    }
    paf_ctx::GraphKey key{0, 0, 0, 0};
    const uint64_t* words = reinterpret_cast<const uint64_t*>(&p);
    for (size_t i = 0; i < sizeof(p) / 8; ++i) key.a = mix(key.a, words[i]);
    key.b = mix(mix((uint64_t)eng, (uint64_t)emax), (uint64_t)L.waves_per_block);
    key.c = mix(mix(mix(sh.blocks, sh.lds_bytes), L.tiles_per_grab), L.chunk_tiles);
    key.d = p.n_pairs;
    return run_graph(ctx, key, stream, [&](hipStream_t s) -> paf_status {
        PAF_HIP(launch_fill_u32(ctx->d_queue, 0u, 1, s), "queue reset");
        PAF_HIP(launch_filter(p, eng, general, emax, sh, s), "filter launch");
        return PAF_OK;
    });
}

paf_status ensure_bucket_ws(paf_ctx* ctx, uint64_t n) {
    if (ctx->ws_cap >= n && ctx->ws_hist) return PAF_OK;
    hipFree(ctx->ws_pred);
    hipFree(ctx->ws_perm);
    hipFree(ctx->ws_hist);
    hipFree(ctx->ws_bucket);
    hipFree(ctx->ws_counts);
    ctx->ws_pred = nullptr;
    ctx->ws_perm = ctx->ws_hist = ctx->ws_counts = nullptr;
    ctx->ws_bucket = nullptr;
    ctx->ws_cap = 0;
    // Drop cached graphs: they may point at the old workspace.
    for (auto& kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    if (hipMalloc(&ctx->ws_perm, n * 4) != hipSuccess || hipMalloc(&ctx->ws_bucket, n) != hipSuccess ||
        hipMalloc(&ctx->ws_counts, bucket_count_words(n) * 4) != hipSuccess ||
        hipMalloc(&ctx->ws_hist, 16 * 4) != hipSuccess)
        return fail(PAF_ERR_NOMEM, "bucketing workspace");
    ctx->ws_cap = n;
    return PAF_OK;
}

// Launch layout: the forced one, else the autotuned one for this class, else
// the default (work queue for the persistent entry point; for orders given
// by a permutation, paf_filter's full grid of compacting chunks for
// SneakySnake alone, where measured dispatch by the hardware beat the queue).
paf_layout layout_for(paf_ctx* ctx, const FilterParams& p, int emax, bool queue_default = true) {
    if (ctx->layout_forced) return ctx->forced;
    auto it = ctx->tuned.find(std::make_tuple((int)p.wmax, emax, p.filters));
    if (it != ctx->tuned.end()) return it->second;
    if (queue_default) return default_layout();
    return plain_layout(emax);
}

void set_outputs(FilterParams& p, const paf_out* out) {
    for (int f = 0; f < 3; ++f) {
        p.acc[f] = ((p.filters >> f) & 1u) ? out->accept_bits[f] : nullptr;
        p.cnt[f] = ((p.filters >> f) & 1u) ? out->count[f] : nullptr;
    }
}

}  // namespace

extern "C" {

const char* paf_last_error(void) { return g_err.c_str(); }

paf_status paf_create(paf_ctx** out, int device) {
    if (!out) return fail(PAF_ERR_ARG, "ctx pointer is NULL");
    *out = nullptr;
    int n = 0;
    PAF_HIP(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(PAF_ERR_ARG, "no such device");
    PAF_HIP(hipSetDevice(device), "hipSetDevice");
    paf_ctx* c = new (std::nothrow) paf_ctx();
    if (!c) return fail(PAF_ERR_NOMEM, "host allocation failed");
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->num_cus = cus;
    if (hipMalloc(&c->d_err, 2 * sizeof(uint32_t)) != hipSuccess) {
        delete c;
        return fail(PAF_ERR_NOMEM, "device allocation failed");
    }
    c->d_queue = c->d_err + 1;
    if (hipMemset(c->d_err, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
        hipEventCreateWithFlags(&c->scratch_ev, hipEventDisableTiming) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        hipFree(c->d_err);
        if (c->scratch_ev) (void)hipEventDestroy(c->scratch_ev);
        delete c;
        return fail(PAF_ERR_DEVICE, "device initialisation failed");
    }
    // The static workspace of paf_filter_magnet_noalloc: its address on this
    // device (the device is current here).  A failed lookup only disables
    // that entry point.
    c->magnet_scratch_err = magnet_noalloc_address(&c->magnet_scratch);
    if (c->magnet_scratch_err != hipSuccess) c->magnet_scratch = nullptr;
    *out = c;
    return PAF_OK;
}

paf_status paf_destroy(paf_ctx* ctx) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (auto& kv : ctx->graphs) hipGraphExecDestroy(kv.second);
    if (ctx->scratch_ev) (void)hipEventDestroy(ctx->scratch_ev);
    hipFree(ctx->d_err);
    mlp_free(ctx->mlp);
    hipFree(ctx->ws_pred);
    hipFree(ctx->ws_perm);
    hipFree(ctx->ws_hist);
    hipFree(ctx->ws_bucket);
    hipFree(ctx->ws_counts);
    delete ctx;
    return PAF_OK;
}

paf_status paf_check(paf_ctx* ctx, void* stream) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    hipStream_t s = (hipStream_t)stream;
    uint32_t flag = 0;
    PAF_HIP(hipMemcpyAsync(&flag, ctx->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    PAF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (flag) {
        PAF_HIP(launch_fill_u32(ctx->d_err, 0u, 1, s), "flag reset");
        PAF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        return fail(PAF_ERR_RANGE, "a pair had a length, threshold or base code outside the batch's bounds");
    }
    return PAF_OK;
}

paf_status paf_pack(paf_ctx* ctx, const uint8_t* codes, uint32_t code_stride, const uint16_t* len,
                    uint16_t uniform_len, const uint64_t* word_offset, uint32_t stride_words,
                    uint64_t n, uint64_t* words, void* stream) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (!codes || !words) return fail(PAF_ERR_ARG, "codes/words is NULL");
    if (n == 0) return fail(PAF_ERR_ARG, "n is zero");
    if (!len && (uniform_len < 1 || uniform_len > PAF_MAX_LEN))
        return fail(PAF_ERR_RANGE, "uniform_len outside [1, PAF_MAX_LEN]");
    const uint32_t maxm = len ? PAF_MAX_LEN : uniform_len;
    if (code_stride < (len ? 1u : (uint32_t)uniform_len)) return fail(PAF_ERR_ARG, "code_stride too small");
    if (!word_offset && stride_words < words_for(maxm) && !len)
        return fail(PAF_ERR_ARG, "stride_words too small");
    // With per-pair lengths every length must fit the stride; lengths are
    // device data, so the kernel clips with the threads it launches.
    const uint32_t wmax = len ? std::min<uint32_t>(words_for(PAF_MAX_LEN),
                                                   word_offset ? words_for(PAF_MAX_LEN) : stride_words)
                              : words_for(uniform_len);
    PAF_HIP(launch_pack(codes, code_stride, len, uniform_len, word_offset, stride_words, n, wmax, words,
                        ctx->d_err, (hipStream_t)stream),
            "pack launch");
    return PAF_OK;
}

}  // extern "C"

namespace {
// Host encoding of n rows into the planar two-bit words (layout of paf.h).
// code(byte) gives the base value 0..3, or a value above 3 for a byte that is
// not a base.  The rows are validated first (lengths against the stride, every
// byte of every row); only when all are good are the words written, so a
// rejected call leaves `words` untouched.  Returns 0, 1 (bad byte) or 2 (bad
// length).
template <typename Code>
int pack_rows_host(const uint8_t* rows, uint32_t row_stride, const uint16_t* len, uint16_t uniform_len,
                   const uint64_t* word_offset, uint32_t stride_words, uint64_t n, uint64_t* words,
                   int threads, Code code) {
    if (threads <= 0) threads = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    std::vector<int> bad((size_t)threads, 0);
    auto span = [&](int t, uint64_t& a, uint64_t& b) {
        a = n * (uint64_t)t / threads;
        b = n * (uint64_t)(t + 1) / threads;
    };
    auto check = [&](int t) {
        uint64_t a, b;
        span(t, a, b);
        for (uint64_t p = a; p < b && !bad[t]; ++p) {
            const uint32_t m = len ? len[p] : uniform_len;
            if (m < 1 || m > PAF_MAX_LEN || m > row_stride || (!word_offset && words_for(m) > stride_words)) {
                bad[t] = 2;
                break;
            }
            const uint8_t* row = rows + p * (uint64_t)row_stride;
            for (uint32_t j = 0; j < m; ++j)
                if (code(row[j]) > 3u) {
                    bad[t] = 1;
                    break;
                }
        }
    };
    auto encode = [&](int t) {
        uint64_t a, b;
        span(t, a, b);
        for (uint64_t p = a; p < b; ++p) {
            const uint32_t m = len ? len[p] : uniform_len;
            const uint8_t* row = rows + p * (uint64_t)row_stride;
            uint64_t* dst = words + (word_offset ? word_offset[p] : p * (uint64_t)stride_words);
            for (uint32_t k = 0; k < words_for(m); ++k) {
                uint32_t lo = 0, hi = 0;
                const uint32_t cnt = std::min(32u, m - 32u * k);
                for (uint32_t j = 0; j < cnt; ++j) {
                    const uint32_t v = code(row[32u * k + j]);
                    lo |= (v & 1u) << j;
                    hi |= ((v >> 1) & 1u) << j;
                }
                dst[k] = ((uint64_t)hi << 32) | lo;
            }
        }
    };
    auto run = [&](auto&& f) {
        std::vector<std::thread> pool;
        for (int t = 1; t < threads; ++t) pool.emplace_back(f, t);
        f(0);
        for (auto& th : pool) th.join();
    };
    run(check);
    int worst = 0;
    for (int v : bad) worst = std::max(worst, v);
    if (worst) return worst;
    run(encode);
    return 0;
}

// ASCII bases: A/a = 0, C/c = 1, G/g = 2, T/t = 3; every other byte 0xFF.
struct AsciiTable {
    uint8_t v[256];
    AsciiTable() {
        memset(v, 0xFF, sizeof(v));
        const char* up = "ACGT";
        const char* lo = "acgt";
        for (int i = 0; i < 4; ++i) {
            v[(uint8_t)up[i]] = (uint8_t)i;
            v[(uint8_t)lo[i]] = (uint8_t)i;
        }
    }
};
const AsciiTable kAscii;
}  // namespace

extern "C" {

paf_status paf_pack_host(const uint8_t* codes, uint32_t code_stride, const uint16_t* len,
                         uint16_t uniform_len, const uint64_t* word_offset, uint32_t stride_words,
                         uint64_t n, uint64_t* words, int threads) {
    if (!codes || !words) return fail(PAF_ERR_ARG, "codes/words is NULL");
    if (n == 0) return fail(PAF_ERR_ARG, "n is zero");
    if (!len && (uniform_len < 1 || uniform_len > PAF_MAX_LEN))
        return fail(PAF_ERR_RANGE, "uniform_len outside [1, PAF_MAX_LEN]");
    const int r = pack_rows_host(codes, code_stride, len, uniform_len, word_offset, stride_words, n, words, threads,
                                 [](uint8_t b) { return (uint32_t)b; });
    if (r) return fail(PAF_ERR_RANGE, r == 1 ? "base code above 3" : "pair length outside range or stride");
    return PAF_OK;
}

paf_status paf_pack_ascii(const char* seqs, uint32_t row_stride, const uint16_t* len, uint16_t uniform_len,
                          const uint64_t* word_offset, uint32_t stride_words, uint64_t n, uint64_t* words,
                          int threads) {
    if (!seqs || !words) return fail(PAF_ERR_ARG, "seqs/words is NULL");
    if (n == 0) return fail(PAF_ERR_ARG, "n is zero");
    if (!len && (uniform_len < 1 || uniform_len > PAF_MAX_LEN))
        return fail(PAF_ERR_RANGE, "uniform_len outside [1, PAF_MAX_LEN]");
    const int r = pack_rows_host(reinterpret_cast<const uint8_t*>(seqs), row_stride, len, uniform_len, word_offset,
                                 stride_words, n, words, threads, [](uint8_t b) { return (uint32_t)kAscii.v[b]; });
    if (r == 1) return fail(PAF_ERR_ARG, "a byte that is not A, C, G or T (either case) inside a sequence");
    if (r == 2) return fail(PAF_ERR_RANGE, "pair length outside range or stride");
    return PAF_OK;
}

paf_status paf_filter(paf_ctx* ctx, const paf_batch* batch, uint32_t filters, const paf_out* out,
                      void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    // Several stages: one map for all of them up to max_E 7.  From 8 on,
    // SneakySnake runs on its own compacting engine (faster than its share
    // of the whole-map kernel), and from 15 on GateKeeper and Shouji get a
    // kernel each (the combined kernel's per-lane state no longer fits at a
    // useful occupancy).  Every launch writes only its own stages' outputs.
    const bool several = (filters & (filters - 1u)) != 0u;
    if (several && (emax >= 15 || (emax >= 8 && (filters & PAF_SNEAKYSNAKE)))) {
        // Each group below is a single stage, or GateKeeper and Shouji
        // together under max_E 15, which the test above does not split again.
        const uint32_t rest = filters & ~(uint32_t)PAF_SNEAKYSNAKE;
        uint32_t groups[3];
        int ng = 0;
        if (filters & PAF_SNEAKYSNAKE) groups[ng++] = PAF_SNEAKYSNAKE;
        if (emax >= 15) {
            if (rest & PAF_GATEKEEPER) groups[ng++] = PAF_GATEKEEPER;
            if (rest & PAF_SHOUJI) groups[ng++] = PAF_SHOUJI;
        } else if (rest) {
            groups[ng++] = rest;
        }
        for (int i = 0; i < ng; ++i)
            if ((st = paf_filter(ctx, batch, groups[i], out, stream)) != PAF_OK) return st;
        return PAF_OK;
    }
    set_outputs(p, out);
    const bool general = batch->len || batch->E || batch->word_offset;
    Engine eng = engine_for(filters);
    LaunchShape sh;
    sh.waves_per_block = p.wmax > 8 ? 2 : 4;
    sh.lds_bytes = filter_lds_bytes(sh.waves_per_block, p.wmax);
    uint64_t units = p.n_tiles;
    // SneakySnake alone: the compacting engine, as a full grid of chunks
    // (a forced layout may set its chunk size and block shape, or turn it off).
    const paf_layout PL = ctx->layout_forced ? ctx->forced : plain_layout(emax);
    if (eng == Engine::Snake && PL.chunk_tiles > 0) {
        eng = compacting_engine(PL, emax, st);
        if (st != PAF_OK) return st;
        p.chunk = PL.chunk_tiles;
        p.span0 = std::max(1u, PL.first_pass_windows);
        p.span = std::max(1u, PL.pass_windows);
        sh.waves_per_block = PL.waves_per_block;
        sh.lds_bytes = chunk_lds_bytes(sh.waves_per_block, general, emax, p.chunk, PL.lanes_per_pair);
        if (sh.lds_bytes > 160 * 1024) return fail(PAF_ERR_RANGE, "layout needs more LDS than a CU has");
        units = (p.n_tiles + p.chunk - 1) / p.chunk;
    }
    sh.blocks = (uint32_t)((units + sh.waves_per_block - 1) / sh.waves_per_block);
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PAF_HIP(allow_lds(filter_kernel_ptr(eng, general, emax, p.filters), sh.lds_bytes), "hipFuncSetAttribute");
    PAF_HIP(launch_filter(p, eng, general, emax, sh, (hipStream_t)stream), "filter launch");
    return PAF_OK;
}

paf_status paf_filter_partitioned(paf_ctx* ctx, const paf_batch* batch, uint32_t t, uint32_t y,
                                  const paf_out* out, void* stream) {
    const uint32_t filters = PAF_SNEAKYSNAKE;
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    if (t < 1 || t > PAF_MAX_PART) return fail(PAF_ERR_RANGE, "partition width outside [1, PAF_MAX_PART]");
    if (y > PAF_MAX_REPL) return fail(PAF_ERR_RANGE, "replications outside [0, PAF_MAX_REPL]");
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    set_outputs(p, out);
    p.part = t;
    p.part_cap = y ? y : ~0u;
    const bool general = batch->len || batch->E || batch->word_offset;
    // The compacting engine, as a full grid of chunks (a forced layout that
    // compacts sets the chunk size, block shape and pass widths).
    const paf_layout PL = ctx->layout_forced && ctx->forced.chunk_tiles > 0 ? ctx->forced : part_layout(emax);
    p.chunk = PL.chunk_tiles;
    p.span0 = std::max(1u, PL.first_pass_windows);
    p.span = std::max(1u, PL.pass_windows);
    LaunchShape sh;
    sh.waves_per_block = PL.waves_per_block;
    sh.lds_bytes = chunk_lds_bytes(sh.waves_per_block, general, emax, p.chunk, 1);
    if (sh.lds_bytes > 160 * 1024) return fail(PAF_ERR_RANGE, "layout needs more LDS than a CU has");
    const uint64_t units = (p.n_tiles + p.chunk - 1) / p.chunk;
    sh.blocks = (uint32_t)((units + sh.waves_per_block - 1) / sh.waves_per_block);
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PAF_HIP(allow_lds(filter_kernel_ptr(Engine::ChunkPart, general, emax, p.filters), sh.lds_bytes),
            "hipFuncSetAttribute");
    PAF_HIP(launch_filter(p, Engine::ChunkPart, general, emax, sh, (hipStream_t)stream), "filter launch");
    return PAF_OK;
}

paf_status paf_filter_magnet(paf_ctx* ctx, const paf_batch* batch, const paf_out* out, void* stream) {
    const uint32_t filters = PAF_SNEAKYSNAKE;   // output slot 0
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    set_outputs(p, out);
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    if ((st = ensure_bucket_ws(ctx, p.n_pairs)) != PAF_OK) return st;
    PAF_HIP(launch_magnet(p, emax, ctx->ws_bucket, ctx->ws_counts, ctx->ws_perm, ctx->ws_hist, ctx->num_cus,
                          (hipStream_t)stream),
            "MAGNET launch");
    return PAF_OK;
}

paf_status paf_filter_magnet_noalloc(paf_ctx* ctx, const paf_batch* batch, const paf_out* out, void* stream) {
    const uint32_t filters = PAF_SNEAKYSNAKE;   // output slot 0
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    if (p.n_pairs > (uint64_t)PAF_MAGNET_NOALLOC_MAX_PAIRS)
        return fail(PAF_ERR_RANGE, "batch larger than the static workspace (PAF_MAGNET_NOALLOC_MAX_PAIRS pairs)");
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    if (!ctx->magnet_scratch)
        return hip_fail(ctx->magnet_scratch_err, "device address of the static MAGNET workspace");
    set_outputs(p, out);
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PAF_HIP(launch_magnet_noalloc(p, emax, ctx->magnet_scratch, ctx->num_cus, (hipStream_t)stream),
            "MAGNET launch");
    return PAF_OK;
}

paf_status paf_verify(paf_ctx* ctx, const paf_batch* batch, const uint32_t* select_bits, uint16_t* dist,
                      void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, PAF_SNEAKYSNAKE, p);
    if (st != PAF_OK) return st;
    if (!dist) return fail(PAF_ERR_ARG, "dist is NULL");
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PAF_HIP(launch_verify(p, emax, select_bits, dist, (hipStream_t)stream),
            "verify launch");
    return PAF_OK;
}

paf_status paf_filter_persistent(paf_ctx* ctx, const paf_batch* batch, uint32_t filters,
                                 const paf_out* out, void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    set_outputs(p, out);
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    const paf_layout L = layout_for(ctx, p, emax);
    return run_persistent(ctx, p, engine_for(filters), emax, L, (hipStream_t)stream, true);
}

paf_status paf_set_layout(paf_ctx* ctx, const paf_layout* layout) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (!layout) {
        ctx->layout_forced = false;
        return PAF_OK;
    }
    if (!layout_ok(*layout)) return fail(PAF_ERR_ARG, "unsupported layout");
    ctx->forced = *layout;
    ctx->layout_forced = true;
    return PAF_OK;
}

paf_status paf_tuned_export(paf_ctx* ctx, paf_tuned_entry* entries, uint32_t cap, uint32_t* count) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (!count) return fail(PAF_ERR_ARG, "count is NULL");
    if (cap > 0 && !entries) return fail(PAF_ERR_ARG, "entries is NULL");
    uint32_t i = 0;
    for (const auto& kv : ctx->tuned) {
        if (i < cap) {
            entries[i].max_words = (uint32_t)std::get<0>(kv.first);
            entries[i].max_E = (uint32_t)std::get<1>(kv.first);
            entries[i].filters = std::get<2>(kv.first);
            entries[i].layout = kv.second;
        }
        ++i;
    }
    *count = i;
    return PAF_OK;
}

paf_status paf_tuned_import(paf_ctx* ctx, const paf_tuned_entry* entries, uint32_t count) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (count > 0 && !entries) return fail(PAF_ERR_ARG, "entries is NULL");
    // Every entry is checked before any is taken, so a bad file changes nothing.
    for (uint32_t i = 0; i < count; ++i) {
        const paf_tuned_entry& t = entries[i];
        if (t.max_words < 1 || t.max_words > (PAF_MAX_LEN + 31) / 32)
            return fail(PAF_ERR_ARG, "tuned entry: max_words outside 1..16");
        if (t.max_E > PAF_MAX_E || emax_bucket((int)t.max_E) != (int)t.max_E)
            return fail(PAF_ERR_ARG, "tuned entry: max_E is not a threshold class of the library");
        if (t.filters < 1 || t.filters > 7u)
            return fail(PAF_ERR_ARG, "tuned entry: filters outside 1..7");
        if (!layout_ok(t.layout)) return fail(PAF_ERR_ARG, "tuned entry: unsupported layout");
        if (t.layout.lanes_per_pair == 2 && (t.max_E < 10 || t.filters != PAF_SNEAKYSNAKE))
            return fail(PAF_ERR_ARG, "tuned entry: two lanes per pair need SneakySnake alone and max_E >= 9");
    }
    for (uint32_t i = 0; i < count; ++i) {
        const paf_tuned_entry& t = entries[i];
        ctx->tuned[std::make_tuple((int)t.max_words, (int)t.max_E, t.filters)] = t.layout;
    }
    return PAF_OK;
}

paf_status paf_autotune(paf_ctx* ctx, const paf_batch* batch, uint32_t filters, const paf_out* out,
                        void* stream, paf_layout* chosen, float* best_ms, float* default_ms) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    set_outputs(p, out);
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    hipStream_t s = (hipStream_t)stream;
    const Engine eng = engine_for(filters);
    std::vector<paf_layout> cands;
    for (uint32_t wpb : {1u, 2u, 4u, 8u}) {
        if (wpb > max_waves(eng)) continue;
        cands.push_back(paf_layout{1u, wpb, 0u, 1u, 0u});   // full grid, no queue
        for (uint32_t bpc : {1u, 2u, 4u, 8u, 16u})
            for (uint32_t grab : {1u, 2u, 4u, 8u}) {
                paf_layout l{1u, wpb, bpc, grab, 0u};
                if (filter_lds_bytes(wpb, p.wmax) * bpc > 160 * 1024) continue;
                if (wpb * bpc > 32) continue;
                cands.push_back(l);
            }
        if (eng != Engine::Snake) continue;
        // Compacting layouts, with one lane per pair and (the whole maze from
        // max_E 9 on) two.
        for (uint32_t lpp : {1u, 2u}) {
            if (lpp == 2 && emax < 10) continue;
            for (uint32_t K : {4u, 6u, 8u, 16u}) {
                const size_t lds = chunk_lds_bytes(wpb, true, emax, K, lpp);
                if (lds > 160 * 1024) continue;
                for (uint32_t sp : {1u, 2u}) {
                    cands.push_back(paf_layout{lpp, wpb, 0u, 1u, K, sp, sp});
                    for (uint32_t bpc : {2u, 4u}) {
                        if (lds * bpc > 160 * 1024 || wpb * bpc > 32) continue;
                        cands.push_back(paf_layout{lpp, wpb, bpc, 1u, K, sp, sp});
                    }
                }
            }
        }
    }
    hipEvent_t e0, e1;
    PAF_HIP(hipEventCreate(&e0), "hipEventCreate");
    PAF_HIP(hipEventCreate(&e1), "hipEventCreate");
    auto time_layout = [&](const paf_layout& l, float& ms) -> paf_status {
        paf_status r = run_persistent(ctx, p, eng, emax, l, s, false);  // warm-up
        if (r != PAF_OK) return r;
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            PAF_HIP(hipEventRecord(e0, s), "hipEventRecord");
            r = run_persistent(ctx, p, eng, emax, l, s, false);
            if (r != PAF_OK) return r;
            PAF_HIP(hipEventRecord(e1, s), "hipEventRecord");
            PAF_HIP(hipEventSynchronize(e1), "hipEventSynchronize");
            float t = 0;
            PAF_HIP(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
            best = std::min(best, t);
        }
        ms = best;
        return PAF_OK;
    };
    paf_layout best_l = default_layout();
    float best_t = 1e30f, def_t = 0;
    st = time_layout(default_layout(), def_t);
    if (st == PAF_OK) {
        best_t = def_t;
        for (const auto& l : cands) {
            float t = 0;
            st = time_layout(l, t);
            if (st != PAF_OK) break;
            if (t < best_t) {
                best_t = t;
                best_l = l;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != PAF_OK) return st;
    ctx->tuned[std::make_tuple((int)p.wmax, emax, p.filters)] = best_l;
    if (chosen) *chosen = best_l;
    if (best_ms) *best_ms = best_t;
    if (default_ms) *default_ms = def_t;
    return PAF_OK;
}

paf_status paf_mlp_predict(paf_ctx* ctx, const paf_batch* batch, float* pred, void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, PAF_SNEAKYSNAKE, p);
    if (st != PAF_OK) return st;
    if (!pred) return fail(PAF_ERR_ARG, "pred is NULL");
    if (!ctx->mlp_ready) return fail(PAF_ERR_STATE, "no cost model: call paf_mlp_set_params first");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    PAF_HIP(launch_learned_buckets(ctx->mlp, p, ctx->num_cus, pred, nullptr, (hipStream_t)stream),
            "cost model launch");
    return PAF_OK;
}

paf_status paf_bucket(paf_ctx* ctx, const paf_batch* batch, const float* pred, uint32_t* perm, uint32_t* hist,
                      void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, PAF_SNEAKYSNAKE, p);
    if (st != PAF_OK) return st;
    if (!pred || !perm || !hist) return fail(PAF_ERR_ARG, "pred/perm/hist is NULL");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    if ((st = ensure_bucket_ws(ctx, p.n_pairs)) != PAF_OK) return st;
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    hipStream_t s = (hipStream_t)stream;
    PAF_HIP(launch_bucket_from_pred(p, pred, ctx->ws_bucket, s), "bucket keys");
    PAF_HIP(launch_bucket_sort(ctx->ws_bucket, p.n_pairs, ctx->ws_counts, perm, hist, s), "bucket sort");
    return PAF_OK;
}

paf_status paf_filter_ordered(paf_ctx* ctx, const paf_batch* batch, uint32_t filters, const uint32_t* order,
                              const paf_out* out, void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    if (!order) return fail(PAF_ERR_ARG, "order is NULL");
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    FilterParams q = p;
    q.perm = order;
    for (int f = 0; f < 3; ++f) {
        q.acc[f] = nullptr;
        q.cnt[f] = ((filters >> f) & 1u) ? out->count[f] : nullptr;
    }
    hipStream_t s = (hipStream_t)stream;
    const paf_layout L = layout_for(ctx, p, emax, false);
    if ((st = run_persistent(ctx, q, engine_for(filters), emax, L, s, true)) != PAF_OK) return st;
    for (int f = 0; f < 3; ++f)
        if ((filters >> f) & 1u)
            PAF_HIP(launch_accept_from_counts(out->count[f], p.len, p.uniform_len, p.E, p.uniform_E, p.max_len,
                                              p.max_E, p.n_pairs, out->accept_bits[f], s),
                    "accept bits");
    return PAF_OK;
}

paf_status paf_filter_bucketed(paf_ctx* ctx, const paf_batch* batch, uint32_t filters, const paf_out* out,
                               void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    if (!ctx->mlp_ready) return fail(PAF_ERR_STATE, "no cost model: call paf_mlp_set_params first");
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    if ((st = ensure_bucket_ws(ctx, p.n_pairs)) != PAF_OK) return st;
    FilterParams q = p;
    q.perm = ctx->ws_perm;
    for (int f = 0; f < 3; ++f) {
        q.acc[f] = nullptr;
        q.cnt[f] = ((filters >> f) & 1u) ? out->count[f] : nullptr;
    }
    const Engine eng = engine_for(filters);
    const paf_layout L = layout_for(ctx, p, emax, false);
    paf_ctx::GraphKey key{0, 0, 0, 0};
    const uint64_t* words = reinterpret_cast<const uint64_t*>(&q);
    for (size_t i = 0; i < sizeof(q) / 8; ++i) key.a = mix(key.a, words[i]);
    key.b = mix(mix(0xB0C4E7ull, (uint64_t)emax), (uint64_t)L.waves_per_block);
    key.c = mix(mix(mix(L.blocks_per_cu, L.tiles_per_grab), L.chunk_tiles),
                (uint64_t)(uintptr_t)out->accept_bits[0]);
    key.d = mix(mix((uint64_t)(uintptr_t)out->accept_bits[1], (uint64_t)(uintptr_t)out->accept_bits[2]),
                p.n_pairs);
    return run_graph(ctx, key, (hipStream_t)stream, [&](hipStream_t s) -> paf_status {
        PAF_HIP(launch_learned_buckets(ctx->mlp, p, ctx->num_cus, nullptr, ctx->ws_bucket, s), "cost model");
        PAF_HIP(launch_bucket_sort(ctx->ws_bucket, p.n_pairs, ctx->ws_counts, ctx->ws_perm, ctx->ws_hist, s),
                "bucket sort");
        paf_status r = run_persistent(ctx, q, eng, emax, L, s, false);
        if (r != PAF_OK) return r;
        for (int f = 0; f < 3; ++f)
            if ((filters >> f) & 1u)
                PAF_HIP(launch_accept_from_counts(out->count[f], p.len, p.uniform_len, p.E, p.uniform_E, p.max_len,
                                                  p.max_E, p.n_pairs, out->accept_bits[f], s),
                        "accept bits");
        return PAF_OK;
    });
}

paf_status paf_cost_levels(paf_ctx* ctx, const paf_batch* batch, uint8_t* key, void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, PAF_SNEAKYSNAKE, p);
    if (st != PAF_OK) return st;
    if (!key) return fail(PAF_ERR_ARG, "key is NULL");
    if (!ctx->mlp_ready) return fail(PAF_ERR_STATE, "no cost model: call paf_mlp_set_params first");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    PAF_HIP(launch_learned_buckets(ctx->mlp, p, ctx->num_cus, nullptr, key, (hipStream_t)stream, true),
            "cost model launch");
    return PAF_OK;
}

// Layout of the keyed compacting launch: the forced or tuned one if it
// compacts, else paf_filter's.
paf_layout keyed_layout(paf_ctx* ctx, const FilterParams& p, int emax) {
    paf_layout L = layout_for(ctx, p, emax, false);
    if (L.chunk_tiles == 0) L = plain_layout(emax);
    return L;
}

paf_status paf_filter_keyed(paf_ctx* ctx, const paf_batch* batch, const uint8_t* key, const paf_out* out,
                            void* stream) {
    const uint32_t filters = PAF_SNEAKYSNAKE;
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    if (!key) return fail(PAF_ERR_ARG, "key is NULL");
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    set_outputs(p, out);
    p.order_key = key;
    return run_persistent(ctx, p, Engine::Snake, emax, keyed_layout(ctx, p, emax), (hipStream_t)stream, true);
}

paf_status paf_filter_bucketed_local(paf_ctx* ctx, const paf_batch* batch, const paf_out* out, void* stream) {
    const uint32_t filters = PAF_SNEAKYSNAKE;
    FilterParams p;
    paf_status st = check_batch(ctx, batch, filters, p);
    if (st != PAF_OK) return st;
    if ((st = check_out(out, filters)) != PAF_OK) return st;
    if (!ctx->mlp_ready) return fail(PAF_ERR_STATE, "no cost model: call paf_mlp_set_params first");
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    if ((st = ensure_bucket_ws(ctx, p.n_pairs)) != PAF_OK) return st;
    set_outputs(p, out);
    FilterParams q = p;
    q.order_key = ctx->ws_bucket;
    const paf_layout L = keyed_layout(ctx, p, emax);
    paf_ctx::GraphKey key{0, 0, 0, 0};
    const uint64_t* words = reinterpret_cast<const uint64_t*>(&q);
    for (size_t i = 0; i < sizeof(q) / 8; ++i) key.a = mix(key.a, words[i]);
    key.b = mix(mix(0x10CA1ull, (uint64_t)emax), (uint64_t)L.waves_per_block);
    key.c = mix(mix(L.blocks_per_cu, L.tiles_per_grab), L.chunk_tiles);
    key.d = p.n_pairs;
    return run_graph(ctx, key, (hipStream_t)stream, [&](hipStream_t s) -> paf_status {
        PAF_HIP(launch_learned_buckets(ctx->mlp, p, ctx->num_cus, nullptr, ctx->ws_bucket, s, true), "cost model");
        return run_persistent(ctx, q, Engine::Snake, emax, L, s, false);
    });
}

}  // extern "C"
