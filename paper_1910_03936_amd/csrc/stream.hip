// Streaming filter: pairs held in host memory are copied chunk by chunk to
// the device on a copy stream while the previous chunk is filtered on a
// compute stream (double-buffered), the way the FPGA system streamed pairs
// over PCIe and returned one decision bit per pair (Ch. 4, Secs. 4.2-4.4).
#include <string.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <vector>

#include "paf_internal.h"

using namespace paf;

namespace {

// Word offsets of a chunk's pairs from their lengths: an exclusive scan of
// ceil(len / 32) in three passes (block sums, scan of the sums, apply).
constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(256) words_block_sum_kernel(const uint16_t* len, uint64_t n, uint32_t* sums) {
    __shared__ uint32_t red[256];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
    for (uint32_t i = threadIdx.x; i < kScanBlock; i += blockDim.x) {
        const uint64_t p = base + i;
        if (p < n) s += (len[p] + 31u) >> 5;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// One block: exclusive scan of the block sums into 64-bit bases.
__global__ void __launch_bounds__(1024) block_base_kernel(const uint32_t* sums, uint32_t nb, uint64_t* base) {
    __shared__ uint64_t wtot[16];
    __shared__ uint64_t carry;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
        const uint64_t v = b0 + t < nb ? sums[b0 + t] : 0u;
        uint64_t inc = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t o = __shfl_up(inc, off);
            if (lane >= (uint32_t)off) inc += o;
        }
        if (lane == 63) wtot[wv] = inc;
        __syncthreads();
        uint64_t before = carry;
        for (uint32_t w = 0; w < wv; ++w) before += wtot[w];
        if (b0 + t < nb) base[b0 + t] = before + inc - v;
        __syncthreads();
        if (t == 0) {
            uint64_t tot = 0;
            for (int w = 0; w < 16; ++w) tot += wtot[w];
            carry += tot;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanBlock) words_offset_kernel(const uint16_t* len, uint64_t n,
                                                                   const uint64_t* base, uint64_t* off) {
    __shared__ uint32_t wtot[16];
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint64_t p = (uint64_t)blockIdx.x * kScanBlock + t;
    const uint32_t v = p < n ? ((len[p] + 31u) >> 5) : 0u;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t x = __shfl_up(inc, o);
        if (lane >= (uint32_t)o) inc += x;
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t w = 0; w < wv; ++w) before += wtot[w];
    if (p < n) off[p] = base[blockIdx.x] + before + inc - v;
}

struct Slot {
    uint64_t* rd = nullptr;
    uint64_t* rf = nullptr;
    uint16_t* len = nullptr;
    uint8_t* E = nullptr;
    uint64_t* off = nullptr;
    uint32_t* sums = nullptr;
    uint64_t* base = nullptr;
    uint32_t* acc[3] = {nullptr, nullptr, nullptr};
    uint16_t* cnt[3] = {nullptr, nullptr, nullptr};
    hipEvent_t copied = nullptr, computed = nullptr, drained = nullptr;
};

void free_slot(Slot& s) {
    for (void* p : {(void*)s.rd, (void*)s.rf, (void*)s.len, (void*)s.E, (void*)s.off, (void*)s.sums, (void*)s.base})
        if (p) hipFree(p);
    for (int f = 0; f < 3; ++f) {
        if (s.acc[f]) hipFree(s.acc[f]);
        if (s.cnt[f]) hipFree(s.cnt[f]);
    }
    if (s.copied) hipEventDestroy(s.copied);
    if (s.computed) hipEventDestroy(s.computed);
    if (s.drained) hipEventDestroy(s.drained);
    s = Slot{};
}

}  // namespace

extern "C" {

paf_status paf_stream_filter(paf_ctx* ctx, const paf_host_batch* hb, uint64_t chunk_pairs, uint32_t filters,
                             int learned, const paf_out* host_out, paf_stream_stats* stats) {
    if (!ctx || !hb || !host_out) return fail(PAF_ERR_ARG, "ctx/batch/out is NULL");
    if (!hb->reads || !hb->refs || !hb->len || !hb->E) return fail(PAF_ERR_ARG, "host batch has a NULL array");
    if (hb->n_pairs == 0) return fail(PAF_ERR_ARG, "batch has no pairs");
    if (chunk_pairs == 0 || chunk_pairs % 64 != 0) return fail(PAF_ERR_ARG, "chunk_pairs must be a positive multiple of 64");
    if (filters == 0 || filters > 7u) return fail(PAF_ERR_ARG, "filters must be a nonzero mask of PAF_* bits");
    if (hb->max_len < 1 || hb->max_len > PAF_MAX_LEN || hb->max_E > PAF_MAX_E)
        return fail(PAF_ERR_RANGE, "max_len/max_E outside the supported range");
    for (int f = 0; f < 3; ++f)
        if ((filters >> f) & 1u)
            if (!host_out->accept_bits[f] || !host_out->count[f])
                return fail(PAF_ERR_ARG, "a requested filter has a NULL output pointer");
    if (learned && !ctx->mlp_ready) return fail(PAF_ERR_STATE, "no cost model: call paf_mlp_set_params first");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");

    const uint64_t n = hb->n_pairs;
    const uint64_t nchunks = (n + chunk_pairs - 1) / chunk_pairs;
    // Word position of every chunk's first pair (pairs are stored back to back).
    std::vector<uint64_t> cw(nchunks + 1, 0);
    {
        const int T = (int)std::min<uint64_t>(16, std::max<uint64_t>(1, nchunks));
        std::vector<std::thread> pool;
        for (int t = 0; t < T; ++t)
            pool.emplace_back([&, t]() {
                for (uint64_t c = t; c < nchunks; c += T) {
                    const uint64_t a = c * chunk_pairs, b = std::min(n, a + chunk_pairs);
                    uint64_t w = 0;
                    for (uint64_t p = a; p < b; ++p) {
                        if (hb->len[p] < 1 || hb->len[p] > hb->max_len) w = UINT64_MAX / 4;
                        w += (hb->len[p] + 31u) >> 5;
                    }
                    cw[c + 1] = w;
                }
            });
        for (auto& th : pool) th.join();
        for (uint64_t c = 0; c < nchunks; ++c) {
            if (cw[c + 1] >= UINT64_MAX / 4) return fail(PAF_ERR_RANGE, "a pair length is outside [1, max_len]");
            cw[c + 1] += cw[c];
        }
    }
    uint64_t max_words = 0;
    for (uint64_t c = 0; c < nchunks; ++c) max_words = std::max(max_words, cw[c + 1] - cw[c]);

    hipStream_t copy = nullptr, comp = nullptr;
    PAF_HIP(hipStreamCreateWithFlags(&copy, hipStreamNonBlocking), "hipStreamCreate");
    if (hipStreamCreateWithFlags(&comp, hipStreamNonBlocking) != hipSuccess) {
        hipStreamDestroy(copy);
        return fail(PAF_ERR_DEVICE, "hipStreamCreate");
    }
    Slot slots[2];
    paf_status st = PAF_OK;
    const uint32_t nsb = (uint32_t)((chunk_pairs + kScanBlock - 1) / kScanBlock);
    for (auto& s : slots) {
        bool ok = hipMalloc(&s.rd, max_words * 8) == hipSuccess && hipMalloc(&s.rf, max_words * 8) == hipSuccess &&
                  hipMalloc(&s.len, chunk_pairs * 2) == hipSuccess && hipMalloc(&s.E, chunk_pairs) == hipSuccess &&
                  hipMalloc(&s.off, chunk_pairs * 8) == hipSuccess && hipMalloc(&s.sums, nsb * 4) == hipSuccess &&
                  hipMalloc(&s.base, nsb * 8) == hipSuccess;
        for (int f = 0; f < 3 && ok; ++f)
            if ((filters >> f) & 1u)
                ok = hipMalloc(&s.acc[f], chunk_pairs / 8) == hipSuccess &&
                     hipMalloc(&s.cnt[f], chunk_pairs * 2) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&s.copied, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&s.computed, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&s.drained, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            st = fail(PAF_ERR_NOMEM, "streaming buffers");
            break;
        }
    }
    double h2d = 0;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint64_t c = 0; c < nchunks && st == PAF_OK; ++c) {
        Slot& s = slots[c % 2];
        const uint64_t a = c * chunk_pairs, m = std::min(chunk_pairs, n - a);
        const uint64_t w0 = cw[c], nw = cw[c + 1] - cw[c];
        // The slot's previous chunk must have been filtered and drained.
        if (c >= 2 && hipStreamWaitEvent(copy, s.drained, 0) != hipSuccess) { st = fail(PAF_ERR_DEVICE, "wait"); break; }
        bool ok = hipMemcpyAsync(s.rd, hb->reads + w0, nw * 8, hipMemcpyHostToDevice, copy) == hipSuccess &&
                  hipMemcpyAsync(s.rf, hb->refs + w0, nw * 8, hipMemcpyHostToDevice, copy) == hipSuccess &&
                  hipMemcpyAsync(s.len, hb->len + a, m * 2, hipMemcpyHostToDevice, copy) == hipSuccess &&
                  hipMemcpyAsync(s.E, hb->E + a, m, hipMemcpyHostToDevice, copy) == hipSuccess &&
                  hipEventRecord(s.copied, copy) == hipSuccess && hipStreamWaitEvent(comp, s.copied, 0) == hipSuccess;
        if (!ok) { st = fail(PAF_ERR_DEVICE, "chunk copy"); break; }
        h2d += (double)nw * 16 + (double)m * 3;
        const uint32_t nb = (uint32_t)((m + kScanBlock - 1) / kScanBlock);
        hipLaunchKernelGGL(words_block_sum_kernel, dim3(nb), dim3(256), 0, comp, s.len, m, s.sums);
        hipLaunchKernelGGL(block_base_kernel, dim3(1), dim3(1024), 0, comp, s.sums, nb, s.base);
        hipLaunchKernelGGL(words_offset_kernel, dim3(nb), dim3(kScanBlock), 0, comp, s.len, m, s.base, s.off);
        paf_batch b{};
        b.reads = s.rd;
        b.refs = s.rf;
        b.word_offset = s.off;
        b.len = s.len;
        b.E = s.E;
        b.max_len = hb->max_len;
        b.max_E = hb->max_E;
        b.n_pairs = m;
        paf_out o{};
        for (int f = 0; f < 3; ++f) {
            o.accept_bits[f] = s.acc[f];
            o.count[f] = s.cnt[f];
        }
        st = !learned ? paf_filter(ctx, &b, filters, &o, comp)
             : filters == PAF_SNEAKYSNAKE ? paf_filter_bucketed_local(ctx, &b, &o, comp)
                                          : paf_filter_bucketed(ctx, &b, filters, &o, comp);
        if (st != PAF_OK) break;
        ok = hipEventRecord(s.computed, comp) == hipSuccess && hipStreamWaitEvent(copy, s.computed, 0) == hipSuccess;
        for (int f = 0; f < 3 && ok; ++f)
            if ((filters >> f) & 1u)
                ok = hipMemcpyAsync(host_out->accept_bits[f] + a / 32, s.acc[f], (m + 31) / 32 * 4,
                                    hipMemcpyDeviceToHost, copy) == hipSuccess &&
                     hipMemcpyAsync(host_out->count[f] + a, s.cnt[f], m * 2, hipMemcpyDeviceToHost, copy) ==
                         hipSuccess;
        ok = ok && hipEventRecord(s.drained, copy) == hipSuccess;
        if (!ok) st = fail(PAF_ERR_DEVICE, "chunk results");
    }
    hipStreamSynchronize(comp);
    hipStreamSynchronize(copy);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (auto& s : slots) free_slot(s);
    hipStreamDestroy(copy);
    hipStreamDestroy(comp);
    if (st != PAF_OK) return st;
    if (stats) {
        stats->seconds = secs;
        stats->h2d_bytes = h2d;
        stats->chunks = nchunks;
    }
    return PAF_OK;
}

}  // extern "C"
