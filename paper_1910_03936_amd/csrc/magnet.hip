// MAGNET decision stage (Ch. 7) on the neighbourhood map of Ch. 6 (vacant
// cells blocked).  Extraction: the longest run of free cells over all 2E+1
// diagonals among the columns still in the search space (ties: the smallest
// start column, then the first diagonal in order -E..E).  Encapsulation: the
// run's columns and one column on each side leave the search space of every
// diagonal.  The search repeats, longest run first, until E + 1 runs are
// found or no free cell is left (the hardware form of Sec. 7.4: one problem
// of fixed size, excluded columns set to ones).  count = min(m - covered,
// E + 1), accept = count <= E.
//
// One lane per pair.  A wave owns a chunk of tiles: the first pass stages
// each group of 64 pairs, makes the first extraction and decides the pairs
// whose longest run is shorter than ceil((m - E) / (E + 1)) (Sec. 7.2's first
// test: E + 1 runs that short cannot cover m - E columns), those whose run
// covers the pair, and E = 0; the others go on a list in LDS with their first
// run, and later groups of 64 of them make the remaining extractions.
//
// A diagonal's longest run is found word by word: the run that enters a
// 32-column word from below ends at the word's first blocked column (a
// trailing-zero count), the longest run inside the word comes from a binary
// lifting over the word's runs of 1, 2, 4, 8 and 16 free cells, and the free
// cells at the word's top carry into the next word.
#include "paf_tile.h"

namespace paf {

namespace {

constexpr uint32_t kMagnetTiles = 16;

struct Run {
    uint32_t L, s;
    int d;
};

// a beats b: longer; else starts earlier; else the earlier diagonal.
__device__ __forceinline__ bool run_better(uint32_t L, uint32_t s, int d, const Run& b) {
    return L > b.L || (L == b.L && L > 0 && (s < b.s || (s == b.s && d < b.d)));
}

__device__ __forceinline__ void run_offer(Run& b, uint32_t L, uint32_t s, int d) {
    if (run_better(L, s, d, b)) b = Run{L, s, d};
}

// Longest run of ones inside one word x != ~0 and its lowest start.
__device__ __forceinline__ void word_longest(uint32_t x, uint32_t& L, uint32_t& s) {
    const uint32_t a1 = x;
    const uint32_t a2 = a1 & (a1 >> 1);
    const uint32_t a4 = a2 & (a2 >> 2);
    const uint32_t a8 = a4 & (a4 >> 4);
    const uint32_t a16 = a8 & (a8 >> 8);
    uint32_t cur = ~0u, len = 0;
    uint32_t c;
    c = cur & (a16 >> len); if (c) { cur = c; len += 16; }
    c = cur & (a8 >> len);  if (c) { cur = c; len += 8; }
    c = cur & (a4 >> len);  if (c) { cur = c; len += 4; }
    c = cur & (a2 >> len);  if (c) { cur = c; len += 2; }
    c = cur & (a1 >> len);  if (c) { cur = c; len += 1; }
    L = len;
    s = len ? (uint32_t)__builtin_ctz(cur) : 0u;
}

// One extraction over the lane's staged pair: the best run among the columns
// whose bit in the lane's `gone` row is clear.
template <int EMAX, int I = 0>
__device__ __forceinline__ void magnet_word(const WindowWords& q, uint32_t blocked, uint32_t k, int E,
                                            uint32_t* carry, Run& best) {
    if constexpr (I < 2 * EMAX + 1) {
        constexpr int d = I - EMAX;
        const bool on = (d < 0 ? -d : d) <= E;
        const uint32_t x = on ? ~(diag_raw<d>(q) | diag_vacant<d>(q) | blocked) : 0u;
        if (x == ~0u) {
            carry[I] += 32u;
        } else {
            // The run entering from below ends at this word's first blocked
            // column.
            const uint32_t t = (uint32_t)__builtin_ctz(~x);
            run_offer(best, carry[I] + t, 32u * k - carry[I], d);
            // Runs inside the word, when one could beat the best so far.
            const uint32_t pc = popc(x);
            const bool try_in = pc > best.L || (pc == best.L && 32u * k < best.s);
            if (wave_any(try_in)) {
                uint32_t L, s;
                word_longest(x, L, s);
                run_offer(best, L, 32u * k + s, d);
            }
            carry[I] = x == 0u ? 0u : (uint32_t)__builtin_clz(~x);
        }
        magnet_word<EMAX, I + 1>(q, blocked, k, E, carry, best);
    }
}

template <int EMAX>
__device__ Run magnet_extract(const uint64_t* rdL, const uint64_t* rfL, const uint32_t* goneL, int lane,
                              uint32_t wmax, int m, int E) {
    constexpr int D = 2 * EMAX + 1;
    uint32_t carry[D];
#pragma unroll
    for (int i = 0; i < D; ++i) carry[i] = 0u;
    Run best{0u, 0u, 0};
    for (uint32_t k = 0; k < wmax; ++k) {
        const WindowWords q = window_words(rdL, rfL, lane, (int)k, wmax, m);
        // Columns past the pair's end and columns out of the search space.
        const uint32_t blocked = q.vc | goneL[k * kLdsRow + lane];
        magnet_word<EMAX>(q, blocked, k, E, carry, best);
    }
    // Runs that reach the last word's top (m a multiple of 32).
#pragma unroll
    for (int i = 0; i < D; ++i) run_offer(best, carry[i], 32u * wmax - carry[i], i - EMAX);
    return best;
}

// Columns [a, b) leave the search space.
__device__ __forceinline__ void magnet_exclude(uint32_t* goneL, int lane, uint32_t wmax, uint32_t a, uint32_t b) {
    for (uint32_t k = 0; k < wmax; ++k) {
        const uint32_t lo = 32u * k;
        const uint32_t x0 = a > lo ? min(a - lo, 32u) : 0u;
        const uint32_t x1 = b > lo ? min(b - lo, 32u) : 0u;
        // bits [x0, x1) of the word
        const uint32_t hi_mask = x1 >= 32u ? ~0u : ((1u << x1) - 1u);
        const uint32_t lo_mask = x0 >= 32u ? ~0u : ((1u << x0) - 1u);
        goneL[k * kLdsRow + lane] |= hi_mask & ~lo_mask;
    }
}

__device__ __forceinline__ void magnet_encapsulate(uint32_t* goneL, int lane, uint32_t wmax, uint32_t m,
                                                   uint32_t s, uint32_t L) {
    magnet_exclude(goneL, lane, wmax, s > 0 ? s - 1u : 0u, min(s + L + 1u, m));
}

template <int EMAX>
__global__ void __launch_bounds__(256) magnet_kernel(FilterParams P) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t wmax = P.wmax;
    const size_t per_wave = (size_t)2 * wmax * kLdsRow + ((size_t)wmax * kLdsRow + 1) / 2 + kMagnetTiles * 64 / 2;
    uint64_t* rdL = lds + (size_t)wave * per_wave;
    uint64_t* rfL = rdL + (size_t)wmax * kLdsRow;
    uint32_t* goneL = reinterpret_cast<uint32_t*>(rfL + (size_t)wmax * kLdsRow);
    uint32_t* list = goneL + (size_t)wmax * kLdsRow;
    const uint64_t chunk = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    const uint64_t slot0 = chunk * kMagnetTiles * 64;
    if (slot0 >= P.n_pairs) return;
    const uint32_t n_here = (uint32_t)min<uint64_t>((uint64_t)kMagnetTiles * 64, P.n_pairs - slot0);

    // Pass 1: first extraction of every pair of the chunk.
    uint32_t n_sel = 0;
    for (uint32_t g = 0; g < n_here; g += 64) {
        const uint32_t i = g + (uint32_t)lane;
        PairSlot s;
        s.in_batch = i < n_here;
        s.valid = s.in_batch;
        s.slot = s.id = slot0 + i;
        s.m = P.uniform_len;
        s.E = P.uniform_E;
        uint64_t off = 0;
        if (s.valid) {
            if (P.len) s.m = P.len[s.id];
            if (P.E) s.E = P.E[s.id];
            off = P.word_offset ? P.word_offset[s.id] : s.id * (uint64_t)P.stride_words;
            if (s.m < 1 || s.m > P.max_len || s.E > P.max_E) {
                atomicOr(P.err, 1u);
                P.cnt[0][s.id] = 0;
                s.valid = false;
            }
        }
        if (!s.valid) s.m = 0;
        s.W = (s.m + 31) >> 5;
        stage_tile<true>(P, 0, lane, s, off, rdL, rfL);
        for (uint32_t k = 0; k < wmax; ++k) goneL[k * kLdsRow + lane] = 0u;
        const Run r = magnet_extract<EMAX>(rdL, rfL, goneL, lane, wmax, (int)s.m, (int)s.E);
        bool more = false;
        if (s.valid) {
            const uint32_t m = s.m, E = s.E;
            // Shorter than ceil((m - E) / (E + 1)) = floor(m / (E + 1)): the
            // E + 1 runs, none longer than this one, cannot cover m - E
            // columns.
            const bool short_run = r.L < m / (E + 1u);
            if (E == 0 || short_run || r.L == 0 || r.L >= m) {
                const uint32_t left = short_run ? E + 1u : m - r.L;
                P.cnt[0][s.id] = (uint16_t)min(left, E + 1u);
            } else {
                more = true;
            }
        }
        const uint64_t bal = __ballot(more);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (more) list[n_sel + below] = i | (r.s << 10) | (r.L << 19);
        n_sel += (uint32_t)__builtin_popcountll(bal);
        wave_lds_sync();
    }

    // Pass 2: the remaining extractions of the pairs still undecided.
    for (uint32_t h = 0; h < n_sel; h += 64) {
        const uint32_t j = h + (uint32_t)lane;
        const bool valid = j < n_sel;
        const uint32_t e = valid ? list[j] : 0u;
        PairSlot s;
        s.valid = s.in_batch = valid;
        s.slot = s.id = slot0 + (e & 1023u);
        s.m = valid ? (P.len ? P.len[s.id] : P.uniform_len) : 0u;
        s.E = valid ? (P.E ? P.E[s.id] : P.uniform_E) : 0u;
        s.W = (s.m + 31) >> 5;
        const uint64_t off = !valid ? 0 : P.word_offset ? P.word_offset[s.id] : s.id * (uint64_t)P.stride_words;
        stage_tile<true>(P, 0, lane, s, off, rdL, rfL);
        for (uint32_t k = 0; k < wmax; ++k) goneL[k * kLdsRow + lane] = 0u;
        uint32_t covered = 0;
        bool act = valid;
        if (valid) {
            const uint32_t s1 = (e >> 10) & 511u, L1 = (e >> 19) & 1023u;
            covered = L1;
            magnet_encapsulate(goneL, lane, wmax, s.m, s1, L1);
        }
        wave_lds_sync();
        for (uint32_t it = 1; wave_any(act); ++it) {
            const Run r = magnet_extract<EMAX>(rdL, rfL, goneL, lane, wmax, act ? (int)s.m : 0, (int)s.E);
            if (act) {
                if (r.L == 0) {
                    act = false;
                } else {
                    covered += r.L;
                    magnet_encapsulate(goneL, lane, wmax, s.m, r.s, r.L);
                    if (it >= s.E || covered >= s.m) act = false;
                }
            }
            wave_lds_sync();
        }
        if (valid) P.cnt[0][s.id] = (uint16_t)min(s.m - covered, s.E + 1u);
        wave_lds_sync();
    }
}

const void* magnet_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&magnet_kernel<X>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

}  // namespace

hipError_t launch_magnet(const FilterParams& p, int emax, hipStream_t s) {
    const void* k = magnet_kernel_for(emax);
    if (!k) return hipErrorInvalidValue;
    const uint32_t waves = 4;
    const size_t per_wave = ((size_t)2 * p.wmax * kLdsRow + ((size_t)p.wmax * kLdsRow + 1) / 2 +
                             kMagnetTiles * 64 / 2) * sizeof(uint64_t);
    const size_t lds = waves * per_wave;
    const uint64_t chunks = (p.n_pairs + kMagnetTiles * 64 - 1) / (kMagnetTiles * 64);
    const uint32_t blocks = (uint32_t)((chunks + waves - 1) / waves);
    FilterParams arg = p;
    void* args[] = {&arg};
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipLaunchKernel(k, dim3(blocks), dim3(64 * waves), args, lds, s);
    if (e != hipSuccess) return e;
    return launch_accept_from_counts(p.cnt[0], p.len, p.uniform_len, p.E, p.uniform_E, p.max_len, p.max_E,
                                     p.n_pairs, p.acc[0], s);
}

}  // namespace paf
