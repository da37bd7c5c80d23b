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
// One lane per pair, two kernels.  The first reads each pair's words
// straight from memory and only asks whether some diagonal has a run of at
// least ceil((m - E) / (E + 1)) = floor(m / (E + 1)) free cells: without one
// the pair is rejected (Sec. 7.2's first test: E + 1 runs that short cannot
// cover m - E columns), and with E = 0 the answer decides the pair; the
// others are flagged.  A stable counting sort of the flags (the bucketing
// kernels) lists the flagged pairs first, and the second kernel's waves take
// that list 64 pairs at a time through the extractions;
// a pair is also rejected as soon as the runs still to come, none longer than
// the last one, cannot reach m - E columns.
//
// A diagonal's longest run is found word by word: the run that enters a
// 32-column word from below ends at the word's first blocked column (a
// trailing-zero count), the longest run inside the word comes from a binary
// lifting over the word's runs of 1, 2, 4, 8 and 16 free cells, and the free
// cells at the word's top carry into the next word.
#include <algorithm>

#include "paf_tile.h"

namespace paf {

namespace {

// LDS of one wave, in 8-byte words: the excluded-column rows (4 bytes per
// word and lane) and the best-run cache (4 bytes per diagonal and lane).
__host__ __device__ constexpr size_t magnet_wave_words(uint32_t wmax, int D) {
    return ((size_t)wmax * kLdsRow + 1) / 2 + (size_t)D * 32;
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

// Whether some diagonal has a run of at least `need` free cells: per word,
// the run entering from below (carry + trailing free cells) and the runs
// inside the word (x AND-ed with itself shifted by sh[0..5], which add up to
// need - 1, leaves the starts of runs of need cells).
template <int EMAX, int I = 0>
__device__ __forceinline__ void magnet_has_run(const WindowWords& q, uint32_t blocked, int E, uint32_t need,
                                               const uint32_t* sh, uint32_t* carry, bool& found) {
    if constexpr (I < 2 * EMAX + 1) {
        constexpr int d = I - EMAX;
        const bool on = (d < 0 ? -d : d) <= E;
        const uint32_t x = on ? ~(diag_raw<d>(q) | diag_vacant<d>(q) | blocked) : 0u;
        const uint32_t t = x == ~0u ? 32u : (uint32_t)__builtin_ctz(~x);
        uint32_t r = x;
#pragma unroll
        for (int j = 0; j < 6; ++j) r &= r >> sh[j];
        found = found || carry[I] + t >= need || (need <= 32u && r != 0u);
        carry[I] = x == ~0u ? carry[I] + 32u : (x == 0u ? 0u : (uint32_t)__builtin_clz(~x));
        magnet_has_run<EMAX, I + 1>(q, blocked, E, need, sh, carry, found);
    }
}

template <int EMAX>
__device__ bool magnet_first_test(const uint64_t* rd, const uint64_t* rf, int W, int m, int E, uint32_t need) {
    constexpr int D = 2 * EMAX + 1;
    uint32_t carry[D];
#pragma unroll
    for (int i = 0; i < D; ++i) carry[i] = 0u;
    // Shifts that add up to need - 1 (each at most the run length so far).
    uint32_t sh[6];
    uint32_t len = 1;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const uint32_t want = need > len ? need - len : 0u;
        sh[j] = min(len, min(want, 31u));
        len += sh[j];
    }
    bool found = need == 0u;
    for (int k = 0; k < W; ++k) {
        const WindowWords q = window_words_direct(rd, rf, k, W, m);
        magnet_has_run<EMAX>(q, q.vc, E, need, sh, carry, found);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) found = found || carry[i] >= need;
    return found;
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

// A diagonal's best run (the longest, then the earliest) packed as L << 16 | s.
__device__ __forceinline__ uint32_t run_pack(uint32_t L, uint32_t s) { return (L << 16) | s; }

// Offer the run [s, s + L) of one diagonal to that diagonal's best.
__device__ __forceinline__ void diag_offer(uint32_t& bL, uint32_t& bS, uint32_t L, uint32_t s) {
    const bool take = L > bL || (L == bL && L > 0 && s < bS);
    bL = take ? L : bL;
    bS = take ? s : bS;
}

// One word x of a diagonal: the run entering from below ends at the word's
// first blocked column; runs inside the word are searched when one could
// beat the diagonal's best; the free cells at the top carry on.
__device__ __forceinline__ void diag_word(uint32_t x, uint32_t k, uint32_t& carry, uint32_t& bL, uint32_t& bS) {
    if (x == ~0u) {
        carry += 32u;
        return;
    }
    const uint32_t t = (uint32_t)__builtin_ctz(~x);
    diag_offer(bL, bS, carry + t, 32u * k - carry);
    const uint32_t pc = popc(x);
    if (pc > bL || (pc == bL && 32u * k < bS)) {
        uint32_t L, s;
        word_longest(x, L, s);
        diag_offer(bL, bS, L, 32u * k + s);
    }
    carry = x == 0u ? 0u : (uint32_t)__builtin_clz(~x);
}

// The best run of one diagonal d (chosen at run time, |d| <= 31) of the pair
// whose W words start at rd and rf.
__device__ uint32_t scan_one(const uint64_t* rd, const uint64_t* rf, const uint32_t* goneL, int lane, uint32_t W,
                             int m, int d) {
    uint32_t carry = 0, bL = 0, bS = 0;
    const uint32_t sp = (uint32_t)d, sn = (uint32_t)(32 + d);
    for (uint32_t k = 0; k < W; ++k) {
        const WindowWords q = window_words_direct(rd, rf, (int)k, (int)W, m);
        uint32_t lo, hi, v;
        if (d > 0) {
            lo = funnel(q.nlo, q.clo, sp);
            hi = funnel(q.nhi, q.chi, sp);
            v = funnel(q.vn, q.vc, sp);
        } else if (d < 0) {
            lo = funnel(q.clo, q.plo, sn);
            hi = funnel(q.chi, q.phi, sn);
            v = funnel(q.vc, q.vp, sn);
        } else {
            lo = q.clo;
            hi = q.chi;
            v = q.vc;
        }
        const uint32_t x = ~((lo ^ q.flo) | (hi ^ q.fhi) | v | q.vc | goneL[k * kLdsRow + lane]);
        diag_word(x, k, carry, bL, bS);
    }
    diag_offer(bL, bS, carry, 32u * W - carry);
    return run_pack(bL, bS);
}

// Threshold test of every pair; flag[p] = 0 for the pairs left undecided,
// 1 for the others (the order the counting sort puts them in).
template <int EMAX, bool GENERAL>
__global__ void __launch_bounds__(256) magnet_test_kernel(FilterParams P, uint8_t* flag) {
    const int lane = threadIdx.x & 63;
    const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= P.n_tiles) return;
    uint64_t off = 0;
    PairSlot s = load_slot<GENERAL>(P, tile, lane, off);
    if (!s.in_batch) return;
    if (!s.valid) {
        P.cnt[0][s.id] = 0;
        flag[s.id] = 1;
        return;
    }
    const uint32_t need = s.m / (s.E + 1u);
    const bool found = magnet_first_test<EMAX>(P.reads + off, P.refs + off, (int)s.W, (int)s.m, (int)s.E, need);
    if (!found) P.cnt[0][s.id] = (uint16_t)(s.E + 1u);
    else if (s.E == 0) P.cnt[0][s.id] = 0;
    flag[s.id] = found && s.E > 0 ? 0 : 1;
}

template <int EMAX>
__global__ void __launch_bounds__(256) magnet_kernel(FilterParams P, const uint32_t* order, const uint32_t* count) {
    constexpr int D = 2 * EMAX + 1;
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t wmax = P.wmax;
    const size_t per_wave = magnet_wave_words(wmax, D);
    uint32_t* goneL = reinterpret_cast<uint32_t*>(lds + (size_t)wave * per_wave);
    uint32_t* cache = goneL + (size_t)wmax * kLdsRow;
    const uint32_t n_sel = *count;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);

    // The extractions of the flagged pairs, 64 at a time.
    // Each diagonal's best run is kept in `cache`; after an extraction only
    // the diagonals whose best run meets the excluded columns are searched
    // again (the others keep their best: excluding columns only shortens
    // runs).
    for (uint32_t h = (blockIdx.x * (blockDim.x >> 6) + wave) * 64u; h < n_sel; h += waves * 64u) {
        const uint32_t j = h + (uint32_t)lane;
        const bool valid = j < n_sel;
        PairSlot s;
        s.valid = s.in_batch = valid;
        s.slot = s.id = valid ? order[j] : 0u;
        s.m = valid ? (P.len ? P.len[s.id] : P.uniform_len) : 0u;
        s.E = valid ? (P.E ? P.E[s.id] : P.uniform_E) : 0u;
        s.W = (s.m + 31) >> 5;
        const uint64_t off = !valid ? 0 : P.word_offset ? P.word_offset[s.id] : s.id * (uint64_t)P.stride_words;
        // The pair's words are read straight from memory (they stay in the
        // caches across its extractions).
        const uint64_t* rd = P.reads + off;
        const uint64_t* rf = P.refs + off;
        for (uint32_t k = 0; k < wmax; ++k) goneL[k * kLdsRow + lane] = 0u;
        for (int i = 0; i < D; ++i) {
            const int d = i - EMAX;
            const bool on = valid && (d < 0 ? -d : d) <= (int)s.E;
            cache[i * 64 + lane] = on ? scan_one(rd, rf, goneL, lane, s.W, (int)s.m, d) : 0u;
        }
        uint32_t covered = 0;
        bool act = valid, rejected = false;
        for (uint32_t it = 1; act; ++it) {
            // The best run over all diagonals (ties: earliest start, then
            // the first diagonal).
            uint32_t bL = 0, bS = 0;
            for (int i = 0; i < D; ++i) {
                const uint32_t v = cache[i * 64 + lane];
                diag_offer(bL, bS, v >> 16, v & 0xFFFFu);
            }
            if (bL == 0) break;
            covered += bL;
            const uint32_t a = bS > 0 ? bS - 1u : 0u, b = min(bS + bL + 1u, s.m);
            magnet_exclude(goneL, lane, wmax, a, b);
            // The E + 1 - it runs still to come are no longer than this one.
            if (covered + (s.E + 1u - it) * bL + s.E < s.m) {
                rejected = true;
                break;
            }
            if (it > s.E || covered >= s.m) break;
            uint64_t dirty = 0;
            for (int i = 0; i < D; ++i) {
                const uint32_t v = cache[i * 64 + lane];
                const uint32_t L = v >> 16, st = v & 0xFFFFu;
                if (L > 0 && st < b && st + L > a) dirty |= 1ull << i;
            }
            while (dirty) {
                const int i = __builtin_ctzll(dirty);
                dirty &= dirty - 1;
                cache[i * 64 + lane] = scan_one(rd, rf, goneL, lane, s.W, (int)s.m, i - EMAX);
            }
        }
        if (valid) P.cnt[0][s.id] = (uint16_t)(rejected ? s.E + 1u : min(s.m - covered, s.E + 1u));
        wave_lds_sync();
    }
}

template <bool GENERAL>
const void* magnet_test_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&magnet_test_kernel<X, GENERAL>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
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

hipError_t launch_magnet(const FilterParams& p, int emax, uint8_t* flag, uint32_t* counts, uint32_t* order,
                         uint32_t* hist, int num_cus, hipStream_t s) {
    const bool general = p.len || p.E || p.word_offset;
    const void* kt = general ? magnet_test_kernel_for<true>(emax) : magnet_test_kernel_for<false>(emax);
    const void* k = magnet_kernel_for(emax);
    if (!kt || !k) return hipErrorInvalidValue;
    FilterParams arg = p;
    const uint32_t waves = 4;
    {
        const uint32_t blocks = (uint32_t)((p.n_tiles + waves - 1) / waves);
        void* args[] = {&arg, &flag};
        hipError_t e = hipLaunchKernel(kt, dim3(blocks), dim3(64 * waves), args, 0, s);
        if (e != hipSuccess) return e;
    }
    // Undecided pairs first (flag 0), in pair order.
    hipError_t e = launch_bucket_sort(flag, p.n_pairs, counts, order, hist, s);
    if (e != hipSuccess) return e;
    // A grid that fills the chip; its waves stride over the list.
    const size_t lds = waves * magnet_wave_words(p.wmax, 2 * emax + 1) * sizeof(uint64_t);
    if (lds > 65536) {
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int nb = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * waves, lds) != hipSuccess || nb < 1) nb = 1;
    const uint64_t groups = (p.n_pairs + 63) / 64;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)num_cus * nb,
                                                                               (groups + waves - 1) / waves));
    const uint32_t* o = order;
    const uint32_t* c = hist;
    void* args[] = {&arg, &o, &c};
    e = hipLaunchKernel(k, dim3(blocks), dim3(64 * waves), args, lds, s);
    if (e != hipSuccess) return e;
    return launch_accept_from_counts(p.cnt[0], p.len, p.uniform_len, p.E, p.uniform_E, p.max_len, p.max_E,
                                     p.n_pairs, p.acc[0], s);
}

}  // namespace paf
