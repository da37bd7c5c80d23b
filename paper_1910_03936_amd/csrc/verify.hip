// Verification of the pairs a filter passes: the banded edit distance of each
// (read, reference segment) pair, min(distance, E + 1), restricted to the
// 2E+1 diagonals of the filter's map (Ukkonen's band).  This is the step the
// filter hands its accepted pairs to (Ch. 1, seed-and-extend), in the form of
// Sec. 8.7's prefix edit distance: the work grows with the number of edits
// found so far, and stops as soon as E is exceeded.
//
// One lane per pair, by diagonal transition (Ukkonen 1985; Landau and Vishkin
// 1989): F_k[d] is the furthest reference column c such that ref[0..c) and
// read[0..c+d) align with at most k edits inside the band.  From F_{k-1} on
// diagonals d-1, d and d+1 one edit more reaches column
//   x = max(F_{k-1}[d] + 1  (substitution),
//           F_{k-1}[d+1] + 1 (a reference base left out),
//           F_{k-1}[d-1]     (a read base left out)),
// and the diagonal's run of matches from x (a pipe of the map, Eq. 8.2) then
// comes for free.  The distance is the first k with F_k[0] = m.  Runs are
// found 32 bases at a time from the planar two-bit words: an XOR per code
// plane, an OR, and a count of trailing zeros.
//
// A selection (optional, e.g. the accept bits of a filter) names the pairs
// to verify; the others get E + 1.
#include "paf_tile.h"

namespace paf {

namespace {

constexpr int kNeg = -(1 << 20);

// 32 bases of one staged sequence from base position p on (planes lo, hi).
__device__ __forceinline__ void bases32(const uint64_t* rows, int lane, uint32_t p, uint32_t W, uint32_t& lo,
                                        uint32_t& hi) {
    const uint32_t k = p >> 5, sh = p & 31u;
    const uint64_t w0 = rows[k * kLdsRow + lane];
    const uint64_t w1 = k + 1 < W ? rows[(k + 1) * kLdsRow + lane] : 0ull;
    lo = funnel((uint32_t)w1, (uint32_t)w0, sh);
    hi = funnel((uint32_t)(w1 >> 32), (uint32_t)(w0 >> 32), sh);
}

// Furthest column reached on diagonal d from column x (x <= end): the run of
// matches ref[c] == read[c + d] for c = x, x+1, ... stops at the first
// mismatch or at end = min(m, m - d).
__device__ __forceinline__ int slide(const uint64_t* rdL, const uint64_t* rfL, int lane, int x, int d,
                                     int end, uint32_t W) {
    int c = x;
    while (c < end) {
        uint32_t alo, ahi, blo, bhi;
        bases32(rfL, lane, (uint32_t)c, W, alo, ahi);
        bases32(rdL, lane, (uint32_t)(c + d), W, blo, bhi);
        const uint32_t mism = (alo ^ blo) | (ahi ^ bhi);
        if (mism != 0u) {
            c += (int)__builtin_ctz(mism);
            break;
        }
        c += 32;
    }
    return min(c, end);
}

template <int EMAX>
__device__ uint32_t band_distance(const uint64_t* rdL, const uint64_t* rfL, int lane, bool act, int m, int E,
                                  uint32_t W) {
    constexpr int D = 2 * EMAX + 1;
    int F[D];
#pragma unroll
    for (int i = 0; i < D; ++i) F[i] = kNeg;
    uint32_t dist = (uint32_t)E + 1u;
    if (act) {
        F[EMAX] = slide(rdL, rfL, lane, 0, 0, m, W);
        if (F[EMAX] >= m) dist = 0;
        if (F[EMAX] >= m || E == 0) act = false;
    }
    // Diagonals beyond the pair's threshold or length stay unreachable.  A
    // path on diagonal d after k edits needs |d| more to end on diagonal 0,
    // so round k only extends the diagonals with k + |d| <= E: the others
    // cannot lie on an alignment within E edits (and the rounds after k
    // only read diagonals that round k kept).
    const int lim = min(E, m);
    for (int k = 1; wave_any(act); ++k) {
        if (act) {
            int left = kNeg;   // F_{k-1}[d-1]
            const int reach = min(k, min(lim, E - k));
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int d = i - EMAX;
                const int old = F[i];
                const int ad = d < 0 ? -d : d;
                if (ad <= reach) {
                    int x = old + 1;
                    if (i + 1 < D) x = max(x, F[i + 1] + 1);
                    x = max(x, left);
                    const int end = d > 0 ? m - d : m;
                    x = min(x, end);
                    F[i] = slide(rdL, rfL, lane, x, d, end, W);
                }
                left = old;
            }
            if (F[EMAX] >= m) {
                dist = (uint32_t)k;
                act = false;
            } else if (k >= E) {
                act = false;
            }
        }
    }
    return dist;
}

// Verification in chunks: a wave owns K tiles of 64 consecutive pairs
// (K <= kVerifyTiles), lists the ones selected (bit p of `sel`, or all when sel is NULL) in
// its LDS, writes E + 1 for the others, and then takes the list 64 entries at
// a time: their words are staged in the wave's LDS rows, word-major, and
// every lane runs its pair.  Filtered batches keep a few pairs in a hundred,
// so the list turns a chunk's scattered survivors into full waves, with no
// pass over the whole batch and no global atomics.  With every pair selected
// a chunk is one tile (the groups are full anyway, and more waves run).
constexpr uint32_t kVerifyTiles = 16;

template <int EMAX>
__global__ void __launch_bounds__(256) verify_kernel(FilterParams P, const uint32_t* sel, uint16_t* dist,
                                                     uint32_t K) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const size_t rows = (size_t)2 * P.wmax * kLdsRow;
    uint64_t* rdL = lds + (size_t)wave * (rows + kVerifyTiles * 64 / 4);
    uint64_t* rfL = rdL + (size_t)P.wmax * kLdsRow;
    uint16_t* list = reinterpret_cast<uint16_t*>(rdL + rows);
    const uint64_t chunk = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    const uint64_t slot0 = chunk * K * 64;
    if (slot0 >= P.n_pairs) return;
    const uint32_t n_here = (uint32_t)min<uint64_t>((uint64_t)K * 64, P.n_pairs - slot0);
    uint32_t n_sel = 0;
    for (uint32_t g = 0; g < n_here; g += 64) {
        const uint32_t i = g + (uint32_t)lane;
        const uint64_t p = slot0 + i;
        bool take = false;
        if (i < n_here) {
            const uint32_t m = P.len ? P.len[p] : P.uniform_len;
            const uint32_t E = P.E ? P.E[p] : P.uniform_E;
            if (m < 1 || m > P.max_len || E > P.max_E) {
                atomicOr(P.err, 1u);
                dist[p] = 0;
            } else if (sel == nullptr || ((sel[p >> 5] >> (p & 31u)) & 1u) != 0u) {
                take = true;
            } else {
                dist[p] = (uint16_t)(E + 1u);
            }
        }
        const uint64_t bal = __ballot(take);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (take) list[n_sel + below] = (uint16_t)i;
        n_sel += (uint32_t)__builtin_popcountll(bal);
    }
    wave_lds_sync();
    for (uint32_t h = 0; h < n_sel; h += 64) {
        const uint32_t j = h + (uint32_t)lane;
        PairSlot s;
        s.valid = j < n_sel;
        s.in_batch = s.valid;
        s.slot = s.id = s.valid ? slot0 + list[j] : 0;
        s.m = s.valid ? (P.len ? P.len[s.id] : P.uniform_len) : 0u;
        s.E = s.valid ? (P.E ? P.E[s.id] : P.uniform_E) : 0u;
        s.W = (s.m + 31) >> 5;
        const uint64_t off = !s.valid ? 0
                             : P.word_offset ? P.word_offset[s.id]
                                             : s.id * (uint64_t)P.stride_words;
        stage_tile<true>(P, 0, lane, s, off, rdL, rfL);
        const uint32_t dd = band_distance<EMAX>(rdL, rfL, lane, s.valid, (int)s.m, (int)s.E, s.W);
        if (s.valid) dist[s.id] = (uint16_t)dd;
        wave_lds_sync();
    }
}

const void* verify_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&verify_kernel<X>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

}  // namespace

hipError_t launch_verify(const FilterParams& p, int emax, const uint32_t* sel, uint16_t* dist, hipStream_t s) {
    const void* k = verify_kernel_for(emax);
    if (!k) return hipErrorInvalidValue;
    // Four waves (four chunks) per block.
    const uint32_t waves = 4;
    uint32_t K = sel ? kVerifyTiles : 1u;
    const size_t lds = (size_t)waves * ((size_t)2 * p.wmax * kLdsRow * sizeof(uint64_t) + kVerifyTiles * 64 * 2);
    const uint64_t chunks = (p.n_pairs + K * 64 - 1) / (K * 64);
    const uint32_t blocks = (uint32_t)((chunks + waves - 1) / waves);
    FilterParams arg = p;
    const uint32_t* sl = sel;
    uint16_t* d = dist;
    void* args[] = {&arg, &sl, &d, &K};
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipLaunchKernel(k, dim3(blocks), dim3(64 * waves), args, lds, s);
}

}  // namespace paf
