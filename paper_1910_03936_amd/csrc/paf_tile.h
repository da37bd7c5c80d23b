// Device code shared by the per-tile engines (the SneakySnake tile kernel
// and the whole-map GateKeeper/Shouji kernel): a lane's view of its pair,
// staging of a tile's words into LDS, map builds of one 32-column window, and
// the tile loop of a launch (full grid or persistent work queue).
#pragma once

#include <type_traits>

#include "paf_internal.h"
#include "paf_map.h"

namespace paf {
namespace {

constexpr int kEmaxList[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 15, 20, 25, 31};

template <int EMAX>
struct DeadMask {
    using T = typename std::conditional<(2 * EMAX + 1 <= 32), uint32_t, uint64_t>::type;
};

// Per-lane view of one pair of the tile.
struct PairSlot {
    uint64_t slot;   // position in the launch order
    uint64_t id;     // original pair index
    bool valid;      // in range and passed the device-side checks
    bool in_batch;   // slot < n_pairs
    uint32_t m, E;
    uint32_t W;      // words per sequence
};

template <bool GENERAL>
__device__ __forceinline__ PairSlot load_slot(const FilterParams& P, uint64_t tile, int lane,
                                              uint64_t& off) {
    PairSlot s;
    s.slot = tile * 64 + (uint64_t)lane;
    s.in_batch = s.slot < P.n_pairs;
    s.valid = s.in_batch;
    s.id = s.slot;
    s.m = P.uniform_len;
    s.E = P.uniform_E;
    off = 0;
    if (GENERAL) {
        if (s.valid && P.perm) s.id = P.perm[s.slot];
        if (s.valid) {
            if (P.len) s.m = P.len[s.id];
            if (P.E) s.E = P.E[s.id];
            off = P.word_offset ? P.word_offset[s.id] : s.id * (uint64_t)P.stride_words;
            if (s.m < 1 || s.m > P.max_len || s.E > P.max_E) {
                atomicOr(P.err, 1u);
                s.valid = false;
            }
        }
    } else {
        off = s.id * (uint64_t)P.stride_words;
    }
    if (!s.valid) s.m = 0;
    s.W = (s.m + 31) >> 5;
    return s;
}

constexpr int kStageBatch = 8;

// Stage the tile's words into the wave's LDS rows.
template <bool GENERAL>
__device__ __forceinline__ void stage_tile(const FilterParams& P, uint64_t tile, int lane,
                                           const PairSlot& s, uint64_t off, uint64_t* rdL,
                                           uint64_t* rfL) {
    const uint32_t WM = P.wmax;
    // Loads go out kStageBatch at a time before their LDS stores, so a
    // wave waits for memory once per batch instead of once per load; a load
    // with nothing to fetch reads word 0 of the array (always there) and is
    // discarded, so no load sits behind a branch.
    constexpr int B = kStageBatch;
    if (!GENERAL) {
        // The tile's pairs are contiguous: pair-major rows of stride_words
        // words.  Coalesced 8-byte loads over the whole tile region, then a
        // transposed write into [word][lane].
        const uint32_t S = P.stride_words;
        const uint64_t base = tile * 64 * (uint64_t)S;
        const uint64_t limit = P.n_pairs * (uint64_t)S;
        const uint32_t total = 64u * S;
        uint32_t q = (uint32_t)lane;
        uint32_t pr = q / S, k = q - pr * S;
        const uint32_t dp = 64u / S, dk = 64u - dp * S;
        while (q < total) {
            uint64_t vr[B], vf[B];
            uint32_t at[B];
            bool use[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const uint64_t g = base + q;
                use[b] = q < total && k < WM;
                const bool ok = use[b] && g < limit;
                const uint64_t a = ok ? g : 0ull;
                const uint64_t xr = P.reads[a], xf = P.refs[a];
                vr[b] = ok ? xr : 0ull;
                vf[b] = ok ? xf : 0ull;
                at[b] = k * kLdsRow + pr;
                q += 64;
                pr += dp;
                k += dk;
                if (k >= S) { k -= S; pr += 1; }
            }
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (use[b]) {
                    rdL[at[b]] = vr[b];
                    rfL[at[b]] = vf[b];
                }
        }
        // Words past a pair's length are zero already (the packer zeroes the
        // tail of the last word and the layout has no words beyond W).
    } else {
        // Pairs sit anywhere (offsets, bucketed order): groups of WM adjacent
        // lanes read one pair's row of words together, so every load
        // instruction covers whole rows; the row's offset and length come
        // from the lane that owns the pair.
        const uint32_t offlo = (uint32_t)off, offhi = (uint32_t)(off >> 32);
        const uint32_t wv = s.valid ? s.W : 0u;
        uint32_t pr = (uint32_t)lane / WM, k = (uint32_t)lane - pr * WM;
        const uint32_t dp = 64u / WM, dk = 64u - dp * WM;
        for (uint32_t r0 = 0; r0 < WM; r0 += B) {
            uint64_t vr[B], vf[B];
            uint32_t at[B];
            bool use[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const uint64_t o = ((uint64_t)__shfl(offhi, (int)pr) << 32) | __shfl(offlo, (int)pr);
                const uint32_t wp = (uint32_t)__shfl(wv, (int)pr);
                use[b] = r0 + (uint32_t)b < WM;
                const bool ok = use[b] && k < wp;
                const uint64_t a = ok ? o + k : 0ull;
                const uint64_t xr = P.reads[a], xf = P.refs[a];
                vr[b] = ok ? xr : 0ull;
                vf[b] = ok ? xf : 0ull;
                at[b] = k * kLdsRow + pr;
                pr += dp;
                k += dk;
                if (k >= WM) { k -= WM; pr += 1; }
            }
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (use[b]) {
                    rdL[at[b]] = vr[b];
                    rfL[at[b]] = vf[b];
                }
        }
    }
    wave_lds_sync();
}

template <int EMAX, int I = 0>
__device__ __forceinline__ void build_snake_map(const WindowWords& q, bool boundary, uint32_t* M) {
    if constexpr (I < 2 * EMAX + 1) {
        constexpr int d = I - EMAX;
        uint32_t x = diag_raw<d>(q);
        if (boundary) x |= diag_vacant<d>(q);
        M[I] = x;
        build_snake_map<EMAX, I + 1>(q, boundary, M);
    }
}

// Whole-map engine: blocked map for SneakySnake/Shouji (vacant and past-end
// cells are 1) and GateKeeper's map (vacant and past-end cells are 0).
template <int d>
__device__ __forceinline__ void diag_both(const WindowWords& q, uint32_t& Mh, uint32_t& G) {
    const uint32_t x = diag_raw<d>(q);
    const uint32_t v = diag_vacant<d>(q);
    Mh = x | v | q.vc;          // q.vc doubles as "column >= m" for this window
    G = x & ~v & ~q.vc;
}

// ---------------------------------------------------------------------------
// SneakySnake: state of one lane's snake.
struct Snake {
    uint32_t c, e;
    bool act, acc;
    uint32_t cnt;
};

__device__ __forceinline__ void snake_finish(Snake& z, bool accept, uint32_t count) {
    z.act = false;
    z.acc = accept;
    z.cnt = count;
}

// Probe every diagonal from column c (window-relative shift s) and move the
// snake: follow the deepest pipe, then cross its obstacle (one edit, one
// column), or finish.  `x` holds the map words of the window; `dead` marks,
// for a lane that enters the window still inside a pipe, the diagonals whose
// pipes ended before the window (bit i = diagonal i); it applies only to the
// window's first column.
template <int EMAX, typename DT>
__device__ __forceinline__ void snake_window(Snake& z, const uint32_t* M, uint32_t w, uint32_t m,
                                             uint32_t E, bool& cont, DT& dead) {
    constexpr int D = 2 * EMAX + 1;
    const uint32_t wend = 32u * (w + 1);
    while (z.act && z.c < wend) {
        const uint32_t s = z.c - 32u * w;
        const uint32_t bs = 1u << s;
        uint32_t runs = 0;
        if (cont) {
            // s == 0 here; dead diagonals are blocked in the first column.
#pragma unroll
            for (int i = 0; i < D; ++i) runs = pipe_runs(runs, M[i] | (uint32_t)((dead >> i) & 1u), bs);
        } else {
#pragma unroll
            for (int i = 0; i < D; ++i) runs = pipe_runs(runs, M[i], bs);
        }
        const uint32_t best = (int32_t)runs < 0 ? 0xFFFFFFFFu : popc(runs);
        if (best == 0xFFFFFFFFu) {
            // Some pipe runs past the window's end.
            if (wend >= m) {
                snake_finish(z, true, z.e);
            } else {
                DT dm = 0;
                if (cont) {
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        dm |= (DT)(((M[i] | (uint32_t)((dead >> i) & 1u)) != 0u) ? 1u : 0u) << i;
                } else {
#pragma unroll
                    for (int i = 0; i < D; ++i) dm |= (DT)(((M[i] >> s) != 0u) ? 1u : 0u) << i;
                }
                dead = dm;
                cont = true;
                z.c = wend;
                return;
            }
        } else {
            cont = false;
            const uint32_t R = z.c + best;     // column of the obstacle
            if (R >= m) {
                snake_finish(z, true, z.e);
            } else {
                z.e += 1;
                z.c = R + 1;
                if (z.e > E) snake_finish(z, false, E + 1);
                else if (z.c >= m) snake_finish(z, true, z.e);
            }
        }
    }
}


// Tiles of one launch: one per wave (full grid), or taken `grab` at a time
// from the persistent work queue until it runs dry.  The next take is issued
// before the current tiles are processed, so the queue's round trip overlaps
// the work; every wave leaves after its first empty take.
template <typename F>
__device__ __forceinline__ void for_each_tile(const FilterParams& P, int lane, int wave, F&& run) {
    if (P.queue == nullptr) {
        const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
        if (tile < P.n_tiles) run(tile);
        return;
    }
    uint32_t t0 = 0;
    if (lane == 0) t0 = atomicAdd(P.queue, P.grab);
    t0 = __shfl(t0, 0);
    while (t0 < P.n_tiles) {
        uint32_t nx = 0;
        if (lane == 0) nx = atomicAdd(P.queue, P.grab);
        const uint32_t t1 = min(P.n_tiles, t0 + P.grab);
        for (uint32_t t = t0; t < t1; ++t) {
            run(t);
            wave_lds_sync();
        }
        t0 = __shfl(nx, 0);
    }
}

}  // namespace
}  // namespace paf
