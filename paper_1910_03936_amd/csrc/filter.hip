// Pre-alignment filter kernels for gfx950.
//
// One lane per (read, reference segment) pair; a wave holds a tile of 64
// pairs.  Sequences arrive 2-bit packed (planar inside each uint64 word, see
// paf.h) and are staged per wave in LDS, word-major ([word][lane]) so that a
// lane reads its own words without bank conflicts.  The neighbourhood map
// (Eq. 6.1; the unweighted maze of Eq. 8.2) is never materialised in HBM: for
// one 32-column window at a time each lane builds the 2E+1 diagonal mismatch
// words in VGPRs with funnel shifts (v_alignbit) and 3-input logic
// (v_bitop3).  Diagonal d compares ref[c] with read[c + d].
//
// Two engines share the map build:
//  * Snake: SneakySnake only (Ch. 8, Sec. 8.4).  Windows are built lazily and
//    a lane stops as soon as its decision is known, so most rejected pairs
//    touch one or two windows.  A probe of all diagonals at column c is
//    max_d ffbl(M_d >> s): the position of the first obstacle of the deepest
//    pipe, found with one shift, one find-first-bit and a third of a max3 per
//    diagonal.
//  * Whole: GateKeeper (Ch. 5) and/or Shouji (Ch. 6), which read the whole map,
//    plus SneakySnake on the same map when asked for.
//
// The window index is wave-uniform: every lane still working is in the same
// window, so the map words live in registers with compile-time indices.
#include "paf_internal.h"
#include "paf_map.h"

namespace paf {

namespace {

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

// Stage the tile's words into the wave's LDS rows.
template <bool GENERAL>
__device__ __forceinline__ void stage_tile(const FilterParams& P, uint64_t tile, int lane,
                                           const PairSlot& s, uint64_t off, uint64_t* rdL,
                                           uint64_t* rfL) {
    const uint32_t WM = P.wmax;
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
        for (; q < total; q += 64) {
            if (k < WM) {
                const uint64_t g = base + q;
                const bool ok = g < limit;
                rdL[k * kLdsRow + pr] = ok ? P.reads[g] : 0ull;
                rfL[k * kLdsRow + pr] = ok ? P.refs[g] : 0ull;
            }
            pr += dp;
            k += dk;
            if (k >= S) { k -= S; pr += 1; }
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
        for (uint32_t r = 0; r < WM; ++r) {
            const uint64_t o = ((uint64_t)__shfl(offhi, (int)pr) << 32) | __shfl(offlo, (int)pr);
            const bool ok = k < (uint32_t)__shfl(wv, (int)pr);
            rdL[k * kLdsRow + pr] = ok ? P.reads[o + k] : 0ull;
            rfL[k * kLdsRow + pr] = ok ? P.refs[o + k] : 0ull;
            pr += dp;
            k += dk;
            if (k >= WM) { k -= WM; pr += 1; }
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
        uint32_t best = 0;
        if (cont) {
            // s == 0 here.
#pragma unroll
            for (int i = 0; i < D; ++i) best = max(best, ffbl(M[i] | (uint32_t)((dead >> i) & 1u)));
        } else {
#pragma unroll
            for (int i = 0; i < D; ++i) best = max(best, ffbl(M[i] >> s));
        }
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

template <int EMAX, bool GENERAL>
__device__ void snake_tile(const FilterParams& P, uint64_t tile, int lane, uint64_t* rdL,
                           uint64_t* rfL) {
    constexpr int D = 2 * EMAX + 1;
    uint64_t off;
    const PairSlot ps = load_slot<GENERAL>(P, tile, lane, off);
    stage_tile<GENERAL>(P, tile, lane, ps, off, rdL, rfL);

    const uint32_t m = ps.m, E = ps.E;
    // Diagonals beyond the pair's own threshold are fully blocked.
    const bool mask_E = GENERAL ? (P.E != nullptr || P.uniform_E < (uint32_t)EMAX)
                                : (P.uniform_E < (uint32_t)EMAX);
    uint32_t c = 0, e = 0;
    bool act = ps.valid, acc = false;
    // A lane whose deepest pipe ran past the end of the previous window enters
    // the next one still inside that pipe: only the diagonals that were clear
    // up to the window's end (from its probe at shift s_prev) may carry it on.
    // Their complement is folded into bit 0 of the new window's map words;
    // bit 0 is only ever read by that first probe (after it, s >= 1).
    uint32_t cont = 0, s_prev = 0;
    uint32_t M[D];
#pragma unroll
    for (int i = 0; i < D; ++i) M[i] = 0u;

    for (uint32_t w = 0; wave_any(act); ++w) {
        if (act) {
            const WindowWords q = window_words(rdL, rfL, lane, (int)w, P.wmax, (int)m);
            // Vacant cells only occur in the first window and near the end.
            const bool boundary = wave_any(w == 0 || 32u * (w + 2) > m);
            const bool any_cont = wave_any(cont != 0u);
            uint32_t T[D];
            build_snake_map<EMAX>(q, boundary, T);
            if (any_cont) {
#pragma unroll
                for (int i = 0; i < D; ++i) M[i] = T[i] | min(M[i] >> s_prev, cont);
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) M[i] = T[i];
            }
            if (mask_E) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const int d = i - EMAX;
                    if ((uint32_t)(d < 0 ? -d : d) > E) M[i] = ~0u;
                }
            }
            cont = 0u;
            // Steps inside this window: probe every diagonal from column c,
            // follow the deepest pipe, cross its obstacle (one edit, one
            // column) or finish.
            const uint32_t w0 = 32u * w, wend = w0 + 32u;
            bool inw = c < wend;
            while (inw) {
                const uint32_t s = c - w0;
                uint32_t best = 0;
#pragma unroll
                for (int i = 0; i < D; ++i) best = max(best, ffbl(M[i] >> s));
                const bool clear = best == 0xFFFFFFFFu;   // a pipe runs past the window
                const uint32_t R = clear ? wend : c + best;
                const bool reach = R >= m;                 // the pipe reaches the last column
                const bool obst = !reach && !clear;
                e += obst ? 1u : 0u;
                c = reach ? c : (clear ? wend : R + 1u);
                const bool rej = e > E;
                const bool fin_acc = reach || (obst && !rej && c >= m);
                acc = fin_acc;
                if (clear && !reach) {
                    cont = 1u;
                    s_prev = s;
                }
                act = !(fin_acc || rej);
                inw = act && c < wend;
            }
        }
    }
    const uint32_t cnt = e;  // e <= E for accepts, E + 1 for rejects

    // Outputs.
    if (GENERAL && P.perm) {
        if (ps.in_batch) P.cnt[0][ps.id] = (uint16_t)(ps.valid ? cnt : 0u);
    } else {
        const uint64_t bal = __ballot(ps.valid && acc);
        if (ps.in_batch) P.cnt[0][ps.slot] = (uint16_t)(ps.valid ? cnt : 0u);
        if (lane == 0) {
            P.acc[0][2 * tile] = (uint32_t)bal;
            if (tile * 64 + 32 < P.n_pairs) P.acc[0][2 * tile + 1] = (uint32_t)(bal >> 32);
        }
    }
}

// ---------------------------------------------------------------------------
// Compacting SneakySnake engine.
//
// A wave owns a chunk of K tiles (64 K pairs) and walks it one 32-column
// window at a time.  The pairs still undecided after window w are packed,
// with their snake state, into a list in the wave's LDS and the next pass
// takes them 64 at a time for window w + 1, so every pass runs full waves
// however early the other pairs of their tiles stopped.  Window words are
// read straight from memory (a lane holds any pair of the chunk); nothing
// but the list lives in LDS.
//
// List entry (64 bits): pair index in the chunk (10 bits), column c (9),
// edits e (5), continuation flag (1), m (10), E (5); plus the dead-diagonal
// mask of a snake that entered the window inside a pipe, and (general
// layout) the pair's word offset.
constexpr uint32_t kChunkMaxTiles = 16;

struct ChunkEntry {
    uint32_t idx, c, e, m, E;
    bool cont;
};

__device__ __forceinline__ uint64_t chunk_pack(const ChunkEntry& t) {
    return (uint64_t)t.idx | ((uint64_t)t.c << 10) | ((uint64_t)t.e << 19) | ((uint64_t)t.cont << 24) |
           ((uint64_t)t.m << 25) | ((uint64_t)t.E << 35);
}

__device__ __forceinline__ ChunkEntry chunk_unpack(uint64_t v) {
    ChunkEntry t;
    t.idx = (uint32_t)v & 1023u;
    t.c = (uint32_t)(v >> 10) & 511u;
    t.e = (uint32_t)(v >> 19) & 31u;
    t.cont = ((v >> 24) & 1u) != 0;
    t.m = (uint32_t)(v >> 25) & 1023u;
    t.E = (uint32_t)(v >> 35) & 31u;
    return t;
}

// Match words of one window for the compacting engine: bit j of Z_d is 1
// when column j is a free cell of diagonal d, i.e. the complement of the
// mismatch word (lo ^ flo) | (hi ^ fhi) over the two code planes.  VAC folds
// in the vacant cells (first and last windows), CONT the dead-diagonal bit of
// a snake that entered inside a pipe (bit 0 of the window).  v_bitop3 takes
// s1 | (s0 ^ s2) (truth table 0xDE) and its complement (0x21) in one
// instruction; both are symmetric in s0 and s2.
__device__ __forceinline__ uint32_t or_xor3(uint32_t a, uint32_t t, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, t, b, 0xDE);
}
__device__ __forceinline__ uint32_t nor_xor3(uint32_t a, uint32_t t, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, t, b, 0x21);
}
// acc | (z & ~y) in one instruction (truth table 0xF4 with s0 = acc).
__device__ __forceinline__ uint32_t or_andn(uint32_t acc, uint32_t z, uint32_t y) {
    return __builtin_amdgcn_bitop3_b32(acc, z, y, 0xF4);
}

template <int EMAX, bool VAC, bool CONT, typename DT, int I = 0>
__device__ __forceinline__ void chunk_map(const WindowWords& q, DT dead, uint32_t* M) {
    if constexpr (I < 2 * EMAX + 1) {
        constexpr int d = I - EMAX;
        uint32_t lo, hi;
        if constexpr (d > 0) {
            lo = funnel(q.nlo, q.clo, d);
            hi = funnel(q.nhi, q.chi, d);
        } else if constexpr (d == 0) {
            lo = q.clo;
            hi = q.chi;
        } else {
            lo = funnel(q.clo, q.plo, 32 + d);
            hi = funnel(q.chi, q.phi, 32 + d);
        }
        uint32_t t;
        if constexpr (VAC || CONT) {
            uint32_t v = 0;
            if constexpr (VAC) v = diag_vacant<d>(q);
            if constexpr (CONT) v |= (uint32_t)((dead >> I) & 1u);
            t = or_xor3(lo, v, q.flo);
        } else {
            t = lo ^ q.flo;
        }
        M[I] = nor_xor3(hi, t, q.fhi);
        chunk_map<EMAX, VAC, CONT, DT, I + 1>(q, dead, M);
    }
}

template <int EMAX, bool GENERAL>
struct ChunkLds {
    using DT = typename DeadMask<EMAX>::T;
    uint64_t* ent;
    DT* dead;
    uint64_t* off;   // GENERAL only
    uint32_t* acc;   // 2 K accept words (plain order)
};

template <int EMAX, bool GENERAL>
__device__ void chunk_snake(const FilterParams& P, uint32_t chunk, uint32_t K, int lane,
                            const ChunkLds<EMAX, GENERAL>& L) {
    constexpr int D = 2 * EMAX + 1;
    using DT = typename DeadMask<EMAX>::T;
    const uint64_t slot0 = (uint64_t)chunk * K * 64u;
    const uint32_t n_here = (uint32_t)min<uint64_t>((uint64_t)K * 64u, P.n_pairs - slot0);
    const bool plain_out = !(GENERAL && P.perm);
    if (plain_out)
        for (uint32_t j = (uint32_t)lane; j < 2 * K; j += 64) L.acc[j] = 0u;
    const bool mask_E = GENERAL ? (P.E != nullptr || P.uniform_E < (uint32_t)EMAX)
                                : (P.uniform_E < (uint32_t)EMAX);
    uint32_t n_ent = n_here;
    // With a key per pair (the cost model's level), the first pass's list
    // holds the chunk's pairs grouped by the key's top two bits (four cost
    // classes, a stable counting sort by wave ballots), so each group of 64
    // takes pairs of like cost.  Finer classes bought less than the sort
    // cost them.
    const bool keyed = P.order_key != nullptr && plain_out;
    if (keyed) {
        constexpr uint32_t NB = 4, NONE = NB;
        // Class of pair i of the chunk (NONE = no entry: outside the batch or
        // outside its bounds), with its length and threshold.
        auto key_of = [&](uint32_t i, ChunkEntry& t) -> uint32_t {
            t = ChunkEntry{};
            t.idx = i;
            t.m = P.uniform_len;
            t.E = P.uniform_E;
            if (i >= n_here) return NONE;
            const uint64_t slot = slot0 + i;
            if (GENERAL) {
                if (P.len) t.m = P.len[slot];
                if (P.E) t.E = P.E[slot];
                if (t.m < 1 || t.m > P.max_len || t.E > P.max_E) return NONE;
            }
            return (P.order_key[slot] & 15u) >> 2;
        };
        // The two pairs of a 128-byte line of sequence words (adjacent
        // pairs) take the costlier class of the two, so they stay side by
        // side in the list and their lines are fetched once.
        auto line_key = [&](uint32_t b) -> uint32_t {
            const uint32_t o = (uint32_t)__shfl_xor((int)b, 1);
            return b < NONE && o < b ? o : b;
        };
        uint32_t base[NB];
#pragma unroll
        for (uint32_t v = 0; v < NB; ++v) base[v] = 0;
        for (uint32_t g = 0; g < n_here; g += 64) {
            ChunkEntry t;
            const uint32_t b = line_key(key_of(g + (uint32_t)lane, t));
#pragma unroll
            for (uint32_t v = 0; v < NB; ++v) base[v] += (uint32_t)__builtin_popcountll(__ballot(b == v));
        }
        uint32_t run = 0;
#pragma unroll
        for (uint32_t v = 0; v < NB; ++v) {
            const uint32_t c = base[v];
            base[v] = run;
            run += c;
        }
        n_ent = run;
        for (uint32_t g = 0; g < n_here; g += 64) {
            const uint32_t i = g + (uint32_t)lane;
            ChunkEntry t;
            const uint32_t b = line_key(key_of(i, t));
            if (i < n_here) {
                const uint64_t slot = slot0 + i;
                if (b == NONE) {
                    atomicOr(P.err, 1u);
                    P.cnt[0][slot] = 0;
                } else if (GENERAL) {
                    L.off[i] = P.word_offset ? P.word_offset[slot] : slot * (uint64_t)P.stride_words;
                }
            }
            uint32_t pos = 0;
#pragma unroll
            for (uint32_t v = 0; v < NB; ++v) {
                const uint64_t mv = __ballot(b == v);
                const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mv >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mv, 0u));
                if (b == v) pos = base[v] + below;
                base[v] += (uint32_t)__builtin_popcountll(mv);
            }
            if (b < NONE) L.ent[pos] = chunk_pack(t);
        }
    }
    // Each pass walks windows [w, w + span) with the same lanes; the pairs
    // still undecided after it are regrouped for the next pass.
    for (uint32_t w = 0, span = P.span0; n_ent > 0; w += span, span = P.span) {
        wave_lds_sync();
        uint32_t n_out = 0;
        for (uint32_t g = 0; g < n_ent; g += 64) {
            const uint32_t i = g + (uint32_t)lane;
            bool act = i < n_ent;
            ChunkEntry t = {};
            DT dead = 0;
            uint64_t off = 0;
            if (w == 0 && !keyed) {
                t.idx = i;
                t.c = 0;
                t.e = 0;
                t.cont = false;
                t.m = P.uniform_len;
                t.E = P.uniform_E;
                if (act) {
                    const uint64_t slot = slot0 + i;
                    if (GENERAL) {
                        const uint64_t id = P.perm ? P.perm[slot] : slot;
                        if (P.len) t.m = P.len[id];
                        if (P.E) t.E = P.E[id];
                        off = P.word_offset ? P.word_offset[id] : id * (uint64_t)P.stride_words;
                        L.off[i] = off;
                        if (t.m < 1 || t.m > P.max_len || t.E > P.max_E) {
                            atomicOr(P.err, 1u);
                            P.cnt[0][id] = 0;
                            act = false;
                        }
                    } else {
                        off = slot * (uint64_t)P.stride_words;
                    }
                }
            } else if (act) {
                t = chunk_unpack(L.ent[i]);
                dead = t.cont ? L.dead[i] : (DT)0;
                off = GENERAL ? L.off[t.idx] : (slot0 + t.idx) * (uint64_t)P.stride_words;
            }
            const uint32_t m = act ? t.m : 0u;
            const uint32_t E = t.E;
            const int W = (int)((m + 31) >> 5);
            uint32_t c = t.c, e = t.e;
            bool cont = t.cont, acc = false;
            for (uint32_t wk = w; wk < w + span && wave_any(act); ++wk) {
                const WindowWords q = window_words_direct(P.reads + off, P.refs + off, (int)wk, W, (int)m);
                // Vacant cells only occur in the first window and near the end.
                // A snake that entered inside a pipe sees the diagonals whose
                // pipes ended before this window blocked in its first column.
                const bool vac = wave_any(act && (wk == 0 || 32u * (wk + 2) > m));
                const bool cnt = wave_any(act && cont);
                uint32_t M[D];
                if (vac) {
                    if (cnt) chunk_map<EMAX, true, true>(q, dead, M);
                    else chunk_map<EMAX, true, false>(q, dead, M);
                } else {
                    if (cnt) chunk_map<EMAX, false, true>(q, dead, M);
                    else chunk_map<EMAX, false, false>(q, dead, M);
                }
                if (mask_E) {
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        const int dd = d - EMAX;
                        if ((uint32_t)(dd < 0 ? -dd : dd) > E) M[d] = 0u;
                    }
                }
                const uint32_t w0 = 32u * wk, wend = w0 + 32u;
                const bool live = act;
                bool ncont = false;
                uint32_t s_prev = 0;
                bool inw = act && c < wend;
                while (inw) {
                    // Pipes from column c: adding 1 << s to a match word
                    // carries through its run of free cells from s, so
                    // Z & ~(Z + (1 << s)) is that run; the OR over the
                    // diagonals is [s, s + deepest run), with bit 31 set when a
                    // pipe reaches the window's end.
                    const uint32_t s = c - w0;
                    const uint32_t bs = 1u << s;
                    uint32_t r0 = 0, r1 = 0;
#pragma unroll
                    for (int d = 0; d < D; d += 2) {
                        r0 = or_andn(r0, M[d], M[d] + bs);
                        if (d + 1 < D) r1 = or_andn(r1, M[d + 1], M[d + 1] + bs);
                    }
                    const uint32_t runs = r0 | r1;
                    const bool clear = (int32_t)runs < 0;
                    const uint32_t R = clear ? wend : c + (uint32_t)__builtin_popcount(runs);
                    const bool reach = R >= m;
                    const bool obst = !reach && !clear;
                    e += obst ? 1u : 0u;
                    c = reach ? c : (clear ? wend : R + 1u);
                    const bool rej = e > E;
                    const bool fin_acc = reach || (obst && !rej && c >= m);
                    acc = fin_acc;
                    if (clear && !reach) {
                        ncont = true;
                        s_prev = s;
                    }
                    act = !(fin_acc || rej);
                    inw = act && c < wend;
                }
                if (live && !act) {
                    const uint64_t slot = slot0 + t.idx;
                    if (plain_out) {
                        P.cnt[0][slot] = (uint16_t)e;
                        if (acc) atomicOr(&L.acc[t.idx >> 5], 1u << (t.idx & 31u));
                    } else {
                        P.cnt[0][P.perm[slot]] = (uint16_t)e;
                    }
                }
                // A diagonal stays alive into the next window when its run
                // from s_prev reaches this window's end, i.e. when adding
                // 1 << s_prev to its match word carries out of bit 31.
                DT dm = 0;
                if (wave_any(act && ncont)) {
                    const uint32_t bs = 1u << s_prev;
                    uint32_t lo = 0, hi = 0;
#pragma unroll
                    for (int d = D - 1; d >= 0; --d) {
                        const uint32_t carry = (uint32_t)(((uint64_t)M[d] + bs) >> 32);
                        if (d >= 32) hi = (hi << 1) | carry;
                        else lo = (lo << 1) | carry;
                    }
                    const DT alive = (DT)lo | (sizeof(DT) > 4 ? (DT)((uint64_t)hi << 32) : (DT)0);
                    constexpr DT all = (D >= 8 * (int)sizeof(DT)) ? ~(DT)0 : (((DT)1 << D) - 1);
                    dm = ~alive & all;
                }
                cont = act && ncont;
                dead = cont ? dm : (DT)0;
            }
            // Survivors go on to the next pass.
            const uint64_t bal = __ballot(act);
            const uint32_t pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (act) {
                ChunkEntry u = t;
                u.c = c;
                u.e = e;
                u.cont = cont;
                L.ent[n_out + pre] = chunk_pack(u);
                L.dead[n_out + pre] = dead;
            }
            n_out += (uint32_t)__builtin_popcountll(bal);
        }
        n_ent = n_out;
    }
    if (plain_out) {
        wave_lds_sync();
        for (uint32_t j = (uint32_t)lane; j < 2 * K; j += 64) {
            const uint64_t s0 = slot0 + 32u * j;
            if (s0 < P.n_pairs) P.acc[0][s0 / 32] = L.acc[j];
        }
    }
}

// Bytes of one wave's list in LDS.
template <int EMAX, bool GENERAL>
__host__ __device__ constexpr size_t chunk_wave_bytes_t(uint32_t K) {
    using DT = typename DeadMask<EMAX>::T;
    return (size_t)K * 64 * (8 + sizeof(DT) + (GENERAL ? 8 : 0)) + (size_t)K * 8;
}

template <int EMAX, bool GENERAL>
__global__ void __launch_bounds__(512) chunk_kernel(FilterParams P) {
    extern __shared__ uint64_t lds[];
    using DT = typename DeadMask<EMAX>::T;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t K = P.chunk;
    const uint32_t NE = K * 64u;
    char* b = reinterpret_cast<char*>(lds) + (size_t)wave * chunk_wave_bytes_t<EMAX, GENERAL>(K);
    ChunkLds<EMAX, GENERAL> L;
    L.ent = reinterpret_cast<uint64_t*>(b);
    b += (size_t)NE * 8;
    if (GENERAL) {
        L.off = reinterpret_cast<uint64_t*>(b);
        b += (size_t)NE * 8;
    } else {
        L.off = nullptr;
    }
    L.dead = reinterpret_cast<DT*>(b);
    b += (size_t)NE * sizeof(DT);
    L.acc = reinterpret_cast<uint32_t*>(b);
    const uint32_t n_chunks = (P.n_tiles + K - 1) / K;
    if (P.queue == nullptr) {
        const uint32_t ch = blockIdx.x * (blockDim.x >> 6) + wave;
        if (ch < n_chunks) chunk_snake<EMAX, GENERAL>(P, ch, K, lane, L);
        return;
    }
    uint32_t c0 = 0;
    if (lane == 0) c0 = atomicAdd(P.queue, 1u);
    c0 = __shfl(c0, 0);
    while (c0 < n_chunks) {
        uint32_t nx = 0;
        if (lane == 0) nx = atomicAdd(P.queue, 1u);
        chunk_snake<EMAX, GENERAL>(P, c0, K, lane, L);
        wave_lds_sync();
        c0 = __shfl(nx, 0);
    }
}

template <bool GENERAL>
const void* chunk_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&chunk_kernel<X, GENERAL>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

template <bool GENERAL>
size_t chunk_bytes_for(int emax, uint32_t K) {
    return emax <= 15 ? chunk_wave_bytes_t<15, GENERAL>(K) : chunk_wave_bytes_t<31, GENERAL>(K);
}

// ---------------------------------------------------------------------------
// Whole-map engine.

// GateKeeper's amendment of one window word (Ch. 5, Sec. 5.2.2; SRS of
// Sec. 3.2.1): a zero inside a streak of one or two zeros bounded by ones on
// both sides becomes one.  L1/L2 are the bits one/two columns to the left,
// R1/R2 to the right (taken from the neighbouring windows).
__device__ __forceinline__ uint32_t amend_word(uint32_t g, uint32_t prev, uint32_t next) {
    const uint32_t L1 = funnel(g, prev, 31);
    const uint32_t L2 = funnel(g, prev, 30);
    const uint32_t R1 = funnel(next, g, 1);
    const uint32_t R2 = funnel(next, g, 2);
    return g | (L1 & (R1 | R2)) | (R1 & (L1 | L2));
}

// Shouji: bit-sliced best 4-column segment per window start column.
struct ShoujiBest {
    uint32_t o0, o1, o2;      // ones in the best segment (bit-sliced, 0..4)
    uint32_t b0, b1, b2, b3;  // the best segment's bits
};

__device__ __forceinline__ void shouji_candidate(ShoujiBest& bs, uint32_t cur, uint32_t nxt,
                                                 bool first) {
    const uint32_t B0 = cur;
    const uint32_t B1 = funnel(nxt, cur, 1);
    const uint32_t B2 = funnel(nxt, cur, 2);
    const uint32_t B3 = funnel(nxt, cur, 3);
    const uint32_t s01 = B0 ^ B1, c01 = B0 & B1, s23 = B2 ^ B3, c23 = B2 & B3;
    const uint32_t o0 = s01 ^ s23;
    const uint32_t cm = s01 & s23;
    const uint32_t o1 = c01 ^ c23 ^ cm;
    const uint32_t o2 = c01 & c23;
    if (first) {
        bs = {o0, o1, o2, B0, B1, B2, B3};
        return;
    }
    // Fewer ones wins; on a tie, a segment that starts with a zero beats one
    // that does not; otherwise the earlier diagonal is kept.
    const uint32_t t0 = ~o0 & bs.o0;
    const uint32_t e1 = ~(o1 ^ bs.o1);
    const uint32_t t1 = (~o1 & bs.o1) | (e1 & t0);
    const uint32_t e2 = ~(o2 ^ bs.o2);
    const uint32_t lt = (~o2 & bs.o2) | (e2 & t1);
    const uint32_t eq = e2 & e1 & ~(o0 ^ bs.o0);
    const uint32_t rep = lt | (eq & ~B0 & bs.b0);
    bs.o0 = (rep & o0) | (~rep & bs.o0);
    bs.o1 = (rep & o1) | (~rep & bs.o1);
    bs.o2 = (rep & o2) | (~rep & bs.o2);
    bs.b0 = (rep & B0) | (~rep & bs.b0);
    bs.b1 = (rep & B1) | (~rep & bs.b1);
    bs.b2 = (rep & B2) | (~rep & bs.b2);
    bs.b3 = (rep & B3) | (~rep & bs.b3);
}

// Sequential store into the Shouji bit-vector for the 32 windows starting in
// this window (Sec. 6.2.2): the best segment overwrites the vector's four
// bits when it holds strictly more zeros.  S covers columns [32w, 32w+64).
template <int J = 0>
__device__ __forceinline__ void shouji_store(const ShoujiBest& bs, uint32_t& S_lo, uint32_t& S_hi,
                                             uint32_t ncols) {
    if constexpr (J < 32) {
        const uint32_t V = ((bs.b0 >> J) & 1u) | (((bs.b1 >> J) & 1u) << 1) |
                           (((bs.b2 >> J) & 1u) << 2) | (((bs.b3 >> J) & 1u) << 3);
        uint32_t cur;
        if constexpr (J <= 28) cur = (S_lo >> J) & 0xFu;
        else cur = funnel(S_hi, S_lo, J) & 0xFu;
        const bool take = (uint32_t)J < ncols && popc(V) < popc(cur);
        if constexpr (J <= 28) {
            const uint32_t nlo = (S_lo & ~(0xFu << J)) | (V << J);
            S_lo = take ? nlo : S_lo;
        } else {
            const uint32_t nlo = (S_lo & ~(0xFu << J)) | (V << J);
            const uint32_t nhi = (S_hi & ~(0xFu >> (32 - J))) | (V >> (32 - J));
            S_lo = take ? nlo : S_lo;
            S_hi = take ? nhi : S_hi;
        }
        shouji_store<J + 1>(bs, S_lo, S_hi, ncols);
    }
}

template <int EMAX, int I = 0>
__device__ __forceinline__ void build_both(const WindowWords& q, uint32_t* Mh, uint32_t* G) {
    if constexpr (I < 2 * EMAX + 1) {
        diag_both<I - EMAX>(q, Mh[I], G[I]);
        build_both<EMAX, I + 1>(q, Mh, G);
    }
}

template <int EMAX, bool GENERAL>
__device__ void whole_tile(const FilterParams& P, uint64_t tile, int lane, uint64_t* rdL,
                           uint64_t* rfL) {
    constexpr int D = 2 * EMAX + 1;
    using DT = typename DeadMask<EMAX>::T;
    uint64_t off;
    const PairSlot ps = load_slot<GENERAL>(P, tile, lane, off);
    stage_tile<GENERAL>(P, tile, lane, ps, off, rdL, rfL);

    const bool doSS = P.filters & PAF_SNEAKYSNAKE;
    const bool doGK = P.filters & PAF_GATEKEEPER;
    const bool doSH = P.filters & PAF_SHOUJI;
    const uint32_t m = ps.m, E = ps.E;
    const bool mask_E = GENERAL ? (P.E != nullptr || P.uniform_E < (uint32_t)EMAX)
                                : (P.uniform_E < (uint32_t)EMAX);

    Snake z{0u, 0u, ps.valid && doSS, false, 0u};
    bool cont = false;
    DT dead = 0;
    uint32_t gk_ham = 0, gk_cnt = 0;
    uint32_t S_lo = ~0u, S_hi = ~0u, sh_cnt = 0;

    uint32_t Mc[D], Gc[D], Gp[D];
    if (ps.valid) {
        const WindowWords q = window_words(rdL, rfL, lane, 0, P.wmax, (int)m);
        build_both<EMAX>(q, Mc, Gc);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) Gp[i] = 0u;
    if (mask_E && ps.valid) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int d = i - EMAX;
            if ((uint32_t)(d < 0 ? -d : d) > E) { Mc[i] = ~0u; Gc[i] = ~0u; Gp[i] = ~0u; }
        }
    }

    for (uint32_t w = 0; wave_any(ps.valid && w < ps.W); ++w) {
        const bool have = ps.valid && w < ps.W;
        if (have) {
            const uint32_t colpast = vacant_word((int)w, (int)m);  // columns >= m
            // SneakySnake on this window.
            if (doSS && z.act) snake_window<EMAX, DT>(z, Mc, w, m, E, cont, dead);
            if (doGK) gk_ham += popc(Mc[EMAX] & ~colpast);
            // Next window's maps, then GateKeeper and Shouji per diagonal.
            const WindowWords qn = window_words(rdL, rfL, lane, (int)w + 1, P.wmax, (int)m);
            uint32_t Fw = ~0u;
            ShoujiBest bs;
            uint32_t Mn[D], Gn[D];
            build_both<EMAX>(qn, Mn, Gn);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (mask_E) {
                    const int d = i - EMAX;
                    if ((uint32_t)(d < 0 ? -d : d) > E) { Mn[i] = ~0u; Gn[i] = ~0u; }
                }
                if (doGK) Fw &= amend_word(Gc[i], Gp[i], Gn[i]);
                if (doSH) shouji_candidate(bs, Mc[i], Mn[i], i == 0);
                Gp[i] = Gc[i];
                Gc[i] = Gn[i];
                Mc[i] = Mn[i];
            }
            if (doGK) gk_cnt += popc(Fw & ~colpast);
            if (doSH) {
                const uint32_t ncols = m - 32u * w;  // >= 1
                shouji_store(bs, S_lo, S_hi, ncols);
                sh_cnt += popc(S_lo & ~colpast);
                S_lo = S_hi;
                S_hi = ~0u;
            }
        }
    }

    const bool gk_acc = gk_ham <= E || gk_cnt <= E;
    const uint32_t gk_out = gk_ham <= E ? gk_ham : gk_cnt;
    const bool sh_acc = sh_cnt <= E;
    bool accs[3] = {z.acc, gk_acc, sh_acc};
    uint32_t cnts[3] = {z.cnt, gk_out, sh_cnt};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        if (!(P.filters & (1u << f))) continue;
        if (GENERAL && P.perm) {
            if (ps.in_batch) P.cnt[f][ps.id] = (uint16_t)(ps.valid ? cnts[f] : 0u);
        } else {
            const uint64_t bal = __ballot(ps.valid && accs[f]);
            if (ps.in_batch) P.cnt[f][ps.slot] = (uint16_t)(ps.valid ? cnts[f] : 0u);
            if (lane == 0) {
                P.acc[f][2 * tile] = (uint32_t)bal;
                if (tile * 64 + 32 < P.n_pairs) P.acc[f][2 * tile + 1] = (uint32_t)(bal >> 32);
            }
        }
    }
}

template <Engine ENG, int EMAX, bool GENERAL>
__global__ void __launch_bounds__(ENG == Engine::Snake ? 512 : 256) filter_kernel(FilterParams P) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint64_t* rdL = lds + (size_t)wave * 2 * P.wmax * kLdsRow;
    uint64_t* rfL = rdL + (size_t)P.wmax * kLdsRow;
    auto run = [&](uint64_t tile) {
        if constexpr (ENG == Engine::Snake) snake_tile<EMAX, GENERAL>(P, tile, lane, rdL, rfL);
        else whole_tile<EMAX, GENERAL>(P, tile, lane, rdL, rfL);
    };
    if (P.queue == nullptr) {
        const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
        if (tile < P.n_tiles) run(tile);
        return;
    }
    // Persistent: each wave takes `grab` tiles at a time from the queue until
    // it runs dry; every wave leaves after its first empty take.  The next
    // take is issued before the current tiles are processed, so the queue's
    // round trip overlaps the work.
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

constexpr int kEmaxList[] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 15, 20, 25, 31};

template <Engine ENG, bool GENERAL>
const void* kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&filter_kernel<ENG, X, GENERAL>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

// ---------------------------------------------------------------------------
// Encoder (Ch. 5, Method 3; planar two-bit layout described in paf.h).
__global__ void pack_kernel(const uint8_t* codes, uint32_t code_stride, const uint16_t* len,
                            uint32_t uniform_len, const uint64_t* word_offset, uint32_t stride_words,
                            uint64_t n, uint32_t wmax, uint64_t* words, uint32_t* err) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t p = t / wmax;
    const uint32_t k = (uint32_t)(t - p * wmax);
    if (p >= n) return;
    const uint32_t m = len ? len[p] : uniform_len;
    if (m < 1 || m > code_stride || m > 32u * wmax) {
        if (k == 0) atomicOr(err, 1u);
        return;
    }
    const uint32_t W = (m + 31) >> 5;
    if (k >= W) return;
    const uint8_t* row = codes + p * (uint64_t)code_stride + 32u * k;
    const uint32_t cnt = min(32u, m - 32u * k);
    uint32_t lo = 0, hi = 0, bad = 0;
    for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t b = row[j];
        bad |= b >> 2;
        lo |= (b & 1u) << j;
        hi |= ((b >> 1) & 1u) << j;
    }
    if (bad) atomicOr(err, 1u);
    const uint64_t o = word_offset ? word_offset[p] : p * (uint64_t)stride_words;
    words[o + k] = ((uint64_t)hi << 32) | lo;
}

// Decisions from counts (bucketed order writes counts at the original index;
// every filter accepts exactly when its count is at most E).
__global__ void accept_kernel(const uint16_t* cnt, const uint16_t* len, uint32_t uniform_len,
                              const uint8_t* E, uint32_t uniform_E, uint32_t max_len, uint32_t max_E,
                              uint64_t n, uint32_t* acc) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool a = false;
    if (p < n) {
        const uint32_t m = len ? len[p] : uniform_len;
        const uint32_t e = E ? E[p] : uniform_E;
        a = m >= 1 && m <= max_len && e <= max_E && cnt[p] <= e;
    }
    const uint64_t bal = __ballot(a);
    const int lane = threadIdx.x & 63;
    const uint64_t base = p - (uint64_t)lane;
    if (lane == 0 && base < n) acc[base / 32] = (uint32_t)bal;
    if (lane == 32 && base + 32 < n) acc[base / 32 + 1] = (uint32_t)(bal >> 32);
}

__global__ void fill_kernel(uint32_t* p, uint32_t v, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

int emax_bucket(int max_E) {
    for (int e : kEmaxList)
        if (e >= max_E) return e;
    return -1;
}

const void* filter_kernel_ptr(Engine eng, bool general, int emax) {
    if (eng == Engine::Chunk) return general ? chunk_kernel_for<true>(emax) : chunk_kernel_for<false>(emax);
    if (eng == Engine::Snake)
        return general ? kernel_for<Engine::Snake, true>(emax) : kernel_for<Engine::Snake, false>(emax);
    return general ? kernel_for<Engine::Whole, true>(emax) : kernel_for<Engine::Whole, false>(emax);
}

size_t filter_lds_bytes(uint32_t waves_per_block, uint32_t wmax) {
    return (size_t)waves_per_block * 2 * wmax * kLdsRow * sizeof(uint64_t);
}

size_t chunk_lds_bytes(uint32_t waves_per_block, bool general, int emax, uint32_t chunk_tiles) {
    return (size_t)waves_per_block *
           (general ? chunk_bytes_for<true>(emax, chunk_tiles) : chunk_bytes_for<false>(emax, chunk_tiles));
}

hipError_t launch_filter(const FilterParams& p, Engine eng, bool general, int emax,
                         const LaunchShape& shape, hipStream_t stream) {
    const void* k = filter_kernel_ptr(eng, general, emax);
    if (!k) return hipErrorInvalidValue;
    FilterParams arg = p;
    void* args[] = {&arg};
    return hipLaunchKernel(k, dim3(shape.blocks), dim3(64 * shape.waves_per_block), args,
                           shape.lds_bytes, stream);
}

hipError_t launch_pack(const uint8_t* codes, uint32_t code_stride, const uint16_t* len,
                       uint32_t uniform_len, const uint64_t* word_offset, uint32_t stride_words,
                       uint64_t n, uint32_t wmax, uint64_t* words, uint32_t* err, hipStream_t s) {
    const uint64_t threads = n * wmax;
    const uint32_t blocks = (uint32_t)((threads + 255) / 256);
    hipLaunchKernelGGL(pack_kernel, dim3(blocks), dim3(256), 0, s, codes, code_stride, len,
                       uniform_len, word_offset, stride_words, n, wmax, words, err);
    return hipGetLastError();
}

hipError_t launch_accept_from_counts(const uint16_t* cnt, const uint16_t* len, uint32_t uniform_len,
                                     const uint8_t* E, uint32_t uniform_E, uint32_t max_len,
                                     uint32_t max_E, uint64_t n, uint32_t* acc, hipStream_t s) {
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    hipLaunchKernelGGL(accept_kernel, dim3(blocks), dim3(256), 0, s, cnt, len, uniform_len, E,
                       uniform_E, max_len, max_E, n, acc);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace paf
