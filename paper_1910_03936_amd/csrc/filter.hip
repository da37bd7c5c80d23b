// Pre-alignment filter kernels for gfx950: SneakySnake engines, encoder and
// small helpers.  (GateKeeper and Shouji, which read the whole map, are in
// whole.hip.)
//
// One lane per (read, reference segment) pair.  Sequences arrive 2-bit
// packed (planar inside each uint64 word, see paf.h).  The neighbourhood map
// (Eq. 6.1; the unweighted maze of Eq. 8.2) is never materialised in HBM: for
// one 32-column window at a time each lane builds the 2E+1 diagonal words in
// VGPRs with funnel shifts (v_alignbit) and 3-input logic (v_bitop3).
// Diagonal d compares ref[c] with read[c + d].
//
// Two SneakySnake engines (Ch. 8, Sec. 8.4):
//  * per tile: a wave holds 64 pairs staged in LDS, word-major ([word][lane]),
//    and walks the windows in step until all 64 are decided;
//  * compacting: a wave owns a chunk of tiles and regroups the pairs still
//    undecided into full waves between passes (see chunk_snake).
#include "paf_tile.h"

namespace paf {

namespace {

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
                const uint32_t bs = 1u << s;
                uint32_t r0 = 0, r1 = 0;
#pragma unroll
                for (int i = 0; i < D; i += 2) {
                    r0 = pipe_runs(r0, M[i], bs);
                    if (i + 1 < D) r1 = pipe_runs(r1, M[i + 1], bs);
                }
                const uint32_t runs = r0 | r1;
                const bool clear = (int32_t)runs < 0;      // a pipe runs past the window
                // The obstacle's column (the window's end when clear).
                const uint32_t R = c + popc(runs);
                const bool reach = R >= m;                 // the pipe reaches the last column
                const bool obst = !reach && !clear;
                e += obst ? 1u : 0u;
                c = R + 1u + (uint32_t)((int32_t)runs >> 31);
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
// edits e (5), continuation flag (1), m (10), E (5), and for a partitioned
// maze the edits counted in the current sub-maze (5); plus the dead-diagonal
// mask of a snake that entered the window inside a pipe, and (general
// layout) the pair's word offset.
constexpr uint32_t kChunkMaxTiles = 16;

struct ChunkEntry {
    uint32_t idx, c, e, m, E, ep;
    bool cont;
};

__device__ __forceinline__ uint64_t chunk_pack(const ChunkEntry& t) {
    return (uint64_t)t.idx | ((uint64_t)t.c << 10) | ((uint64_t)t.e << 19) | ((uint64_t)t.cont << 24) |
           ((uint64_t)t.m << 25) | ((uint64_t)t.E << 35) | ((uint64_t)min(t.ep, 31u) << 40);
}

__device__ __forceinline__ ChunkEntry chunk_unpack(uint64_t v) {
    ChunkEntry t;
    t.idx = (uint32_t)v & 1023u;
    t.c = (uint32_t)(v >> 10) & 511u;
    t.e = (uint32_t)(v >> 19) & 31u;
    t.cont = ((v >> 24) & 1u) != 0;
    t.m = (uint32_t)(v >> 25) & 1023u;
    t.E = (uint32_t)(v >> 35) & 31u;
    t.ep = (uint32_t)(v >> 40) & 31u;
    return t;
}

// Match words of one window for the compacting engine: bit j of Z_d is 1
// when column j is a free cell of diagonal d, i.e. the complement of the
// mismatch word (lo ^ flo) | (hi ^ fhi) over the two code planes.  VAC folds
// in the vacant cells: kVacFirst for window 0 of pairs of 64 columns or more
// (only the read positions before 0 are vacant: the low -d bits of diagonal
// d < 0, a constant), kVacAny from the per-lane vacancy words (short pairs and
// the last windows).  CONT folds in the dead-diagonal bit of a snake that
// entered inside a pipe (bit 0 of the window).  v_bitop3 takes s1 | (s0 ^ s2)
// (truth table 0xDE) and its complement (0x21) in one instruction; both are
// symmetric in s0 and s2.
constexpr int kVacNone = 0, kVacFirst = 1, kVacAny = 2;
__device__ __forceinline__ uint32_t or_xor3(uint32_t a, uint32_t t, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, t, b, 0xDE);
}
__device__ __forceinline__ uint32_t nor_xor3(uint32_t a, uint32_t t, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, t, b, 0x21);
}

template <int EMAX, int VAC, bool CONT, typename DT, int I = 0>
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
        if constexpr (VAC == kVacFirst && !CONT && d < 0) {
            t = or_xor3(lo, (1u << -d) - 1u, q.flo);
        } else if constexpr (VAC == kVacAny || CONT) {
            uint32_t v = 0;
            if constexpr (VAC == kVacAny) v = diag_vacant<d>(q);
            if constexpr (VAC == kVacFirst && d < 0) v = (1u << -d) - 1u;
            if constexpr (CONT) v |= (uint32_t)((dead >> I) & 1u);
            t = or_xor3(lo, v, q.flo);
        } else {
            t = lo ^ q.flo;
        }
        M[I] = nor_xor3(hi, t, q.fhi);
        chunk_map<EMAX, VAC, CONT, DT, I + 1>(q, dead, M);
    }
}

// Two lanes per pair: lane h = 0 builds the match words of diagonals
// d = -EMAX..0 and lane h = 1 those of d = 0..EMAX (EMAX + 1 slots each; the
// main diagonal is in both, which changes neither the deepest pipe nor its
// continuation).  Slot I of lane h reads the read plane shifted by I + s_h:
// s_1 = 0 (words c, n) and s_0 = 32 - EMAX (words p, c), so after one
// funnel shift per plane at the window's start (A, B below) every slot is a
// funnel shift by the compile-time I, as in chunk_map.  Vacancy comes from the
// per-lane vacancy words (VAC), the dead bits of a snake inside a pipe from
// this lane's half of the mask.
struct HalfWords {
    uint32_t alo, blo, ahi, bhi, flo, fhi, va, vb;
};

template <int EMAX>
__device__ __forceinline__ HalfWords half_words(const WindowWords& q, int h) {
    constexpr uint32_t s0 = 32u - (uint32_t)EMAX;
    HalfWords r;
    r.alo = h ? q.clo : funnel(q.clo, q.plo, s0);
    r.blo = h ? q.nlo : (q.clo >> s0);
    r.ahi = h ? q.chi : funnel(q.chi, q.phi, s0);
    r.bhi = h ? q.nhi : (q.chi >> s0);
    r.va = h ? q.vc : funnel(q.vc, q.vp, s0);
    r.vb = h ? q.vn : (q.vc >> s0);
    r.flo = q.flo;
    r.fhi = q.fhi;
    return r;
}

template <int EMAX, bool VAC, bool CONT, int I = 0>
__device__ __forceinline__ void chunk_map_half(const HalfWords& q, uint32_t dead, uint32_t* M) {
    if constexpr (I < EMAX + 1) {
        const uint32_t lo = funnel(q.blo, q.alo, I);
        const uint32_t hi = funnel(q.bhi, q.ahi, I);
        uint32_t v = 0;
        if constexpr (VAC) v = funnel(q.vb, q.va, I);
        if constexpr (CONT) v |= (dead >> I) & 1u;
        const uint32_t t = (VAC || CONT) ? or_xor3(lo, v, q.flo) : lo ^ q.flo;
        M[I] = nor_xor3(hi, t, q.fhi);
        chunk_map_half<EMAX, VAC, CONT, I + 1>(q, dead, M);
    }
}

// Dead-diagonal mask of one lane: with two lanes per pair each lane keeps the
// bits of its own half of the diagonals (EMAX + 1 of them, so 32 bits do).
template <int EMAX, int LPP>
struct ChunkDead {
    using T = typename std::conditional<LPP == 2, uint32_t, typename DeadMask<EMAX>::T>::type;
};

template <typename DT, bool GENERAL>
struct ChunkLds {
    uint64_t* ent;    // the list: K*64 entries
    uint64_t* off;    // GENERAL only: word offset of each pair of the chunk (by pair index)
    DT* dead;         // dead-diagonal mask of each pair (by pair index; two halves, one per
                      // lane, with two lanes per pair)
    uint32_t* acc;    // 2K accept words (plain order)
    uint16_t* cnt;    // K*64 counts (plain order)
};

// The first pass's windows 0 and 1 read words 0..2 of the read and words 0
// and 1 of the reference.  Each lane loads its own pair's five at the start
// of the group, all at once, so the group waits for memory once:
// w = read words 0..2, then reference words 0 and 1 (zero past the pair).
__device__ __forceinline__ void first_words(const uint64_t* rd, const uint64_t* rf, uint32_t W, uint64_t (&w)[5]) {
    w[0] = W > 0u ? rd[0] : 0ull;
    w[1] = W > 1u ? rd[1] : 0ull;
    w[2] = W > 2u ? rd[2] : 0ull;
    w[3] = W > 0u ? rf[0] : 0ull;
    w[4] = W > 1u ? rf[1] : 0ull;
}

// Window k (0 or 1) from those words.
__device__ __forceinline__ WindowWords window_words_first(const uint64_t (&w)[5], int k, int m) {
    WindowWords q;
    const bool one = k != 0;
    const uint64_t p = one ? w[0] : 0ull, c = one ? w[1] : w[0], n = one ? w[2] : w[1], f = one ? w[4] : w[3];
    q.plo = (uint32_t)p; q.phi = (uint32_t)(p >> 32);
    q.clo = (uint32_t)c; q.chi = (uint32_t)(c >> 32);
    q.nlo = (uint32_t)n; q.nhi = (uint32_t)(n >> 32);
    q.flo = (uint32_t)f; q.fhi = (uint32_t)(f >> 32);
    q.vp = vacant_word(k - 1, m);
    q.vc = vacant_word(k, m);
    q.vn = vacant_word(k + 1, m);
    return q;
}

// Window k's words read from memory, the read words carried over from window
// k - 1 of the same pass (first = true at a pass's first window, which loads
// all of them).
struct Carry {
    uint64_t c, n;
};

__device__ __forceinline__ WindowWords window_words_carried(const uint64_t* rd, const uint64_t* rf, int k,
                                                            int W, int m, bool first, Carry& cy) {
    WindowWords q;
    uint64_t p, c;
    if (first) {
        p = (k > 0 && k - 1 < W) ? rd[k - 1] : 0ull;
        c = k < W ? rd[k] : 0ull;
    } else {
        p = cy.c;
        c = cy.n;
    }
    const uint64_t n = k + 1 < W ? rd[k + 1] : 0ull;
    const uint64_t f = k < W ? rf[k] : 0ull;
    cy.c = c;
    cy.n = n;
    q.plo = (uint32_t)p; q.phi = (uint32_t)(p >> 32);
    q.clo = (uint32_t)c; q.chi = (uint32_t)(c >> 32);
    q.nlo = (uint32_t)n; q.nhi = (uint32_t)(n >> 32);
    q.flo = (uint32_t)f; q.fhi = (uint32_t)(f >> 32);
    q.vp = vacant_word(k - 1, m);
    q.vc = vacant_word(k, m);
    q.vn = vacant_word(k + 1, m);
    return q;
}

// PART: the maze is cut into sub-mazes of P.part columns, each solved on its
// own (Sec. 8.6; SneakySnake-t of Sec. 9.3.1).  A lane then also tracks pe,
// the first column of the next sub-maze: a probe's run is cut at pe, reaching
// pe costs nothing, and the snake leaves pe free to take any diagonal.  With
// a cap y (P.part_cap), a sub-maze counts at most y obstacles: the hardware's
// y replications each cross one, so after the y-th the snake moves on to pe
// (a sub-maze then counts min(y, its fewest obstacles), the hardware's
// min(y, w - sum x)).
//
// Passes.  The first pass takes the chunk's pairs in order, 64 at a time:
// up to EMAX 10 each lane loads the words of its pair's first two windows at
// the group's start (first_words), and the group walks windows [0, span0)
// (later windows of a wider first pass, and every window above EMAX 10, read
// their words from memory).  The pairs still undecided are appended to the
// list (in key order when a key is given) and the later passes take the
// list 64 at a time through `span` windows each, reading their words from
// memory (up to EMAX 8 carrying a pair's read words from one window to the
// next).  Counts and accept bits of the chunk are collected in LDS and
// written once at the end.
//
// LPP = 2: two lanes per pair (whole maze only, EMAX 10 and up): a group is
// 32 pairs, lane 2j + h holds pair j's half h of the diagonals (chunk_map_half)
// and both lanes of a pair OR their runs after every probe (one DPP move), so
// they walk the same snake; lane h = 0 writes the pair's outputs and list
// entry, each lane its half of the dead-diagonal mask.
template <int EMAX, bool GENERAL, bool PART, int LPP>
__device__ void chunk_snake(const FilterParams& P, uint32_t chunk, uint32_t K, int lane,
                            const ChunkLds<typename ChunkDead<EMAX, LPP>::T, GENERAL>& L) {
    constexpr int D = 2 * EMAX + 1;
    // Up to EMAX 8 the kernel waits on memory more than it issues: there the
    // first two windows' words are loaded together at a group's start and a
    // pair's read words are carried from window to window.  Above, it is
    // bound by instruction issue and every later window reads its words
    // straight from memory; the first two windows' words are still loaded
    // together up to EMAX 10 (measured 2% faster there; from EMAX 12 on the
    // five extra live words cost a wave per SIMD).
    constexpr bool FIRST_REGS = LPP == 1 && EMAX <= 10;
    constexpr bool CARRY = EMAX <= 8;
    static_assert(LPP == 1 || (LPP == 2 && !PART && !FIRST_REGS && !CARRY),
                  "two lanes per pair: whole maze, EMAX >= 9");
    constexpr int DL = LPP == 2 ? EMAX + 1 : D;   // map words per lane
    constexpr uint32_t GS = 64 / LPP;             // pairs per group
    using DT = typename ChunkDead<EMAX, LPP>::T;
    const int h = LPP == 2 ? (lane & 1) : 0;      // this lane's half of the diagonals
    const uint32_t pl = (uint32_t)lane / LPP;     // the pair of the group this lane works on
    const uint64_t slot0 = (uint64_t)chunk * K * 64u;
    const uint32_t n_here = (uint32_t)min<uint64_t>((uint64_t)K * 64u, P.n_pairs - slot0);
    const bool plain_out = !(GENERAL && P.perm);
    if (plain_out)
        for (uint32_t j = (uint32_t)lane; j < 2 * K; j += 64) L.acc[j] = 0u;
    const bool mask_E = GENERAL ? (P.E != nullptr || P.uniform_E < (uint32_t)EMAX)
                                : (P.uniform_E < (uint32_t)EMAX);
    const bool keyed = P.order_key != nullptr && plain_out;
    uint32_t n_ent = 0;
    // Each pass walks windows [w, w + span) with the same lanes; the pairs
    // still undecided after it are regrouped for the next pass.
    for (uint32_t w = 0, span = P.span0; w == 0 || n_ent > 0; w += span, span = P.span) {
        wave_lds_sync();
        const bool first_pass = w == 0;
        const uint32_t n_in = first_pass ? n_here : n_ent;
        uint32_t n_out = 0;
        for (uint32_t g = 0; g < n_in; g += GS) {
            const uint32_t i = g + pl;
            bool act = i < n_in;
            ChunkEntry t = {};
            DT dead = 0;
            uint64_t off = 0;
            uint64_t fw[5] = {};
            if (first_pass) {
                t.idx = i;
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
                            if (plain_out) L.cnt[i] = 0;
                            else P.cnt[0][id] = 0;
                            act = false;
                        }
                    } else {
                        off = slot * (uint64_t)P.stride_words;
                    }
                }
                if constexpr (FIRST_REGS)
                    first_words(P.reads + off, P.refs + off, act ? (t.m + 31u) >> 5 : 0u, fw);
            } else if (act) {
                t = chunk_unpack(L.ent[i]);
                dead = t.cont ? L.dead[t.idx * LPP + h] : (DT)0;
                off = GENERAL ? L.off[t.idx] : (slot0 + t.idx) * (uint64_t)P.stride_words;
            }
            const uint32_t m = act ? t.m : 0u;
            const uint32_t E = t.E;
            const int W = (int)((m + 31) >> 5);
            uint32_t c = t.c, e = t.e;
            bool cont = t.cont;
            // A snake inside a pipe at a window's start is never at a
            // sub-maze's first column (reaching that column ends the pipe), so
            // pe follows from c alone.
            uint32_t pe = PART ? (c / P.part + 1u) * P.part : 0u;
            uint32_t ep = t.ep;
            Carry cy = {0ull, 0ull};
            for (uint32_t wk = w; wk < w + span && wave_any(act); ++wk) {
                WindowWords q;
                if (FIRST_REGS && first_pass && wk < 2u) {
                    q = window_words_first(fw, (int)wk, (int)m);
                } else if constexpr (CARRY) {
                    q = window_words_carried(P.reads + off, P.refs + off, (int)wk, act ? W : 0, (int)m,
                                             wk == (first_pass && FIRST_REGS ? 2u : w), cy);
                } else {
                    q = window_words_direct(P.reads + off, P.refs + off, (int)wk, act ? W : 0, (int)m);
                }
                // Vacant cells only occur in the first window and near the
                // pair's end.  A snake that entered inside a pipe sees the
                // diagonals whose pipes ended before this window blocked in
                // its first column.
                const bool near_end = wave_any(act && 32u * (wk + 2) > m);
                const bool cnt = wave_any(act && cont);
                uint32_t M[DL];
                if constexpr (LPP == 2) {
                    const HalfWords hq = half_words<EMAX>(q, h);
                    if (near_end || wk == 0) {
                        if (cnt) chunk_map_half<EMAX, true, true>(hq, (uint32_t)dead, M);
                        else chunk_map_half<EMAX, true, false>(hq, (uint32_t)dead, M);
                    } else {
                        if (cnt) chunk_map_half<EMAX, false, true>(hq, (uint32_t)dead, M);
                        else chunk_map_half<EMAX, false, false>(hq, (uint32_t)dead, M);
                    }
                } else if (near_end) {
                    if (cnt) chunk_map<EMAX, kVacAny, true>(q, dead, M);
                    else chunk_map<EMAX, kVacAny, false>(q, dead, M);
                } else if (wk == 0) {
                    // No snake is inside a pipe at column 0.
                    chunk_map<EMAX, kVacFirst, false>(q, dead, M);
                } else {
                    if (cnt) chunk_map<EMAX, kVacNone, true>(q, dead, M);
                    else chunk_map<EMAX, kVacNone, false>(q, dead, M);
                }
                if (mask_E) {
#pragma unroll
                    for (int d = 0; d < DL; ++d) {
                        const int dd = LPP == 2 ? (h ? d : d - EMAX) : d - EMAX;
                        if ((uint32_t)(dd < 0 ? -dd : dd) > E) M[d] = 0u;
                    }
                }
                const uint32_t w0 = 32u * wk;
                const bool live = act;
                uint32_t clear = 0, bs = 0;
                if constexpr (PART) {
                    // The snake state stays in plain integers (column c,
                    // edits e, the sub-maze's end pe and its edits ep), so the
                    // loop carries no lane masks beyond its own condition: the
                    // lane probes while c is inside both the window and the
                    // pair and e <= E.
                    const uint32_t w31 = w0 + 31u;
                    const uint32_t lim = min(m, w0 + 32u);
                    while (act && (int32_t)((c - lim) & (e - E - 1u)) < 0) {
                        // Pipes from column c: adding 1 << s to a match word
                        // carries through its run of free cells from s, so
                        // Z & ~(Z + (1 << s)) is that run; the OR over the
                        // diagonals is [s, s + deepest run), with bit 31 set
                        // when a pipe reaches the window's end.
                        bs = 0x80000000u >> (w31 - c);
                        uint32_t r0 = 0, r1 = 0;
#pragma unroll
                        for (int d = 0; d < D; d += 2) {
                            r0 = or_andn(r0, M[d], M[d] + bs);
                            if (d + 1 < D) r1 = or_andn(r1, M[d + 1], M[d + 1] + bs);
                        }
                        uint32_t runs = r0 | r1;
                        // The run stops at the sub-maze's end pe; reaching it
                        // is free (at), and so is the window's end when pe
                        // lies beyond it (clear: the pipe goes on).
                        const uint32_t cut = pe - w0;
                        runs &= cut < 32u ? (1u << cut) - 1u : ~0u;
                        const uint32_t R = c + (uint32_t)__builtin_popcount(runs);
                        const uint32_t at = R == pe ? 1u : 0u;
                        clear = (runs >> 31) & (at ^ 1u);
                        const uint32_t ob = ((R - m) >> 31) & ((clear | at) ^ 1u);
                        e += ob;
                        ep += ob;
                        c = R + 1u - clear - at;
                        c = ep >= P.part_cap ? pe : c;
                        const bool nx = c == pe;
                        pe += nx ? P.part : 0u;
                        ep = nx ? 0u : ep;
                    }
                } else {
                    // Every lane still undecided enters the window at its
                    // first column (it left the last one at its end), so the
                    // snake's column lives in a one-hot word b: a probe from
                    // b gives the run [s, s + L) as above, and runs + b is
                    // the bit of the obstacle at s + L (zero when a pipe runs
                    // through the window's end); the next probe starts one
                    // column after it, (runs + b) << 1.  The lane probes
                    // while b is a column of the pair (so the last probe's
                    // obstacle was inside the pair and cost an edit) and the
                    // edits stay within E: every probe but the last costs one
                    // edit, so the loop only counts probes and the last one
                    // is settled after it.
                    const uint32_t inpair = m >= w0 + 32u ? ~0u : (1u << (m - w0)) - 1u;
                    uint32_t b = act ? 1u : 0u, runs = 0;
                    int32_t budget = (int32_t)E - (int32_t)e;
                    while ((b & inpair) != 0u && budget >= 0) {
                        uint32_t r0 = 0, r1 = 0;
#pragma unroll
                        for (int d = 0; d < DL; d += 2) {
                            r0 = or_andn(r0, M[d], M[d] + b);
                            if (d + 1 < DL) r1 = or_andn(r1, M[d + 1], M[d + 1] + b);
                        }
                        runs = r0 | r1;
                        // The partner lane's half (quad_perm [1, 0, 3, 2]).
                        if constexpr (LPP == 2)
                            runs |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)runs, 0xB1, 0xF, 0xF, false);
                        b = (runs + b) << 1;
                        --budget;
                    }
                    if (live) {
                        const uint32_t probes = (uint32_t)((int32_t)E - (int32_t)e - budget);
                        clear = runs >> 31;
                        // The last probe's obstacle (none when its pipe ran
                        // through the window's end; bit 31 when b wrapped to 0).
                        const uint32_t ob = clear ? 0u : (b != 0u ? b >> 1 : 0x80000000u);
                        e += probes - (probes != 0u && (ob & inpair) == 0u ? 1u : 0u);
                        // The column reached: past the pair's end inside the
                        // window, or the next window's first column.
                        c = b != 0u ? w0 + (uint32_t)__builtin_ctz(b) : w0 + 32u;
                        // The last probe's start, for the dead-diagonal mask
                        // of a pipe running on (its run is [s, 32)).
                        bs = runs & (0u - runs);
                    }
                }
                // A lane is decided once it crossed the pair's end (accept
                // exactly when e <= E) or counted E + 1 edits.
                if (live && (c >= m || e > E)) {
                    act = false;
                    if (h == 0) {
                        if (plain_out) {
                            L.cnt[t.idx] = (uint16_t)e;
                            if (e <= E) atomicOr(&L.acc[t.idx >> 5], 1u << (t.idx & 31u));
                        } else {
                            P.cnt[0][P.perm[slot0 + t.idx]] = (uint16_t)e;
                        }
                    }
                }
                const bool ncont = act && clear != 0u;
                // A diagonal stays alive into the next window when its run
                // from the last probe's start reaches this window's end: bit
                // 31 of Z & ~(Z + bs), shifted into the alive mask.
                DT dm = 0;
                if (wave_any(ncont)) {
                    // That run reaches bit 31 exactly when Z + bs carries out
                    // of it; the carries are shifted in as they come.
                    uint32_t lo = 0, hi = 0;
#pragma unroll
                    for (int d = DL - 1; d >= 0; --d) {
                        uint32_t sum;
                        const uint32_t cy = __builtin_add_overflow(M[d], bs, &sum) ? 1u : 0u;
                        if (d >= 32) hi = hi + hi + cy;
                        else lo = lo + lo + cy;
                    }
                    const DT alive = (DT)lo | (sizeof(DT) > 4 ? (DT)((uint64_t)hi << 32) : (DT)0);
                    constexpr DT all = (DL >= 8 * (int)sizeof(DT)) ? ~(DT)0 : (((DT)1 << DL) - 1);
                    dm = ~alive & all;
                }
                cont = ncont;
                dead = cont ? dm : (DT)0;
            }
            // Survivors go on to the next pass (written behind the read
            // position: n_out + pre <= i).  With two lanes per pair the
            // pair's first lane counts it.
            const uint64_t bal = __ballot(act) & (LPP == 2 ? 0x5555555555555555ull : ~0ull);
            const uint32_t first_lane = (uint32_t)lane & ~(uint32_t)(LPP - 1);
            const uint64_t below = first_lane ? bal & (~0ull >> (64 - first_lane)) : 0ull;
            const uint32_t pre = (uint32_t)__builtin_popcountll(below);
            if (act) {
                ChunkEntry u = t;
                u.c = c;
                u.e = e;
                u.cont = cont;
                u.ep = PART ? ep : 0u;
                if (h == 0) L.ent[n_out + pre] = chunk_pack(u);
                if (cont) L.dead[t.idx * LPP + h] = dead;
            }
            n_out += (uint32_t)__builtin_popcountll(bal);
        }
        n_ent = n_out;
        if (first_pass && keyed && n_ent > 1 && 2 * n_ent <= K * 64u) {
            // The undecided pairs enter the later passes grouped into four
            // classes by the key's bits 2-3 (a stable counting sort by wave
            // ballots, into the list's unused tail and back), so each group of
            // 64 takes pairs of like predicted cost.  (More survivors than
            // half the list keep their order: the key only orders work.)
            uint64_t* const stage = L.ent + (K * 64u - n_ent);
            wave_lds_sync();
            constexpr uint32_t NB = 4;
            uint32_t base[NB];
#pragma unroll
            for (uint32_t v = 0; v < NB; ++v) base[v] = 0;
            for (uint32_t g = 0; g < n_ent; g += 64) {
                const uint32_t i = g + (uint32_t)lane;
                const uint32_t cls = i < n_ent ? (P.order_key[slot0 + ((uint32_t)L.ent[i] & 1023u)] & 15u) >> 2 : NB;
#pragma unroll
                for (uint32_t v = 0; v < NB; ++v) base[v] += (uint32_t)__builtin_popcountll(__ballot(cls == v));
            }
            uint32_t run = 0;
#pragma unroll
            for (uint32_t v = 0; v < NB; ++v) {
                const uint32_t cv = base[v];
                base[v] = run;
                run += cv;
            }
            for (uint32_t g = 0; g < n_ent; g += 64) {
                const uint32_t i = g + (uint32_t)lane;
                const uint64_t v64 = i < n_ent ? L.ent[i] : 0ull;
                const uint32_t cls = i < n_ent ? (P.order_key[slot0 + ((uint32_t)v64 & 1023u)] & 15u) >> 2 : NB;
                uint32_t pos = 0;
#pragma unroll
                for (uint32_t v = 0; v < NB; ++v) {
                    const uint64_t mv = __ballot(cls == v);
                    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mv >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mv, 0u));
                    if (cls == v) pos = base[v] + below;
                    base[v] += (uint32_t)__builtin_popcountll(mv);
                }
                if (cls < NB) stage[pos] = v64;
            }
            wave_lds_sync();
            for (uint32_t i = (uint32_t)lane; i < n_ent; i += 64) L.ent[i] = stage[i];
        }
    }
    if (plain_out) {
        wave_lds_sync();
        for (uint32_t j = (uint32_t)lane; j < 2 * K; j += 64) {
            const uint64_t s0 = slot0 + 32u * j;
            if (s0 < P.n_pairs) P.acc[0][s0 / 32] = L.acc[j];
        }
        // Counts: two per 4-byte store when the output is 4-byte aligned
        // (slot0 is a multiple of 64).
        uint16_t* dst = P.cnt[0] + slot0;
        if (((uintptr_t)dst & 3u) == 0) {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(L.cnt);
            uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
            for (uint32_t j = (uint32_t)lane; 2 * j + 1 < n_here; j += 64) d32[j] = src[j];
            if ((n_here & 1u) && lane == 0) dst[n_here - 1] = L.cnt[n_here - 1];
        } else {
            for (uint32_t j = (uint32_t)lane; j < n_here; j += 64) dst[j] = L.cnt[j];
        }
    }
}

// Bytes of one wave's LDS: list, offsets (general layout), dead masks,
// accept words and counts.
template <int EMAX, bool GENERAL, int LPP = 1>
__host__ __device__ constexpr size_t chunk_wave_bytes_t(uint32_t K) {
    using DT = typename ChunkDead<EMAX, LPP>::T;
    return (size_t)K * 64 * (8 + (GENERAL ? 8 : 0) + LPP * sizeof(DT) + 2) + (size_t)K * 8;
}

// Up to EMAX 8 the kernel is held to the registers of five waves per SIMD:
// measured faster than four waves with the registers it would take otherwise.
// At EMAX 20 and 31 four waves with a few spilled registers measured faster
// than three without (1.28 -> 1.22 and 2.42 -> 2.21 ms per 10M pairs of
// 250 bp); at 25 they did not (1.64 either way), nor are they needed up to 15.
template <int EMAX, bool GENERAL, bool PART, int LPP>
__global__ void __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(LPP == 2 ? 4 : (EMAX <= 8 ? 5 : ((EMAX == 20 || EMAX == 31) ? 4 : 1)))))
chunk_kernel(FilterParams P) {
    extern __shared__ uint64_t lds[];
    using DT = typename ChunkDead<EMAX, LPP>::T;
    const int lane = threadIdx.x & 63;
    // Wave-uniform, so the LDS pointers below live in scalar registers.
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t K = P.chunk;
    const uint32_t NE = K * 64u;
    char* b = reinterpret_cast<char*>(lds) + (size_t)wave * chunk_wave_bytes_t<EMAX, GENERAL, LPP>(K);
    ChunkLds<DT, GENERAL> L;
    L.ent = reinterpret_cast<uint64_t*>(b);
    b += (size_t)NE * 8;
    if (GENERAL) {
        L.off = reinterpret_cast<uint64_t*>(b);
        b += (size_t)NE * 8;
    } else {
        L.off = nullptr;
    }
    L.dead = reinterpret_cast<DT*>(b);
    b += (size_t)NE * LPP * sizeof(DT);
    L.acc = reinterpret_cast<uint32_t*>(b);
    b += (size_t)K * 8;
    L.cnt = reinterpret_cast<uint16_t*>(b);
    const uint32_t n_chunks = (P.n_tiles + K - 1) / K;
    if (P.queue == nullptr) {
        const uint32_t ch = blockIdx.x * (blockDim.x >> 6) + wave;
        if (ch < n_chunks) chunk_snake<EMAX, GENERAL, PART, LPP>(P, ch, K, lane, L);
        return;
    }
    uint32_t c0 = 0;
    if (lane == 0) c0 = atomicAdd(P.queue, 1u);
    c0 = __shfl(c0, 0);
    while (c0 < n_chunks) {
        uint32_t nx = 0;
        if (lane == 0) nx = atomicAdd(P.queue, 1u);
        chunk_snake<EMAX, GENERAL, PART, LPP>(P, c0, K, lane, L);
        wave_lds_sync();
        c0 = __shfl(nx, 0);
    }
}

template <bool GENERAL, bool PART>
const void* chunk_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&chunk_kernel<X, GENERAL, PART, 1>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

// Two lanes per pair: the whole maze from EMAX 10 on.
template <bool GENERAL>
const void* chunk2_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&chunk_kernel<X, GENERAL, false, 2>);
        PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25) PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

template <bool GENERAL>
size_t chunk_bytes_for(int emax, uint32_t K, uint32_t lpp) {
    if (lpp == 2) return chunk_wave_bytes_t<31, GENERAL, 2>(K);
    return emax <= 15 ? chunk_wave_bytes_t<15, GENERAL>(K) : chunk_wave_bytes_t<31, GENERAL>(K);
}

template <int EMAX, bool GENERAL>
__global__ void __launch_bounds__(512) snake_kernel(FilterParams P) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint64_t* rdL = lds + (size_t)wave * 2 * P.wmax * kLdsRow;
    uint64_t* rfL = rdL + (size_t)P.wmax * kLdsRow;
    for_each_tile(P, lane, wave, [&](uint64_t tile) { snake_tile<EMAX, GENERAL>(P, tile, lane, rdL, rfL); });
}

template <bool GENERAL>
const void* snake_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&snake_kernel<X, GENERAL>);
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

const void* filter_kernel_ptr(Engine eng, bool general, int emax, uint32_t filters) {
    if (eng == Engine::Chunk) return general ? chunk_kernel_for<true, false>(emax) : chunk_kernel_for<false, false>(emax);
    if (eng == Engine::Chunk2) return general ? chunk2_kernel_for<true>(emax) : chunk2_kernel_for<false>(emax);
    if (eng == Engine::ChunkPart)
        return general ? chunk_kernel_for<true, true>(emax) : chunk_kernel_for<false, true>(emax);
    if (eng == Engine::Snake) return general ? snake_kernel_for<true>(emax) : snake_kernel_for<false>(emax);
    return whole_kernel_ptr(general, emax, filters);
}

size_t filter_lds_bytes(uint32_t waves_per_block, uint32_t wmax) {
    return (size_t)waves_per_block * 2 * wmax * kLdsRow * sizeof(uint64_t);
}

size_t chunk_lds_bytes(uint32_t waves_per_block, bool general, int emax, uint32_t chunk_tiles, uint32_t lpp) {
    return (size_t)waves_per_block * (general ? chunk_bytes_for<true>(emax, chunk_tiles, lpp)
                                              : chunk_bytes_for<false>(emax, chunk_tiles, lpp));
}

hipError_t launch_filter(const FilterParams& p, Engine eng, bool general, int emax,
                         const LaunchShape& shape, hipStream_t stream) {
    const void* k = filter_kernel_ptr(eng, general, emax, p.filters);
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
