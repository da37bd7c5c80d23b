// Whole-map decision stages for gfx950: GateKeeper (Ch. 5) and Shouji
// (Ch. 6), which read every window of the map, plus SneakySnake on the same
// map when asked for.  One lane per pair, 64 pairs per wave staged in LDS
// (word-major); windows are walked in step.
#include "paf_tile.h"

namespace paf {

namespace {

// ---------------------------------------------------------------------------
// Whole-map engine.


// Shouji: bit-sliced best 4-column segment per window start column.
struct ShoujiBest {
    uint32_t o0, o1, o2;      // ones in the best segment (bit-sliced, 0..4)
    uint32_t b0, b1, b2, b3;  // the best segment's bits
};

// Three-input logic in one v_bitop3 each (truth table bit s0 * 4 + s1 * 2 + s2):
// m ? x : y; a ^ b ^ c; and one step of a bit-sliced less-than from the low
// bit up, (~n & o) | (~(n ^ o) & t).
__device__ __forceinline__ uint32_t sel3(uint32_t m, uint32_t x, uint32_t y) {
    return __builtin_amdgcn_bitop3_b32(m, x, y, 0xCA);
}
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t lt_step(uint32_t n, uint32_t o, uint32_t t) {
    return __builtin_amdgcn_bitop3_b32(n, o, t, 0x8E);
}

__device__ __forceinline__ void shouji_candidate(ShoujiBest& bs, uint32_t cur, uint32_t nxt,
                                                 bool first) {
    const uint32_t B0 = cur;
    const uint32_t B1 = funnel(nxt, cur, 1);
    const uint32_t B2 = funnel(nxt, cur, 2);
    const uint32_t B3 = funnel(nxt, cur, 3);
    // Ones in the segment, bit-sliced: n = B0 + B1 + B2 + B3 (0..4).
    const uint32_t s01 = B0 ^ B1, c01 = B0 & B1, s23 = B2 ^ B3, c23 = B2 & B3;
    const uint32_t n0 = s01 ^ s23;
    const uint32_t n1 = xor3(c01, c23, s01 & s23);
    const uint32_t n2 = c01 & c23;
    if (first) {
        bs = {n0, n1, n2, B0, B1, B2, B3};
        return;
    }
    // Fewer ones wins; on a tie, a segment that starts with a zero beats one
    // that does not; otherwise the earlier diagonal is kept.  That is one
    // strict comparison of the keys 2 n + B0 and 2 o + b0, bit-sliced from
    // the lowest bit up: t = new < best on the bits seen so far.
    const uint32_t t0 = ~B0 & bs.b0;
    const uint32_t rep = lt_step(n2, bs.o2, lt_step(n1, bs.o1, lt_step(n0, bs.o0, t0)));
    bs.o0 = sel3(rep, n0, bs.o0);
    bs.o1 = sel3(rep, n1, bs.o1);
    bs.o2 = sel3(rep, n2, bs.o2);
    bs.b0 = sel3(rep, B0, bs.b0);
    bs.b1 = sel3(rep, B1, bs.b1);
    bs.b2 = sel3(rep, B2, bs.b2);
    bs.b3 = sel3(rep, B3, bs.b3);
}

// Bits 0..7 of x spread to bits 0, 4, ..., 28.
__device__ __forceinline__ uint32_t spread8(uint32_t x) {
    x = (x | (x << 12)) & 0x000F000Fu;
    x = (x | (x << 6)) & 0x03030303u;
    return (x | (x << 3)) & 0x11111111u;
}

// The best segments of the window's 32 start columns as nibbles: word k holds
// the segment of column j = 8k + i in bits 4i..4i+3 (bit t = the segment's
// column j + t).
__device__ __forceinline__ void shouji_nibbles(const ShoujiBest& bs, uint32_t* nib) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int sh = 8 * k;
        nib[k] = spread8((bs.b0 >> sh) & 0xFFu) | (spread8((bs.b1 >> sh) & 0xFFu) << 1) |
                 (spread8((bs.b2 >> sh) & 0xFFu) << 2) | (spread8((bs.b3 >> sh) & 0xFFu) << 3);
    }
}

// Sequential store into the Shouji bit-vector for the 32 windows starting in
// this window (Sec. 6.2.2): the best segment overwrites the vector's four
// bits when it holds strictly more zeros.  S covers columns [32w, 32w+64).
// Window starts past the pair's end hold segment 1111 (see below), which
// never holds strictly more zeros than the vector, so they store nothing.
template <int J = 0>
__device__ __forceinline__ void shouji_store_nib(const uint32_t* nib, uint32_t& S_lo, uint32_t& S_hi) {
    if constexpr (J < 32) {
        const uint32_t V = (nib[J >> 3] >> (4 * (J & 7))) & 0xFu;
        uint32_t cur;
        if constexpr (J <= 28) cur = (S_lo >> J) & 0xFu;
        else cur = funnel(S_hi, S_lo, J) & 0xFu;
        const bool take = popc(V) < popc(cur);
        if constexpr (J <= 28) {
            const uint32_t nlo = (S_lo & ~(0xFu << J)) | (V << J);
            S_lo = take ? nlo : S_lo;
        } else {
            const uint32_t nlo = (S_lo & ~(0xFu << J)) | (V << J);
            const uint32_t nhi = (S_hi & ~(0xFu >> (32 - J))) | (V >> (32 - J));
            S_lo = take ? nlo : S_lo;
            S_hi = take ? nhi : S_hi;
        }
        shouji_store_nib<J + 1>(nib, S_lo, S_hi);
    }
}

template <int EMAX, int I = 0>
__device__ __forceinline__ void build_both(const WindowWords& q, uint32_t* Mh, uint32_t* G) {
    if constexpr (I < 2 * EMAX + 1) {
        diag_both<I - EMAX>(q, Mh[I], G[I]);
        build_both<EMAX, I + 1>(q, Mh, G);
    }
}

// Only the blocked map (SneakySnake, Shouji): vacant and past-end cells 1.
template <int EMAX, int I = 0>
__device__ __forceinline__ void build_blocked(const WindowWords& q, uint32_t* Mh) {
    if constexpr (I < 2 * EMAX + 1) {
        constexpr int d = I - EMAX;
        Mh[I] = diag_raw<d>(q) | diag_vacant<d>(q) | q.vc;
        build_blocked<EMAX, I + 1>(q, Mh);
    }
}

// Window k of every active lane's pair is inner: k >= 1 and its columns,
// plus max_E beyond, lie before the pair's end, so no cell of any diagonal
// is vacant there.
template <int EMAX>
__device__ __forceinline__ bool inner_window(bool active, uint32_t k, uint32_t m) {
    return !wave_any(active && (k == 0u || 32u * (k + 1u) + (uint32_t)EMAX > m));
}

// Only GateKeeper's map: vacant and past-end cells 0 (INNER: an inner window,
// the raw mismatch words).
template <int EMAX, bool INNER = false, int I = 0>
__device__ __forceinline__ void build_gk(const WindowWords& q, uint32_t* G) {
    if constexpr (I < 2 * EMAX + 1) {
        constexpr int d = I - EMAX;
        if constexpr (INNER) G[I] = diag_raw<d>(q);
        else G[I] = diag_raw<d>(q) & ~(diag_vacant<d>(q) | q.vc);
        build_gk<EMAX, INNER, I + 1>(q, G);
    }
}

// Fw AND GateKeeper's amendment of one window word g (Ch. 5, Sec. 5.2.2; SRS
// of Sec. 3.2.1): a zero inside a streak of one or two zeros bounded by ones
// on both sides becomes one.  L1/L2 are the bits one/two columns to the left,
// R1/R2 to the right (taken from the neighbouring windows); the amended word
// g | L1 (R1 | R2) | R1 (L1 | L2) = L1 (R1 | R2) | (R1 L2 | g) takes three
// 3-input operations with the AND.
__device__ __forceinline__ uint32_t and_amended(uint32_t Fw, uint32_t g, uint32_t prev, uint32_t next) {
    const uint32_t L1 = funnel(g, prev, 31);
    const uint32_t L2 = funnel(g, prev, 30);
    const uint32_t R1 = funnel(next, g, 1);
    const uint32_t R2 = funnel(next, g, 2);
    const uint32_t t = __builtin_amdgcn_bitop3_b32(L1, R1, R2, 0xE0);  // L1 & (R1 | R2)
    const uint32_t u = __builtin_amdgcn_bitop3_b32(R1, L2, g, 0xEA);   // (R1 & L2) | g
    return __builtin_amdgcn_bitop3_b32(Fw, t, u, 0xE0);                // Fw & (t | u)
}

// FS: the decision stages this instantiation runs (bits of PAF_*), or 0 for
// any mask given at run time.  Only the words the stages read are built.
template <int EMAX, bool GENERAL, int FS>
__device__ void whole_tile(const FilterParams& P, uint64_t tile, int lane, uint64_t* rdL,
                           uint64_t* rfL) {
    constexpr int D = 2 * EMAX + 1;
    using DT = typename DeadMask<EMAX>::T;
    uint64_t off;
    const PairSlot ps = load_slot<GENERAL>(P, tile, lane, off);
    stage_tile<GENERAL>(P, tile, lane, ps, off, rdL, rfL);

    constexpr bool RT = FS == 0;
    constexpr bool needG = RT || (FS & PAF_GATEKEEPER);
    constexpr bool needM = RT || (FS & (PAF_SNEAKYSNAKE | PAF_SHOUJI));
    const bool doSS = RT ? (P.filters & PAF_SNEAKYSNAKE) != 0 : (FS & PAF_SNEAKYSNAKE) != 0;
    const bool doGK = RT ? (P.filters & PAF_GATEKEEPER) != 0 : (FS & PAF_GATEKEEPER) != 0;
    const bool doSH = RT ? (P.filters & PAF_SHOUJI) != 0 : (FS & PAF_SHOUJI) != 0;
    const uint32_t m = ps.m, E = ps.E;
    const bool mask_E = GENERAL ? (P.E != nullptr || P.uniform_E < (uint32_t)EMAX)
                                : (P.uniform_E < (uint32_t)EMAX);

    Snake z{0u, 0u, ps.valid && doSS, false, 0u};
    bool cont = false;
    DT dead = 0;
    uint32_t gk_ham = 0, gk_cnt = 0;
    uint32_t S_lo = ~0u, S_hi = ~0u, sh_cnt = 0;

    uint32_t Mc[needM ? D : 1], Gc[needG ? D : 1], Gp[needG ? D : 1];
    if (ps.valid) {
        const WindowWords q = window_words(rdL, rfL, lane, 0, P.wmax, (int)m);
        if constexpr (needM && needG) build_both<EMAX>(q, Mc, Gc);
        else if constexpr (needM) build_blocked<EMAX>(q, Mc);
        else build_gk<EMAX>(q, Gc);
    }
    if constexpr (needG) {
#pragma unroll
        for (int i = 0; i < D; ++i) Gp[i] = 0u;
    }
    if (mask_E && ps.valid) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int d = i - EMAX;
            if ((uint32_t)(d < 0 ? -d : d) > E) {
                if constexpr (needM) Mc[i] = ~0u;
                if constexpr (needG) { Gc[i] = ~0u; Gp[i] = ~0u; }
            }
        }
    }

    if constexpr (FS == PAF_GATEKEEPER && EMAX <= 10) {
        // GateKeeper alone: the previous, current and next window's masks
        // take turns in three arrays, so no window copies them on (the loop
        // is unrolled by hand; its wave vote keeps the compiler from it).
        // Above max_E 10 the third array would cost occupancy.
        uint32_t Gx[D];
        auto gk_window = [&](uint32_t w, const uint32_t (&Gpv)[D], const uint32_t (&Gcu)[D], uint32_t (&Gnx)[D]) {
            const bool inner = inner_window<EMAX>(ps.valid && w < ps.W, w + 1u, m);
            if (ps.valid && w < ps.W) {
                const uint32_t colpast = vacant_word((int)w, (int)m);  // columns >= m
                gk_ham += popc(Gcu[EMAX] & ~colpast);
                const WindowWords qn = window_words(rdL, rfL, lane, (int)w + 1, P.wmax, (int)m);
                if (inner) build_gk<EMAX, true>(qn, Gnx);
                else build_gk<EMAX>(qn, Gnx);
                uint32_t Fw = ~0u;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    if (mask_E) {
                        const int d = i - EMAX;
                        if ((uint32_t)(d < 0 ? -d : d) > E) Gnx[i] = ~0u;
                    }
                    Fw = and_amended(Fw, Gcu[i], Gpv[i], Gnx[i]);
                }
                gk_cnt += popc(Fw & ~colpast);
            }
        };
        for (uint32_t w = 0;;) {
            if (!wave_any(ps.valid && w < ps.W)) break;
            gk_window(w++, Gp, Gc, Gx);
            if (!wave_any(ps.valid && w < ps.W)) break;
            gk_window(w++, Gc, Gx, Gp);
            if (!wave_any(ps.valid && w < ps.W)) break;
            gk_window(w++, Gx, Gp, Gc);
        }
    } else
    for (uint32_t w = 0; wave_any(ps.valid && w < ps.W); ++w) {
        const bool have = ps.valid && w < ps.W;
        if (have) {
            const uint32_t colpast = vacant_word((int)w, (int)m);  // columns >= m
            // SneakySnake on this window.
            if constexpr (needM)
                if (doSS && z.act) snake_window<EMAX, DT>(z, Mc, w, m, E, cont, dead);
            // GateKeeper's fast path: Hamming distance on diagonal 0 (its
            // mismatches, vacant cells not counted).
            if constexpr (needG)
                if (doGK) gk_ham += popc(Gc[EMAX] & ~colpast);
            // This window's blocked main diagonal (Shouji at E = 0, below).
            const uint32_t mc0 = needM ? Mc[0] : 0u;
            // Next window's maps, then GateKeeper and Shouji per diagonal.
            const WindowWords qn = window_words(rdL, rfL, lane, (int)w + 1, P.wmax, (int)m);
            uint32_t Fw = ~0u;
            ShoujiBest bs;
            uint32_t Mn[needM ? D : 1], Gn[needG ? D : 1];
            if constexpr (needM && needG) build_both<EMAX>(qn, Mn, Gn);
            else if constexpr (needM) build_blocked<EMAX>(qn, Mn);
            else build_gk<EMAX>(qn, Gn);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (mask_E) {
                    const int d = i - EMAX;
                    if ((uint32_t)(d < 0 ? -d : d) > E) {
                        if constexpr (needM) Mn[i] = ~0u;
                        if constexpr (needG) Gn[i] = ~0u;
                    }
                }
                if constexpr (needG) {
                    if (doGK) Fw = and_amended(Fw, Gc[i], Gp[i], Gn[i]);
                    Gp[i] = Gc[i];
                    Gc[i] = Gn[i];
                }
                if constexpr (needM) {
                    if constexpr (EMAX > 0)
                        if (doSH) shouji_candidate(bs, Mc[i], Mn[i], i == 0);
                    Mc[i] = Mn[i];
                }
            }
            if (doGK) gk_cnt += popc(Fw & ~colpast);
            if (doSH && EMAX == 0) {
                // One diagonal (E = 0): the window starting at column j
                // replaces the vector's bits j..j+3, which hold the diagonal's
                // bits j..j+2 and a still unset 1 at j+3, exactly when bit j+3
                // of the diagonal is 0; the first window leaves the vector's
                // first four bits equal to the diagonal's either way.  So the
                // vector ends equal to the diagonal, and the count is its
                // Hamming distance.
                sh_cnt += popc(mc0 & ~colpast);
            } else if (doSH) {
                // Start columns at or past the pair's end get segment 1111.
                const uint32_t ncols = m - 32u * w;  // >= 1
                const uint32_t past = ncols >= 32u ? 0u : ~0u << ncols;
                bs.b0 |= past;
                bs.b1 |= past;
                bs.b2 |= past;
                bs.b3 |= past;
                uint32_t nib[4];
                shouji_nibbles(bs, nib);
                shouji_store_nib(nib, S_lo, S_hi);
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


template <int EMAX, bool GENERAL, int FS>
__global__ void __launch_bounds__(256) whole_kernel(FilterParams P) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint64_t* rdL = lds + (size_t)wave * 2 * P.wmax * kLdsRow;
    uint64_t* rfL = rdL + (size_t)P.wmax * kLdsRow;
    for_each_tile(P, lane, wave, [&](uint64_t tile) { whole_tile<EMAX, GENERAL, FS>(P, tile, lane, rdL, rfL); });
}

template <bool GENERAL, int FS>
const void* whole_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&whole_kernel<X, GENERAL, FS>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

}  // namespace

// GateKeeper alone and Shouji alone get kernels of their own; every other
// mask runs on the kernel that reads the mask at run time.
const void* whole_kernel_ptr(bool general, int emax, uint32_t filters) {
    if (filters == PAF_GATEKEEPER) return general ? whole_for<true, PAF_GATEKEEPER>(emax)
                                                  : whole_for<false, PAF_GATEKEEPER>(emax);
    if (filters == PAF_SHOUJI) return general ? whole_for<true, PAF_SHOUJI>(emax) : whole_for<false, PAF_SHOUJI>(emax);
    return general ? whole_for<true, 0>(emax) : whole_for<false, 0>(emax);
}

}  // namespace paf
