// Device helpers shared by the filter and cost-model kernels: the 2-bit
// planar sequence words of one 32-column window and the diagonal mismatch
// words built from them (neighbourhood map, Eq. 6.1; unweighted maze, Eq. 8.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "paf_internal.h"

namespace paf {

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

__device__ __forceinline__ uint32_t popc(uint32_t x) { return __builtin_popcount(x); }

// acc | (z & ~y) in one v_bitop3 (truth table 0xF4 with s0 = acc, s1 = z,
// s2 = y).
__device__ __forceinline__ uint32_t or_andn(uint32_t acc, uint32_t z, uint32_t y) {
    return __builtin_amdgcn_bitop3_b32(acc, z, y, 0xF4);
}

// Free cells from window-relative column s on, given a mismatch word M
// (1 = blocked): subtracting 1 << s borrows through the zeros of M from s up
// to its next one, so (M - (1 << s)) & ~M is exactly that run of free cells
// (all of [s, 32) when no obstacle follows).  Accumulated over diagonals, the
// OR is [s, s + depth of the deepest pipe).
__device__ __forceinline__ uint32_t pipe_runs(uint32_t acc, uint32_t M, uint32_t bs) {
    return or_andn(acc, M - bs, M);
}

// Read positions 32k..32k+31 that fall outside [0, m): a vacant map cell.
__device__ __forceinline__ uint32_t vacant_word(int k, int m) {
    if (k < 0) return ~0u;
    const int lo = 32 * k;
    if (lo >= m) return ~0u;
    const int r = m - lo;
    return r >= 32 ? 0u : (~0u << r);
}

__device__ __forceinline__ bool wave_any(bool v) { return __ballot(v) != 0ull; }

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// Window k's words of one lane: read words k-1, k, k+1 and reference word k.
struct WindowWords {
    uint32_t plo, phi, clo, chi, nlo, nhi, flo, fhi;
    uint32_t vp, vc, vn;  // vacant read positions of words k-1, k, k+1
};

__device__ __forceinline__ WindowWords window_words(const uint64_t* rdL, const uint64_t* rfL,
                                                    int lane, int k, uint32_t wmax, int m) {
    WindowWords q;
    const uint64_t p = k > 0 ? rdL[(k - 1) * kLdsRow + lane] : 0ull;
    const uint64_t c = (uint32_t)k < wmax ? rdL[k * kLdsRow + lane] : 0ull;
    const uint64_t n = (uint32_t)(k + 1) < wmax ? rdL[(k + 1) * kLdsRow + lane] : 0ull;
    const uint64_t f = (uint32_t)k < wmax ? rfL[k * kLdsRow + lane] : 0ull;
    q.plo = (uint32_t)p; q.phi = (uint32_t)(p >> 32);
    q.clo = (uint32_t)c; q.chi = (uint32_t)(c >> 32);
    q.nlo = (uint32_t)n; q.nhi = (uint32_t)(n >> 32);
    q.flo = (uint32_t)f; q.fhi = (uint32_t)(f >> 32);
    q.vp = vacant_word(k - 1, m);
    q.vc = vacant_word(k, m);
    q.vn = vacant_word(k + 1, m);
    return q;
}

// Raw mismatch bits of diagonal d over the window (read bases shifted by d
// against the reference window), and the vacant bits of the same cells.
template <int d>
__device__ __forceinline__ uint32_t diag_raw(const WindowWords& q) {
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
    return (lo ^ q.flo) | (hi ^ q.fhi);
}

template <int d>
__device__ __forceinline__ uint32_t diag_vacant(const WindowWords& q) {
    if constexpr (d > 0) return funnel(q.vn, q.vc, d);
    else if constexpr (d == 0) return q.vc;
    else return funnel(q.vc, q.vp, 32 + d);
}


// Blocked map words of all 2 EMAX + 1 diagonals (vacant cells are 1).
template <int EMAX, int I = 0>
__device__ __forceinline__ void build_diag_blocked(const WindowWords& q, uint32_t* M) {
    if constexpr (I < 2 * EMAX + 1) {
        M[I] = diag_raw<I - EMAX>(q) | diag_vacant<I - EMAX>(q);
        build_diag_blocked<EMAX, I + 1>(q, M);
    }
}

// Window k's words taken straight from a pair's packed words in memory.
__device__ __forceinline__ WindowWords window_words_direct(const uint64_t* rd, const uint64_t* rf, int k,
                                                           int W, int m) {
    WindowWords q;
    const uint64_t p = (k > 0 && k - 1 < W) ? rd[k - 1] : 0ull;
    const uint64_t c = k < W ? rd[k] : 0ull;
    const uint64_t n = k + 1 < W ? rd[k + 1] : 0ull;
    const uint64_t f = k < W ? rf[k] : 0ull;
    q.plo = (uint32_t)p; q.phi = (uint32_t)(p >> 32);
    q.clo = (uint32_t)c; q.chi = (uint32_t)(c >> 32);
    q.nlo = (uint32_t)n; q.nhi = (uint32_t)(n >> 32);
    q.flo = (uint32_t)f; q.fhi = (uint32_t)(f >> 32);
    q.vp = vacant_word(k - 1, m);
    q.vc = vacant_word(k, m);
    q.vn = vacant_word(k + 1, m);
    return q;
}

}  // namespace paf
