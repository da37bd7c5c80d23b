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
// One lane per pair, two kernels.  The first reads each pair's words (staged
// through LDS up to max_E 7, straight from memory above) and only asks
// whether some diagonal has a run of at least
// ceil((m - E) / (E + 1)) = floor(m / (E + 1)) free cells: without one
// the pair is rejected (Sec. 7.2's first test: E + 1 runs that short cannot
// cover m - E columns), and with E = 0 the answer decides the pair; the
// others are flagged.  A stable counting sort of the flags (the bucketing
// kernels) lists the flagged pairs first.  Each wave of the second kernel
// takes an equal share of that list; each lane holds one pair's words and
// excluded columns in registers and takes the next pair of the share when
// its own is done.  Per diagonal it keeps one ordering key in LDS: the best
// run found by the last scan, or before any scan the pair's length as an
// upper bound.  A step takes the largest key, extracts it when it is exact,
// and scans its diagonal (again).  A pair is also rejected as soon as the
// runs still to come, none longer than the last one, cannot reach m - E
// columns.
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
// inside the word.  How the runs inside a word are tested depends on `need`
// (MODE):
//   0: need > 32, no run inside one word is long enough (the carry finds the
//      runs that cross words);
//   1: 17 <= need <= 32, a run of 17 or more cells inside a 32-bit word
//      covers bits 15 and 16, so the run through the word's middle (free
//      cells up from bit 16 plus down from bit 15) is the only candidate;
//   2: need <= 16, x AND-ed with itself shifted by sh[0..3], which add up to
//      need - 1, leaves the starts of runs of need cells;
//   3: any need (a wave whose lanes differ), the same with sh[0..5].
template <int EMAX, int MODE, int I = 0>
__device__ __forceinline__ void magnet_has_run(const WindowWords& q, uint32_t blocked, int E, uint32_t need,
                                               const uint32_t* sh, uint32_t* carry, uint32_t& found) {
    if constexpr (I < 2 * EMAX + 1) {
        constexpr int d = I - EMAX;
        const bool on = (d < 0 ? -d : d) <= E;
        const uint32_t x = on ? ~(diag_raw<d>(q) | diag_vacant<d>(q) | blocked) : 0u;
        const uint32_t t = x == ~0u ? 32u : (uint32_t)__builtin_ctz(~x);
        uint32_t in_word;
        if constexpr (MODE == 0) {
            in_word = 0u;
        } else if constexpr (MODE == 1) {
            // Both operands have 16 set bits on the far side, so the counts
            // stop at 16.
            const uint32_t up = (uint32_t)__builtin_ctz(~(x >> 16));
            const uint32_t down = (uint32_t)__builtin_clz(~(x << 16));
            in_word = (uint32_t)(up + down >= need);
        } else {
            uint32_t r = x;
#pragma unroll
            for (int j = 0; j < (MODE == 2 ? 4 : 6); ++j) r &= r >> sh[j];
            in_word = (uint32_t)(r != 0u);
        }
        // (bitwise, so that no branch is taken per diagonal)
        found |= (uint32_t)(carry[I] + t >= need) | in_word;
        carry[I] = x == ~0u ? carry[I] + 32u : (x == 0u ? 0u : (uint32_t)__builtin_clz(~x));
        magnet_has_run<EMAX, MODE, I + 1>(q, blocked, E, need, sh, carry, found);
    }
}

// rd, rf: the pair's words in memory, or (STAGED) the wave's LDS rows of the
// tile, read at column `lane`.
template <int EMAX, int MODE, bool STAGED>
__device__ __forceinline__ bool magnet_first_test_mode(const uint64_t* rd, const uint64_t* rf, int lane,
                                                       uint32_t wmax, int W, int m, int E, uint32_t need) {
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
    uint32_t found = need == 0u ? 1u : 0u;
    for (int k = 0; k < W; ++k) {
        const WindowWords q = STAGED ? window_words(rd, rf, lane, k, wmax, m) : window_words_direct(rd, rf, k, W, m);
        magnet_has_run<EMAX, MODE>(q, q.vc, E, need, sh, carry, found);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) found |= (uint32_t)(carry[i] >= need);
    return found != 0u;
}

// The in-word test is chosen once per wave: the one of the lanes' common
// mode, else the general one.
template <int EMAX, bool STAGED>
__device__ __forceinline__ bool magnet_first_test(const uint64_t* rd, const uint64_t* rf, int lane, uint32_t wmax,
                                                  int W, int m, int E, uint32_t need) {
    const uint32_t mode = need > 32u ? 0u : (need >= 17u ? 1u : 2u);
    const uint64_t all = __ballot(true);
    if (__ballot(mode == 0u) == all)
        return magnet_first_test_mode<EMAX, 0, STAGED>(rd, rf, lane, wmax, W, m, E, need);
    if (__ballot(mode == 1u) == all)
        return magnet_first_test_mode<EMAX, 1, STAGED>(rd, rf, lane, wmax, W, m, E, need);
    if (__ballot(mode == 2u) == all)
        return magnet_first_test_mode<EMAX, 2, STAGED>(rd, rf, lane, wmax, W, m, E, need);
    return magnet_first_test_mode<EMAX, 3, STAGED>(rd, rf, lane, wmax, W, m, E, need);
}

// The lane's pair held in registers: WM words of each sequence (zero past its
// W words), the vacant columns (m and above) of each word, and the mask of
// columns that left the search space (vacant ones included).
template <int WM>
struct PairRegs {
    uint64_t rd[WM], rf[WM];
    uint32_t vac[WM], gone[WM];
    uint32_t m, W;
};

// Bits of word k for the columns at or above t (a clamp and one shift of
// a 64-bit constant, whose low half is zero once t passes the word).
__device__ __forceinline__ uint32_t cols_from(int k, uint32_t t) {
    const int x = min(max((int)t - 32 * k, 0), 32);
    return (uint32_t)(0xFFFFFFFFull << x);
}

// Bits of columns [a, b) that fall in word k.
__device__ __forceinline__ uint32_t cols_mask(int k, uint32_t a, uint32_t b) {
    return cols_from(k, a) & ~cols_from(k, b);
}

// Columns [a, b) leave the search space.
template <int WM>
__device__ __forceinline__ void exclude_cols(PairRegs<WM>& r, uint32_t a, uint32_t b) {
#pragma unroll
    for (int k = 0; k < WM; ++k) r.gone[k] |= cols_mask(k, a, b);
}

// Whether some column of [a, b) has left the search space.
template <int WM>
__device__ __forceinline__ bool meets_gone(const PairRegs<WM>& r, uint32_t a, uint32_t b) {
    uint32_t hit = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k) hit |= r.gone[k] & cols_mask(k, a, b);
    return hit != 0u;
}

// Free cells of word k of diagonal d (chosen per lane, |d| <= 31): the read
// words around k funnel-shifted by d & 31 (those of k and k + 1 for d >= 0,
// of k - 1 and k otherwise), compared with the reference word; cells whose
// read base lies outside the read, vacant columns and excluded columns are
// blocked.
template <int WM>
__device__ __forceinline__ uint32_t free_word(const PairRegs<WM>& r, int k, bool pos, uint32_t sh) {
    const uint64_t p = k > 0 ? r.rd[k - 1] : 0ull;
    const uint64_t c = r.rd[k];
    const uint64_t n = k + 1 < WM ? r.rd[k + 1] : 0ull;
    const uint64_t H = pos ? n : c, L = pos ? c : p;
    const uint32_t vp = k > 0 ? r.vac[k - 1] : ~0u, vc = r.vac[k], vn = k + 1 < WM ? r.vac[k + 1] : ~0u;
    const uint32_t lo = funnel((uint32_t)H, (uint32_t)L, sh);
    const uint32_t hi = funnel((uint32_t)(H >> 32), (uint32_t)(L >> 32), sh);
    const uint32_t v = funnel(pos ? vn : vc, pos ? vc : vp, sh);
    return ~((lo ^ (uint32_t)r.rf[k]) | (hi ^ (uint32_t)(r.rf[k] >> 32)) | v | r.gone[k]);
}

// Ordering key of a run of diagonal i: longer first, then the smaller start,
// then the smaller diagonal index (the order of extraction), so the best run
// over all diagonals is the largest key.  Bit 0 is set when a scan found the
// run; a key without it (length m, start 0) is an upper bound.  m <= 512
// fits the 10-bit fields.
__device__ __forceinline__ uint32_t run_key(uint32_t L, uint32_t s) { return (L << 17) | ((1023u - s) << 7); }
__device__ __forceinline__ uint32_t diag_tag(uint32_t i, uint32_t scanned) { return ((63u - i) << 1) | scanned; }
__device__ __forceinline__ uint32_t key_len(uint32_t key) { return key >> 17; }
__device__ __forceinline__ uint32_t key_start(uint32_t key) { return 1023u - ((key >> 7) & 1023u); }
__device__ __forceinline__ uint32_t key_diag(uint32_t key) { return 63u - ((key >> 1) & 63u); }

// The best run of diagonal i (d = i - emax), word by word: the run entering
// a word from below ends at its first blocked column; runs inside the word
// are searched only when its free-cell count could beat the best so far; the
// free cells at the top carry on.  (A run still open at a word's top is also
// offered there: it is part of a real run with the same start, which is
// offered in full later.)
template <int WM>
__device__ uint32_t scan_key(const PairRegs<WM>& r, uint32_t i, int emax) {
    const int d = (int)i - emax;
    const bool pos = d >= 0;
    const uint32_t sh = (uint32_t)d & 31u;
    uint32_t carry = 0, best = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k) {
        if ((uint32_t)k < r.W) {
            const uint32_t x = free_word<WM>(r, k, pos, sh);
            const uint32_t t = x == ~0u ? 32u : (uint32_t)__builtin_ctz(~x);
            best = max(best, run_key(carry + t, 32u * k - carry));
            if (x != ~0u && run_key(popc(x), 32u * k) > best) {
                uint32_t L, s;
                word_longest(x, L, s);
                best = max(best, run_key(L, 32u * k + s));
            }
            carry = x == ~0u ? carry + 32u : (uint32_t)__builtin_clz(~x);
        }
    }
    best = max(best, run_key(carry, 32u * r.W - carry));
    return best | diag_tag(i, 1u);
}

// Threshold test of every pair; flag[p] = 0 for the pairs left undecided,
// 1 for the others (the order the counting sort puts them in).  Up to
// max_E 7 the test is light and the kernel would wait on memory, so each
// wave first stages its tile's words in LDS with loads that cover whole
// rows (the per-tile engine's staging); above, each lane reads its pair's
// words itself.
constexpr int kTestStagedMaxE = 7;

template <int EMAX, bool GENERAL>
__global__ void __launch_bounds__(256) magnet_test_kernel(FilterParams P, uint8_t* flag) {
    constexpr bool STAGED = EMAX <= kTestStagedMaxE;
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint64_t tile = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= P.n_tiles) return;
    uint64_t off = 0;
    PairSlot s = load_slot<GENERAL>(P, tile, lane, off);
    const uint64_t* rd = P.reads + off;
    const uint64_t* rf = P.refs + off;
    if constexpr (STAGED) {
        uint64_t* rdL = lds + (size_t)wave * 2 * P.wmax * kLdsRow;
        uint64_t* rfL = rdL + (size_t)P.wmax * kLdsRow;
        stage_tile<GENERAL>(P, tile, lane, s, off, rdL, rfL);
        rd = rdL;
        rf = rfL;
    }
    if (!s.in_batch) return;
    if (!s.valid) {
        P.cnt[0][s.id] = 0;
        flag[s.id] = 1;
        return;
    }
    const uint32_t need = s.m / (s.E + 1u);
    const bool found = magnet_first_test<EMAX, STAGED>(rd, rf, lane, P.wmax, (int)s.W, (int)s.m, (int)s.E, need);
    if (!found) P.cnt[0][s.id] = (uint16_t)(s.E + 1u);
    else if (s.E == 0) P.cnt[0][s.id] = 0;
    flag[s.id] = found && s.E > 0 ? 0 : 1;
}

// Refill a wave's idle lanes once this many are idle (or the wave's share
// has fewer pairs left).
constexpr uint32_t kRefillLanes = 8;

template <int EMAX, int WM>
__global__ void __launch_bounds__(256) magnet_kernel(FilterParams P, const uint32_t* order, const uint32_t* count) {
    constexpr int D = 2 * EMAX + 1;
    extern __shared__ uint32_t lds32[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t* key = lds32 + (size_t)wave * D * 64;
    const uint64_t n_sel = *count;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    // This wave's share of the flagged list.
    uint64_t next = n_sel * w / waves;
    const uint64_t end = n_sel * (w + 1) / waves;

    // Each lane runs its own pair and takes a new one when it is done, so a
    // wave waits for no pair.  A step selects the largest key of the lane's
    // diagonals.  A key from a scan whose run still avoids the excluded
    // columns is exact and is extracted; either way the diagonal is then
    // scanned (again).  Excluding columns only shortens runs, so a stale key
    // is never below the exact one and the largest exact key is the true
    // best.
    PairRegs<WM> r;
    r.m = 0;
    r.W = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k) {
        r.rd[k] = r.rf[k] = 0ull;
        r.vac[k] = r.gone[k] = ~0u;
    }
    uint64_t id = 0;
    uint32_t E = 0, covered = 0, it = 0;
    bool busy = false;
    for (;;) {
        const uint64_t idle = __ballot(!busy);
        const uint32_t n_idle = (uint32_t)__builtin_popcountll(idle);
        const uint64_t left = end - next;
        if (left == 0 && n_idle == 64u) break;
        if (left != 0 && n_idle >= min<uint64_t>(kRefillLanes, left)) {
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
            if (!busy && rank < left) {
                id = order[next + rank];
                r.m = P.len ? P.len[id] : P.uniform_len;
                E = P.E ? P.E[id] : P.uniform_E;
                r.W = (r.m + 31) >> 5;
                const uint64_t off = P.word_offset ? P.word_offset[id] : id * (uint64_t)P.stride_words;
#pragma unroll
                for (int k = 0; k < WM; ++k) {
                    r.rd[k] = (uint32_t)k < r.W ? P.reads[off + k] : 0ull;
                    r.rf[k] = (uint32_t)k < r.W ? P.refs[off + k] : 0ull;
                    r.vac[k] = r.gone[k] = vacant_word(k, (int)r.m);
                }
                covered = 0;
                it = 0;
                // Before any scan, m bounds every diagonal's best run (ties
                // between bounds go to the first diagonal, so the first
                // steps scan the diagonals in order).
                for (int i = 0; i < D; ++i) {
                    const int d = i - EMAX;
                    key[i * 64 + lane] = (d < 0 ? -d : d) <= (int)E ? run_key(r.m, 0u) | diag_tag((uint32_t)i, 0u) : 0u;
                }
                busy = true;
            }
            next += min<uint64_t>(n_idle, left);
        }
        if (busy) {
            uint32_t best = 0;
            for (int i = 0; i < D; ++i) best = max(best, key[i * 64 + lane]);
            const uint32_t L = key_len(best);
            bool done = L == 0u, rejected = false;
            if (!done) {
                const uint32_t s = key_start(best), i = key_diag(best);
                if ((best & 1u) != 0u && !meets_gone<WM>(r, s, s + L)) {
                    // Extraction: the run and one column on each side leave
                    // the search space.
                    ++it;
                    covered += L;
                    exclude_cols<WM>(r, s > 0 ? s - 1u : 0u, min(s + L + 1u, r.m));
                    // The E + 1 - it runs still to come are no longer than this one.
                    rejected = covered + (E + 1u - it) * L + E < r.m;
                    done = rejected || it > E || covered >= r.m;
                }
                // The winner is scanned (again): a bound, a run an exclusion
                // cut, or the run just extracted, whose key stays the largest
                // and would be the next step's stale winner.
                if (!done) key[i * 64 + lane] = scan_key<WM>(r, i, EMAX);
            }
            if (done) {
                P.cnt[0][id] = (uint16_t)(rejected ? E + 1u : min(r.m - covered, E + 1u));
                busy = false;
            }
        }
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

template <int WM>
const void* magnet_kernel_for(int emax) {
    switch (emax) {
#define PAF_CASE(X) \
    case X: return reinterpret_cast<const void*>(&magnet_kernel<X, WM>);
        PAF_CASE(0) PAF_CASE(1) PAF_CASE(2) PAF_CASE(3) PAF_CASE(4) PAF_CASE(5) PAF_CASE(6)
        PAF_CASE(7) PAF_CASE(8) PAF_CASE(10) PAF_CASE(12) PAF_CASE(15) PAF_CASE(20) PAF_CASE(25)
        PAF_CASE(31)
#undef PAF_CASE
        default: return nullptr;
    }
}

}  // namespace

// Workspace of paf_filter_magnet_noalloc: a static device array, one copy on
// every device the library runs on, held until the process ends.  Laid out
// as the bucketing workspace of paf_filter_magnet for up to
// PAF_MAGNET_NOALLOC_MAX_PAIRS pairs: the list order (4 bytes per pair), the
// flags of the first test (1 byte per pair), the counting sort's per-block
// counts and its 16 totals, each part starting on a 256-byte boundary.  Every
// byte a call reads was written earlier in the same call, so nothing needs
// clearing between calls.
namespace {
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNoallocOrder = 0;
constexpr size_t kNoallocFlag = align256(kNoallocOrder + (size_t)PAF_MAGNET_NOALLOC_MAX_PAIRS * 4);
constexpr size_t kNoallocCounts = align256(kNoallocFlag + (size_t)PAF_MAGNET_NOALLOC_MAX_PAIRS);
constexpr size_t kNoallocHist =
    align256(kNoallocCounts + 16 * (((size_t)PAF_MAGNET_NOALLOC_MAX_PAIRS + 4095) / 4096) * 4);
constexpr size_t kNoallocBytes = align256(kNoallocHist + 16 * 4);
}  // namespace

static __device__ __align__(256) uint8_t scratch[kNoallocBytes];

size_t magnet_noalloc_bytes() { return kNoallocBytes; }

// The device address of `scratch` on the current device (the host-side name
// of the array is only a stand-in: kernels and copies take this address).
hipError_t magnet_noalloc_address(uint8_t** ptr) {
    *ptr = nullptr;
    return hipGetSymbolAddress(reinterpret_cast<void**>(ptr), HIP_SYMBOL(scratch));
}

hipError_t launch_magnet_noalloc(const FilterParams& p, int emax, uint8_t* base, int num_cus, hipStream_t s) {
    if (p.n_pairs > (uint64_t)PAF_MAGNET_NOALLOC_MAX_PAIRS || bucket_count_words(p.n_pairs) * 4 > kNoallocHist - kNoallocCounts)
        return hipErrorInvalidValue;
    return launch_magnet(p, emax, base + kNoallocFlag, reinterpret_cast<uint32_t*>(base + kNoallocCounts),
                         reinterpret_cast<uint32_t*>(base + kNoallocOrder), reinterpret_cast<uint32_t*>(base + kNoallocHist),
                         num_cus, s);
}

hipError_t launch_magnet(const FilterParams& p, int emax, uint8_t* flag, uint32_t* counts, uint32_t* order,
                         uint32_t* hist, int num_cus, hipStream_t s) {
    const bool general = p.len || p.E || p.word_offset;
    const void* kt = general ? magnet_test_kernel_for<true>(emax) : magnet_test_kernel_for<false>(emax);
    // Pairs of up to 256 bases keep 8 words per sequence in registers, longer
    // ones 16.
    const void* k = p.wmax <= 8 ? magnet_kernel_for<8>(emax) : magnet_kernel_for<16>(emax);
    if (!kt || !k) return hipErrorInvalidValue;
    FilterParams arg = p;
    const uint32_t waves = 4;
    {
        const size_t lds_t = emax <= kTestStagedMaxE ? filter_lds_bytes(waves, p.wmax) : 0;
        if (lds_t > 65536) {
            hipError_t e = hipFuncSetAttribute(kt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_t);
            if (e != hipSuccess) return e;
        }
        const uint32_t blocks = (uint32_t)((p.n_tiles + waves - 1) / waves);
        void* args[] = {&arg, &flag};
        hipError_t e = hipLaunchKernel(kt, dim3(blocks), dim3(64 * waves), args, lds_t, s);
        if (e != hipSuccess) return e;
    }
    // With max_E 0 the first test decides every pair (only a pair equal to
    // its reference is accepted): no list to build and nothing to extract.
    if (emax == 0)
        return launch_accept_from_counts(p.cnt[0], p.len, p.uniform_len, p.E, p.uniform_E, p.max_len, p.max_E,
                                         p.n_pairs, p.acc[0], s);
    // Undecided pairs first (flag 0), in pair order.
    hipError_t e = launch_bucket_sort(flag, p.n_pairs, counts, order, hist, s);
    if (e != hipSuccess) return e;
    // A grid that fills the chip; each wave takes an equal share of the list.
    const size_t lds = (size_t)waves * (2 * emax + 1) * 64 * sizeof(uint32_t);
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
