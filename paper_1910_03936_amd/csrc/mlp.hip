// Learned cost bucketing for gfx950: pair features, the 64 -> 128 -> 128 -> 1
// cost model on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, fp32
// accumulation) for inference and training, Adam, and the 16-bucket stable
// scatter that reorders pairs before the filter.  The model only changes the
// order in which pairs are filtered; every decision is the filter's.
//
// Matrix-core operand layout of v_mfma_f32_16x16x32_bf16 (checked on the
// device): lane l holds A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16]
// for j = 0..7, and receives C[4 (l / 16) + i][l % 16] for i = 0..3.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "paf_internal.h"
#include "paf_map.h"

namespace paf {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kHid = 128, kFeat = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 8192, OFF_W2 = 8320, OFF_B2 = 24704, OFF_W3 = 24832, OFF_B3 = 24960;
constexpr int kBucketChunk = 4096;  // pairs per block of the bucket scatter

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) short s16x2;

// relu as an integer max on the bit pattern: negative values (sign bit set)
// become +0, the rest pass unchanged.
__device__ __forceinline__ float relu_bits(float x) {
    const int b = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, b > 0 ? b : 0);
}

// relu of two fp32 values rounded to bf16, as the packed bf16 bit patterns.
__device__ __forceinline__ s16x2 relu_pk(float a, float b) {
    const bf16x2 h = __builtin_convertvector(f32x2{a, b}, bf16x2);
    const s16x2 v = __builtin_bit_cast(s16x2, h);
    return __builtin_elementwise_max(v, s16x2{0, 0});
}

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Layer-1 weight fragment (m-tile mt, k-tile kt) of one lane from LDS.
__device__ __forceinline__ bf16x8 a1_at(const uint16_t* sW1, int mt, int kt, int lane) {
    return *reinterpret_cast<const bf16x8*>(&sW1[((mt * 2 + kt) * 64 + lane) * 8]);
}

// Hidden index carried by element j of lane group g in layer-2 k-tile kt.
// Layer 1 leaves hidden units 16 mt + 4 g + i (i = 0..3) of m-tile mt in lane
// group g; pairing m-tiles 2 kt and 2 kt + 1 gives each lane the 8 k-values of
// a layer-2 fragment without moving data.  A and B use the same order, so the
// dot products are unchanged.
__host__ __device__ __forceinline__ int l2_hidden(int kt, int g, int j) {
    return 32 * kt + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

// ---------------------------------------------------------------------------
// Working copies of the weights: bf16 row-major W1 [h][f], W2 [o][h] and its
// transpose, W3 rounded to bf16 values, and matrix-core fragment orders.
__global__ void round_kernel(const float* master, uint16_t* w1b, uint16_t* w2b, uint16_t* w2tb,
                             float* w3r, uint16_t* w1f, uint16_t* w2f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kHid * kFeat) {
        w1b[i] = bf16_bits(master[OFF_W1 + i]);
        const int j = i % 8, lane = (i / 8) % 64, kt = (i / 512) % 2, mt = i / 1024;
        const int h = 16 * mt + lane % 16, f = 32 * kt + 8 * (lane / 16) + j;
        w1f[i] = bf16_bits(master[OFF_W1 + h * kFeat + f]);
    }
    if (i < kHid * kHid) {
        const uint16_t v = bf16_bits(master[OFF_W2 + i]);
        w2b[i] = v;
        w2tb[(i % kHid) * kHid + i / kHid] = v;
        const int j = i % 8, lane = (i / 8) % 64, kt = (i / 512) % 4, mt = i / 2048;
        const int o = 16 * mt + lane % 16, h = l2_hidden(kt, lane / 16, j);
        w2f[i] = bf16_bits(master[OFF_W2 + o * kHid + h]);
    }
    if (i < kHid) w3r[i] = bf16_round(master[OFF_W3 + i]);
}

// ---------------------------------------------------------------------------
// Features of one pair: [0] = m / 512, [1] = E / 32, slot 32 + d = fraction of
// matching map cells (vacant cells blocked) over the first min(m, 64)
// columns of diagonal d, |d| <= min(E, 30).
// Left-edge vacancy of window 0 for diagonal d < 0: read positions below 0.
template <int d>
__device__ __forceinline__ constexpr uint32_t left_vacant() {
    if constexpr (d >= 0) return 0u;
    else return (1u << (-d)) - 1u;
}

template <int EF, int K, int I = 0>
__device__ __forceinline__ void count_long(const WindowWords& q, uint32_t* z) {
    if constexpr (I < 2 * EF + 1) {
        constexpr int d = I - EF;
        // m >= 64 + EF: no read position of the first two windows lies past the
        // read, so the only vacant cells are the constant left edge of window 0.
        // z counts blocked cells here.
        const uint32_t mw = diag_raw<d>(q) | (K == 0 ? left_vacant<d>() : 0u);
        z[I] += __builtin_popcount(mw);
        count_long<EF, K, I + 1>(q, z);
    }
}

// Fraction features of the diagonals inside the pair's own threshold; those
// beyond it are 0.  `masked` is false when every lane of the wave has E >= EF.
// Slot of diagonal index i (d = i - EF) in the feature vector: 32 + d in the
// 64-slot layout, 2 + i in the compact one (m/512, E/32, then the 2 EF + 1
// diagonals; the model's other inputs are zero and contribute nothing).
template <int EF, bool CK>
__device__ __forceinline__ constexpr int diag_slot(int i) {
    return CK ? 2 + i : 32 + i - EF;
}

template <int EF, bool CK>
__device__ __forceinline__ void store_fractions(const float* v, uint32_t E, bool masked, float* f) {
    constexpr int D = 2 * EF + 1;
    if (EF <= 15 && !masked) {
#pragma unroll
        for (int i = 0; i < D; ++i) f[diag_slot<EF, CK>(i)] = v[i];
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int d = i - EF;
            const uint32_t ad = (uint32_t)(d < 0 ? -d : d);
            f[diag_slot<EF, CK>(i)] = ad <= E ? v[i] : 0.0f;
        }
    }
}

// Which pairs go through the model when only the compacting filter's
// in-chunk order needs their level.  That order is read only for the pairs
// a chunk still holds after its first pass (the first 64 columns), and a
// pair survives that pass only if some diagonal inside its threshold is
// mostly free there.  So the model runs on the pairs with a diagonal |d| <= E
// whose matching cells make up at least 2/5 of the first min(m, 64) columns;
// the others get the cheapest level without running it.  Integer test on the
// counts: 5 matches >= 2 columns.
__device__ __forceinline__ bool model_gate(uint32_t matches, uint32_t cols) {
    return 5u * matches >= 2u * cols;
}

// NF = 64: the model's own input layout; NF < 64: the compact one (only the
// non-zero inputs, in slots 0 .. 2 EF + 2).
template <int EF, int NF = 64>
__device__ __forceinline__ void pair_features(const uint64_t* rd, const uint64_t* rf, uint32_t m,
                                              uint32_t E, float* f, bool all_long, bool masked,
                                              bool* gate = nullptr) {
    constexpr int D = 2 * EF + 1;
    constexpr bool CK = NF < 64;
    uint32_t z[D];
#pragma unroll
    for (int i = 0; i < D; ++i) z[i] = 0;
    const int W = (int)((m + 31) >> 5);
    float v[D];
#pragma unroll
    for (int i = 0; i < NF; ++i) f[i] = 0.0f;
    f[0] = (float)m * (1.0f / 512.0f);
    f[1] = (float)E * (1.0f / 32.0f);
    // The fast path doubles the feature code; above 15 diagonals per side it
    // would push the fused model kernel past its register budget.
    if (EF <= 15 && all_long) {
        count_long<EF, 0>(window_words_direct(rd, rf, 0, W, (int)m), z);
        count_long<EF, 1>(window_words_direct(rd, rf, 1, W, (int)m), z);
        // 64 columns: the fraction (64 - blocked) / 64 = 1 - blocked / 64, exact.
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] = __builtin_fmaf((float)z[i], -1.0f / 64.0f, 1.0f);
        if (gate) {
            bool g = false;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int d = i - EF;
                g |= (uint32_t)(d < 0 ? -d : d) <= E && model_gate(64u - z[i], 64u);
            }
            *gate = g;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const WindowWords q = window_words_direct(rd, rf, k, W, (int)m);
            const uint32_t colvalid = ~q.vc;
            uint32_t M[D];
            build_diag_blocked<EF>(q, M);
#pragma unroll
            for (int i = 0; i < D; ++i) z[i] += __builtin_popcount(~M[i] & colvalid);
        }
        const uint32_t cols = m < 64 ? m : 64;
        const float rcp = 1.0f / (float)cols;
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] = (float)z[i] * rcp;
        if (gate) {
            bool g = false;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int d = i - EF;
                g |= (uint32_t)(d < 0 ? -d : d) <= E && model_gate(z[i], cols);
            }
            *gate = g;
        }
    }
    store_fractions<EF, CK>(v, E, masked, f);
}

// A feature vector rounded to bf16, eight inputs per 16-byte word.
template <int NF>
__device__ __forceinline__ void pack_row(const float* v, uint4 (&row)[NF / 8]) {
#pragma unroll
    for (int c = 0; c < NF / 8; ++c) {
        row[c].x = bf16_bits(v[8 * c + 0]) | ((uint32_t)bf16_bits(v[8 * c + 1]) << 16);
        row[c].y = bf16_bits(v[8 * c + 2]) | ((uint32_t)bf16_bits(v[8 * c + 3]) << 16);
        row[c].z = bf16_bits(v[8 * c + 4]) | ((uint32_t)bf16_bits(v[8 * c + 5]) << 16);
        row[c].w = bf16_bits(v[8 * c + 6]) | ((uint32_t)bf16_bits(v[8 * c + 7]) << 16);
    }
}

// Fast path of the compact layout (every read of the wave at least 64 + EF
// long, every lane's E >= EF): blocked-cell counts of the first two windows
// straight from the packed words, converted to the bf16 inputs and stored
// as the pair's staged row.
__device__ __forceinline__ uint32_t or_xor3_m(uint32_t a, uint32_t t, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(a, t, b, 0xDE);   // t | (a ^ b)
}

template <int EF, int K, int I = 0>
__device__ __forceinline__ void blocked_counts(uint32_t plo, uint32_t phi, uint32_t clo, uint32_t chi,
                                               uint32_t nlo, uint32_t nhi, uint32_t flo, uint32_t fhi,
                                               uint32_t* z) {
    if constexpr (I < 2 * EF + 1) {
        constexpr int d = I - EF;
        uint32_t lo, hi;
        if constexpr (d > 0) {
            lo = funnel(nlo, clo, d);
            hi = funnel(nhi, chi, d);
        } else if constexpr (d == 0) {
            lo = clo;
            hi = chi;
        } else {
            lo = funnel(clo, plo, 32 + d);
            hi = funnel(chi, phi, 32 + d);
        }
        uint32_t t = lo ^ flo;
        if constexpr (K == 0) t |= left_vacant<d>();
        z[I] += __builtin_popcount(or_xor3_m(hi, t, fhi));
        blocked_counts<EF, K, I + 1>(plo, phi, clo, chi, nlo, nhi, flo, fhi, z);
    }
}

template <int EF, int NF>
__device__ __forceinline__ void stage_compact_fast(uint64_t r0, uint64_t r1, uint64_t r2, uint64_t f0,
                                                   uint64_t f1, uint32_t m, uint32_t E, uint4 (&row)[NF / 8],
                                                   bool& gate) {
    constexpr int D = 2 * EF + 1;
    uint32_t z[D];
#pragma unroll
    for (int i = 0; i < D; ++i) z[i] = 0;
    const uint32_t r0l = (uint32_t)r0, r0h = (uint32_t)(r0 >> 32), r1l = (uint32_t)r1,
                   r1h = (uint32_t)(r1 >> 32), r2l = (uint32_t)r2, r2h = (uint32_t)(r2 >> 32);
    blocked_counts<EF, 0>(0u, 0u, r0l, r0h, r1l, r1h, (uint32_t)f0, (uint32_t)(f0 >> 32), z);
    blocked_counts<EF, 1>(r0l, r0h, r1l, r1h, r2l, r2h, (uint32_t)f1, (uint32_t)(f1 >> 32), z);
    float v[NF];
    v[0] = (float)m * (1.0f / 512.0f);
    v[1] = (float)E * (1.0f / 32.0f);
#pragma unroll
    for (int i = 0; i < D; ++i) v[2 + i] = __builtin_fmaf((float)z[i], -1.0f / 64.0f, 1.0f);
#pragma unroll
    for (int i = D + 2; i < NF; ++i) v[i] = 0.0f;
    pack_row<NF>(v, row);
    // Every lane of the wave has E >= EF here: all diagonals are inside it.
    bool g = false;
#pragma unroll
    for (int i = 0; i < D; ++i) g |= model_gate(64u - z[i], 64u);
    gate = g;
}

struct PairRef {
    const uint64_t* rd;
    const uint64_t* rf;
    uint32_t m, E;
    bool valid;
};

__device__ __forceinline__ PairRef pair_ref(const FilterParams& P, uint64_t p) {
    PairRef r;
    r.valid = p < P.n_pairs;
    r.m = P.uniform_len;
    r.E = P.uniform_E;
    r.rd = r.rf = nullptr;
    if (!r.valid) return r;
    if (P.len) r.m = P.len[p];
    if (P.E) r.E = P.E[p];
    const uint64_t off = P.word_offset ? P.word_offset[p] : p * (uint64_t)P.stride_words;
    r.rd = P.reads + off;
    r.rf = P.refs + off;
    if (r.m < 1 || r.m > P.max_len || r.E > P.max_E) {
        atomicOr(P.err, 1u);
        r.valid = false;
    }
    return r;
}

template <int EF>
__global__ void __launch_bounds__(256) features_kernel(FilterParams P, float* out) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n_pairs) return;
    const PairRef r = pair_ref(P, p);
    float f[64];
    if (r.valid) {
        pair_features<EF>(r.rd, r.rf, r.m, r.E, f, false, true);
    } else {
#pragma unroll
        for (int i = 0; i < 64; ++i) f[i] = 0.0f;
    }
    float4* o = reinterpret_cast<float4*>(out + p * 64);
#pragma unroll
    for (int i = 0; i < 16; ++i) o[i] = make_float4(f[4 * i], f[4 * i + 1], f[4 * i + 2], f[4 * i + 3]);
}

// ---------------------------------------------------------------------------
// Cost key of a pair from the model's prediction y (SneakySnake's count at the
// largest threshold, i.e. how many obstacles the whole maze holds).  The
// filter's waves walk the 32-column windows in step, so what makes a wave
// long is how many windows its lanes traverse: the snake stops after E + 1
// obstacles, covering about m (E + 1) / y columns when y > E + 1, else all m.
// The key is that window count, refined by the expected number of steps, on a
// 16-level scale.  Integer arithmetic after one exact scaling, so the host can
// reproduce it.  Pairs are stored as bucket 15 - level, so that the longest
// work is scheduled first.
__host__ __device__ __forceinline__ uint32_t cost_bucket(float y, uint32_t m, uint32_t E,
                                                         uint32_t max_len, uint32_t max_E) {
    float yc = y > 0.0f ? y : 0.0f;   // NaN -> 0
    yc = yc < 32.0f ? yc : 32.0f;
    const uint32_t yq = (uint32_t)floorf(yc * 8.0f);         // eighths, 0..256
    const uint32_t lim = 8u * (E + 1u);
    const uint32_t steps8 = (yq < lim ? yq : lim) + 8u;      // expected steps, in eighths
    const uint32_t trav = yq <= lim ? m : (m * lim) / yq;    // columns the snake is expected to cover
    const uint32_t win = trav ? (trav + 31u) / 32u : 1u;
    const uint32_t u = 8u * (win - 1u) + (8u * steps8) / (lim + 8u + 1u);   // 0 .. 8 W - 1
    const uint32_t umax = 8u * ((max_len + 31u) / 32u);
    const uint32_t b = (16u * u) / umax;
    (void)max_E;
    return b < 15u ? b : 15u;
}

// Level of a pair for the compacting filter's in-chunk order: the prediction
// on 16 levels of width 2 (0..32 obstacles), stored as 15 - level so that
// ascending order puts the costliest pairs first.  Pairs with similar counts
// take similar numbers of steps in each window, which is what makes a window
// pass of the compacting engine long.
__host__ __device__ __forceinline__ uint32_t chunk_level(float y) {
    float yc = y > 0.0f ? y : 0.0f;   // NaN -> 0
    yc = yc < 32.0f ? yc : 32.0f;
    const uint32_t l = (uint32_t)floorf(yc * 0.5f);
    return l < 15u ? l : 15u;
}

// ---------------------------------------------------------------------------
// Fused inference: features -> layer 1 -> layer 2 -> head -> bucket, one
// 64-pair tile per wave; weights stay in LDS for the whole (persistent) launch.
struct KeyParams {
    FilterParams P;
    const uint16_t* w1f;
    const uint16_t* w1b;   // row-major bf16 W1 [128][64] (compact-feature gather)
    const uint16_t* w2f;
    const float* master;
    const float* w3r;
    float* pred;       // optional
    uint8_t* bucket;   // optional
    uint32_t chunk_key;  // bucket = 15 - chunk_level (in-chunk order) instead of 15 - cost_bucket
    uint32_t gate;       // with chunk_key and no pred: only pairs that pass model_gate run the model
};

constexpr int kKeyWaves = 8;  // waves per block of the fused kernel (weights shared in LDS)

// The words the features need: read words 0..2 and reference words 0..1.
struct FeatWords {
    uint64_t r0, r1, r2, f0, f1;
    uint32_t m, E;
    bool valid;
};

__device__ __forceinline__ FeatWords feat_words(const FilterParams& P, uint64_t p) {
    FeatWords q{0, 0, 0, 0, 0, 0, 0, false};
    const PairRef r = pair_ref(P, p);
    q.valid = r.valid;
    q.m = r.m;
    q.E = r.E;
    if (r.valid) {
        const uint32_t W = (r.m + 31) >> 5;
        q.r0 = r.rd[0];
        q.f0 = r.rf[0];
        if (W > 1) { q.r1 = r.rd[1]; q.f1 = r.rf[1]; }
        if (W > 2) q.r2 = r.rd[2];
    }
    return q;
}

// The words of pair p of a batch with one length and one threshold (`ok`:
// both in range), loaded without a branch: a lane past the batch reads pair
// 0's words, and a word at or past the pair's W repeats its word 0 (the
// feature code reads only words below W).  With no branch around them, the
// loads of later tiles stay in flight while earlier tiles are worked on.
__device__ __forceinline__ FeatWords feat_words_uniform(const FilterParams& P, uint64_t p, bool ok) {
    FeatWords q;
    q.valid = ok && p < P.n_pairs;
    q.m = P.uniform_len;
    q.E = P.uniform_E;
    const uint32_t W = ok ? (q.m + 31) >> 5 : 1u;
    const uint64_t off = (q.valid ? p : 0ull) * (uint64_t)P.stride_words;
    const uint64_t* rd = P.reads + off;
    const uint64_t* rf = P.refs + off;
    const uint32_t k1 = W > 1 ? 1u : 0u, k2 = W > 2 ? 2u : 0u;
    q.r0 = rd[0];
    q.r1 = rd[k1];
    q.r2 = rd[k2];
    q.f0 = rf[0];
    q.f1 = rf[k1];
    return q;
}

template <int EF, int NF>
__device__ __forceinline__ void features_from_words(const FeatWords& w, float* f, bool all_long,
                                                    bool masked, bool* gate) {
    uint64_t rd[3] = {w.r0, w.r1, w.r2};
    uint64_t rf[2] = {w.f0, w.f1};
    pair_features<EF, NF>(rd, rf, w.m, w.E, f, all_long, masked, gate);
}

// With at most 14 diagonals per side the non-zero inputs (m/512, E/32 and
// the 2 EF + 1 fractions) fit one 32-wide k-tile: the kernel stages that
// compact vector and layer 1 takes one matrix product per tile instead of
// two (the other 32 inputs are zero and add nothing).  Up to 18 per side
// they fit 40 slots: still two k-tiles, but the staged rows (and so the
// rows a gated wave can hold) stay small.
//
// UNIFORM (gated launches on batches with no per-pair lengths, thresholds or
// offsets): each wave keeps two tiles of words in flight, in two register
// sets used in turn (a copy from one set to the other would wait for its
// loads), and computes layer 2 in two halves to make room for them.
template <int EF, bool UNIFORM>
__global__ void __launch_bounds__(64 * kKeyWaves) key_kernel(KeyParams K) {
    // Staged inputs per pair: the 2 EF + 3 non-zero ones in 32 or 40 slots
    // (compact), else the model's 64.
    constexpr int NF = 2 * EF + 3 <= 32 ? 32 : (2 * EF + 3 <= 40 ? 40 : 64);
    constexpr bool CK = NF < 64;
    constexpr int KT1 = NF > 32 ? 2 : 1;     // layer-1 k-tiles
    __shared__ __attribute__((aligned(16))) uint16_t sW1[8 * KT1 * 64 * 8];
    __shared__ __attribute__((aligned(16))) uint16_t sW2[8 * 4 * 64 * 8];
    __shared__ __attribute__((aligned(16))) float sB1[kHid];
    __shared__ __attribute__((aligned(16))) float sB2[kHid];
    __shared__ float sW3[kHid];
    // Gated launches hold up to 127 rows per wave (a partial tile of rows
    // that passed the gate plus the next tile's).
    constexpr int ROWS = CK ? 128 : 64;
    __shared__ __attribute__((aligned(16))) uint16_t sX[kKeyWaves][ROWS][NF + 8];
    __shared__ uint64_t sIdx[kKeyWaves][CK ? 128 : 1];
    const FilterParams& P = K.P;
    if (P.n_tiles == 0) return;
    if constexpr (CK) {
        // Fragment order: lane (q, g) of m-tile mt, k-tile kt holds
        // W1[16 mt + q][input of compact slot 32 kt + 8 g + j], j = 0..7.
        for (int i = threadIdx.x; i < 8 * KT1 * 64 * 8; i += blockDim.x) {
            const int j = i & 7, ln = (i >> 3) & 63, kt = (i >> 9) % KT1, mt = (i >> 9) / KT1;
            const int h = 16 * mt + (ln & 15), slot = 32 * kt + 8 * (ln >> 4) + j;
            const int in = slot < 2 ? slot : (slot - 2 <= 2 * EF ? 32 - EF + (slot - 2) : -1);
            sW1[i] = in < 0 ? (uint16_t)0 : K.w1b[h * kFeat + in];
        }
    } else {
        for (int i = threadIdx.x; i < 8 * 2 * 64; i += blockDim.x)
            reinterpret_cast<uint4*>(sW1)[i] = reinterpret_cast<const uint4*>(K.w1f)[i];
    }
    for (int i = threadIdx.x; i < 8 * 4 * 64; i += blockDim.x)
        reinterpret_cast<uint4*>(sW2)[i] = reinterpret_cast<const uint4*>(K.w2f)[i];
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        sB1[i] = K.master[OFF_B1 + i];
        sB2[i] = K.master[OFF_B2 + i];
        sW3[i] = K.w3r[i];
    }
    const float b3 = K.master[OFF_B3];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q16 = lane & 15, grp = lane >> 4;
    const uint32_t stride = gridDim.x * kKeyWaves;
    // Gated (compact layout, in-chunk levels only): the wave collects the
    // pairs that pass model_gate from its tiles into full 64-row tiles of
    // sX (with their pair indices in sIdx) and runs the model on those; the
    // others get the cheapest level at once.  Otherwise every tile goes
    // through the model, pair p in row p % 64.
    const bool gated = CK && K.gate != 0u;
    uint32_t n_buf = 0;
    uint32_t tile = blockIdx.x * kKeyWaves + wave;
    // One length and threshold for the whole batch: checked once.
    const bool uni_ok = P.uniform_len >= 1 && P.uniform_len <= P.max_len && P.uniform_E <= P.max_E;
    if (UNIFORM && !uni_ok && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(P.err, 1u);
    auto fetch = [&](uint32_t t) -> FeatWords {
        if constexpr (UNIFORM)
            return feat_words_uniform(P, (uint64_t)(t < P.n_tiles ? t : P.n_tiles - 1) * 64 + lane, uni_ok);
        else
            return feat_words(P, (uint64_t)t * 64 + lane);
    };
    // One tile: the features (and gate) of its pairs from the words in cur,
    // which are then refilled with those of the tile `ahead` strides on; then
    // the model on a full tile of staged rows, if there is one.  Returns
    // false after the wave's last tile.
    auto step = [&](FeatWords& cur, uint32_t ahead) -> bool {
        const bool have = tile < P.n_tiles;
        const uint64_t p = (uint64_t)tile * 64 + lane;
        uint32_t m = 0, E = 0;
        bool valid = false;
        if (have) {
            const bool all_long = !wave_any(cur.valid && cur.m < 64u + EF);
            const bool masked = wave_any(cur.valid && cur.E < (uint32_t)EF);
            uint4 row[NF / 8];
            bool pass = false;
            if (CK && all_long && !masked) {
                stage_compact_fast<EF, NF>(cur.r0, cur.r1, cur.r2, cur.f0, cur.f1, cur.m, cur.E, row, pass);
            } else {
                float f[NF];
                if (cur.valid) {
                    features_from_words<EF, NF>(cur, f, all_long, masked, &pass);
                } else {
#pragma unroll
                    for (int i = 0; i < NF; ++i) f[i] = 0.0f;
                }
                pack_row<NF>(f, row);
            }
            m = cur.m;
            E = cur.E;
            valid = cur.valid;
            int r = lane;
            if (gated) {
                pass = pass && valid;
                const uint64_t bal = __ballot(pass);
                r = (int)n_buf + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                if (pass) sIdx[wave][r] = p;
                else if (p < P.n_pairs && K.bucket) K.bucket[p] = 15u;   // level 0
                n_buf += (uint32_t)__builtin_popcountll(bal);
            }
            if (!gated || pass) {
#pragma unroll
                for (int c = 0; c < NF / 8; ++c) *reinterpret_cast<uint4*>(&sX[wave][r][8 * c]) = row[c];
            }
            // Next tile's words are fetched while this one goes through the model.
            if constexpr (!UNIFORM)
                if (tile + stride < P.n_tiles) cur = fetch(tile + stride);
        }
        // Uniform batches: the words of the tile `ahead` strides on, on every
        // path (a fetch past the last tile reads the last tile's words again),
        // so that every path into the next step has the same loads in flight
        // and the wait before using a set of words covers only that set.
        if constexpr (UNIFORM) cur = fetch(tile + ahead * stride);
        const uint32_t rows = gated ? (n_buf >= 64u ? 64u : (have ? 0u : n_buf)) : (have ? 64u : 0u);
        if (rows > 0) {
            wave_lds_sync();
            // Layer-1 operand B: X^T, lane (row 16 nt + q16, group grp) holds
            // features 32 kt + 8 grp .. +7 of its row.
            bf16x8 xf[KT1][4];
#pragma unroll
            for (int kt = 0; kt < KT1; ++kt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    xf[kt][nt] = 32 * kt + 8 * grp < NF
                                     ? *reinterpret_cast<const bf16x8*>(&sX[wave][16 * nt + q16][32 * kt + 8 * grp])
                                     : bf16x8{};
            auto layer1 = [&](int kt2, bf16x8* b2) {
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int mt1 = 2 * kt2 + half;
                    const f32x4 bias1 = *reinterpret_cast<const f32x4*>(&sB1[16 * mt1 + 4 * grp]);
                    f32x4 acc1[4];
                    const bf16x8 a1a = *reinterpret_cast<const bf16x8*>(&sW1[((mt1 * KT1 + 0) * 64 + lane) * 8]);
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) acc1[nt] = mfma(a1a, xf[0][nt], bias1);
                    if constexpr (KT1 == 2) {
                        const bf16x8 a1b =
                            *reinterpret_cast<const bf16x8*>(&sW1[((mt1 * KT1 + 1) * 64 + lane) * 8]);
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) acc1[nt] = mfma(a1b, xf[KT1 - 1][nt], acc1[nt]);
                    }
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; i += 2) {
                            const s16x2 v = relu_pk(acc1[nt][i], acc1[nt][i + 1]);
                            b2[nt][4 * half + i] = __builtin_bit_cast(__bf16, (short)v[0]);
                            b2[nt][4 * half + i + 1] = __builtin_bit_cast(__bf16, (short)v[1]);
                        }
                }
            };
            float yv = 0.0f;
            if constexpr (UNIFORM) {
                // Layer 2 and the head in two halves of the 128 hidden units (m-tiles
                // 0..3, then 4..7), recomputing layer 1 for the second: half the
                // accumulators, so a wave keeps registers for more words in flight.
                // Each head sum takes its terms in the same order as over all eight
                // m-tiles at once (m-tile, then element), so the result is the same.
                float th[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll 1
                for (int h2 = 0; h2 < 2; ++h2) {
                    f32x4 acc2[4][4];
                    {
                        // k-tile 0: the accumulators start from the bias (C operand).
                        bf16x8 b2[4];
                        layer1(0, b2);
    #pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int mt2 = 4 * h2 + j;
                            const f32x4 bias2 = *reinterpret_cast<const f32x4*>(&sB2[16 * mt2 + 4 * grp]);
                            const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(&sW2[((mt2 * 4 + 0) * 64 + lane) * 8]);
    #pragma unroll
                            for (int nt = 0; nt < 4; ++nt) acc2[j][nt] = mfma(a2, b2[nt], bias2);
                        }
                    }
    #pragma unroll 1
                    for (int kt2 = 1; kt2 < 4; ++kt2) {
                        bf16x8 b2[4];
                        layer1(kt2, b2);
    #pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int mt2 = 4 * h2 + j;
                            const bf16x8 a2 =
                                *reinterpret_cast<const bf16x8*>(&sW2[((mt2 * 4 + kt2) * 64 + lane) * 8]);
    #pragma unroll
                            for (int nt = 0; nt < 4; ++nt) acc2[j][nt] = mfma(a2, b2[nt], acc2[j][nt]);
                        }
                    }
                    // Head: y = w3 . relu(layer 2) + b3.
    #pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
    #pragma unroll
                        for (int j = 0; j < 4; ++j)
    #pragma unroll
                            for (int i = 0; i < 4; ++i)
                                th[nt] += sW3[16 * (4 * h2 + j) + 4 * grp + i] * relu_bits(acc2[j][nt][i]);
                }
                // Lane l ends with row l.
    #pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    float t = th[nt];
                    t += __shfl_xor(t, 16);
                    t += __shfl_xor(t, 32);
                    if (grp == nt) yv = t;
                }
            } else {
                f32x4 acc2[8][4];
                {
                    // k-tile 0: the accumulators start from the bias (C operand).
                    bf16x8 b2[4];
                    layer1(0, b2);
    #pragma unroll
                    for (int mt2 = 0; mt2 < 8; ++mt2) {
                        const f32x4 bias2 = *reinterpret_cast<const f32x4*>(&sB2[16 * mt2 + 4 * grp]);
                        const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(&sW2[((mt2 * 4 + 0) * 64 + lane) * 8]);
    #pragma unroll
                        for (int nt = 0; nt < 4; ++nt) acc2[mt2][nt] = mfma(a2, b2[nt], bias2);
                    }
                }
    #pragma unroll 1
                for (int kt2 = 1; kt2 < 4; ++kt2) {
                    bf16x8 b2[4];
                    layer1(kt2, b2);
    #pragma unroll
                    for (int mt2 = 0; mt2 < 8; ++mt2) {
                        const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(&sW2[((mt2 * 4 + kt2) * 64 + lane) * 8]);
    #pragma unroll
                        for (int nt = 0; nt < 4; ++nt) acc2[mt2][nt] = mfma(a2, b2[nt], acc2[mt2][nt]);
                    }
                }
                // Head: y = w3 . relu(layer 2) + b3; lane l ends with row l.
    #pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    float t = 0.0f;
    #pragma unroll
                    for (int mt2 = 0; mt2 < 8; ++mt2)
    #pragma unroll
                        for (int i = 0; i < 4; ++i) t += sW3[16 * mt2 + 4 * grp + i] * relu_bits(acc2[mt2][nt][i]);
                    t += __shfl_xor(t, 16);
                    t += __shfl_xor(t, 32);
                    if (grp == nt) yv = t;
                }
            }
            const float y = yv + b3;
            if (gated) {
                if ((uint32_t)lane < rows && K.bucket) K.bucket[sIdx[wave][lane]] = (uint8_t)(15u - chunk_level(y));
            } else if (p < P.n_pairs) {
                if (K.pred) K.pred[p] = valid ? y : 0.0f;
                if (K.bucket) {
                    const uint32_t lv = K.chunk_key ? chunk_level(y) : cost_bucket(y, m, E, P.max_len, P.max_E);
                    K.bucket[p] = (uint8_t)(valid ? 15u - lv : 15u);
                }
            }
            wave_lds_sync();
            if (gated) {
                // Rows past the first 64 move to the front for the next tile.
                const uint32_t rest = n_buf - rows;
                if (rows == 64u && (uint32_t)lane < rest) {
#pragma unroll
                    for (int c = 0; c < NF / 8; ++c)
                        *reinterpret_cast<uint4*>(&sX[wave][lane][8 * c]) =
                            *reinterpret_cast<const uint4*>(&sX[wave][64 + lane][8 * c]);
                    sIdx[wave][lane] = sIdx[wave][64 + lane];
                }
                n_buf = rest;
                wave_lds_sync();
            }
        }
        if (!have) return false;
        tile += stride;
        return true;
    };
    if constexpr (UNIFORM) {
        FeatWords a = fetch(tile), b = fetch(tile + stride);
        for (;;) {
            // Both steps run on every pass (a step past the wave's last tile
            // only refills), so every path round the loop has issued the
            // loads of both sets in the same order.
            const bool more_a = step(a, 2u);
            const bool more_b = step(b, 2u);
            if (!(more_a && more_b)) break;
        }
    } else {
        FeatWords a = fetch(tile);
        while (step(a, 1u)) {
        }
    }
}

// Bucket of each pair from given predictions.
__global__ void bucket_from_pred_kernel(FilterParams P, const float* pred, uint8_t* bucket) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n_pairs) return;
    const uint32_t m = P.len ? P.len[p] : P.uniform_len;
    const uint32_t E = P.E ? P.E[p] : P.uniform_E;
    const bool ok = m >= 1 && m <= P.max_len && E <= P.max_E;
    if (!ok) atomicOr(P.err, 1u);
    bucket[p] = (uint8_t)(ok ? 15u - cost_bucket(pred[p], m, E, P.max_len, P.max_E) : 15u);
}

// ---------------------------------------------------------------------------
// Stable 16-bucket scatter (one 4-bit radix pass).
// counts[b * nblk + blk] = pairs of block blk in bucket b.
__global__ void __launch_bounds__(256) bucket_count_kernel(const uint8_t* bucket, uint64_t n, uint32_t nblk,
                                                           uint32_t* counts) {
    __shared__ uint32_t c[16];
    if (threadIdx.x < 16) c[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kBucketChunk;
    for (uint32_t i = threadIdx.x; i < kBucketChunk; i += blockDim.x) {
        const uint64_t p = base + i;
        if (p < n) atomicAdd(&c[bucket[p] & 15u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 16) counts[threadIdx.x * nblk + blockIdx.x] = c[threadIdx.x];
}

// Exclusive scan of `len` words in place (one block of 1024 threads, tiles of
// 4096 words read with coalesced loads), and the 16 bucket totals (the array
// is bucket-major, nblk entries per bucket).
__global__ void __launch_bounds__(1024) scan_kernel(uint32_t* a, uint32_t len, uint32_t nblk, uint32_t* hist) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry_s;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (uint32_t base = 0; base < len; base += 4096) {
        uint32_t v[4], s = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = base + 4 * t + j;
            v[j] = i < len ? a[i] : 0u;
            s += v[j];
        }
        // inclusive scan of the thread sums inside the wave
        uint32_t inc = s;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off);
            if (lane >= (uint32_t)off) inc += o;
        }
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        uint32_t before = carry_s;
        for (uint32_t w = 0; w < wv; ++w) before += wsum[w];
        uint32_t run = before + inc - s;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t i = base + 4 * t + j;
            if (i < len) a[i] = run;
            run += v[j];
        }
        __syncthreads();
        if (t == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < 16; ++w) tot += wsum[w];
            carry_s += tot;
        }
        __syncthreads();
    }
    if (hist && t < 16) {
        const uint32_t end = t < 15 ? a[(t + 1) * nblk] : carry_s;
        hist[t] = end - a[t * nblk];
    }
}

__global__ void __launch_bounds__(256) bucket_scatter_kernel(const uint8_t* bucket, uint64_t n, uint32_t nblk,
                                                             const uint32_t* offsets, uint32_t* perm) {
    __shared__ uint32_t base[16];
    __shared__ uint32_t wcnt[4][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < 16) base[threadIdx.x] = offsets[threadIdx.x * nblk + blockIdx.x];
    __syncthreads();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint64_t start = (uint64_t)blockIdx.x * kBucketChunk;
    for (uint32_t r = 0; r < kBucketChunk; r += blockDim.x) {
        const uint64_t p = start + r + threadIdx.x;
        const bool in = p < n;
        const uint32_t b = in ? (bucket[p] & 15u) : 16u;
        uint32_t rank = 0;
        for (uint32_t k = 0; k < 16; ++k) {
            const uint64_t msk = __ballot(b == k);
            if (b == k) rank = (uint32_t)__builtin_popcountll(msk & lt);
            if (lane == 0) wcnt[wave][k] = (uint32_t)__builtin_popcountll(msk);
        }
        __syncthreads();
        if (in) {
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += wcnt[w][b];
            perm[base[b] + before + rank] = (uint32_t)p;
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            uint32_t tot = 0;
            for (int w = 0; w < 4; ++w) tot += wcnt[w][threadIdx.x];
            base[threadIdx.x] += tot;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Training.  TN GEMM on the matrix cores: C[m][n] = sum_k A[m][k] B[n][k]
// (both operands k-contiguous bf16), fp32 accumulation; M, N multiples of
// 64, K and the k-chunk multiples of 32.  Block = 4 waves, 64 x 64 tile.
enum GemmMode { G_PARTIAL = 0, G_BIAS_RELU = 1, G_MASK = 2 };
struct Gemm {
    const uint16_t* A;
    int lda;
    const uint16_t* B;
    int ldb;
    int M, N, K, kchunk;
    int mode;
    const float* bias;
    float* outf;
    int ldo;
    uint16_t* outb;
    int ldob;
    uint16_t* outbT;
    int ldobT;
    const uint16_t* mask;
    int ldmask;
};

__global__ void __launch_bounds__(256) gemm_tn_kernel(Gemm g) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q16 = lane & 15, grp = lane >> 4;
    const int m0 = blockIdx.x * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.y * 64 + (wave & 1) * 32;
    const int kb = blockIdx.z * g.kchunk;
    const int ke = min(g.K, kb + g.kchunk);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = kb; k < ke; k += 32) {
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(g.A + (size_t)(m0 + 16 * i + q16) * g.lda + k + 8 * grp);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(g.B + (size_t)(n0 + 16 * j + q16) * g.ldb + k + 8 * grp);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + 16 * i + 4 * grp + e;
                const int col = n0 + 16 * j + q16;
                float v = acc[i][j][e];
                if (g.mode == G_PARTIAL) {
                    g.outf[(size_t)blockIdx.z * g.M * g.N + (size_t)row * g.N + col] = v;
                    continue;
                }
                if (g.mode == G_BIAS_RELU) {
                    v = fmaxf(v + g.bias[col], 0.0f);
                } else {  // G_MASK: gradient through the ReLU of the stored activation
                    const uint16_t h = g.mask[(size_t)row * g.ldmask + col];
                    v = ((h & 0x7fffu) != 0u && !(h & 0x8000u)) ? v : 0.0f;
                }
                if (g.outf) g.outf[(size_t)row * g.ldo + col] = v;
                const uint16_t vb = bf16_bits(v);
                if (g.outb) g.outb[(size_t)row * g.ldob + col] = vb;
                if (g.outbT) g.outbT[(size_t)col * g.ldobT + row] = vb;
            }
}

// Features (fp32, n rows) -> bf16 [Np][64] and its transpose [64][Np]; rows
// past n are zero.
__global__ void to_bf16_kernel(const float* f, uint32_t n, uint32_t Np, uint16_t* X, uint16_t* XT) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Np * kFeat) return;
    const uint32_t p = i / kFeat, c = i % kFeat;
    const uint16_t v = p < n ? bf16_bits(f[(size_t)p * kFeat + c]) : (uint16_t)0;
    X[i] = v;
    XT[(size_t)c * Np + p] = v;
}

// Head, loss and its gradient: y = w3 . h2 + b3 per row; for rows < n,
// dy = 2 (y - t) / n and dL/dh2 = dy w3 where h2 > 0.
// Rows p < n are real; predictions are written for them only.  Without
// targets (inference) the gradients are zero.
__global__ void head_kernel(const float* H2, const float* w3r, const float* master, const float* tgt,
                            uint32_t n, uint32_t Np, float* pred, float* sq, float* dy, uint16_t* dH2b,
                            uint16_t* dH2T, float* dH2f) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Np) return;
    const float* h = H2 + (size_t)p * kHid;
    float y = 0.0f;
    for (int o = 0; o < kHid; ++o) y += w3r[o] * h[o];
    y += master[OFF_B3];
    float d = 0.0f;
    if (p < n && tgt) {
        const float e = y - tgt[p];
        sq[p] = e * e;
        d = 2.0f * e / (float)n;
    } else {
        sq[p] = 0.0f;
    }
    if (p < n) pred[p] = y;
    dy[p] = d;
    for (int o = 0; o < kHid; ++o) {
        const float g = h[o] > 0.0f ? d * w3r[o] : 0.0f;
        dH2f[(size_t)p * kHid + o] = g;
        const uint16_t gb = bf16_bits(g);
        dH2b[(size_t)p * kHid + o] = gb;
        dH2T[(size_t)o * Np + p] = gb;
    }
}

// out[j] = scale * sum_p w[p] X[p][j] (w = 1 when NULL); fixed reduction order.
__global__ void __launch_bounds__(256) reduce_rows_kernel(const float* X, uint32_t rows, uint32_t cols,
                                                          const float* w, float scale, float* out) {
    __shared__ float red[256];
    const uint32_t j = blockIdx.x;
    float s = 0.0f;
    for (uint32_t p = threadIdx.x; p < rows; p += blockDim.x) s += (w ? w[p] : 1.0f) * X[(size_t)p * cols + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0] * scale;
}

__global__ void splitk_reduce_kernel(const float* part, uint32_t S, uint32_t MN, float* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MN) return;
    float s = 0.0f;
    for (uint32_t k = 0; k < S; ++k) s += part[(size_t)k * MN + i];
    out[i] = s;
}

// Adam (Kingma and Ba, 2015) on the fp32 master weights.
__global__ void adam_kernel(float* w, const float* g, float* m, float* v, uint32_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void u16_to_f32_kernel(const uint16_t* a, uint64_t n, float* out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)a[i];
}

template <int EF>
const void* features_ptr() { return reinterpret_cast<const void*>(&features_kernel<EF>); }
// The two-sets form up to 12 diagonals per side; above, its registers spill.
template <int EF>
const void* key_ptr(bool two_sets) {
    if constexpr (EF <= 12)
        if (two_sets) return reinterpret_cast<const void*>(&key_kernel<EF, true>);
    return reinterpret_cast<const void*>(&key_kernel<EF, false>);
}

// Diagonals the features use: min(E bucket, 30).
int feature_ef(int emax) { return emax > 30 ? 30 : emax; }

const void* feature_kernel_for(int ef, bool fused, bool two_sets = false) {
    switch (ef) {
#define PAF_FCASE(X) \
    case X: return fused ? key_ptr<X>(two_sets) : features_ptr<X>();
        PAF_FCASE(0) PAF_FCASE(1) PAF_FCASE(2) PAF_FCASE(3) PAF_FCASE(4) PAF_FCASE(5) PAF_FCASE(6)
        PAF_FCASE(7) PAF_FCASE(8) PAF_FCASE(10) PAF_FCASE(12) PAF_FCASE(15) PAF_FCASE(20) PAF_FCASE(25)
        PAF_FCASE(30)
#undef PAF_FCASE
        default: return nullptr;
    }
}

// ---------------------------------------------------------------------------
// Training workspace carved from one allocation.
struct TrainWs {
    uint16_t *X, *XT, *H1b, *H1T, *dH2b, *dH2T, *dH1T;
    float *H2f, *pred, *sq, *dy, *dH2f, *dH1f, *part, *tgt;
};
constexpr uint32_t kMaxSplit = 64;

size_t train_ws_bytes(size_t Np) {
    return Np * kFeat * 2 * 2 + Np * kHid * 2 * 5 + Np * kHid * 4 * 3 + Np * 4 * 4 +
           (size_t)kMaxSplit * kHid * kHid * 4 + 4096;
}

TrainWs carve(void* base, size_t Np) {
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 255) & ~size_t(255);
        return r;
    };
    TrainWs w;
    w.X = (uint16_t*)take(Np * kFeat * 2);
    w.XT = (uint16_t*)take(Np * kFeat * 2);
    w.H1b = (uint16_t*)take(Np * kHid * 2);
    w.H1T = (uint16_t*)take(Np * kHid * 2);
    w.dH2b = (uint16_t*)take(Np * kHid * 2);
    w.dH2T = (uint16_t*)take(Np * kHid * 2);
    w.dH1T = (uint16_t*)take(Np * kHid * 2);
    w.H2f = (float*)take(Np * kHid * 4);
    w.dH2f = (float*)take(Np * kHid * 4);
    w.dH1f = (float*)take(Np * kHid * 4);
    w.pred = (float*)take(Np * 4);
    w.sq = (float*)take(Np * 4);
    w.dy = (float*)take(Np * 4);
    w.tgt = (float*)take(Np * 4);
    w.part = (float*)take((size_t)kMaxSplit * kHid * kHid * 4);
    return w;
}

hipError_t gemm(const Gemm& g, hipStream_t s) {
    const int splits = g.mode == G_PARTIAL ? (g.K + g.kchunk - 1) / g.kchunk : 1;
    hipLaunchKernelGGL(gemm_tn_kernel, dim3(g.M / 64, g.N / 64, splits), dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace

hipError_t mlp_alloc(MlpDev& m) {
    const size_t P = PAF_MLP_NPARAMS;
    hipError_t e;
    if ((e = hipMalloc(&m.master, P * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.adam_m, P * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.adam_v, P * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.grad, P * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.w1b, kHid * kFeat * 2)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.w2b, kHid * kHid * 2)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.w2tb, kHid * kHid * 2)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.w3r, kHid * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.w1f, kHid * kFeat * 2)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.w2f, kHid * kHid * 2)) != hipSuccess) return e;
    return hipSuccess;
}

void mlp_free(MlpDev& m) {
    for (void* p : {(void*)m.master, (void*)m.adam_m, (void*)m.adam_v, (void*)m.grad, (void*)m.w1b, (void*)m.w2b,
                    (void*)m.w2tb, (void*)m.w3r, (void*)m.w1f, (void*)m.w2f, m.ws})
        if (p) hipFree(p);
    m = MlpDev{};
}

size_t bucket_count_words(uint64_t n) { return 16 * ((n + kBucketChunk - 1) / kBucketChunk); }

hipError_t launch_learned_buckets(const MlpDev& m, const FilterParams& p, int num_cus, float* pred,
                                  uint8_t* bucket, hipStream_t s, bool chunk_key) {
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return hipErrorInvalidValue;
    // Gated launches of uniform batches take the two-sets form (the model
    // runs on a third of the tiles there, so its halves cost little).
    const bool two_sets = !p.len && !p.E && !p.word_offset && chunk_key && !pred;
    const void* k = feature_kernel_for(feature_ef(emax), true, two_sets);
    if (!k) return hipErrorInvalidValue;
    KeyParams kp;
    kp.P = p;
    kp.w1f = m.w1f;
    kp.w1b = m.w1b;
    kp.w2f = m.w2f;
    kp.master = m.master;
    kp.w3r = m.w3r;
    kp.pred = pred;
    kp.bucket = bucket;
    kp.chunk_key = chunk_key ? 1u : 0u;
    kp.gate = chunk_key && !pred ? 1u : 0u;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * kKeyWaves, 0) != hipSuccess || nb < 1) nb = 1;
    const uint32_t want = (uint32_t)(num_cus * nb);
    const uint32_t need = (p.n_tiles + kKeyWaves - 1) / kKeyWaves;
    void* args[] = {&kp};
    return hipLaunchKernel(k, dim3(std::max(1u, std::min(want, need))), dim3(64 * kKeyWaves), args, 0, s);
}

hipError_t launch_bucket_from_pred(const FilterParams& p, const float* pred, uint8_t* bucket, hipStream_t s) {
    hipLaunchKernelGGL(bucket_from_pred_kernel, dim3((uint32_t)((p.n_pairs + 255) / 256)), dim3(256), 0, s, p,
                       pred, bucket);
    return hipGetLastError();
}

hipError_t launch_bucket_sort(const uint8_t* bucket, uint64_t n, uint32_t* counts, uint32_t* perm,
                              uint32_t* hist, hipStream_t s) {
    const uint32_t nblk = (uint32_t)((n + kBucketChunk - 1) / kBucketChunk);
    hipLaunchKernelGGL(bucket_count_kernel, dim3(nblk), dim3(256), 0, s, bucket, n, nblk, counts);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, counts, 16 * nblk, nblk, hist);
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(nblk), dim3(256), 0, s, bucket, n, nblk,
                       (const uint32_t*)counts, perm);
    return hipGetLastError();
}

hipError_t mlp_round_weights(MlpDev& m, hipStream_t s) {
    hipLaunchKernelGGL(round_kernel, dim3(kHid * kHid / 256), dim3(256), 0, s, m.master, m.w1b, m.w2b, m.w2tb,
                       m.w3r, m.w1f, m.w2f);
    return hipGetLastError();
}

}  // namespace paf

using namespace paf;

namespace {

paf_status need_model(paf_ctx* ctx) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (!ctx->mlp_ready) return fail(PAF_ERR_STATE, "no cost model: call paf_mlp_set_params first");
    return PAF_OK;
}

paf_status ensure_train_ws(paf_ctx* ctx, size_t Np) {
    MlpDev& m = ctx->mlp;
    if (m.ws_rows >= Np) return PAF_OK;
    if (m.ws) hipFree(m.ws);
    m.ws = nullptr;
    m.ws_rows = 0;
    if (hipMalloc(&m.ws, train_ws_bytes(Np)) != hipSuccess) return fail(PAF_ERR_NOMEM, "training workspace");
    m.ws_rows = Np;
    return PAF_OK;
}

// Forward, loss and gradients of one minibatch; Adam step when lr > 0.
paf_status train_step(paf_ctx* ctx, const float* feat, const float* tgt, uint32_t n, float lr, hipStream_t s,
                      float* loss_out) {
    MlpDev& m = ctx->mlp;
    const uint32_t Np = (n + 63u) & ~63u;
    paf_status st = ensure_train_ws(ctx, Np);
    if (st != PAF_OK) return st;
    TrainWs w = carve(m.ws, Np);
    hipLaunchKernelGGL(to_bf16_kernel, dim3((Np * kFeat + 255) / 256), dim3(256), 0, s, feat, n, Np, w.X, w.XT);
    Gemm g{};
    // Layer 1: H1 = relu(X W1^T + b1)
    g = Gemm{w.X, kFeat, m.w1b, kFeat, (int)Np, kHid, kFeat, kFeat, G_BIAS_RELU, m.master + OFF_B1,
             nullptr, 0, w.H1b, kHid, w.H1T, (int)Np, nullptr, 0};
    PAF_HIP(gemm(g, s), "layer 1");
    // Layer 2: H2 = relu(H1 W2^T + b2)
    g = Gemm{w.H1b, kHid, m.w2b, kHid, (int)Np, kHid, kHid, kHid, G_BIAS_RELU, m.master + OFF_B2,
             w.H2f, kHid, nullptr, 0, nullptr, 0, nullptr, 0};
    PAF_HIP(gemm(g, s), "layer 2");
    hipLaunchKernelGGL(head_kernel, dim3((Np + 255) / 256), dim3(256), 0, s, w.H2f, m.w3r, m.master, tgt, n, Np,
                       w.pred, w.sq, w.dy, w.dH2b, w.dH2T, w.dH2f);
    float* G = m.grad;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(kHid), dim3(256), 0, s, w.H2f, Np, (uint32_t)kHid, w.dy, 1.0f,
                       G + OFF_W3);
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(256), 0, s, w.dy, Np, 1u, (const float*)nullptr, 1.0f,
                       G + OFF_B3);
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(kHid), dim3(256), 0, s, w.dH2f, Np, (uint32_t)kHid,
                       (const float*)nullptr, 1.0f, G + OFF_B2);
    if (loss_out)
        hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(256), 0, s, w.sq, Np, 1u, (const float*)nullptr,
                           1.0f / (float)n, loss_out);
    // dW2 = dH2^T H1 (split over the batch)
    const int kc = (int)std::max<uint32_t>(64u, ((Np + kMaxSplit - 1) / kMaxSplit + 31u) & ~31u);
    const uint32_t S = (Np + kc - 1) / kc;
    g = Gemm{w.dH2T, (int)Np, w.H1T, (int)Np, kHid, kHid, (int)Np, kc, G_PARTIAL, nullptr,
             w.part, kHid, nullptr, 0, nullptr, 0, nullptr, 0};
    PAF_HIP(gemm(g, s), "dW2");
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(kHid * kHid / 256), dim3(256), 0, s, w.part, S,
                       (uint32_t)(kHid * kHid), G + OFF_W2);
    // dH1 = (dH2 W2) * relu'(H1)
    g = Gemm{w.dH2b, kHid, m.w2tb, kHid, (int)Np, kHid, kHid, kHid, G_MASK, nullptr,
             w.dH1f, kHid, nullptr, 0, w.dH1T, (int)Np, w.H1b, kHid};
    PAF_HIP(gemm(g, s), "dH1");
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(kHid), dim3(256), 0, s, w.dH1f, Np, (uint32_t)kHid,
                       (const float*)nullptr, 1.0f, G + OFF_B1);
    // dW1 = dH1^T X
    g = Gemm{w.dH1T, (int)Np, w.XT, (int)Np, kHid, kFeat, (int)Np, kc, G_PARTIAL, nullptr,
             w.part, kFeat, nullptr, 0, nullptr, 0, nullptr, 0};
    PAF_HIP(gemm(g, s), "dW1");
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(kHid * kFeat / 256), dim3(256), 0, s, w.part, S,
                       (uint32_t)(kHid * kFeat), G + OFF_W1);
    if (lr > 0.0f) {
        m.step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - powf(b1, (float)m.step), c2 = 1.0f - powf(b2, (float)m.step);
        hipLaunchKernelGGL(adam_kernel, dim3((PAF_MLP_NPARAMS + 255) / 256), dim3(256), 0, s, m.master, G,
                           m.adam_m, m.adam_v, (uint32_t)PAF_MLP_NPARAMS, lr, b1, b2, 1e-8f, c1, c2);
        PAF_HIP(mlp_round_weights(m, s), "weight rounding");
    }
    PAF_HIP(hipGetLastError(), "training step");
    return PAF_OK;
}

const void* checked_feature_kernel(const FilterParams& p, bool fused, int& ef) {
    const int emax = emax_bucket((int)p.max_E);
    if (emax < 0) return nullptr;
    ef = feature_ef(emax);
    return feature_kernel_for(ef, fused);
}

}  // namespace

extern "C" {

paf_status paf_features(paf_ctx* ctx, const paf_batch* batch, float* features, void* stream) {
    FilterParams p;
    paf_status st = check_batch(ctx, batch, PAF_SNEAKYSNAKE, p);
    if (st != PAF_OK) return st;
    if (!features) return fail(PAF_ERR_ARG, "features is NULL");
    int ef = 0;
    const void* k = checked_feature_kernel(p, false, ef);
    if (!k) return fail(PAF_ERR_RANGE, "max_E exceeds PAF_MAX_E");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    float* out = features;
    void* args[] = {&p, &out};
    PAF_HIP(hipLaunchKernel(k, dim3((uint32_t)((p.n_pairs + 255) / 256)), dim3(256), args, 0, (hipStream_t)stream),
            "features launch");
    return PAF_OK;
}

paf_status paf_mlp_set_params(paf_ctx* ctx, const float* params) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (!params) return fail(PAF_ERR_ARG, "params is NULL");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    MlpDev& m = ctx->mlp;
    if (!m.master) {
        if (mlp_alloc(m) != hipSuccess) {
            mlp_free(m);
            return fail(PAF_ERR_NOMEM, "model allocation");
        }
    }
    PAF_HIP(hipMemcpy(m.master, params, PAF_MLP_NPARAMS * 4, hipMemcpyHostToDevice), "hipMemcpy");
    PAF_HIP(hipMemset(m.adam_m, 0, PAF_MLP_NPARAMS * 4), "hipMemset");
    PAF_HIP(hipMemset(m.adam_v, 0, PAF_MLP_NPARAMS * 4), "hipMemset");
    PAF_HIP(hipMemset(m.grad, 0, PAF_MLP_NPARAMS * 4), "hipMemset");
    m.step = 0;
    PAF_HIP(mlp_round_weights(m, nullptr), "weight rounding");
    PAF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    ctx->mlp_ready = true;
    return PAF_OK;
}

paf_status paf_mlp_get_params(paf_ctx* ctx, float* params) {
    paf_status st = need_model(ctx);
    if (st != PAF_OK) return st;
    if (!params) return fail(PAF_ERR_ARG, "params is NULL");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PAF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    PAF_HIP(hipMemcpy(params, ctx->mlp.master, PAF_MLP_NPARAMS * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    return PAF_OK;
}

paf_status paf_mlp_get_state(paf_ctx* ctx, float* params, float* adam_m, float* adam_v, uint32_t* step) {
    paf_status st = need_model(ctx);
    if (st != PAF_OK) return st;
    if (!params || !adam_m || !adam_v || !step) return fail(PAF_ERR_ARG, "state pointer is NULL");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    PAF_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    const MlpDev& m = ctx->mlp;
    PAF_HIP(hipMemcpy(params, m.master, PAF_MLP_NPARAMS * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    PAF_HIP(hipMemcpy(adam_m, m.adam_m, PAF_MLP_NPARAMS * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    PAF_HIP(hipMemcpy(adam_v, m.adam_v, PAF_MLP_NPARAMS * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    *step = (uint32_t)m.step;
    return PAF_OK;
}

paf_status paf_mlp_set_state(paf_ctx* ctx, const float* params, const float* adam_m, const float* adam_v,
                             uint32_t step) {
    if (!ctx) return fail(PAF_ERR_ARG, "ctx is NULL");
    if (!params || !adam_m || !adam_v) return fail(PAF_ERR_ARG, "state pointer is NULL");
    if (step > (uint32_t)INT32_MAX) return fail(PAF_ERR_ARG, "step out of range");
    // Adam's second moment is a running mean of squares: a negative or
    // non-finite entry cannot come from training and would poison the update.
    for (uint32_t i = 0; i < PAF_MLP_NPARAMS; ++i)
        if (!std::isfinite(params[i]) || !std::isfinite(adam_m[i]) || !(adam_v[i] >= 0.0f) ||
            !std::isfinite(adam_v[i]))
            return fail(PAF_ERR_ARG, "model state holds a non-finite value or a negative second moment");
    paf_status st = paf_mlp_set_params(ctx, params);
    if (st != PAF_OK) return st;
    MlpDev& m = ctx->mlp;
    PAF_HIP(hipMemcpy(m.adam_m, adam_m, PAF_MLP_NPARAMS * 4, hipMemcpyHostToDevice), "hipMemcpy");
    PAF_HIP(hipMemcpy(m.adam_v, adam_v, PAF_MLP_NPARAMS * 4, hipMemcpyHostToDevice), "hipMemcpy");
    m.step = (int)step;
    return PAF_OK;
}

paf_status paf_mlp_forward(paf_ctx* ctx, const float* features, uint64_t n, float* out, void* stream) {
    paf_status st = need_model(ctx);
    if (st != PAF_OK) return st;
    if (!features || !out) return fail(PAF_ERR_ARG, "features/out is NULL");
    if (n == 0) return fail(PAF_ERR_ARG, "n is zero");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    hipStream_t s = (hipStream_t)stream;
    MlpDev& m = ctx->mlp;
    const uint64_t chunk = 65536;
    for (uint64_t a = 0; a < n; a += chunk) {
        const uint32_t k = (uint32_t)std::min<uint64_t>(chunk, n - a);
        const uint32_t Np = (k + 63u) & ~63u;
        if ((st = ensure_train_ws(ctx, Np)) != PAF_OK) return st;
        TrainWs w = carve(m.ws, Np);
        hipLaunchKernelGGL(to_bf16_kernel, dim3((Np * kFeat + 255) / 256), dim3(256), 0, s, features + a * kFeat,
                           k, Np, w.X, w.XT);
        Gemm g = Gemm{w.X, kFeat, m.w1b, kFeat, (int)Np, kHid, kFeat, kFeat, G_BIAS_RELU, m.master + OFF_B1,
                      nullptr, 0, w.H1b, kHid, nullptr, 0, nullptr, 0};
        PAF_HIP(gemm(g, s), "layer 1");
        g = Gemm{w.H1b, kHid, m.w2b, kHid, (int)Np, kHid, kHid, kHid, G_BIAS_RELU, m.master + OFF_B2,
                 w.H2f, kHid, nullptr, 0, nullptr, 0, nullptr, 0};
        PAF_HIP(gemm(g, s), "layer 2");
        hipLaunchKernelGGL(head_kernel, dim3((Np + 255) / 256), dim3(256), 0, s, w.H2f, m.w3r, m.master,
                           (const float*)nullptr, k, Np, out + a, w.sq, w.dy, w.dH2b, w.dH2T, w.dH2f);
        PAF_HIP(hipGetLastError(), "forward");
    }
    return PAF_OK;
}

paf_status paf_mlp_train_step(paf_ctx* ctx, const float* features, const float* targets, uint64_t n, float lr,
                              float* grads, float* loss, void* stream) {
    paf_status st = need_model(ctx);
    if (st != PAF_OK) return st;
    if (!features || !targets) return fail(PAF_ERR_ARG, "features/targets is NULL");
    if (n == 0 || n > 65536) return fail(PAF_ERR_RANGE, "minibatch size must be in [1, 65536]");
    if (lr < 0.0f) return fail(PAF_ERR_ARG, "lr is negative");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = train_step(ctx, features, targets, (uint32_t)n, lr, s, loss)) != PAF_OK) return st;
    if (grads)
        PAF_HIP(hipMemcpyAsync(grads, ctx->mlp.grad, PAF_MLP_NPARAMS * 4, hipMemcpyDeviceToDevice, s), "grads");
    return PAF_OK;
}

paf_status paf_mlp_train(paf_ctx* ctx, const float* features, const uint16_t* labels, uint64_t n, uint32_t epochs,
                         uint32_t batch, float lr, float* epoch_loss, void* stream) {
    paf_status st = need_model(ctx);
    if (st != PAF_OK) return st;
    if (!features || !labels) return fail(PAF_ERR_ARG, "features/labels is NULL");
    if (n == 0 || batch == 0 || batch > 65536 || epochs == 0) return fail(PAF_ERR_RANGE, "bad n/batch/epochs");
    if (!(lr > 0.0f)) return fail(PAF_ERR_ARG, "lr must be positive");
    PAF_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    ScratchScope scope(ctx, (hipStream_t)stream);
    if (scope.st != PAF_OK) return scope.st;
    hipStream_t s = (hipStream_t)stream;
    float* tg = nullptr;
    float* lbuf = nullptr;
    const uint64_t nb = (n + batch - 1) / batch;
    if (hipMalloc(&tg, n * 4) != hipSuccess) return fail(PAF_ERR_NOMEM, "targets");
    if (hipMalloc(&lbuf, nb * epochs * 4) != hipSuccess) {
        hipFree(tg);
        return fail(PAF_ERR_NOMEM, "loss buffer");
    }
    hipLaunchKernelGGL(u16_to_f32_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, labels, n, tg);
    for (uint32_t ep = 0; ep < epochs && st == PAF_OK; ++ep)
        for (uint64_t b = 0; b < nb && st == PAF_OK; ++b) {
            const uint64_t a = b * batch;
            const uint32_t k = (uint32_t)std::min<uint64_t>(batch, n - a);
            st = train_step(ctx, features + a * kFeat, tg + a, k, lr, s, lbuf + ep * nb + b);
        }
    if (st == PAF_OK && epoch_loss) {
        std::vector<float> h(nb * epochs);
        if (hipMemcpyAsync(h.data(), lbuf, h.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = fail(PAF_ERR_DEVICE, "loss copy");
        } else {
            for (uint32_t ep = 0; ep < epochs; ++ep) {
                double t = 0;
                for (uint64_t b = 0; b < nb; ++b) t += h[ep * nb + b];
                epoch_loss[ep] = (float)(t / nb);
            }
        }
    }
    hipStreamSynchronize(s);
    hipFree(tg);
    hipFree(lbuf);
    return st;
}

}  // extern "C"
