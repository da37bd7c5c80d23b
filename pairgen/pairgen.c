/*
 * pairgen: seeded, counter-based generator of synthetic (read, reference
 * segment) pairs.
 *
 * This module holds no arithmetic of the filtering method.  It only draws
 * random DNA: every pair p of a workload is a pure function of (seed, p), so
 * any subset of pairs can be regenerated on its own (the CPU checker samples
 * single pairs out of batches of tens of millions).  Bases are emitted as
 * uint8 codes 0..3 (A, C, G, T).
 *
 * Workload recipe (stand-in for the thesis's mapped read sets, which rely on
 * real genomes and reads): a read is m i.i.d. uniform bases.  With probability
 * `unrelated` the reference segment is an independent uniform segment of m
 * bases; otherwise it is the read with k edits applied one after another,
 * k ~ U{0..kmax}, each edit a substitution, insertion or deletion with
 * probability 1/3 each, at a uniform position of the current string
 * (a substitution draws one of the 3 other bases, an insertion a uniform base),
 * then trimmed to m or padded with uniform bases up to m.  m is drawn
 * uniformly from a small list of lengths; E is either fixed or
 * floor(m * e_num / e_den).
 *
 * Random numbers: SplitMix64's output function applied to a per-pair key plus
 * a Weyl counter (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

typedef struct {
    uint64_t seed;
    uint32_t n_len;        /* number of length choices (1..8) */
    uint16_t lens[8];      /* length choices, each in [1, 512] */
    uint32_t kmax;         /* edits per related pair ~ U{0..kmax} */
    double   unrelated;    /* probability that a pair is unrelated */
    int32_t  fixed_E;      /* >= 0: every pair gets this E */
    uint32_t e_num, e_den; /* fixed_E < 0: E = floor(m * e_num / e_den) */
} pg_config;

#define PG_GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t pg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t key, ctr; } pg_rng;

static inline void pg_seed(pg_rng* r, uint64_t seed, uint64_t pair) {
    r->key = pg_mix(seed * PG_GOLDEN + pg_mix(pair + 0x632be59bd9b4e019ULL));
    r->ctr = 0;
}
static inline uint64_t pg_next(pg_rng* r) {
    r->ctr += 1;
    return pg_mix(r->key + r->ctr * PG_GOLDEN);
}
/* uniform integer in [0, n) by multiply-high (bias < 2^-32 for n < 2^32). */
static inline uint32_t pg_below(pg_rng* r, uint32_t n) {
    return (uint32_t)(((unsigned __int128)pg_next(r) * n) >> 64);
}
static inline double pg_unit(pg_rng* r) {
    return (double)(pg_next(r) >> 11) * (1.0 / 9007199254740992.0);
}
static void pg_uniform_bases(pg_rng* r, uint8_t* out, uint32_t n) {
    uint32_t i = 0;
    while (i < n) {
        uint64_t x = pg_next(r);
        for (int j = 0; j < 32 && i < n; ++j, ++i) { out[i] = (uint8_t)(x & 3u); x >>= 2; }
    }
}

/* Generate one pair.  `read` and `ref` have room for at least the pair's
 * length; `work` has room for m + kmax + 1 bytes. */
static void pg_one(const pg_config* cfg, uint64_t p, uint8_t* read, uint8_t* ref,
                   uint16_t* len_out, uint8_t* E_out, uint8_t* related_out, uint16_t* k_out,
                   uint8_t* work) {
    pg_rng r;
    pg_seed(&r, cfg->seed, p);
    uint32_t m = cfg->lens[cfg->n_len > 1 ? pg_below(&r, cfg->n_len) : 0];
    uint32_t E = cfg->fixed_E >= 0 ? (uint32_t)cfg->fixed_E : (m * cfg->e_num) / cfg->e_den;
    pg_uniform_bases(&r, read, m);
    int unrelated = pg_unit(&r) < cfg->unrelated;
    uint32_t k = 0;
    if (unrelated) {
        pg_uniform_bases(&r, ref, m);
    } else {
        k = pg_below(&r, cfg->kmax + 1);
        uint32_t n = m;
        memcpy(work, read, m);
        for (uint32_t e = 0; e < k; ++e) {
            uint32_t kind = pg_below(&r, 3);
            if (kind == 0) {                      /* substitution */
                if (n == 0) continue;
                uint32_t pos = pg_below(&r, n);
                work[pos] = (uint8_t)((work[pos] + 1 + pg_below(&r, 3)) & 3u);
            } else if (kind == 1) {               /* insertion */
                uint32_t pos = pg_below(&r, n + 1);
                memmove(work + pos + 1, work + pos, n - pos);
                work[pos] = (uint8_t)pg_below(&r, 4);
                n += 1;
            } else {                              /* deletion */
                if (n == 0) continue;
                uint32_t pos = pg_below(&r, n);
                memmove(work + pos, work + pos + 1, n - pos - 1);
                n -= 1;
            }
        }
        if (n >= m) {
            memcpy(ref, work, m);
        } else {
            memcpy(ref, work, n);
            pg_uniform_bases(&r, ref + n, m - n);
        }
    }
    if (len_out) *len_out = (uint16_t)m;
    if (E_out) *E_out = (uint8_t)E;
    if (related_out) *related_out = (uint8_t)(!unrelated);
    if (k_out) *k_out = (uint16_t)k;
}

/* Pairs [first, first + n) of the workload.  Pair i of the call is written to
 * reads + i*stride and refs + i*stride (stride >= the longest length).  Any of
 * the per-pair side outputs may be NULL.  Returns 0, or -1 on a bad config. */
int pg_generate(const pg_config* cfg, uint64_t first, uint64_t n,
                uint8_t* reads, uint8_t* refs, uint32_t stride,
                uint16_t* len, uint8_t* E, uint8_t* related, uint16_t* k, int nthreads) {
    if (!cfg || cfg->n_len < 1 || cfg->n_len > 8) return -1;
    uint32_t maxlen = 0;
    for (uint32_t i = 0; i < cfg->n_len; ++i) {
        if (cfg->lens[i] < 1 || cfg->lens[i] > 512) return -1;
        if (cfg->lens[i] > maxlen) maxlen = cfg->lens[i];
    }
    if (stride < maxlen) return -1;
    if (cfg->fixed_E < 0 && cfg->e_den == 0) return -1;
    if (nthreads < 1) nthreads = 1;
    int err = 0;
#pragma omp parallel num_threads(nthreads)
    {
        uint8_t* work = (uint8_t*)malloc(maxlen + cfg->kmax + 1);
        if (!work) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static, 4096)
            for (int64_t i = 0; i < (int64_t)n; ++i) {
                pg_one(cfg, first + (uint64_t)i, reads + (uint64_t)i * stride, refs + (uint64_t)i * stride,
                       len ? len + i : NULL, E ? E + i : NULL, related ? related + i : NULL,
                       k ? k + i : NULL, work);
            }
            free(work);
        }
    }
    return err ? -1 : 0;
}

/* Gather variant: generate the pairs with the listed ids (for sampled checks). */
int pg_generate_ids(const pg_config* cfg, const uint64_t* ids, uint64_t n,
                    uint8_t* reads, uint8_t* refs, uint32_t stride,
                    uint16_t* len, uint8_t* E, uint8_t* related, uint16_t* k, int nthreads) {
    if (!cfg || cfg->n_len < 1 || cfg->n_len > 8) return -1;
    uint32_t maxlen = 0;
    for (uint32_t i = 0; i < cfg->n_len; ++i) {
        if (cfg->lens[i] < 1 || cfg->lens[i] > 512) return -1;
        if (cfg->lens[i] > maxlen) maxlen = cfg->lens[i];
    }
    if (stride < maxlen) return -1;
    if (cfg->fixed_E < 0 && cfg->e_den == 0) return -1;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        uint8_t* work = (uint8_t*)malloc(maxlen + cfg->kmax + 1);
#pragma omp for schedule(static, 256)
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            pg_one(cfg, ids[i], reads + (uint64_t)i * stride, refs + (uint64_t)i * stride,
                   len ? len + i : NULL, E ? E + i : NULL, related ? related + i : NULL,
                   k ? k + i : NULL, work);
        }
        free(work);
    }
    return 0;
}

/* Lengths and thresholds only of pairs [first, first + n): the first draws of
 * each pair's stream, without its bases. */
int pg_lengths(const pg_config* cfg, uint64_t first, uint64_t n, uint16_t* len, uint8_t* E, int nthreads) {
    if (!cfg || cfg->n_len < 1 || cfg->n_len > 8) return -1;
    if (cfg->fixed_E < 0 && cfg->e_den == 0) return -1;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static, 65536)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        pg_rng r;
        pg_seed(&r, cfg->seed, first + (uint64_t)i);
        uint32_t m = cfg->lens[cfg->n_len > 1 ? pg_below(&r, cfg->n_len) : 0];
        len[i] = (uint16_t)m;
        E[i] = (uint8_t)(cfg->fixed_E >= 0 ? (uint32_t)cfg->fixed_E : (m * cfg->e_num) / cfg->e_den);
    }
    return 0;
}
