/*
 * paf.h -- C ABI of libpaf, an MI355X (gfx950) library for pre-alignment
 * filtering of (read, reference segment) pairs under an edit threshold E,
 * after Alser's thesis "Accelerating the Understanding of Life's Code Through
 * Better Algorithms and Hardware Design" (arXiv 1910.03936).
 *
 * General conventions
 *  - Every pointer marked [device] is device memory owned by the caller; the
 *    library never frees it.  [host] pointers are host memory.
 *  - Calls that take a `stream` (a hipStream_t passed as void*, NULL = the
 *    null stream) are asynchronous: they enqueue work and return.  The caller
 *    synchronizes before reading outputs.
 *  - Every call validates its arguments on the host before launching
 *    anything; on a bad argument it returns PAF_ERR_ARG or PAF_ERR_RANGE,
 *    launches nothing and leaves a message for paf_last_error().  Per-pair
 *    values that live in device memory (lengths, thresholds) are checked by
 *    the kernels; a violation sets a sticky flag in the context, the pair's
 *    outputs are zero, and the next paf_check() reports PAF_ERR_RANGE.
 *  - No C++ exception crosses this interface.
 *  - A context serves one device; calls on one context from several threads
 *    must be serialized by the caller.
 *  - Calls that use the context's own device memory (the persistent launch's
 *    work-queue counter, the bucketing workspace of the bucketed and MAGNET
 *    calls, the cost model's weights and training workspace) may be made on
 *    different streams: the library orders them, a call on another stream
 *    than the previous such call waiting on the device for that call's work
 *    (an event the context records).  paf_filter, paf_filter_partitioned,
 *    paf_verify, paf_pack and paf_features use no such memory and are not
 *    ordered.  A stream under graph capture should keep such calls on that
 *    one stream.
 *
 * Sequence encoding (Ch. 5, Method 3: two bits per base; the thesis fixes
 * A = 00 and T = 11, this library uses C = 01 and G = 10).  A sequence of m
 * bases occupies ceil(m / 32) uint64 words; word k holds bases 32k..32k+31
 * with the low code bit of base 32k+j in bit j and the high code bit in bit
 * 32 + j.  Bases past m are zero.  paf_pack / paf_pack_host produce this.
 */
#ifndef PAF_H
#define PAF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct paf_ctx paf_ctx;

typedef enum {
    PAF_OK = 0,
    PAF_ERR_ARG = 1,     /* NULL pointer, zero size, inconsistent arguments */
    PAF_ERR_RANGE = 2,   /* length, threshold or size outside the supported range */
    PAF_ERR_DEVICE = 3,  /* a HIP runtime call failed */
    PAF_ERR_NOMEM = 4,   /* device or pinned allocation failed */
    PAF_ERR_STATE = 5    /* call out of order (e.g. predicting with no model) */
} paf_status;

/* Filter selection mask; the bit position is also the index into paf_out. */
enum { PAF_SNEAKYSNAKE = 1u, PAF_GATEKEEPER = 2u, PAF_SHOUJI = 4u };

#define PAF_MAX_LEN 512  /* bases per sequence: 16 words */
#define PAF_MAX_E 31     /* threshold: 2E+1 <= 63 diagonals */

/* A batch of pairs (all pointers [device]).
 * Pair p: read words at reads + off(p), reference words at refs + off(p),
 * off(p) = word_offset[p] if word_offset != NULL else p * stride_words.
 * Length m(p) = len[p] if len != NULL else uniform_len, 1 <= m <= PAF_MAX_LEN.
 * Threshold E(p) = E[p] if E != NULL else uniform_E, 0 <= E <= PAF_MAX_E.
 * max_len / max_E: upper bounds over the batch (equal to the uniform values
 * when those are used); the kernels are specialised on them, and a pair
 * above them is a device-side range violation. */
typedef struct {
    const uint64_t* reads;
    const uint64_t* refs;
    const uint64_t* word_offset;
    uint32_t stride_words;
    const uint16_t* len;
    uint16_t uniform_len;
    const uint8_t* E;
    uint8_t uniform_E;
    uint16_t max_len;
    uint8_t max_E;
    uint64_t n_pairs;
} paf_batch;

/* Outputs (all [device]).  Index 0 = SneakySnake, 1 = GateKeeper,
 * 2 = Shouji.  accept_bits[f] holds ceil(n/32) words: pair p's decision is
 * bit p % 32 of word p / 32 (1 = accept, i.e. pass on to alignment).
 * count[f] holds n uint16: SneakySnake's obstacle count min(e, E+1);
 * GateKeeper's and Shouji's edit estimate (the ones they counted).  A filter
 * requested in the mask needs both of its pointers; the others may be NULL. */
typedef struct {
    uint32_t* accept_bits[3];
    uint16_t* count[3];
} paf_out;

/* Context: binds device `device`, allocates the small device state (error
 * flag, work-queue counter, model weights, autotune cache).  *ctx is NULL on
 * failure. */
paf_status paf_create(paf_ctx** ctx, int device);
paf_status paf_destroy(paf_ctx* ctx);

/* Thread-local message describing the last non-OK status of this thread. */
const char* paf_last_error(void);

/* Waits for `stream`, then reports (and clears) the sticky device-side range
 * flag: PAF_ERR_RANGE if any pair since the last check had a length or
 * threshold outside its batch's bounds. */
paf_status paf_check(paf_ctx* ctx, void* stream);

/* Encoder (Ch. 4 host read encoder; Ch. 5 Method 3).
 * codes [device]: n rows of code_stride bytes, base values 0..3 (A,C,G,T);
 * row p holds m(p) bases (len/uniform_len as in paf_batch).
 * words [device]: output, written at off(p) as in paf_batch; the caller
 * sizes it.  A code above 3 sets the sticky range flag. */
paf_status paf_pack(paf_ctx* ctx, const uint8_t* codes, uint32_t code_stride, const uint16_t* len,
                    uint16_t uniform_len, const uint64_t* word_offset, uint32_t stride_words,
                    uint64_t n, uint64_t* words, void* stream);

/* Host-side encoder with the same layout (for streaming from host memory).
 * All pointers [host].  Uses up to `threads` host threads (0 = library
 * default).  Returns PAF_ERR_RANGE on a code above 3 or a bad length. */
paf_status paf_pack_host(const uint8_t* codes, uint32_t code_stride, const uint16_t* len,
                         uint16_t uniform_len, const uint64_t* word_offset, uint32_t stride_words,
                         uint64_t n, uint64_t* words, int threads);

/* Host encoder from sequence text (the host-side read encoder of Ch. 4,
 * Sec. 4.2, into the two-bit codes of Ch. 5, Method 3).  All pointers
 * [host], owned by the caller.
 * seqs: n rows of row_stride bytes; row p holds the m(p) bases of sequence p
 * as ASCII letters A, C, G, T (lower case a, c, g, t is accepted as the same
 * base; the bytes after m(p) are not read).  len / uniform_len, word_offset /
 * stride_words and words as in paf_pack_host; `threads` host threads (0 =
 * library default).
 * Every row is checked before anything is written: a byte inside a sequence
 * that is not one of those letters (N, IUPAC codes, digits, NUL ...) returns
 * PAF_ERR_ARG, a length outside [1, PAF_MAX_LEN], above row_stride or beyond
 * stride_words returns PAF_ERR_RANGE, and in both cases `words` is left
 * untouched. */
paf_status paf_pack_ascii(const char* seqs, uint32_t row_stride, const uint16_t* len, uint16_t uniform_len,
                          const uint64_t* word_offset, uint32_t stride_words, uint64_t n, uint64_t* words,
                          int threads);

/* Plain batched filter.  For every pair: load its words,
 * build the 2E+1 diagonal match bit-vectors (neighbourhood map, Eq. 6.1 /
 * unweighted maze, Eq. 8.2) and run the requested decision stages on them:
 * SneakySnake's greedy traversal (Ch. 8, Sec. 8.4), GateKeeper's Hamming
 * fast path plus amended shifted masks (Ch. 5, Sec. 5.2) and Shouji's
 * sliding-window search (Ch. 6, Sec. 6.2).  filters: mask of PAF_* bits.
 * SneakySnake alone runs on the compacting engine (see paf_layout's
 * chunk_tiles; up to max_E 15 a first pass of 2 windows, then: up to max_E
 * 3, 4 waves per block, chunks of 4 tiles and later passes of 3 windows;
 * 4..6: 2 waves, 4 tiles, 3 windows; 7..8: 2 waves, 6 tiles, 2 windows;
 * 9..15: 2 waves, 6 tiles, 3 windows; 16..25: 2 waves, 6 tiles, a first
 * pass of 3 windows, then 1; above: the same with a first pass of 4; unless
 * a layout was forced with paf_set_layout,
 * whose waves_per_block, chunk_tiles and pass widths then apply here too;
 * chunk_tiles = 0 selects the per-tile engine).  Several stages share one
 * map and one launch up to max_E 7; from max_E 8 SneakySnake runs as above in a launch of its own,
 * and from max_E 15 GateKeeper and Shouji get a launch each too (all on
 * `stream`, in order; the outputs are the same either way). */
paf_status paf_filter(paf_ctx* ctx, const paf_batch* batch, uint32_t filters, const paf_out* out,
                      void* stream);

/* SneakySnake on a column-partitioned maze (Sec. 8.6: the maze is cut into
 * adjacent, non-overlapping sub-mazes of t columns, all 2E+1 diagonals high,
 * the last one narrower when t does not divide m; Sec. 9.3.1 evaluates the
 * software form, SneakySnake-t, at t = 5, 10, 25 and 50).  Each sub-maze is
 * solved on its own by the greedy of paf_filter: a pipe is probed only up to
 * the sub-maze's last column, reaching that column costs nothing, and the
 * snake enters the next sub-maze free to take any diagonal.  The obstacles of
 * all sub-mazes add up: count = min(sum, E+1), accept = sum <= E.
 * y = 0: no other limit (SneakySnake-t).  y in [1, PAF_MAX_REPL]: the
 * hardware form of Sec. 8.6 (t = 8, y = 3 there), which searches each
 * sub-maze with y replications of leading-zero count, maximum and shift by
 * x + 1 and counts min(y, w - sum x) obstacles in a sub-maze of width w; that
 * is min(y, the sub-maze's fewest obstacles), which is what is computed.
 * The count never exceeds the whole maze's (so there are no false rejects
 * either), and t >= m with y = 0 gives paf_filter's SneakySnake result.
 * t in [1, PAF_MAX_PART].  Writes out->accept_bits[0] and out->count[0] (the
 * SneakySnake slots; the others are ignored).  Runs on the compacting engine
 * with paf_filter's layout, except that from max_E 4 to 6 it takes chunks of
 * 6 tiles and later passes of 1 window (a forced layout applies when its
 * chunk_tiles > 0). */
#define PAF_MAX_PART 65535
#define PAF_MAX_REPL 31
paf_status paf_filter_partitioned(paf_ctx* ctx, const paf_batch* batch, uint32_t t, uint32_t y,
                                  const paf_out* out, void* stream);

/* MAGNET decision stage (Ch. 7) on the neighbourhood map of Ch. 6 (vacant
 * cells blocked).  Repeatedly, up to E+1 times: the longest run of free cells
 * over all 2E+1 diagonals among the columns still searched (extraction; ties
 * go to the smallest start column, then to the first diagonal in order
 * -E..E) is taken, and its columns plus one column on each side leave the
 * search of every diagonal (encapsulation), until no free cell is left.
 * count = min(m - columns covered by the runs, E+1), accept = count <= E
 * (the thesis rejects when the runs cover fewer than m - E columns).  Unlike
 * SneakySnake, MAGNET may reject a pair within E edits (Sec. 9.3.3).  Writes
 * out->accept_bits[0] and out->count[0] (the other slots are ignored).  Uses
 * the context's bucketing workspace (5 bytes per pair, grown on first use
 * with a larger batch). */
paf_status paf_filter_magnet(paf_ctx* ctx, const paf_batch* batch, const paf_out* out, void* stream);

/* paf_filter_magnet without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and outputs as paf_filter_magnet.
 * Its workspace is not the context's: it is a static device array of the
 * library, laid out for up to PAF_MAGNET_NOALLOC_MAX_PAIRS pairs (about
 * 20 MiB), of which each device the library runs on holds one copy until the
 * process ends; its address is looked up once per context by paf_create.  The
 * call makes no hipMalloc, hipFree or other allocating call.  Every call on
 * one device shares that array: calls that overlap on the device (other
 * streams, other contexts of the device) race and their results are
 * undefined; calls on one stream, or ordered by the caller, do not.  Nothing
 * in the array needs clearing between calls.  n_pairs above the maximum
 * returns PAF_ERR_RANGE and launches nothing; PAF_ERR_DEVICE if the array's
 * address could not be looked up at paf_create. */
#define PAF_MAGNET_NOALLOC_MAX_PAIRS 4194304
paf_status paf_filter_magnet_noalloc(paf_ctx* ctx, const paf_batch* batch, const paf_out* out, void* stream);

/* Verification of filtered pairs: dist[p] = min(edit distance, E+1) of the
 * pair's reference segment and read, over alignments that stay inside the
 * band of the 2E+1 diagonals the filter examined (Ukkonen's banded edit
 * distance; Sec. 8.7 restricts exact edit distance to the cells that are
 * needed, and Sec. 9.3.1 pairs SneakySnake with such an aligner).  A value
 * <= E is the pair's exact edit distance; E+1 means more than E edits.
 * select_bits [device, ceil(n/32) words] or NULL: only the pairs whose bit is
 * set (bit p % 32 of word p / 32, the layout of paf_out's accept bits) are
 * verified, the others get E+1 (they were rejected); NULL verifies every
 * pair.  Passing SneakySnake's accept bits gives exactly the result of
 * verifying every pair, since SneakySnake never rejects a pair within E
 * edits.  dist [device]: n_pairs uint16, at the original pair index.  Work
 * grows with each pair's distance (by diagonal transition, E+1 rounds at
 * most); each wave gathers the selected pairs of 1024 consecutive ones into
 * full groups of 64, so only the selected pairs cost time.  Needs no
 * workspace. */
paf_status paf_verify(paf_ctx* ctx, const paf_batch* batch, const uint32_t* select_bits, uint16_t* dist,
                      void* stream);

/* Persistent launch: the same filter as one launch over 64-pair tiles, or
 * over compacting chunks of tiles for SneakySnake alone, handed out by a work
 * queue (the Read Controller's role, Sec. 4.2.1) or by the hardware
 * dispatcher as a full grid, for batches of uneven lengths and per-pair
 * thresholds.  The launch (queue reset + kernel) is captured once into a HIP
 * graph per (layout, filters, bounds, stream) and replayed; the layout is the
 * forced one, else the one paf_autotune chose for this batch's (max_len,
 * max_E, filters) class, else the default (per-tile engine, work queue of
 * 4 waves x 4 blocks per CU, 2 tiles per take).  Outputs as paf_filter. */
paf_status paf_filter_persistent(paf_ctx* ctx, const paf_batch* batch, uint32_t filters,
                                 const paf_out* out, void* stream);

/* Launch layout of the persistent, ordered and learned launches (paf_filter
 * takes waves_per_block, chunk_tiles and the pass widths from a forced
 * layout). */
typedef struct {
    uint32_t lanes_per_pair;   /* 1 (pair per lane), or 2: SneakySnake on the compacting engine
                                  with a pair's diagonals split between two lanes that OR their
                                  runs after every probe (max_E 9 and up; paf_filter_partitioned
                                  always runs one lane per pair) */
    uint32_t waves_per_block;  /* 1, 2, 4 or 8 */
    uint32_t blocks_per_cu;    /* resident blocks per compute unit in the persistent grid;
                                  0 = no work queue: a full grid, one tile per wave */
    uint32_t tiles_per_grab;   /* 64-pair tiles taken per queue access */
    uint32_t chunk_tiles;      /* SneakySnake alone: 0 = every wave keeps its 64 pairs until
                                  all are decided; K in 1..16 = a wave owns K tiles and, after
                                  each 32-column window, regroups the pairs still undecided
                                  into full waves (the queue then hands out chunks) */
    uint32_t first_pass_windows;   /* compacting engine: windows the lanes walk together
                                      before the first regrouping (0 = 1), 1..16 */
    uint32_t pass_windows;         /* ... and between later regroupings (0 = 1), 1..16 */
} paf_layout;

/* Times each candidate layout on `batch` (synchronously, on `stream`),
 * caches the fastest for the batch's class and returns it (and, if not NULL,
 * the time of the fastest and of the default layout in ms).  Outputs in
 * `out` are overwritten. */
paf_status paf_autotune(paf_ctx* ctx, const paf_batch* batch, uint32_t filters, const paf_out* out,
                        void* stream, paf_layout* chosen, float* best_ms, float* default_ms);
paf_status paf_set_layout(paf_ctx* ctx, const paf_layout* layout); /* NULL = back to autotuned */

/* Checkpoint of the autotuner's cache.  The cache lives in the context and
 * ends with it; a saved copy spares a later process the timing runs.  One
 * entry per tuned class (the classes paf_autotune forms: the batch's
 * ceil(max_len / 32), its max_E rounded up to the next threshold the library
 * has a kernel for, and the filter mask). */
typedef struct {
    uint32_t max_words;  /* 1..16 */
    uint32_t max_E;      /* one of 0..8, 10, 12, 15, 20, 25, 31 */
    uint32_t filters;    /* 1..7 */
    paf_layout layout;
} paf_tuned_entry;

/* Copies the first min(cap, *count) cached entries into entries [host] (may
 * be NULL when cap is 0) and sets *count to the number the cache holds. */
paf_status paf_tuned_export(paf_ctx* ctx, paf_tuned_entry* entries, uint32_t cap, uint32_t* count);
/* Adds (or replaces) `count` entries [host].  Every entry is checked first
 * (its class as above, the layout as paf_set_layout checks it, two lanes per
 * pair only for SneakySnake alone at max_E 10 and up); PAF_ERR_ARG on the
 * first bad one, and then nothing is added.  A layout whose chunks need more
 * LDS than a compute unit holds is refused at launch, as a forced one is. */
paf_status paf_tuned_import(paf_ctx* ctx, const paf_tuned_entry* entries, uint32_t count);

/* Learned cost bucketing.
 * Features of each pair (fp32, 64 per pair, row-major [n][64]): [0] = m/512,
 * [1] = E/32, slot 32+d = fraction of matching map cells over the first
 * min(m, 64) columns of diagonal d, |d| <= min(E, 30); other slots 0. */
paf_status paf_features(paf_ctx* ctx, const paf_batch* batch, float* features, void* stream);

/* Cost model: dense 64 -> 128 -> 128 -> 1, ReLU on the hidden layers.
 * Parameters are fp32 master copies with bf16 working copies used by the
 * matrix-core kernels (fp32 accumulation).  Host layout of `params`
 * (PAF_MLP_NPARAMS floats): W1[128][64], b1[128], W2[128][128], b2[128],
 * W3[128], b3. */
#define PAF_MLP_NPARAMS 24961
paf_status paf_mlp_set_params(paf_ctx* ctx, const float* params /* [host] */);
paf_status paf_mlp_get_params(paf_ctx* ctx, float* params /* [host] */);
/* Checkpoint of the model with its optimizer: master weights, Adam's first
 * and second moments (PAF_MLP_NPARAMS floats each, [host], the layout of
 * `params`) and the number of Adam steps taken, so that training resumed
 * from a saved state takes the same steps as training never stopped.
 * get_state needs a model (PAF_ERR_STATE).  set_state returns PAF_ERR_ARG,
 * leaving the context as it was, if a value is not finite or a second
 * moment is negative; it clears the stored gradients (as set_params does). */
paf_status paf_mlp_get_state(paf_ctx* ctx, float* params, float* adam_m, float* adam_v, uint32_t* step);
paf_status paf_mlp_set_state(paf_ctx* ctx, const float* params, const float* adam_m, const float* adam_v,
                             uint32_t step);
/* Predictions for n feature rows [device] -> out [device] fp32. */
paf_status paf_mlp_forward(paf_ctx* ctx, const float* features, uint64_t n, float* out, void* stream);
/* One training step on a minibatch: forward, MSE loss against targets,
 * backward, and an Adam update (lr, beta1 0.9, beta2 0.999, eps 1e-8) of
 * the master weights, then bf16 re-rounding.  features [device] [n][64],
 * targets [device] fp32 [n], n <= 65536.  If grads != NULL [device,
 * PAF_MLP_NPARAMS floats] the gradients are copied there; if loss != NULL
 * [device] the mean loss is stored there.  If lr == 0 the weights are left
 * unchanged (gradient only). */
paf_status paf_mlp_train_step(paf_ctx* ctx, const float* features, const float* targets, uint64_t n,
                              float lr, float* grads, float* loss, void* stream);

/* Predictions of the cost model for every pair of a batch, computed by the
 * fused kernel the bucketed filter uses (features -> model on the matrix
 * cores).  pred [device] fp32 [n]; pairs that fail the device-side checks
 * get 0.  Needs a model (PAF_ERR_STATE otherwise). */
paf_status paf_mlp_predict(paf_ctx* ctx, const paf_batch* batch, float* pred, void* stream);

/* Trains the model on n labelled feature rows for `epochs` passes over
 * consecutive minibatches of `batch` rows (the caller shuffles the rows),
 * with paf_mlp_train_step's Adam update.  features [device] fp32 [n][64],
 * labels [device] uint16 [n] (the target counts).  epoch_loss [host,
 * `epochs` floats] receives each epoch's mean minibatch loss if not NULL.
 * Synchronizes `stream` before returning. */
paf_status paf_mlp_train(paf_ctx* ctx, const float* features, const uint16_t* labels, uint64_t n,
                         uint32_t epochs, uint32_t batch, float lr, float* epoch_loss, void* stream);

/* Bucketing.  From a prediction y (the model's estimate of SneakySnake's
 * obstacle count over the whole maze) and the pair's m and E, the number of
 * 32-column windows the snake is expected to traverse at the pair's own
 * threshold is estimated (it stops after E+1 obstacles, so it covers about
 * m (E+1)/y columns when y > E+1, else all m), refined by the expected number
 * of steps, and quantised to a level 0..15 against the longest pair the
 * batch's bounds allow; bucket = 15 - level, so the longest work comes first.
 * Writes a permutation of 0..n-1 grouped by bucket, stable within a bucket
 * (perm [device] uint32 [n]) and the 16 bucket sizes (hist [device] uint32
 * [16]).  pred [device] fp32 [n]. */
paf_status paf_bucket(paf_ctx* ctx, const paf_batch* batch, const float* pred, uint32_t* perm,
                      uint32_t* hist, void* stream);

/* The filter of paf_filter_persistent over a caller-given order of the pairs
 * (order [device] uint32 [n], a permutation of 0..n-1; a repeated or
 * out-of-range id is undefined behaviour).  Outputs land at each pair's
 * original index, identical to paf_filter's. */
paf_status paf_filter_ordered(paf_ctx* ctx, const paf_batch* batch, uint32_t filters,
                              const uint32_t* order, const paf_out* out, void* stream);

/* The learned pipeline end to end: features -> model -> buckets -> persistent
 * filter over the bucketed order -> decisions written at each pair's original
 * index.  Decisions are identical to paf_filter's; only the order of work
 * changes.  Needs a model (PAF_ERR_STATE otherwise).  Workspace is held by
 * the context and grows to the largest batch seen. */
paf_status paf_filter_bucketed(paf_ctx* ctx, const paf_batch* batch, uint32_t filters,
                               const paf_out* out, void* stream);

/* Chunk-local learned bucketing, stage 1: features and cost model of every
 * pair; key[p] = 15 - level, level = min(15, floor(clamp(y, 0, 32) / 2)),
 * y the predicted SneakySnake count at E = 31 (key: uint8 [device],
 * n_pairs entries, original order).  The compacting filter reads a pair's
 * key only if the pair is still undecided after the first pass (its first
 * 64 columns), so up to max_E 15 (the compact feature layouts) the model
 * runs only on the pairs with a diagonal |d| <= E whose matching cells make
 * up at least 2/5 of the first min(m, 64) columns (5 matches >= 2 columns);
 * the others, which that pass almost always decides, get level 0 (key 15)
 * without it.  Above max_E 15 every pair runs the model. */
paf_status paf_cost_levels(paf_ctx* ctx, const paf_batch* batch, uint8_t* key, void* stream);

/* Stage 2: SneakySnake alone on the compacting engine, the pairs of each
 * chunk still undecided after the first pass entering the later passes
 * grouped into four classes by bits 2-3 of their key (key: uint8 per pair
 * [device], original order; class = (key & 15) >> 2, class 0 first; a
 * stable sort, skipped when a chunk keeps more than 320 pairs).  Any key
 * gives the outputs of paf_filter; a key that groups pairs of like cost
 * makes the groups of 64 more even.  Layout as paf_filter_bucketed_local. */
paf_status paf_filter_keyed(paf_ctx* ctx, const paf_batch* batch, const uint8_t* key, const paf_out* out,
                            void* stream);

/* Chunk-local learned bucketing (SneakySnake alone).  The cost model's
 * prediction puts every pair on one of 16 levels (width 2 obstacles, highest
 * first).  The compacting filter then groups the undecided pairs of each of
 * its chunks into four classes of four levels after the first pass
 * (paf_filter_keyed), so each group of 64 takes pairs of like cost, while the
 * pairs stay in place in memory (no global permutation, no gathers).  Model and filter are captured in one HIP graph per (batch,
 * layout, outputs).  Outputs as paf_filter, in the original order.  The
 * launch layout is the forced or autotuned one if it has chunk_tiles > 0,
 * else paf_filter's. */
paf_status paf_filter_bucketed_local(paf_ctx* ctx, const paf_batch* batch, const paf_out* out, void* stream);

/* Streaming from host memory (the host-to-accelerator stream of
 * Ch. 4, Secs. 4.2-4.4).  All pointers [host]; page-locked (pinned) memory
 * lets the copies overlap the filtering.  Pairs are stored back to back:
 * pair p's words start at word sum_{q<p} ceil(len[q] / 32) of reads and of
 * refs (the encoding of paf.h). */
typedef struct {
    const uint64_t* reads;
    const uint64_t* refs;
    const uint16_t* len;   /* per-pair lengths, 1..max_len */
    const uint8_t* E;      /* per-pair thresholds, 0..max_E */
    uint16_t max_len;
    uint8_t max_E;
    uint64_t n_pairs;
} paf_host_batch;

typedef struct {
    double seconds;    /* wall time of the whole stream */
    double h2d_bytes;  /* bytes copied host to device */
    uint64_t chunks;
} paf_stream_stats;

/* Filters every pair of a host batch, chunk_pairs pairs at a time (a positive
 * multiple of 64): each chunk is copied on a copy stream into one of two
 * device buffers while the previous chunk is filtered on a compute stream
 * (plain batching, or when `learned` is nonzero the learned pipeline:
 * paf_filter_bucketed_local for SneakySnake alone, paf_filter_bucketed for
 * other masks), and its decisions are copied back into host_out
 * (paf_out with [host] pointers: accept bits and counts for all n pairs).
 * Blocks until every chunk is done.  Decisions equal paf_filter's. */
paf_status paf_stream_filter(paf_ctx* ctx, const paf_host_batch* batch, uint64_t chunk_pairs,
                             uint32_t filters, int learned, const paf_out* host_out,
                             paf_stream_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* PAF_H */
