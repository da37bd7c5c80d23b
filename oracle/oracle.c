/*
 * CPU oracle for the pre-alignment filters -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar implementation of what the GPU path computes, written
 * straight from the definitions in Alser's thesis (arXiv 1910.03936).  It is
 * used by the tests, by the package's smoke check and by the benchmark's CPU
 * baseline leg; nothing on the product path may call it.  It shares no code,
 * header or table with the GPU library.
 *
 * Sequences are uint8 codes 0..3, one per base, read[0..m) and ref[0..m)
 * (the filter compares a read with a reference segment of the same length,
 * Ch. 1, seed-and-extend overview).
 *
 * Readings of points the thesis leaves open (each is listed with its evidence
 * in the design notes):
 *  - Columns run along the reference; diagonal d in [-E, E] compares ref[c]
 *    with read[c + d] (fixed by the worked example of Figs. 8.1/8.2 and by
 *    Fig. 6.2; traversing along the read gives different pipes).
 *  - A map cell whose read index c + d falls outside [0, m) is blocked (1)
 *    for SneakySnake and Shouji (the maze has E+1 entrances, Sec. 8.2; Shouji
 *    fills vacant bits with ones, Sec. 6.4) and a match (0) for GateKeeper
 *    (it inherits SHD's zero fill, Sec. 3.2.3).
 *  - Every filter accepts when its count is <= E.
 *  - Crossing an obstacle costs one edit and advances one column; the snake
 *    then chooses again (Sec. 8.2 pipes and obstacles; the hardware tile
 *    shifts by x + 1, Sec. 8.6).
 *  - SneakySnake reports min(e, E + 1) (it stops after E + 1 obstacles);
 *    GateKeeper and Shouji report their raw popcount.
 *  - Shouji: m windows of 4 columns, columns >= m padded with ones; among the
 *    diagonals with the most zeros in the window the first (in order -E..E)
 *    whose first bit is a zero wins, else the first; the window's 4 bits
 *    overwrite the Shouji bit-vector only when they hold strictly more zeros.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_LEN 512
#define OR_MAX_E 31

/* Neighborhood map cell (Eq. 6.1; unweighted maze, Eq. 8.2): 0 when the two
 * bases match, 1 when they differ.  `vacant` is the value used when the read
 * index c + d lies outside the read. */
static int map_cell(const uint8_t* read, const uint8_t* ref, int m, int c, int d, int vacant) {
    int j = c + d;
    if (j < 0 || j >= m) return vacant;
    return ref[c] != read[j];
}

/* Depth of the pipe that starts at column c on diagonal d: the number of
 * consecutive available cells (Sec. 8.4.2, depth-first probe of one diagonal). */
static int pipe_depth(const uint8_t* read, const uint8_t* ref, int m, int c, int d) {
    int L = 0;
    while (c + L < m && map_cell(read, ref, m, c + L, d, 1) == 0) L++;
    return L;
}

/* SneakySnake on the unweighted maze (Secs. 8.2 and 8.4).  From the current column the
 * snake probes every diagonal, upper ones first, to its first obstacle and
 * follows the deepest pipe (the first of equal depth).  At the pipe's end it
 * crosses the obstacle, which costs one of its E tries and one column; an
 * all-blocked column is a pipe of depth 0.  It survives when it reaches the
 * last column having crossed at most E obstacles.
 *
 * Returns accept (0/1); *count = obstacles crossed, at most E + 1.  When
 * `pipes` is non-NULL, up to max_pipes (start column, diagonal, depth)
 * triples of the followed pipes with depth > 0 are written, and *n_pipes is
 * set. */
int or_sneakysnake(const uint8_t* read, const uint8_t* ref, int m, int E, int* count,
                   int* pipes, int max_pipes, int* n_pipes) {
    int c = 0, e = 0, np = 0;
    while (c < m) {
        int best = -1, best_d = 0;
        for (int d = -E; d <= E; ++d) {          /* upper diagonals (d < 0) first */
            int L = pipe_depth(read, ref, m, c, d);
            if (L > best) { best = L; best_d = d; }
        }
        if (best > 0 && pipes && np < max_pipes) {
            pipes[3 * np + 0] = c; pipes[3 * np + 1] = best_d; pipes[3 * np + 2] = best;
            np++;
        }
        c += best;
        if (c < m) {                              /* an obstacle: cross it */
            e += 1;
            c += 1;
            if (e > E) break;                     /* all E tries used */
        }
    }
    if (n_pipes) *n_pipes = np;
    *count = e;
    return e <= E;
}

/* SneakySnake on a column-partitioned maze (Sec. 8.6, the hardware design's
 * sub-matrices; its software form with t = 5, 10, 25 or 50 columns is the
 * SneakySnake-t of Sec. 9.3.1).  The maze is cut into adjacent,
 * non-overlapping sub-mazes of t columns each (the last one narrower when t
 * does not divide m), all 2E+1 diagonals high, and each sub-maze is solved on
 * its own by the same greedy: a pipe is probed only up to the sub-maze's last
 * column, reaching that column costs nothing, and the snake enters the next
 * sub-maze free to take any diagonal.  The obstacles crossed in all sub-mazes
 * add up; the search stops once the sum exceeds E.  With t >= m there is one
 * sub-maze, the whole maze.
 * Returns accept (0/1); *count = min(total obstacles, E + 1). */
int or_sneakysnake_t(const uint8_t* read, const uint8_t* ref, int m, int E, int t, int* count) {
    int e = 0;
    for (int p0 = 0; p0 < m && e <= E; p0 += t) {
        int p1 = p0 + t < m ? p0 + t : m;         /* this sub-maze: columns [p0, p1) */
        int c = p0;
        while (c < p1) {
            int best = 0;
            for (int d = -E; d <= E; ++d) {
                int L = 0;
                while (c + L < p1 && map_cell(read, ref, m, c + L, d, 1) == 0) L++;
                if (L > best) best = L;
            }
            c += best;
            if (c < p1) {                         /* an obstacle inside the sub-maze */
                e += 1;
                c += 1;
                if (e > E) break;
            }
        }
    }
    *count = e;
    return e <= E;
}

/* The hardware form of SneakySnake (Sec. 8.6): sub-mazes of t columns (the
 * last one narrower when t does not divide m), each searched by y
 * replications of three steps: a leading-zero count of every row from the
 * current column (the search starts at a row's least significant bit, and
 * bits shifted in past the sub-maze's end are ones), the largest count x over
 * the rows, and a shift of every row by x + 1.  A sub-maze of width w then
 * counts min(y, w - sum of its x) obstacles.  The pair's count is min(sum over
 * the sub-mazes, E + 1); accept = sum <= E.
 * Reading: the text also says a sub-maze counts y obstacles whenever every
 * replication found x > 0, which gives 2 for its own step-4 example (one row
 * 00010000, t = 8, y = 2: x = 4 then 3, one obstacle); min(y, w - sum x)
 * gives 1 and is used for every sub-maze. */
int or_sneakysnake_fpga(const uint8_t* read, const uint8_t* ref, int m, int E, int t, int y, int* count) {
    int e = 0;
    for (int p0 = 0; p0 < m; p0 += t) {
        int p1 = p0 + t < m ? p0 + t : m;
        int c = p0, sx = 0;
        for (int r = 0; r < y; ++r) {
            int x = 0;
            for (int d = -E; d <= E; ++d) {
                int L = 0;
                while (c + L < p1 && map_cell(read, ref, m, c + L, d, 1) == 0) L++;
                if (L > x) x = L;
            }
            sx += x;
            c += x + 1;
        }
        int ob = (p1 - p0) - sx;
        e += ob < y ? ob : y;
    }
    *count = e > E ? E + 1 : e;
    return e <= E;
}

/* SneakySnake on the weighted maze (Sec. 8.3, Eq. 8.1): each available cell holds the
 * number of available cells from it to the end of its pipe, filled from the
 * lower right; the snake reads the largest weight in its column instead of
 * probing.  Same result as the unweighted maze by construction; kept as a
 * second, independently written route. */
int or_sneakysnake_weighted(const uint8_t* read, const uint8_t* ref, int m, int E, int* count) {
    int D = 2 * E + 1;
    int* WN = (int*)calloc((size_t)D * (m + 1), sizeof(int));
    for (int k = 0; k < D; ++k) {
        int d = k - E;
        WN[k * (m + 1) + m] = 0;
        for (int c = m - 1; c >= 0; --c)
            WN[k * (m + 1) + c] = map_cell(read, ref, m, c, d, 1) ? 0 : WN[k * (m + 1) + c + 1] + 1;
    }
    int c = 0, e = 0;
    while (c < m) {
        int best = 0;
        for (int k = 0; k < D; ++k)
            if (WN[k * (m + 1) + c] > best) best = WN[k * (m + 1) + c];
        c += best;
        if (c < m) {
            e += 1;
            c += 1;
            if (e > E) break;
        }
    }
    free(WN);
    *count = e;
    return e <= E;
}

/* SHD/GateKeeper amendment (Sec. 3.2.1; Sec. 5.2.2): a zero whose streak of
 * zeros has length 1 or 2 and is bounded by ones on both sides is flipped to
 * one ("101" -> "111", "1001" -> "1111").  Streaks that touch either end of
 * the mask are kept (the first and last bits are copied unchanged). */
static void amend(const uint8_t* in, uint8_t* out, int m) {
    memcpy(out, in, (size_t)m);
    int i = 0;
    while (i < m) {
        if (in[i]) { i++; continue; }
        int a = i;
        while (i < m && in[i] == 0) i++;
        int b = i;                                /* zeros occupy [a, b) */
        if (a >= 1 && b <= m - 1 && (b - a) <= 2)
            for (int t = a; t < b; ++t) out[t] = 1;
    }
}

/* The amendment alone, exposed so that its bit rules can be checked. */
void or_amend(const uint8_t* in, uint8_t* out, int m) { amend(in, out, m); }

/* GateKeeper (Ch. 5).  Method 1: count the ones of the unshifted Hamming mask;
 * at most E accepts at once.  Method 2: build the 2E+1 shifted masks (vacant
 * bits zero), amend each, AND them all, and count the ones of the result;
 * accept when that count is at most E.  Method 3 (one mismatch bit per base
 * pair) is how the masks are represented here: one entry per base.
 * Returns accept; *count = the count the decision used. */
int or_gatekeeper(const uint8_t* read, const uint8_t* ref, int m, int E, int* count) {
    int H = 0;
    for (int c = 0; c < m; ++c) H += map_cell(read, ref, m, c, 0, 0);
    if (H <= E) { *count = H; return 1; }
    uint8_t G[OR_MAX_LEN], A[OR_MAX_LEN], F[OR_MAX_LEN];
    for (int c = 0; c < m; ++c) F[c] = 1;
    for (int d = -E; d <= E; ++d) {
        for (int c = 0; c < m; ++c) G[c] = (uint8_t)map_cell(read, ref, m, c, d, 0);
        amend(G, A, m);
        for (int c = 0; c < m; ++c) F[c] = (uint8_t)(F[c] & A[c]);
    }
    int n = 0;
    for (int c = 0; c < m; ++c) n += F[c];
    *count = n;
    return n <= E;
}

/* Shouji (Ch. 6).  A 4-column search window slides one column at a time over
 * the neighborhood map, m windows in all.  In each window the diagonal
 * segment with the most zeros is selected (ties: the first one that starts
 * with a zero, else the first); if it holds more zeros than the Shouji
 * bit-vector at the same four positions, it is copied there.  The number of
 * ones left in the bit-vector is the edit estimate; accept when <= E.
 * Returns accept; *count = ones in the bit-vector; S (m entries) optional. */
int or_shouji(const uint8_t* read, const uint8_t* ref, int m, int E, int* count, uint8_t* S_out) {
    uint8_t S[OR_MAX_LEN + 4];
    for (int c = 0; c < m + 3; ++c) S[c] = 1;
    for (int c = 0; c < m; ++c) {
        int best_z = -1, best_lead = 0;
        uint8_t best_v[4] = {1, 1, 1, 1};
        for (int d = -E; d <= E; ++d) {
            uint8_t v[4];
            int z = 0;
            for (int t = 0; t < 4; ++t) {
                int col = c + t;
                v[t] = (uint8_t)(col < m ? map_cell(read, ref, m, col, d, 1) : 1);
                z += (v[t] == 0);
            }
            int lead = (v[0] == 0);
            if (z > best_z || (z == best_z && lead && !best_lead)) {
                best_z = z; best_lead = lead;
                memcpy(best_v, v, 4);
            }
        }
        int zs = 0;
        for (int t = 0; t < 4; ++t) zs += (S[c + t] == 0);
        if (best_z > zs)
            for (int t = 0; t < 4; ++t) S[c + t] = best_v[t];
    }
    int n = 0;
    for (int c = 0; c < m; ++c) n += S[c];
    if (S_out) memcpy(S_out, S, (size_t)m);
    *count = n;
    return n <= E;
}

/* MAGNET (Ch. 7) on the neighborhood map of Ch. 6 (vacant cells blocked).
 * Extraction: the longest run of consecutive zeros over all 2E+1 diagonals,
 * among the columns still in the search space.  Encapsulation: the run's
 * columns and the one column on each side of it leave the search space of
 * every diagonal.  The two sides are searched again the same way, longest
 * run first (the hardware form keeps one problem and sets the excluded
 * columns to ones in every bit-vector, Sec. 7.4), until E + 1 runs are found
 * or no zero is left.  The pair is rejected when the runs found cover fewer
 * than m - E columns.
 * Readings: among runs of equal length the one with the smallest start
 * column is taken, then the first diagonal in order -E..E; count = min(m -
 * covered, E + 1) (the columns the runs leave uncovered, an edit estimate)
 * and accept = count <= E.  The thesis's test after the first extraction
 * (reject when the longest run is shorter than ceil((m - E) / (E + 1))) can
 * only reject pairs the final test rejects, and changes neither output, so it
 * is not repeated here.
 * segs (optional, 3 (E + 1) ints): (diagonal, start column, length) of each
 * run in the order found; *n_segs = their number. */
int or_magnet(const uint8_t* read, const uint8_t* ref, int m, int E, int* count, int* segs, int* n_segs) {
    uint8_t gone[OR_MAX_LEN];                     /* 1 = column left the search space */
    memset(gone, 0, (size_t)m);
    int covered = 0, ns = 0;
    for (int it = 0; it <= E; ++it) {
        int best = 0, best_c = 0, best_d = 0;
        for (int c = 0; c < m; ++c)
            for (int d = -E; d <= E; ++d) {
                int L = 0;
                while (c + L < m && !gone[c + L] && map_cell(read, ref, m, c + L, d, 1) == 0) L++;
                if (L > best) { best = L; best_c = c; best_d = d; }
            }
        if (best == 0) break;
        if (segs) { segs[3 * ns + 0] = best_d; segs[3 * ns + 1] = best_c; segs[3 * ns + 2] = best; }
        ns++;
        covered += best;
        int a = best_c > 0 ? best_c - 1 : 0;
        int b = best_c + best + 1 < m ? best_c + best + 1 : m;
        for (int c = a; c < b; ++c) gone[c] = 1;
    }
    int left = m - covered;
    if (n_segs) *n_segs = ns;
    *count = left > E ? E + 1 : left;
    return left <= E;
}

/* MAGNET over a batch (pairs as in or_filter_batch). */
void or_magnet_batch(const uint8_t* reads, const uint8_t* refs, uint32_t stride, const uint16_t* len,
                     const uint8_t* E, uint64_t n, uint8_t* acc, uint16_t* cnt, int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        int c = 0;
        acc[i] = (uint8_t)or_magnet(reads + (uint64_t)i * stride, refs + (uint64_t)i * stride, len[i], E[i],
                                    &c, NULL, NULL);
        cnt[i] = (uint16_t)c;
    }
}

/* Levenshtein distance restricted to the 2E+1 diagonals around the main one
 * (Ukkonen's band, Sec. 2.2.2), for two strings of length m.  Returns
 * min(distance, E + 1).  When the true distance is at most E it equals the
 * true distance, since such an alignment never leaves the band. */
int or_banded_levenshtein(const uint8_t* a, const uint8_t* b, int m, int E) {
    const int INF = 1 << 28;
    int W = m + 1;
    int* Dm = (int*)malloc(sizeof(int) * (size_t)W * W);
    for (int i = 0; i <= m; ++i)
        for (int j = 0; j <= m; ++j) {
            int v;
            if (abs(i - j) > E) v = INF;
            else if (i == 0) v = j;
            else if (j == 0) v = i;
            else {
                int sub = Dm[(i - 1) * W + (j - 1)] + (a[i - 1] != b[j - 1]);
                int del = Dm[(i - 1) * W + j] + 1;
                int ins = Dm[i * W + (j - 1)] + 1;
                v = sub < del ? sub : del;
                if (ins < v) v = ins;
            }
            Dm[i * W + j] = v;
        }
    int r = Dm[m * W + m];
    free(Dm);
    return r > E ? E + 1 : r;
}

/* Full Levenshtein distance of a[0..n) and b[0..k). */
int or_levenshtein(const uint8_t* a, int n, const uint8_t* b, int k) {
    int* prev = (int*)malloc(sizeof(int) * (size_t)(k + 1));
    int* cur = (int*)malloc(sizeof(int) * (size_t)(k + 1));
    for (int j = 0; j <= k; ++j) prev[j] = j;
    for (int i = 1; i <= n; ++i) {
        cur[0] = i;
        for (int j = 1; j <= k; ++j) {
            int sub = prev[j - 1] + (a[i - 1] != b[j - 1]);
            int del = prev[j] + 1, ins = cur[j - 1] + 1;
            int v = sub < del ? sub : del;
            cur[j] = ins < v ? ins : v;
        }
        int* t = prev; prev = cur; cur = t;
    }
    int r = prev[k];
    free(prev);
    free(cur);
    return r;
}

/* Hamming distance of two equal-length strings. */
int or_hamming(const uint8_t* a, const uint8_t* b, int m) {
    int n = 0;
    for (int i = 0; i < m; ++i) n += a[i] != b[i];
    return n;
}

/* Features of one pair for the cost model: [0] = m / 512, [1] = E / 32, and
 * for each diagonal |d| <= min(E, 30), slot 32 + d holds the fraction of the
 * first min(m, 64) columns whose map cell is a match (out-of-range cells are
 * blocked).  Every other slot is zero. */
void or_features(const uint8_t* read, const uint8_t* ref, int m, int E, double* f) {
    for (int i = 0; i < 64; ++i) f[i] = 0.0;
    f[0] = m / 512.0;
    f[1] = E / 32.0;
    int cols = m < 64 ? m : 64;
    int Ef = E < 30 ? E : 30;
    for (int d = -Ef; d <= Ef; ++d) {
        int z = 0;
        for (int c = 0; c < cols; ++c) z += map_cell(read, ref, m, c, d, 1) == 0;
        f[32 + d] = cols > 0 ? (double)z / cols : 0.0;
    }
}

/* Batch driver: pair i has read reads[i*stride ..], ref refs[i*stride ..],
 * length len[i] and threshold E[i].  For each requested filter (bit 0
 * SneakySnake, bit 1 GateKeeper, bit 2 Shouji) writes accept (one byte per
 * pair) and count.  Pairs are independent; they are spread over threads. */
void or_filter_batch(const uint8_t* reads, const uint8_t* refs, uint32_t stride,
                     const uint16_t* len, const uint8_t* E, uint64_t n, uint32_t filters,
                     uint8_t* acc_ss, uint16_t* cnt_ss, uint8_t* acc_gk, uint16_t* cnt_gk,
                     uint8_t* acc_sh, uint16_t* cnt_sh, int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 256)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        const uint8_t* rd = reads + (uint64_t)i * stride;
        const uint8_t* rf = refs + (uint64_t)i * stride;
        int m = len[i], e = E[i], cnt = 0;
        if (filters & 1u) {
            acc_ss[i] = (uint8_t)or_sneakysnake(rd, rf, m, e, &cnt, NULL, 0, NULL);
            cnt_ss[i] = (uint16_t)cnt;
        }
        if (filters & 2u) {
            acc_gk[i] = (uint8_t)or_gatekeeper(rd, rf, m, e, &cnt);
            cnt_gk[i] = (uint16_t)cnt;
        }
        if (filters & 4u) {
            acc_sh[i] = (uint8_t)or_shouji(rd, rf, m, e, &cnt, NULL);
            cnt_sh[i] = (uint16_t)cnt;
        }
    }
}

/* SneakySnake-t over a batch (pairs as in or_filter_batch). */
void or_sneakysnake_t_batch(const uint8_t* reads, const uint8_t* refs, uint32_t stride,
                            const uint16_t* len, const uint8_t* E, uint64_t n, int t,
                            uint8_t* acc, uint16_t* cnt, int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 256)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        int c = 0;
        acc[i] = (uint8_t)or_sneakysnake_t(reads + (uint64_t)i * stride, refs + (uint64_t)i * stride,
                                           len[i], E[i], t, &c);
        cnt[i] = (uint16_t)c;
    }
}

/* Hardware-form SneakySnake over a batch (pairs as in or_filter_batch). */
void or_sneakysnake_fpga_batch(const uint8_t* reads, const uint8_t* refs, uint32_t stride, const uint16_t* len,
                               const uint8_t* E, uint64_t n, int t, int y, uint8_t* acc, uint16_t* cnt,
                               int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 256)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        int c = 0;
        acc[i] = (uint8_t)or_sneakysnake_fpga(reads + (uint64_t)i * stride, refs + (uint64_t)i * stride, len[i],
                                              E[i], t, y, &c);
        cnt[i] = (uint16_t)c;
    }
}

/* Ground-truth batch: min(banded Levenshtein, E + 1) per pair. */
void or_banded_batch(const uint8_t* reads, const uint8_t* refs, uint32_t stride,
                     const uint16_t* len, const uint8_t* E, uint64_t n, uint16_t* dist, int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64)
    for (int64_t i = 0; i < (int64_t)n; ++i)
        dist[i] = (uint16_t)or_banded_levenshtein(reads + (uint64_t)i * stride,
                                                  refs + (uint64_t)i * stride, len[i], E[i]);
}

/* Feature batch (doubles, 64 per pair). */
void or_features_batch(const uint8_t* reads, const uint8_t* refs, uint32_t stride,
                       const uint16_t* len, const uint8_t* E, uint64_t n, double* out, int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1024)
    for (int64_t i = 0; i < (int64_t)n; ++i)
        or_features(reads + (uint64_t)i * stride, refs + (uint64_t)i * stride, len[i], E[i],
                    out + (uint64_t)i * 64);
}
