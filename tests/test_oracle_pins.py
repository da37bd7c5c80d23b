"""Pins of the CPU oracle against what the thesis and the mathematics fix.

Each check comes from outside the oracle's own code: the thesis's worked
examples (tests/golden), closed forms, textbook special cases, brute force on
tiny inputs, and invariants that a dropped term, a wrong sign or a transposed
operand would break."""
import itertools

import numpy as np
import pytest

import oracle
import pairgen
from tests.conftest import read_golden

enc = pairgen.encode


# ---------------------------------------------------------------- worked examples
def test_sneakysnake_fig8_worked_example():
    g = read_golden("sneakysnake_fig8.txt")
    ref, read, E = g["ref"], g["read"], int(g["E"])
    acc, cnt, pipes = oracle.sneakysnake(enc(read), enc(ref), E, with_pipes=True)
    assert acc == bool(int(g["accept"]))
    assert cnt == int(g["obstacles"])
    # The bases each followed pipe covers (columns run along the reference).
    spelled = [ref[c:c + L] for (c, d, L) in pipes]
    assert spelled == g["pipes"].split(",")
    # The reference bases of each pipe equal the read bases on its diagonal.
    for c, d, L in pipes:
        assert ref[c:c + L] == read[c + d:c + d + L]


def test_sneakysnake_orientation_matters():
    # Traversing along the read (swapping the roles) gives other pipes, so the
    # worked example does fix the orientation.
    g = read_golden("sneakysnake_fig8.txt")
    _, _, pipes = oracle.sneakysnake(enc(g["ref"]), enc(g["read"]), int(g["E"]), with_pipes=True)
    spelled = [g["read"][c:c + L] for (c, d, L) in pipes]
    assert spelled != g["pipes"].split(",")


def test_shouji_fig6_worked_example():
    g = read_golden("shouji_fig6.txt")
    T, P, E = g["text"], g["pattern"], int(g["E"])
    acc, cnt, S = oracle.shouji(enc(P), enc(T), E, with_vector=True)
    runs = []
    c = 0
    while c < len(S):
        if S[c] == "0":
            a = c
            while c < len(S) and S[c] == "0":
                c += 1
            runs.append(T[a:c])
        else:
            c += 1
    assert runs == g["common"].split(",")
    assert cnt == len(T) - sum(len(r) for r in runs)
    assert acc


def test_levenshtein_not_additive_example():
    g = read_golden("prefix_cgcg.txt")
    a, b = enc(g["a"]), enc(g["b"])
    assert oracle.hamming(a, b) == int(g["per_base"])
    assert oracle.levenshtein(a, b) == int(g["distance"])
    assert oracle.banded_levenshtein(a, b, 2) == int(g["distance"])
    assert oracle.banded_levenshtein(a, b, 1) == 2  # band of 1 also reaches 2 (shift by one)


def test_amend_rules():
    with open("tests/golden/amend_srs.txt") as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            src, dst = [s.strip() for s in line.split("->")]
            got = oracle.amend(np.array([int(ch) for ch in src], np.uint8))
            assert "".join(str(int(v)) for v in got) == dst, src


def test_lzc_tile_example_as_single_diagonal():
    g = read_golden("lzc_tile.txt")
    row = g["row_msb_first"][::-1]          # column c = bit c
    m = len(row)
    # Periodic ACGT reference: every shifted comparison mismatches, so only the
    # main diagonal carries pipes.  Read = reference with a substitution at
    # each 1-bit, chosen to match neither neighbour diagonal.
    ref = [i % 4 for i in range(m)]
    read = list(ref)
    for c, bit in enumerate(row):
        if bit == "1":
            read[c] = (ref[c] + 2) % 4
    acc, cnt, pipes = oracle.sneakysnake(np.array(read), np.array(ref), 1, with_pipes=True)
    assert [L for (_, d, L) in pipes] == [int(x) for x in g["pipes"].split(",")]
    assert all(d == 0 for (_, d, _) in pipes)
    assert cnt == int(g["obstacles"]) and acc


# ---------------------------------------------------------------- Levenshtein
def _bfs_distance(a, b, limit):
    """Edit distance by breadth-first search over single-edit neighbours (a
    route that shares nothing with the dynamic programme); None if > limit."""
    a, b = tuple(a), tuple(b)
    if a == b:
        return 0
    frontier, seen = {a}, {a}
    for depth in range(1, limit + 1):
        nxt = set()
        for s in frontier:
            n = len(s)
            cands = []
            for i in range(n):
                cands.append(s[:i] + s[i + 1:])
                for x in range(4):
                    if x != s[i]:
                        cands.append(s[:i] + (x,) + s[i + 1:])
            for i in range(n + 1):
                for x in range(4):
                    cands.append(s[:i] + (x,) + s[i:])
            for t in cands:
                if t == b:
                    return depth
                if t not in seen:
                    seen.add(t)
                    nxt.add(t)
        frontier = nxt
    return None


def test_levenshtein_against_bfs():
    rng = np.random.default_rng(1)
    for _ in range(300):
        m = int(rng.integers(1, 6))
        a = rng.integers(0, 4, m)
        # b: a with up to 3 random edits, so short distances are well covered
        b = list(a)
        for _ in range(int(rng.integers(0, 4))):
            kind = rng.integers(0, 3)
            if kind == 0 and b:
                i = rng.integers(0, len(b)); b[i] = (b[i] + 1 + rng.integers(0, 3)) % 4
            elif kind == 1:
                b.insert(int(rng.integers(0, len(b) + 1)), int(rng.integers(0, 4)))
            elif b:
                b.pop(int(rng.integers(0, len(b))))
        d = _bfs_distance(a, b, 2)
        got = oracle.levenshtein(np.array(a), np.array(b, dtype=np.uint8))
        if d is None:
            assert got > 2
        else:
            assert got == d


def test_banded_equals_full_within_band():
    rng = np.random.default_rng(2)
    for _ in range(400):
        m = int(rng.integers(1, 20))
        a = rng.integers(0, 4, m)
        b = a.copy()
        for _ in range(int(rng.integers(0, 6))):
            b[int(rng.integers(0, m))] = rng.integers(0, 4)
        if rng.random() < 0.5 and m > 2:  # an indel pair keeping the length
            i, j = sorted(rng.integers(0, m, 2))
            b = np.concatenate([b[:i], b[i + 1:j + 1], [rng.integers(0, 4)], b[j + 1:]])[:m]
        E = int(rng.integers(0, 6))
        full = oracle.levenshtein(a, b)
        band = oracle.banded_levenshtein(a, b, E)
        if full <= E:
            assert band == full
        else:
            assert band == E + 1
        assert band <= E + 1


# ---------------------------------------------------------------- SneakySnake
def _all_pairs(m):
    seqs = np.array(list(itertools.product(range(4), repeat=m)), np.uint8)
    idx = np.array(list(itertools.product(range(len(seqs)), repeat=2)))
    return seqs[idx[:, 0]], seqs[idx[:, 1]]


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_sneakysnake_never_rejects_within_E_exhaustive(m):
    reads, refs = _all_pairs(m)
    n = reads.shape[0]
    for E in range(0, m + 2):
        ss = oracle.filter_batch(reads, refs, np.full(n, m), np.full(n, E))[1]
        band = oracle.banded_batch(reads, refs, np.full(n, m), np.full(n, E))
        acc, cnt = ss
        # Lower bound: the obstacle count never exceeds the banded distance.
        assert np.all(cnt.astype(int) <= band.astype(int))
        # Hence zero false rejects.
        assert np.all(acc[band <= E] == 1)
        assert np.all((cnt <= E) == (acc == 1))


def test_sneakysnake_lower_bound_random_16():
    rng = np.random.default_rng(3)
    n, m = 20000, 16
    reads = rng.integers(0, 4, (n, m)).astype(np.uint8)
    refs = reads.copy()
    for i in range(n):
        for _ in range(rng.integers(0, 5)):
            kind = rng.integers(0, 3)
            r = list(refs[i])
            if kind == 0:
                j = rng.integers(0, m); r[j] = (r[j] + 1 + rng.integers(0, 3)) % 4
            elif kind == 1:
                r.insert(int(rng.integers(0, m + 1)), int(rng.integers(0, 4))); r = r[:m]
            else:
                r.pop(int(rng.integers(0, m))); r.append(int(rng.integers(0, 4)))
            refs[i] = r
    for E in (0, 1, 2, 3, 5):
        acc, cnt = oracle.filter_batch(reads, refs, np.full(n, m), np.full(n, E))[1]
        band = oracle.banded_batch(reads, refs, np.full(n, m), np.full(n, E))
        assert np.all(cnt.astype(int) <= band.astype(int))
        assert np.all(acc[band <= E] == 1)


def test_sneakysnake_E0_is_hamming_capped():
    # With one diagonal the snake stops at the first mismatch: min(H, 1).
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 3000)
    acc, cnt = oracle.filter_batch(p.reads, p.refs, p.len, 0)[1]
    ham = (p.reads != p.refs).sum(1)
    assert np.array_equal(cnt, np.minimum(ham, 1))
    assert np.array_equal(acc, (ham == 0).astype(np.uint8))


def test_sneakysnake_bounded_by_hamming_and_identical_zero():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 3000)
    for E in (1, 5, 12):
        acc, cnt = oracle.filter_batch(p.reads, p.refs, p.len, E)[1]
        ham = (p.reads != p.refs).sum(1)
        assert np.all(cnt <= np.minimum(ham, E + 1))
    acc, cnt = oracle.filter_batch(p.reads, p.reads, p.len, 5)[1]
    assert np.all(cnt == 0) and np.all(acc == 1)


def test_weighted_equals_unweighted():
    p = pairgen.generate(pairgen.FIXED_250BP, 0, 600)
    for i in range(p.n):
        for E in (0, 3, 10):
            a = oracle.sneakysnake(p.reads[i], p.refs[i], E)
            b = oracle.sneakysnake_weighted(p.reads[i], p.refs[i], E)
            assert a == b


def test_sneakysnake_monotone_in_E():
    p = pairgen.generate(pairgen.FIXED_250BP, 0, 4000)
    prev = None
    for E in range(0, 16):
        acc, _ = oracle.filter_batch(p.reads, p.refs, p.len, E)[1]
        if prev is not None:
            assert np.all(acc >= prev)
        prev = acc


def test_sneakysnake_E_at_least_m_accepts():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 200)
    short = p.reads[:, :7].copy(), p.refs[:, :7].copy()
    acc, cnt = oracle.filter_batch(short[0], short[1], np.full(200, 7), 7)[1]
    # 2E+1 diagonals cover every cell; the greedy needs at most m - 1 ... but
    # the count is still bounded by the banded distance <= m.
    band = oracle.banded_batch(short[0], short[1], np.full(200, 7), 7)
    assert np.all(acc[band <= 7] == 1)


# ---------------------------------------------------------------- GateKeeper
def test_gatekeeper_E0_is_exact_match():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 3000)
    acc, cnt = oracle.filter_batch(p.reads, p.refs, p.len, 0, oracle.GATEKEEPER)[2]
    ham = (p.reads != p.refs).sum(1)
    assert np.array_equal(acc, (ham == 0).astype(np.uint8))


def test_gatekeeper_fast_path_and_amended_count():
    # Substitution-only pair whose Hamming distance is <= E: Method 1 accepts
    # with count = Hamming distance.
    rng = np.random.default_rng(5)
    a = rng.integers(0, 4, 100).astype(np.uint8)
    b = a.copy()
    for j in (10, 40, 77):
        b[j] = (b[j] + 1) % 4
    assert oracle.gatekeeper(a, b, 3) == (True, 3)
    # E = 0 on a pair whose main-diagonal mask is 1 0 1 0 0 1 ...: the reject
    # count is the popcount of the amended mask (Sec. 5.2.2 rule).
    mask = np.array([int(c) for c in "0110100111000101"], np.uint8)
    ref = np.zeros(mask.size, np.uint8)
    read = (ref + mask).astype(np.uint8)
    acc, cnt = oracle.gatekeeper(read, ref, 0)
    # Hand-amended: zeros at 3 (101), 5-6 (1001) and 14 (101) flip; 10-12 (a
    # run of 3) stays, and so does 0, which touches the start.
    assert not acc and cnt == sum(int(c) for c in "0111111111000111")


def test_gatekeeper_identical_is_zero():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 300)
    acc, cnt = oracle.filter_batch(p.reads, p.reads, p.len, 5, oracle.GATEKEEPER)[2]
    assert np.all(cnt == 0) and np.all(acc == 1)


# ---------------------------------------------------------------- Shouji
def test_shouji_E0_is_hamming():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 3000)
    acc, cnt = oracle.filter_batch(p.reads, p.refs, p.len, 0, oracle.SHOUJI)[4]
    ham = (p.reads != p.refs).sum(1)
    assert np.array_equal(cnt.astype(int), ham)


def test_shouji_identical_is_zero_and_count_le_m():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 300)
    acc, cnt = oracle.filter_batch(p.reads, p.reads, p.len, 5, oracle.SHOUJI)[4]
    assert np.all(cnt == 0)
    acc, cnt = oracle.filter_batch(p.reads, p.refs, p.len, 5, oracle.SHOUJI)[4]
    assert np.all(cnt <= 100)


# ---------------------------------------------------------------- features
def test_features_closed_form():
    # All-A pair of length 10, E = 3: every in-range cell matches, so the match
    # fraction of diagonal d is (10 - |d|) / 10.
    a = np.zeros(10, np.uint8)
    f = oracle.features(a, a, 3)
    assert f[0] == 10 / 512 and f[1] == 3 / 32
    for d in range(-3, 4):
        assert f[32 + d] == pytest.approx((10 - abs(d)) / 10)
    assert np.count_nonzero(f) == 2 + 7
    # Only the first 64 columns count: a 100-base pair that differs only after
    # column 64 has main-diagonal fraction 1.
    rng = np.random.default_rng(0)
    x = rng.integers(0, 4, 100).astype(np.uint8)
    y = x.copy()
    y[70:] = (y[70:] + 1) % 4
    assert oracle.features(x, y, 5)[32] == 1.0


# ---------------------------------------------------------------- SneakySnake-t
def _maze(read, ref, E):
    """Blocked (1) / free (0) cells of the unweighted maze, rows d = -E..E,
    built with numpy straight from the cell definition."""
    m = len(ref)
    read, ref = np.asarray(read), np.asarray(ref)
    Z = np.ones((2 * E + 1, m), np.uint8)
    for k, d in enumerate(range(-E, E + 1)):
        for c in range(m):
            if 0 <= c + d < m:
                Z[k, c] = int(read[c + d] != ref[c])
    return Z


def _least_obstacles(Z, p0, p1):
    """Fewest obstacles a snake crosses from column p0 to the end of the
    sub-maze [p0, p1), by dynamic programming over every choice of pipe (no
    greedy rule): from a free column it may follow any row to its first
    obstacle (or to the sub-maze's end, at no cost) and cross that obstacle
    for one."""
    f = [0] * (p1 - p0 + 2)
    for c in range(p1 - 1, p0 - 1, -1):
        best = None
        for row in Z:
            r = 0
            while c + r < p1 and row[c + r] == 0:
                r += 1
            cost = 0 if c + r == p1 else 1 + f[c + r + 1 - p0]
            best = cost if best is None else min(best, cost)
        f[c - p0] = best
    return f[0]


def test_sneakysnake_t_greedy_takes_least_obstacles():
    # Sec. 8.6: within each sub-maze the greedy finds the path with the fewest
    # obstacles; the partitioned count is the sum over sub-mazes.
    rng = np.random.default_rng(11)
    for _ in range(600):
        m = int(rng.integers(1, 25))
        E = int(rng.integers(0, 5))
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = a.copy()
        for _ in range(int(rng.integers(0, 6))):
            b[int(rng.integers(0, m))] = rng.integers(0, 4)
        if rng.random() < 0.5 and m > 2:
            i = int(rng.integers(0, m))
            b = np.concatenate([b[:i], b[i + 1:], rng.integers(0, 4, 1)]).astype(np.uint8)
        Z = _maze(a, b, E)
        for t in (1, 2, 3, 5, 7, m, m + 3):
            total = sum(_least_obstacles(Z, p0, min(p0 + t, m)) for p0 in range(0, m, t))
            acc, cnt = oracle.sneakysnake_t(a, b, E, t)
            assert cnt == min(total, E + 1), (m, E, t)
            assert acc == (total <= E)
        # One sub-maze is the whole maze.
        assert oracle.sneakysnake(a, b, E)[1] == min(_least_obstacles(Z, 0, m), E + 1)


def test_sneakysnake_t_single_columns_count_blocked_columns():
    # t = 1: every column is its own sub-maze, which costs one exactly when all
    # of its 2E+1 cells are blocked.
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 300)
    for i in range(p.n):
        for E in (0, 1, 3):
            blocked = int(_maze(p.reads[i], p.refs[i], E).min(0).sum())
            assert oracle.sneakysnake_t(p.reads[i], p.refs[i], E, 1) == (blocked <= E, min(blocked, E + 1))


def test_sneakysnake_t_wide_partition_is_whole_maze():
    p = pairgen.generate(pairgen.FIXED_250BP, 0, 500)
    for E in (0, 5, 10):
        whole = oracle.filter_batch(p.reads, p.refs, p.len, E)[1]
        for t in (250, 251, 512):
            a, c = oracle.sneakysnake_t_batch(p.reads, p.refs, p.len, E, t)
            assert np.array_equal(a, whole[0]) and np.array_equal(c, whole[1])


def test_sneakysnake_t_nested_partitions_and_zero_false_rejects():
    # A partition that refines another can only lose obstacles (each sub-maze
    # path restricted to a finer sub-maze is a path there), so t | t' gives
    # count_t <= count_t' <= the whole maze's count <= the banded distance.
    p = pairgen.generate(pairgen.FIXED_250BP, 1, 2000)
    E = 10
    whole = oracle.filter_batch(p.reads, p.refs, p.len, E)[1][1].astype(int)
    band = oracle.banded_batch(p.reads, p.refs, p.len, E).astype(int)
    c = {t: oracle.sneakysnake_t_batch(p.reads, p.refs, p.len, E, t)[1].astype(int) for t in (5, 10, 25, 50)}
    assert np.all(c[5] <= c[10]) and np.all(c[10] <= c[50]) and np.all(c[25] <= c[50])
    assert np.all(c[50] <= whole) and np.all(whole <= band)
    # ... and on tiny inputs exhaustively, for every partition width.
    reads, refs = _all_pairs(4)
    n = reads.shape[0]
    for E in range(0, 3):
        band = oracle.banded_batch(reads, refs, np.full(n, 4), np.full(n, E)).astype(int)
        for t in (1, 2, 3):
            a, cnt = oracle.sneakysnake_t_batch(reads, refs, np.full(n, 4), np.full(n, E), t)
            assert np.all(cnt.astype(int) <= band) and np.all(a[band <= E] == 1)


def test_sneakysnake_t_E0_is_hamming_capped():
    # One diagonal: every mismatch is an obstacle of its sub-maze.
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 2000)
    ham = (p.reads != p.refs).sum(1)
    for t in (1, 5, 10, 100):
        a, c = oracle.sneakysnake_t_batch(p.reads, p.refs, p.len, 0, t)
        assert np.array_equal(c, np.minimum(ham, 1)) and np.array_equal(a, (ham == 0).astype(np.uint8))


# ---------------------------------------------------------------- MAGNET
def test_magnet_identical_is_one_run():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 50)
    for i in range(p.n):
        for E in (0, 3, 10):
            assert oracle.magnet(p.reads[i], p.reads[i], E, with_segments=True) == (True, 0, [(0, 0, 100)])


def _periodic_with_substitutions(m, subs):
    # Reference ACGTACGT...: every diagonal with |d| in {1, 2, 3} mismatches
    # everywhere.  A substitution to the base two steps on leaves diagonal 0
    # blocked there and adds an isolated free cell on diagonals +-2 only.
    ref = np.array([i % 4 for i in range(m)], np.uint8)
    read = ref.copy()
    for j in subs:
        read[j] = (ref[j] + 2) % 4
    return read, ref


def test_magnet_isolated_substitutions_closed_form():
    # The free runs of diagonal 0 are the gaps between substitutions; MAGNET
    # takes the E+1 longest of them (each is longer than the isolated cells of
    # diagonals +-2), and encapsulation drops exactly the substituted columns.
    # So the uncovered columns are m minus the sum of the E+1 longest gaps.
    rng = np.random.default_rng(21)
    m = 100
    for _ in range(300):
        k = int(rng.integers(0, 9))
        subs = []
        while len(subs) < k:
            j = int(rng.integers(0, m))
            if all(abs(j - q) >= 3 for q in subs):
                subs.append(j)
        subs.sort()
        read, ref = _periodic_with_substitutions(m, subs)
        bounds = [-1] + subs + [m]
        gaps = sorted((b - a - 1 for a, b in zip(bounds, bounds[1:]) if b - a - 1 > 0), reverse=True)
        for E in (1, 2, 3):
            left = m - sum(gaps[:E + 1])
            acc, cnt, segs = oracle.magnet(read, ref, E, with_segments=True)
            assert cnt == min(left, E + 1) and acc == (left <= E), (subs, E)
            assert all(d == 0 for d, _, _ in segs)
            if k <= E:
                assert cnt == k


def test_magnet_E0_accepts_only_exact_matches():
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 2000)
    acc, cnt = oracle.magnet_batch(p.reads, p.refs, p.len, 0)
    ham = (p.reads != p.refs).sum(1)
    assert np.array_equal(acc, (ham == 0).astype(np.uint8))
    assert np.array_equal(cnt, np.minimum(ham, 1))


def test_magnet_runs_are_disjoint_longest_first_and_free():
    # Invariants of extraction + encapsulation: every run found is free on its
    # diagonal, runs never touch (one column at least between them), they come
    # longest first, there are at most E+1, and the count is what they leave.
    p = pairgen.generate(pairgen.SMALL_100BP, 5, 300)
    for i in range(p.n):
        for E in (2, 5):
            acc, cnt, segs = oracle.magnet(p.reads[i], p.refs[i], E, with_segments=True)
            Z = _maze(p.reads[i], p.refs[i], E)
            assert 1 <= len(segs) <= E + 1
            lens = [L for _, _, L in segs]
            assert lens == sorted(lens, reverse=True)
            spans = sorted((s, s + L) for _, s, L in segs)
            assert all(b1 < a2 for (_, b1), (a2, _) in zip(spans, spans[1:]))
            for d, s, L in segs:
                assert not Z[d + E, s:s + L].any()
            left = 100 - sum(lens)
            assert cnt == min(left, E + 1) and acc == (left <= E)


# ---------------------------------------------------------------- hardware form (t columns, y replications)
def test_fpga_tile_worked_example():
    # Sec. 8.6 step 4: one row 00010000 (t = 8) searched by two replications
    # finds x = 4 and x = 3, and the sub-maze holds one obstacle.
    g = read_golden("lzc_tile.txt")
    row = g["row_msb_first"][::-1]
    m = len(row)
    ref = np.array([i % 4 for i in range(m)], np.uint8)
    read = ref.copy()
    for c, bit in enumerate(row):
        if bit == "1":
            read[c] = (ref[c] + 2) % 4
    assert oracle.sneakysnake_fpga(read, ref, 1, 8, 2) == (True, int(g["obstacles"]))
    # One replication finds the first pipe only: min(1, 8 - 4) = 1.
    assert oracle.sneakysnake_fpga(read, ref, 1, 8, 1) == (True, 1)


def test_fpga_tile_counts_least_obstacles_capped_by_replications():
    # Each replication crosses at most one obstacle, and the greedy is optimal
    # in a sub-maze (Sec. 8.6), so a sub-maze counts min(y, its fewest
    # obstacles): checked against the dynamic programme over every pipe.
    rng = np.random.default_rng(31)
    for _ in range(400):
        m = int(rng.integers(1, 30))
        E = int(rng.integers(0, 4))
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = a.copy()
        for _ in range(int(rng.integers(0, 8))):
            b[int(rng.integers(0, m))] = rng.integers(0, 4)
        if rng.random() < 0.5 and m > 2:
            i = int(rng.integers(0, m))
            b = np.concatenate([b[:i], b[i + 1:], rng.integers(0, 4, 1)]).astype(np.uint8)
        Z = _maze(a, b, E)
        for t in (3, 5, 8):
            for y in (1, 2, 3, 8):
                total = sum(min(y, _least_obstacles(Z, p0, min(p0 + t, m))) for p0 in range(0, m, t))
                assert oracle.sneakysnake_fpga(a, b, E, t, y) == (total <= E, min(total, E + 1)), (m, E, t, y)


def test_fpga_tile_enough_replications_is_partitioned_maze():
    p = pairgen.generate(pairgen.SMALL_100BP, 3, 1500)
    for E in (2, 5):
        for t in (5, 8):
            a, c = oracle.sneakysnake_fpga_batch(p.reads, p.refs, p.len, E, t, t)
            a2, c2 = oracle.sneakysnake_t_batch(p.reads, p.refs, p.len, E, t)
            assert np.array_equal(a, a2) and np.array_equal(c, c2)


def test_magnet_first_run_test_is_implied_by_the_final_one():
    # Sec. 7.2 rejects at once when the longest run is shorter than
    # ceil((m - E) / (E + 1)); the E + 1 runs found later are no longer, so
    # such a pair is rejected by the final test anyway (count E + 1).
    p = pairgen.generate(pairgen.SMALL_100BP, 9, 600)
    m = 100
    for E in (2, 5, 9):
        need = -(-(m - E) // (E + 1))
        assert need == m // (E + 1)      # the form the GPU test uses
        for i in range(p.n):
            acc, cnt, segs = oracle.magnet(p.reads[i], p.refs[i], E, with_segments=True)
            if segs[0][2] < need:
                assert not acc and cnt == E + 1


# ---------------------------------------------------------------- decision rules that
# the closed forms above leave open.  Each pin below is also run against a
# deliberately altered copy of the oracle (tests/mutants.py) to show that the
# alteration it is meant to catch makes it fail.
from mutants import mutant  # noqa: E402

GK_OR = ("F[c] = (uint8_t)(F[c] & A[c]);", "F[c] = (uint8_t)(F[c] | A[c]);")
GK_VACANT_ONE = ("G[c] = (uint8_t)map_cell(read, ref, m, c, d, 0);",
                 "G[c] = (uint8_t)map_cell(read, ref, m, c, d, 1);")
GK_SHIFTS_UNAMENDED = ("        amend(G, A, m);\n        for (int c = 0; c < m; ++c) F[c]",
                       "        if (d == 0) amend(G, A, m); else memcpy(A, G, (size_t)m);\n"
                       "        for (int c = 0; c < m; ++c) F[c]")
SH_FIRST_TIED = ("(z > best_z || (z == best_z && lead && !best_lead))", "(z > best_z)")
SH_STORE_ON_EQUAL = ("if (best_z > zs)", "if (best_z >= zs)")
SH_REVERSED_ORDER = ("        for (int d = -E; d <= E; ++d) {\n            uint8_t v[4];",
                     "        for (int d = E; d >= -E; --d) {\n            uint8_t v[4];")
MG_LATER_START = ("if (L > best) { best = L; best_c = c; best_d = d; }",
                  "if (L >= best) { best = L; best_c = c; best_d = d; }")


def _gk_masks(read, ref, E):
    """G_d straight from the definition (Sec. 5.2.2 with SHD's zero fill,
    Sec. 3.2.3): bit c = 1 when ref[c] != read[c + d], vacant read index 0."""
    m = len(ref)
    out = {}
    for d in range(-E, E + 1):
        out[d] = np.array([0 if not 0 <= c + d < m else int(ref[c] != read[c + d]) for c in range(m)], np.uint8)
    return out


def test_gatekeeper_method2_worked_example():
    g = read_golden("gatekeeper_method2.txt")
    ref, read, E = enc(g["ref"]), enc(g["read"]), int(g["E"])
    assert int((ref != read).sum()) == int(g["hamming"])
    # the hand-derived masks of the fixture, from the definition
    G = _gk_masks(read, ref, E)
    F = np.ones(len(ref), np.uint8)
    for d in G:
        F &= oracle.amend(G[d])
    assert "".join(map(str, F)) == g["F"]
    assert oracle.gatekeeper(read, ref, E) == (bool(int(g["accept"])), int(g["count"]))
    for edit, key in ((GK_OR, "count_or"), (GK_VACANT_ONE, "count_vacant_one"),
                      (GK_SHIFTS_UNAMENDED, "count_unamended_shifts")):
        with mutant(edit):
            assert oracle.gatekeeper(read, ref, E)[1] == int(g[key])


def _shifted_pairs(n, m, E, seed):
    """Reads that are the reference shifted by k, 1 <= |k| <= E (the bases
    shifted in are random), with Hamming distance > E."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        ref = rng.integers(0, 4, m).astype(np.uint8)
        k = int(rng.integers(1, E + 1)) * (1 if rng.random() < 0.5 else -1)
        read = rng.integers(0, 4, m).astype(np.uint8)
        for j in range(m):
            if 0 <= j - k < m:
                read[j] = ref[j - k]
        if int((ref != read).sum()) > E:
            out.append((read, ref, k))
    return out


def _gk_shift_pin_holds(cases, E):
    return all(oracle.gatekeeper(read, ref, E) == (True, 0) for read, ref, _ in cases)


@pytest.mark.parametrize("E", [1, 3, 10])
def test_gatekeeper_pure_shift_counts_zero(E):
    # Diagonal d = k matches everywhere and its vacant bits are zeros, so its
    # amended mask is all zeros and so is the AND: count 0, accept, although
    # the Hamming fast path does not apply (Secs. 5.2.1-5.2.2).
    cases = _shifted_pairs(60, 100, E, seed=E)
    assert _gk_shift_pin_holds(cases, E)
    for edit in (GK_OR, GK_VACANT_ONE):
        with mutant(edit):
            assert not _gk_shift_pin_holds(cases, E), edit


def _gk_and_invariant_holds(pairs, E):
    """count <= ones(amend(G_d)) for every d: F is the AND of the amended masks."""
    for read, ref in pairs:
        if int((read != ref).sum()) <= E:
            continue
        cnt = oracle.gatekeeper(read, ref, E)[1]
        for d, G in _gk_masks(read, ref, E).items():
            if cnt > int(oracle.amend(G).sum()):
                return False
    return True


def _gk_zeros_from_long_streaks(pairs, E):
    """Every zero of F sits in a zero streak of some G_d that the amendment
    keeps: three or more zeros, or a streak touching an end."""
    for read, ref in pairs:
        if int((read != ref).sum()) <= E:
            continue
        G = _gk_masks(read, ref, E)
        m = len(ref)
        F = np.ones(m, np.uint8)
        for d in G:
            F &= oracle.amend(G[d])
        if int(F.sum()) != oracle.gatekeeper(read, ref, E)[1]:
            return False
        for c in np.nonzero(F == 0)[0]:
            ok = False
            for g in G.values():
                if g[c]:
                    continue
                a = c
                while a > 0 and g[a - 1] == 0:
                    a -= 1
                b = c
                while b < m - 1 and g[b + 1] == 0:
                    b += 1
                if b - a + 1 >= 3 or a == 0 or b == m - 1:
                    ok = True
                    break
            if not ok:
                return False
    return True


def test_gatekeeper_and_of_amended_shifted_masks():
    p = pairgen.generate(pairgen.SMALL_100BP.with_E(4), 0, 300)
    pairs = [(p.reads[i], p.refs[i]) for i in range(p.n)]
    assert _gk_and_invariant_holds(pairs, 4)
    assert _gk_zeros_from_long_streaks(pairs, 4)
    with mutant(GK_OR):
        assert not _gk_and_invariant_holds(pairs, 4)
    with mutant(GK_SHIFTS_UNAMENDED):
        assert not _gk_zeros_from_long_streaks(pairs, 4)


def test_shouji_tie_break_and_store_rule_worked_example():
    g = read_golden("shouji_tie_store.txt")
    ref, read, E = enc(g["ref"]), enc(g["read"]), int(g["E"])
    assert oracle.shouji(read, ref, E, with_vector=True) == (bool(int(g["accept"])), int(g["count"]), g["S"])
    with mutant(SH_FIRST_TIED):
        assert oracle.shouji(read, ref, E, with_vector=True)[1:] == (int(g["count_first_tied"]), g["S_first_tied"])
    with mutant(SH_STORE_ON_EQUAL):
        assert oracle.shouji(read, ref, E, with_vector=True)[1:] == (int(g["count_store_on_equal"]),
                                                                      g["S_store_on_equal"])
    with mutant(SH_REVERSED_ORDER):
        assert oracle.shouji(read, ref, E, with_vector=True)[1:] == (int(g["count_reversed_order"]),
                                                                      g["S_reversed_order"])


def test_magnet_tie_rule_worked_example():
    g = read_golden("magnet_tie.txt")
    ref, read, E = enc(g["ref"]), enc(g["read"]), int(g["E"])
    segs = [tuple(int(x) for x in s.split(":")) for s in g["segments"].split(",")]
    assert oracle.magnet(read, ref, E, with_segments=True) == (bool(int(g["accept"])), int(g["count"]), segs)
    with mutant(MG_LATER_START):
        assert oracle.magnet(read, ref, E)[1] == int(g["count_later_start_first"])
