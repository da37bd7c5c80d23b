"""Compacting SneakySnake engine (pairs regrouped between 32-column windows)
against the oracle: uniform and per-pair layouts, caller-given orders, both
dead-mask widths, chunk sizes that leave ragged last chunks, and the launch
shapes the autotuner may pick."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import pairgen
import paper_1910_03936_amd as paf
from gpu_util import assert_parity, oracle_for, results, to_device

pytestmark = pytest.mark.gpu
SS = paf.SNEAKYSNAKE


def _layout(wpb, bpc, K, span0=1, span=1):
    return {"lanes_per_pair": 1, "waves_per_block": wpb, "blocks_per_cu": bpc, "tiles_per_grab": 1,
            "chunk_tiles": K, "first_pass_windows": span0, "pass_windows": span}


@pytest.fixture
def ctx(gpu_ctx):
    yield gpu_ctx
    gpu_ctx.set_layout(None)


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_chunk_fixed_250bp(ctx, E):
    w = pairgen.FIXED_250BP.with_E(E)
    p = pairgen.generate(w, 17, 64 * 37 + 5)
    want = oracle_for(p, SS)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    for wpb, K, s0, s1 in ((4, 8, 1, 1), (1, 1, 2, 1), (8, 3, 2, 2), (2, 16, 3, 1), (2, 6, 16, 16)):
        ctx.set_layout(_layout(wpb, 0, K, s0, s1))
        tag = f"E={E} wpb={wpb} K={K} spans={s0},{s1}"
        assert_parity(results(ctx.filter(b, SS), p.n), want, f"plain {tag}")
        assert_parity(results(ctx.filter_persistent(b, SS), p.n), want, f"full grid {tag}")
        ctx.set_layout(_layout(wpb, 2, K, s0, s1))
        assert_parity(results(ctx.filter_persistent(b, SS), p.n), want, f"queue {tag}")
    ctx.check()


def test_chunk_uneven_offsets_and_orders(ctx):
    p = pairgen.generate(pairgen.UNEVEN_MIX, 23, 6000)
    want = oracle_for(p, SS)
    g = torch.Generator().manual_seed(5)
    for offsets in (True, False):
        b = to_device(p, ctx, per_pair=True, offsets=offsets)
        for lay in (_layout(4, 0, 8), _layout(8, 1, 4, 2, 1), _layout(1, 4, 16, 1, 2)):
            ctx.set_layout(lay)
            assert_parity(results(ctx.filter(b, SS), p.n), want, f"plain {lay}")
            assert_parity(results(ctx.filter_persistent(b, SS), p.n), want, f"persistent {lay}")
            o = torch.randperm(p.n, generator=g).to(torch.int32).cuda()
            assert_parity(results(ctx.filter_ordered(b, o, SS), p.n), want, f"ordered {lay}")
    ctx.check()


def test_chunk_edge_lengths_and_thresholds(ctx):
    """Lengths 1..512 around word edges, E from 0 to 31 (and E >= m), pairs
    that match exactly (pipes that run across every window) and pairs that
    differ everywhere."""
    rng = np.random.default_rng(29)
    rows = []
    for m in (1, 2, 31, 32, 33, 63, 64, 65, 95, 96, 97, 255, 256, 257, 480, 511, 512):
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = a.copy()
        b[rng.integers(0, m, max(1, m // 40))] ^= 2
        for ref in (a, b, np.roll(a, 2), np.roll(a, -3), (a + 1) % 4, rng.integers(0, 4, m).astype(np.uint8)):
            for E in sorted({0, 1, 2, 7, 15, 16, min(31, m - 1), min(31, m), 31}):
                rows.append((a, ref, m, E))
    n = len(rows)
    R = np.zeros((n, 512), np.uint8)
    F = np.zeros((n, 512), np.uint8)
    L = np.zeros(n, np.uint16)
    Ev = np.zeros(n, np.uint8)
    for i, (a, r, m, E) in enumerate(rows):
        R[i, :m], F[i, :m], L[i], Ev[i] = a, r, m, E
    p = pairgen.Pairs(R, F, L, Ev, np.zeros(n, np.uint8), np.zeros(n, np.uint16))
    want = oracle_for(p, SS)
    for me in (15, 31):   # 32-bit and 64-bit dead masks
        sel = np.nonzero(Ev <= me)[0]
        q = pairgen.Pairs(R[sel], F[sel], L[sel], Ev[sel], np.zeros(sel.size, np.uint8),
                          np.zeros(sel.size, np.uint16))
        wq = {SS: (want[SS][0][sel], want[SS][1][sel])}
        b = to_device(q, ctx, per_pair=True, offsets=True, max_len=512, max_E=me)
        for lay in (_layout(4, 0, 8), _layout(2, 2, 5, 2, 3)):
            ctx.set_layout(lay)
            assert_parity(results(ctx.filter(b, SS), q.n), wq, f"edges max_E={me} {lay}")
            assert_parity(results(ctx.filter_persistent(b, SS), q.n), wq, f"edges persistent max_E={me} {lay}")
    ctx.check()


@pytest.mark.parametrize("unrelated", [0.0, 0.5, 0.7])
def test_keyed_sort_taken_and_skipped(ctx, unrelated):
    """Keyed launches sort a chunk's first-pass survivors by key class only
    while they fill at most half of the chunk's list.  Related pairs only
    (nearly all accepted, so nearly all survive the first 64 columns and
    every chunk skips the sort), an even mix (chunks on both sides of half)
    and the benchmark's 70% unrelated mix (about 30% survive: sorted), each
    under several chunk sizes, against the oracle."""
    w = pairgen.Workload("keyed sort", 64 * 53 + 7, (250,), 8, unrelated, fixed_E=10, seed=4242)
    p = pairgen.generate(w, 0, w.n_pairs)
    want = oracle_for(p, SS)
    if unrelated == 0.0:
        # An accepted pair is still undecided after the first pass (64 of
        # its 250 columns).
        assert float((np.asarray(want[SS][0]) == 1).mean()) > 0.99
    b = to_device(p, ctx, per_pair=False, offsets=False)
    g = torch.Generator().manual_seed(3)
    key = torch.randint(0, 16, (p.n,), generator=g, dtype=torch.uint8).cuda()
    for lay in (None, _layout(2, 0, 6, 2, 3), _layout(2, 0, 2, 2, 3), _layout(4, 2, 16, 1, 2)):
        ctx.set_layout(lay)
        assert_parity(results(ctx.filter_keyed(b, key), p.n), want, f"keyed unrelated={unrelated} {lay}")
    ctx.check()


@pytest.mark.parametrize("n", [1, 63, 64, 65, 511, 512, 513])
def test_chunk_tiny_batches(ctx, n):
    p = pairgen.generate(pairgen.FIXED_250BP, 300, n)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    want = oracle_for(p, SS)
    assert_parity(results(ctx.filter(b, SS), n), want, f"n={n}")
    ctx.set_layout(_layout(8, 0, 16))
    assert_parity(results(ctx.filter(b, SS), n), want, f"n={n} K=16")


def test_chunk_range_violation(ctx):
    """A pair outside the batch's bounds: count 0, reject, sticky flag; the
    other pairs are unaffected."""
    p = pairgen.generate(pairgen.UNEVEN_MIX, 0, 700)
    E = p.E.copy()
    E[100] = 20
    p2 = pairgen.Pairs(p.reads, p.refs, p.len, E, p.related, p.k)
    b = to_device(p2, ctx, per_pair=True, offsets=True, max_E=15)
    got = results(ctx.filter(b, SS), p.n)
    with pytest.raises(paf.PafError):
        ctx.check()
    assert got[SS][0][100] == 0 and got[SS][1][100] == 0
    want = oracle_for(p, SS)
    mask = np.arange(p.n) != 100
    assert np.array_equal(got[SS][1][mask], want[SS][1][mask])
    assert np.array_equal(got[SS][0][mask], want[SS][0][mask])


def _layout2(wpb, bpc, K, span0=1, span=1):
    return {"lanes_per_pair": 2, "waves_per_block": wpb, "blocks_per_cu": bpc, "tiles_per_grab": 1,
            "chunk_tiles": K, "first_pass_windows": span0, "pass_windows": span}


@pytest.mark.parametrize("E", [9, 10, 12, 15, 20, 25, 31])
def test_two_lanes_per_pair_fixed_250bp(ctx, E):
    """A pair's diagonals split between two lanes (whole maze, max_E 9 and
    up): bit-exact against the oracle under full-grid and queue layouts, chunk
    sizes and pass widths, with a ragged last chunk."""
    w = pairgen.FIXED_250BP.with_E(E)
    p = pairgen.generate(w, 29, 64 * 23 + 17)
    want = oracle_for(p, SS)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    for wpb, bpc, K, s0, s1 in ((2, 0, 6, 2, 3), (4, 0, 1, 1, 1), (1, 2, 3, 2, 2), (4, 1, 16, 3, 1)):
        ctx.set_layout(_layout2(wpb, bpc, K, s0, s1))
        tag = f"E={E} lpp=2 wpb={wpb} bpc={bpc} K={K} spans={s0},{s1}"
        assert_parity(results(ctx.filter(b, SS), p.n), want, f"plain {tag}")
        assert_parity(results(ctx.filter_persistent(b, SS), p.n), want, f"persistent {tag}")
    ctx.check()


def test_two_lanes_per_pair_uneven_orders_and_keys(ctx):
    p = pairgen.generate(pairgen.UNEVEN_MIX, 31, 5000)
    want = oracle_for(p, SS)
    g = torch.Generator().manual_seed(9)
    for offsets in (True, False):
        b = to_device(p, ctx, per_pair=True, offsets=offsets)
        for lay in (_layout2(2, 0, 6, 2, 2), _layout2(4, 2, 4, 1, 2)):
            ctx.set_layout(lay)
            assert_parity(results(ctx.filter(b, SS), p.n), want, f"plain {lay}")
            assert_parity(results(ctx.filter_persistent(b, SS), p.n), want, f"persistent {lay}")
            o = torch.randperm(p.n, generator=g).to(torch.int32).cuda()
            assert_parity(results(ctx.filter_ordered(b, o, SS), p.n), want, f"ordered {lay}")
            key = torch.randint(0, 16, (p.n,), generator=g, dtype=torch.uint8).cuda()
            assert_parity(results(ctx.filter_keyed(b, key), p.n), want, f"keyed {lay}")
    ctx.check()


def test_two_lanes_per_pair_word_edges_and_small_thresholds(ctx):
    """Lengths around every word edge with per-pair thresholds 0..31 under a
    launch bound of 31 (pairs with E below 9 run with the two-lane split
    too), and the error for a batch whose bound is below 9."""
    rng = np.random.default_rng(3)
    n = 3000
    lens = rng.choice([1, 2, 31, 32, 33, 63, 64, 65, 96, 127, 128, 129, 255, 256, 257, 300, 511, 512], n)
    Es = rng.integers(0, 32, n)
    reads = rng.integers(0, 4, (n, 512)).astype(np.uint8)
    refs = reads.copy()
    flip = rng.random((n, 512)) < 0.05
    refs[flip] = (refs[flip] + 1) % 4
    p = pairgen.Pairs(reads, refs, lens.astype(np.uint16), Es.astype(np.uint8), np.ones(n, np.uint8),
                      np.zeros(n, np.uint16))
    want = oracle_for(p, SS)
    b = to_device(p, ctx, per_pair=True, offsets=True, max_len=512, max_E=31)
    ctx.set_layout(_layout2(2, 0, 4, 2, 2))
    assert_parity(results(ctx.filter(b, SS), p.n), want, "word edges, lpp=2")
    small = pairgen.generate(pairgen.FIXED_250BP.with_E(5), 0, 200)
    bs = to_device(small, ctx, per_pair=False, offsets=False)
    with pytest.raises(paf.PafError):
        ctx.filter(bs, SS)
    ctx.set_layout(None)
    ctx.check()
