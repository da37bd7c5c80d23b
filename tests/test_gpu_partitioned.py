"""SneakySnake on a column-partitioned maze (sub-mazes of t columns, each
solved on its own) on the compacting engine, against the oracle: the
thesis's partition widths 5, 10, 25 and 50 at every threshold of the 250 bp
workload, widths on and around the 32-column window edges, the uneven mix with
per-pair thresholds and offsets, lengths around every word edge, and range
errors."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
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


def _want(p, t):
    a, c = oracle.sneakysnake_t_batch(p.reads, p.refs, p.len, p.E, t)
    return {SS: (a, c)}


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_partitioned_fixed_250bp(ctx, E):
    p = pairgen.generate(pairgen.FIXED_250BP.with_E(E), 41, 64 * 29 + 7)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    for t in (1, 5, 10, 25, 31, 32, 33, 50, 64, 100):
        want = _want(p, t)
        assert_parity(results(ctx.filter_partitioned(b, t), p.n), want, f"E={E} t={t}")
        for lay in (_layout(4, 0, 8), _layout(1, 0, 3, 2, 3)):
            ctx.set_layout(lay)
            assert_parity(results(ctx.filter_partitioned(b, t), p.n), want, f"E={E} t={t} {lay}")
        ctx.set_layout(None)
    # One sub-maze: the whole maze.
    whole = oracle_for(p, SS)
    for t in (250, 256, 512, paf.MAX_PART):
        assert_parity(results(ctx.filter_partitioned(b, t), p.n), whole, f"E={E} t={t} whole maze")
    ctx.check()


def test_partitioned_uneven_offsets(ctx):
    p = pairgen.generate(pairgen.UNEVEN_MIX, 43, 5000)
    for offsets in (True, False):
        b = to_device(p, ctx, per_pair=True, offsets=offsets)
        for t in (3, 5, 10, 25, 50):
            assert_parity(results(ctx.filter_partitioned(b, t), p.n), _want(p, t), f"uneven t={t} off={offsets}")
    ctx.check()


def test_partitioned_edge_lengths(ctx):
    rng = np.random.default_rng(47)
    rows = []
    for m in (1, 2, 5, 31, 32, 33, 63, 64, 65, 96, 97, 255, 256, 257, 511, 512):
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = a.copy()
        b[rng.integers(0, m, max(1, m // 30))] ^= 1
        for ref in (a, b, np.roll(a, 1), np.roll(a, -2), (a + 3) % 4, rng.integers(0, 4, m).astype(np.uint8)):
            for E in sorted({0, 2, 9, 15, min(31, m), 31}):
                rows.append((a, ref, m, E))
    n = len(rows)
    R = np.zeros((n, 512), np.uint8)
    F = np.zeros((n, 512), np.uint8)
    L = np.zeros(n, np.uint16)
    Ev = np.zeros(n, np.uint8)
    for i, (a, r, m, E) in enumerate(rows):
        R[i, :m], F[i, :m], L[i], Ev[i] = a, r, m, E
    for me in (15, 31):
        sel = np.nonzero(Ev <= me)[0]
        q = pairgen.Pairs(R[sel], F[sel], L[sel], Ev[sel], np.zeros(sel.size, np.uint8),
                          np.zeros(sel.size, np.uint16))
        b = to_device(q, ctx, per_pair=True, offsets=True, max_len=512, max_E=me)
        for t in (1, 2, 5, 16, 31, 32, 33, 100, 300):
            assert_parity(results(ctx.filter_partitioned(b, t), q.n), _want(q, t), f"edges max_E={me} t={t}")
    ctx.check()


def test_partitioned_range_errors(ctx):
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 100)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    for t in (0, paf.MAX_PART + 1):
        with pytest.raises(paf.PafError):
            ctx.filter_partitioned(b, t)


def _want_fpga(p, t, y):
    a, c = oracle.sneakysnake_fpga_batch(p.reads, p.refs, p.len, p.E, t, y)
    return {SS: (a, c)}


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_hardware_form_fixed_250bp(ctx, E):
    """The hardware form (t-column sub-mazes, y replications each) against the
    oracle that follows its steps: leading-zero counts, maximum, shift."""
    p = pairgen.generate(pairgen.FIXED_250BP.with_E(E), 73, 64 * 19 + 3)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    for t, y in ((8, 3), (8, 1), (8, 2), (5, 1), (10, 3), (32, 4), (33, 2), (64, 31)):
        want = _want_fpga(p, t, y)
        assert_parity(results(ctx.filter_partitioned(b, t, y), p.n), want, f"E={E} t={t} y={y}")
        ctx.set_layout(_layout(2, 0, 5, 2, 3))
        assert_parity(results(ctx.filter_partitioned(b, t, y), p.n), want, f"E={E} t={t} y={y} spans 2,3")
        ctx.set_layout(None)
    ctx.check()


def test_hardware_form_uneven_and_edges(ctx):
    p = pairgen.generate(pairgen.UNEVEN_MIX, 79, 4000)
    b = to_device(p, ctx, per_pair=True, offsets=True)
    for t, y in ((8, 3), (5, 2), (16, 1)):
        assert_parity(results(ctx.filter_partitioned(b, t, y), p.n), _want_fpga(p, t, y), f"uneven t={t} y={y}")
    rng = np.random.default_rng(83)
    rows = []
    for m in (1, 7, 8, 9, 31, 32, 33, 64, 65, 255, 256, 257, 512):
        a = rng.integers(0, 4, m).astype(np.uint8)
        b2 = a.copy()
        b2[rng.integers(0, m, max(1, m // 12))] ^= 1
        for ref in (a, b2, np.roll(a, 1), (a + 2) % 4):
            for E in sorted({0, 3, 15, min(31, m), 31}):
                rows.append((a, ref, m, E))
    n = len(rows)
    R = np.zeros((n, 512), np.uint8)
    F = np.zeros((n, 512), np.uint8)
    L = np.zeros(n, np.uint16)
    Ev = np.zeros(n, np.uint8)
    for i, (a, r, m, E) in enumerate(rows):
        R[i, :m], F[i, :m], L[i], Ev[i] = a, r, m, E
    q = pairgen.Pairs(R, F, L, Ev, np.zeros(n, np.uint8), np.zeros(n, np.uint16))
    bq = to_device(q, ctx, per_pair=True, offsets=True, max_len=512, max_E=31)
    for t, y in ((8, 3), (1, 1), (3, 2), (40, 5)):
        assert_parity(results(ctx.filter_partitioned(bq, t, y), q.n), _want_fpga(q, t, y), f"edges t={t} y={y}")
    with pytest.raises(paf.PafError):
        ctx.filter_partitioned(bq, 8, paf.MAX_REPL + 1)
    ctx.check()
