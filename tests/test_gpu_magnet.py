"""MAGNET on the GPU against the oracle: every threshold of the 250 bp
workload, the uneven mix with and without offsets, lengths around every word
edge (runs that reach the last word's top), E >= m, exact matches, isolated
substitutions, batches large enough that lanes take new pairs as they finish,
and a range violation."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import pairgen
import paper_1910_03936_amd as paf
from gpu_util import assert_parity, results, to_device

pytestmark = pytest.mark.gpu
SS = paf.SNEAKYSNAKE


def _want(p):
    return {SS: oracle.magnet_batch(p.reads, p.refs, p.len, p.E)}


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_magnet_fixed_250bp(gpu_ctx, E):
    p = pairgen.generate(pairgen.FIXED_250BP.with_E(E), 61, 64 * 21 + 11)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    assert_parity(results(gpu_ctx.filter_magnet(b), p.n), _want(p), f"E={E}")
    gpu_ctx.check()


def test_magnet_uneven_offsets(gpu_ctx):
    p = pairgen.generate(pairgen.UNEVEN_MIX, 67, 4000)
    # also with every threshold at most 7 (the first test then stages the
    # tile's words in LDS)
    low = pairgen.Pairs(p.reads, p.refs, p.len, np.minimum(p.E, 7).astype(p.E.dtype), p.related, p.k)
    for q, tag in ((p, "E<=15"), (low, "E<=7")):
        want = _want(q)
        for offsets in (True, False):
            b = to_device(q, gpu_ctx, per_pair=True, offsets=offsets)
            assert_parity(results(gpu_ctx.filter_magnet(b), q.n), want, f"uneven {tag} offsets={offsets}")
    gpu_ctx.check()


def test_magnet_edge_lengths(gpu_ctx):
    rng = np.random.default_rng(71)
    rows = []
    for m in (1, 2, 3, 31, 32, 33, 63, 64, 65, 96, 97, 255, 256, 257, 511, 512):
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = a.copy()
        b[rng.integers(0, m, max(1, m // 30))] ^= 2
        per = np.array([i % 4 for i in range(m)], np.uint8)
        sub = per.copy()
        sub[rng.integers(0, m, max(1, m // 20))] ^= 2
        ins = np.concatenate([a[: m // 3], [3], a[m // 3:]])[:m].astype(np.uint8)
        for read, ref in ((a, a), (a, b), (a, ins), (a, np.roll(a, 2)), (sub, per), (a, (a + 1) % 4),
                          (a, rng.integers(0, 4, m).astype(np.uint8))):
            for E in sorted({0, 1, 3, 9, 15, min(31, m), min(31, m + 2), 31}):
                rows.append((read, ref, m, E))
    n = len(rows)
    R = np.zeros((n, 512), np.uint8)
    F = np.zeros((n, 512), np.uint8)
    L = np.zeros(n, np.uint16)
    Ev = np.zeros(n, np.uint8)
    for i, (a, r, m, E) in enumerate(rows):
        R[i, :m], F[i, :m], L[i], Ev[i] = a, r, m, E
    # max_E 0: the first test decides every pair (no list, no extraction).
    for me in (0, 7, 15, 31):
        sel = np.nonzero(Ev <= me)[0]
        q = pairgen.Pairs(R[sel], F[sel], L[sel], Ev[sel], np.zeros(sel.size, np.uint8),
                          np.zeros(sel.size, np.uint16))
        b = to_device(q, gpu_ctx, per_pair=True, offsets=True, max_len=512, max_E=me)
        assert_parity(results(gpu_ctx.filter_magnet(b), q.n), _want(q), f"edges max_E={me}")
    gpu_ctx.check()


@pytest.mark.parametrize("lens", [(260,), (100, 150, 250)])
def test_magnet_refill_large_batch(gpu_ctx, lens):
    # A wave's share of the undecided list exceeds its 64 lanes only in large
    # batches (the grid is capped at what fits the chip), so only these make
    # lanes take new pairs as they finish.  Related pairs only, so that most
    # pairs pass the first test; 260 bp pairs keep 16 words per sequence in
    # registers, the mix 8; per-pair lengths and thresholds, word offsets.
    n = 1_000_000
    w = pairgen.Workload("related pairs, E = floor(0.05 m), k <= 20", n, lens, 20, 0.0,
                         e_num=5, e_den=100, seed=pairgen.SEED_BASE + 41)
    p = pairgen.generate(w, 0, n)
    b = to_device(p, gpu_ctx, per_pair=True, offsets=True)
    acc, cnt = results(gpu_ctx.filter_magnet(b), n)[SS]
    gpu_ctx.check()
    E = p.E.astype(np.int64)
    assert np.all(cnt.astype(np.int64) <= E + 1)
    assert np.array_equal(acc.astype(bool), cnt.astype(np.int64) <= E)
    ids = pairgen.sample_ids(n, 20000)
    wa, wc = oracle.magnet_batch(p.reads[ids], p.refs[ids], p.len[ids], p.E[ids])
    bad = np.nonzero((acc[ids] != wa) | (cnt[ids] != wc))[0]
    assert bad.size == 0, (f"{bad.size} of {ids.size} sampled pairs differ, first id {ids[bad[0]]}: "
                           f"gpu {acc[ids[bad[0]]]},{cnt[ids[bad[0]]]} oracle {wa[bad[0]]},{wc[bad[0]]}")
    # every accepted pair (E > 0 here) went through the extraction kernel
    assert (cnt <= E).mean() > 0.3


def test_magnet_range_violation(gpu_ctx):
    p = pairgen.generate(pairgen.UNEVEN_MIX, 0, 300)
    E = p.E.copy()
    E[11] = 20
    p2 = pairgen.Pairs(p.reads, p.refs, p.len, E, p.related, p.k)
    b = to_device(p2, gpu_ctx, per_pair=True, offsets=True, max_E=15)
    got = results(gpu_ctx.filter_magnet(b), p.n)
    with pytest.raises(paf.PafError):
        gpu_ctx.check()
    assert got[SS][0][11] == 0 and got[SS][1][11] == 0
    want = _want(p)
    mask = np.arange(p.n) != 11
    assert np.array_equal(got[SS][1][mask], want[SS][1][mask])
    assert np.array_equal(got[SS][0][mask], want[SS][0][mask])
