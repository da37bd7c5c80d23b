"""Verification of filtered pairs on the GPU (banded edit distance by
diagonal transition) against the oracle's banded dynamic programme: every
threshold of the 250 bp workload, the uneven mix with offsets, lengths around
every word edge with E up to 31 and E >= m, selection by SneakySnake's accept
bits (the same result as verifying every pair, since SneakySnake never
rejects a pair within E edits) and by arbitrary bits, and range errors."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import pairgen
import paper_1910_03936_amd as paf
from gpu_util import to_device

pytestmark = pytest.mark.gpu
SS = paf.SNEAKYSNAKE


def _dist(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return paf.counts_u16(t).cpu().numpy().astype(np.uint16)


def _want(p):
    return oracle.banded_batch(p.reads, p.refs, p.len, p.E)


def _check(got, want, label):
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{label}: {bad.size} mismatches, first at {bad[:5]}: gpu {got[bad[:5]]} oracle {want[bad[:5]]}"


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_verify_fixed_250bp(gpu_ctx, E):
    ctx = gpu_ctx
    p = pairgen.generate(pairgen.FIXED_250BP.with_E(E), 51, 64 * 23 + 9)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    want = _want(p)
    _check(_dist(ctx.verify(b)), want, f"E={E} all pairs")
    out = ctx.filter(b, SS)
    _check(_dist(ctx.verify(b, out[SS][0])), want, f"E={E} SneakySnake survivors")
    ctx.check()


def test_verify_uneven_offsets(gpu_ctx):
    ctx = gpu_ctx
    p = pairgen.generate(pairgen.UNEVEN_MIX, 53, 6000)
    want = _want(p)
    for offsets in (True, False):
        b = to_device(p, ctx, per_pair=True, offsets=offsets)
        _check(_dist(ctx.verify(b)), want, f"uneven offsets={offsets}")
        out = ctx.filter(b, SS)
        _check(_dist(ctx.verify(b, out[SS][0])), want, f"uneven survivors offsets={offsets}")
    ctx.check()


def test_verify_selection_bits(gpu_ctx):
    ctx = gpu_ctx
    p = pairgen.generate(pairgen.SMALL_100BP, 57, 3000)
    b = to_device(p, ctx, per_pair=False, offsets=False)
    want = _want(p)
    rng = np.random.default_rng(3)
    sel = rng.random(p.n) < 0.3
    words = np.zeros((p.n + 31) // 32, np.uint32)
    for i in np.nonzero(sel)[0]:
        words[i // 32] |= np.uint32(1 << (i % 32))
    bits = torch.from_numpy(words.view(np.int32)).cuda()
    got = _dist(ctx.verify(b, bits))
    _check(got[sel], want[sel], "selected")
    assert np.all(got[~sel] == p.E[~sel].astype(np.uint16) + 1)
    none = torch.zeros_like(bits)
    assert np.all(_dist(ctx.verify(b, none)) == p.E.astype(np.uint16) + 1)
    ctx.check()


def test_verify_edge_lengths(gpu_ctx):
    ctx = gpu_ctx
    rng = np.random.default_rng(59)
    rows = []
    for m in (1, 2, 3, 31, 32, 33, 63, 64, 65, 96, 97, 255, 256, 257, 511, 512):
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = a.copy()
        b[rng.integers(0, m, max(1, m // 25))] ^= 1
        ins = np.concatenate([a[: m // 2], [1], a[m // 2:]])[:m].astype(np.uint8)
        for ref in (a, b, ins, np.roll(a, 1), np.roll(a, -3), (a + 1) % 4, rng.integers(0, 4, m).astype(np.uint8)):
            for E in sorted({0, 1, 4, 15, min(31, m), min(31, m + 1), 31}):
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
        bq = to_device(q, ctx, per_pair=True, offsets=True, max_len=512, max_E=me)
        _check(_dist(ctx.verify(bq)), _want(q), f"edges max_E={me}")
    ctx.check()


def test_verify_range_violation(gpu_ctx):
    ctx = gpu_ctx
    p = pairgen.generate(pairgen.UNEVEN_MIX, 0, 500)
    E = p.E.copy()
    E[7] = 20
    p2 = pairgen.Pairs(p.reads, p.refs, p.len, E, p.related, p.k)
    b = to_device(p2, ctx, per_pair=True, offsets=True, max_E=15)
    got = _dist(ctx.verify(b))
    with pytest.raises(paf.PafError):
        ctx.check()
    assert got[7] == 0
    mask = np.arange(p.n) != 7
    _check(got[mask], _want(p)[mask], "others")
