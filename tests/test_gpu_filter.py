"""GPU parity of the filter path (through the C ABI) against the CPU oracle.

Element-by-element, bit-exact: accept bits and counts are integers."""
import numpy as np
import pytest
import torch

import oracle
import pairgen
import paper_1910_03936_amd as paf
from tests.gpu_util import assert_parity, oracle_for, results, to_device

pytestmark = pytest.mark.gpu

SS, GK, SH, ALL = paf.SNEAKYSNAKE, paf.GATEKEEPER, paf.SHOUJI, paf.ALL_FILTERS


def test_gpu_pack_matches_host_pack(gpu_ctx):
    p = pairgen.generate(pairgen.UNEVEN_MIX, 0, 777)
    b = to_device(p, gpu_ctx, per_pair=True, offsets=True)
    torch.cuda.synchronize()
    gpu_words = b.reads.cpu().numpy().view(np.uint64)
    off = b.word_offset.cpu().numpy().astype(np.uint64)
    host = np.zeros_like(gpu_words)
    import ctypes
    lib = paf.load_library()
    st = lib.paf_pack_host(p.reads.ctypes.data_as(ctypes.c_void_p), p.stride,
                           p.len.ctypes.data_as(ctypes.c_void_p), 0,
                           off.ctypes.data_as(ctypes.c_void_p), 0, p.n,
                           host.ctypes.data_as(ctypes.c_void_p), 4)
    assert st == 0
    assert np.array_equal(gpu_words, host)
    gpu_ctx.check()


def test_small_100bp_full_snake(gpu_ctx):
    """100 bp, E=5, all 100k pairs of the workload, SneakySnake."""
    p = pairgen.generate(pairgen.SMALL_100BP)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    got = results(gpu_ctx.filter(b, SS), p.n)
    assert_parity(got, oracle_for(p, SS), "100bp")
    gpu_ctx.check()


@pytest.mark.parametrize("E", [0, 5, 10, 20, 25, 31])
def test_fixed_250bp_all_filters(gpu_ctx, E):
    """250 bp at each threshold: SneakySnake alone (compacting engine, in the
    default layout of each threshold class, up to the longer first pass and
    one-window later passes above 15) and all three filters in one call;
    3001 pairs = 46 full tiles and a ragged tail."""
    p = pairgen.generate(pairgen.FIXED_250BP.with_E(E), 0, 3001)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    want = oracle_for(p, ALL)
    assert_parity(results(gpu_ctx.filter(b, SS), p.n), {SS: want[SS]}, f"E={E} snake")
    assert_parity(results(gpu_ctx.filter(b, ALL), p.n), want, f"E={E} whole")
    for f in (GK, SH, GK | SH, SS | SH):
        assert_parity(results(gpu_ctx.filter(b, f), p.n), {k: want[k] for k in want if k & f},
                      f"E={E} mask {f}")
    gpu_ctx.check()


@pytest.mark.parametrize("filters", [SS, ALL])
def test_uneven_per_pair(gpu_ctx, filters):
    """Uneven lengths {64..300} and E = floor(0.05 m), word offsets: plain
    general kernel and the persistent graph launch."""
    p = pairgen.generate(pairgen.UNEVEN_MIX, 5, 4100)
    want = oracle_for(p, filters)
    for offsets in (True, False):
        b = to_device(p, gpu_ctx, per_pair=True, offsets=offsets)
        assert_parity(results(gpu_ctx.filter(b, filters), p.n), want, f"offsets={offsets} plain")
        assert_parity(results(gpu_ctx.filter_persistent(b, filters), p.n), want,
                      f"offsets={offsets} persistent")
        # Replay of the captured graph.
        assert_parity(results(gpu_ctx.filter_persistent(b, filters), p.n), want, "replay")
    gpu_ctx.check()


@pytest.mark.parametrize("lens,E", [((96,), 4), ((180,), 9), ((270,), 10), ((100,), 3), ((250,), 10)])
def test_gatekeeper_alone_window_counts(gpu_ctx, lens, E):
    """GateKeeper alone (its window loop takes three windows per turn) on
    pairs of 3, 6, 9, 4 and 8 words, so that the loop ends at each of its
    three checks; uniform and per-pair layouts, with and without offsets."""
    w = pairgen.Workload("GateKeeper window counts", 3000, lens, 20, 0.5, fixed_E=E,
                         seed=pairgen.SEED_BASE + 51)
    p = pairgen.generate(w, 0, 3000)
    want = oracle_for(p, GK)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    assert_parity(results(gpu_ctx.filter(b, GK), p.n), want, f"m={lens[0]} uniform")
    for offsets in (True, False):
        b = to_device(p, gpu_ctx, per_pair=True, offsets=offsets)
        assert_parity(results(gpu_ctx.filter(b, GK), p.n), want, f"m={lens[0]} per-pair offsets={offsets}")
    # the uneven mix with thresholds capped at E (mixed word counts per wave)
    u = pairgen.generate(pairgen.UNEVEN_MIX, 9, 2100)
    q = pairgen.Pairs(u.reads, u.refs, u.len, np.minimum(u.E, E).astype(u.E.dtype), u.related, u.k)
    b = to_device(q, gpu_ctx, per_pair=True, offsets=True)
    assert_parity(results(gpu_ctx.filter(b, GK), q.n), oracle_for(q, GK), f"uneven E<={E}")
    gpu_ctx.check()


def _edge_pairs():
    rng = np.random.default_rng(11)
    rows = []
    for m in (1, 2, 3, 31, 32, 33, 63, 64, 65, 96, 255, 256, 257, 511, 512):
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = a.copy()
        b[rng.integers(0, m, max(1, m // 20))] ^= 1
        c = np.roll(a, 1)                       # one indel-like shift
        d = (a + 1) % 4                         # every base differs
        for read, ref in ((a, a), (a, b), (a, c), (a, d), (a, rng.integers(0, 4, m).astype(np.uint8))):
            for E in sorted({0, 1, 3, min(31, m - 1), min(31, m), 31}):
                rows.append((read, ref, m, E))
    return rows


def test_edge_cases(gpu_ctx):
    rows = _edge_pairs()
    n = len(rows)
    R = np.zeros((n, 512), np.uint8)
    F = np.zeros((n, 512), np.uint8)
    L = np.zeros(n, np.uint16)
    Ev = np.zeros(n, np.uint8)
    for i, (a, b, m, E) in enumerate(rows):
        R[i, :m], F[i, :m], L[i], Ev[i] = a, b, m, E
    p = pairgen.Pairs(R, F, L, Ev, np.zeros(n, np.uint8), np.zeros(n, np.uint16))
    want = oracle_for(p, ALL)
    b = to_device(p, gpu_ctx, per_pair=True, offsets=True, max_len=512, max_E=31)
    assert_parity(results(gpu_ctx.filter(b, SS), n), {SS: want[SS]}, "edge snake")
    assert_parity(results(gpu_ctx.filter(b, ALL), n), want, "edge whole")
    assert_parity(results(gpu_ctx.filter_persistent(b, ALL), n), want, "edge persistent")
    gpu_ctx.check()


def test_edge_cases_E0(gpu_ctx):
    """The one-diagonal kernels (max_E 0; Shouji's count there in closed
    form) on the edge lengths 1..512: each filter alone and all three."""
    rows = [r for r in _edge_pairs() if r[3] == 0]
    n = len(rows)
    R = np.zeros((n, 512), np.uint8)
    F = np.zeros((n, 512), np.uint8)
    L = np.zeros(n, np.uint16)
    for i, (a, b, m, E) in enumerate(rows):
        R[i, :m], F[i, :m], L[i] = a, b, m
    p = pairgen.Pairs(R, F, L, np.zeros(n, np.uint8), np.zeros(n, np.uint8), np.zeros(n, np.uint16))
    want = oracle_for(p, ALL)
    b = to_device(p, gpu_ctx, per_pair=True, offsets=True, max_len=512, max_E=0)
    for f in (SS, GK, SH, GK | SH, ALL):
        assert_parity(results(gpu_ctx.filter(b, f), n), {k: want[k] for k in want if k & f}, f"E=0 mask {f}")
    gpu_ctx.check()


@pytest.mark.parametrize("n", [1, 63, 64, 65])
def test_tiny_batches(gpu_ctx, n):
    p = pairgen.generate(pairgen.FIXED_250BP, 100, n)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    assert_parity(results(gpu_ctx.filter(b, ALL), n), oracle_for(p, ALL), f"n={n}")


def test_device_range_violation_sets_flag(gpu_ctx):
    """A pair whose E exceeds the batch's max_E: outputs zero, sticky flag."""
    p = pairgen.generate(pairgen.UNEVEN_MIX, 0, 200)
    E = p.E.copy()
    E[7] = 20
    p2 = pairgen.Pairs(p.reads, p.refs, p.len, E, p.related, p.k)
    b = to_device(p2, gpu_ctx, per_pair=True, offsets=True, max_E=15)
    got = results(gpu_ctx.filter(b, SS), p.n)
    with pytest.raises(paf.PafError) as ei:
        gpu_ctx.check()
    assert ei.value.status == 2
    gpu_ctx.check()  # cleared
    assert got[SS][0][7] == 0 and got[SS][1][7] == 0
    want = oracle_for(p, SS)
    mask = np.arange(p.n) != 7
    assert np.array_equal(got[SS][1][mask], want[SS][1][mask])


def test_host_validation(gpu_ctx):
    p = pairgen.generate(pairgen.SMALL_100BP, 0, 10)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    with pytest.raises(paf.PafError):
        gpu_ctx.filter(b, 0)
    b.uniform_E = 40
    b.max_E = 40
    with pytest.raises(paf.PafError) as ei:
        gpu_ctx.filter(b, SS)
    assert ei.value.status == 2


def test_full_size_fixed_250bp_sampled(gpu_ctx):
    """The benchmark workload at full size (10M pairs, 250 bp, E = 10), in the
    launch configuration the benchmark times: 20k sampled pairs against the
    oracle one by one, and whole-batch properties."""
    w = pairgen.FIXED_250BP
    n = w.n_pairs
    dev = torch.device("cuda", 0)
    chunk = 2_000_000
    words = words_rf = None
    stride = paf.words_for(250)
    rd_w = torch.empty(n * stride, dtype=torch.int64, device=dev)
    rf_w = torch.empty(n * stride, dtype=torch.int64, device=dev)
    for a in range(0, n, chunk):
        q = pairgen.generate(w, a, min(chunk, n - a))
        r = gpu_ctx.pack(torch.from_numpy(q.reads).to(dev), uniform_len=250, stride_words=stride)
        f = gpu_ctx.pack(torch.from_numpy(q.refs).to(dev), uniform_len=250, stride_words=stride)
        rd_w[a * stride:(a + q.n) * stride] = r
        rf_w[a * stride:(a + q.n) * stride] = f
    b = paf.Batch(rd_w, rf_w, n, stride, uniform_len=250, uniform_E=10, max_len=250, max_E=10)
    got = results(gpu_ctx.filter(b, SS), n)
    acc, cnt = got[SS]
    assert np.all(cnt <= 11)
    assert np.array_equal(acc == 1, cnt <= 10)
    ids = pairgen.sample_ids(n, 20000)
    s = pairgen.generate_ids(w, ids)
    want = oracle.filter_batch(s.reads, s.refs, s.len, s.E, SS)[SS]
    assert np.array_equal(acc[ids.astype(np.int64)], want[0])
    assert np.array_equal(cnt[ids.astype(np.int64)], want[1])
    # The persistent launch agrees with the plain one on the whole batch.
    got2 = results(gpu_ctx.filter_persistent(b, SS), n)
    assert np.array_equal(got2[SS][0], acc) and np.array_equal(got2[SS][1], cnt)
    gpu_ctx.check()


@pytest.mark.parametrize("filters", [SS, ALL])
def test_ordered_filter_equals_plain(gpu_ctx, filters):
    """Any caller-given order gives the plain decisions at the original ids."""
    p = pairgen.generate(pairgen.UNEVEN_MIX, 9, 5000)
    b = to_device(p, gpu_ctx, per_pair=True, offsets=True)
    want = oracle_for(p, filters)
    g = torch.Generator().manual_seed(3)
    for order in (torch.randperm(p.n, generator=g), torch.arange(p.n - 1, -1, -1)):
        o = order.to(torch.int32).cuda()
        assert_parity(results(gpu_ctx.filter_ordered(b, o, filters), p.n), want, "ordered")
    gpu_ctx.check()


def test_scratch_calls_on_two_streams(gpu_ctx):
    """Persistent launches (work-queue counter), MAGNET (bucketing workspace)
    and the global-bucket pipeline, issued back to back on two streams of one
    context: the library orders them, so every result equals the oracle's."""
    p = pairgen.generate(pairgen.UNEVEN_MIX, 41, 20_000)
    b = to_device(p, gpu_ctx, per_pair=True, offsets=True)
    want = oracle_for(p, SS)
    want_mg = oracle.magnet_batch(p.reads, p.refs, p.len, p.E)
    gpu_ctx.set_layout({"lanes_per_pair": 1, "waves_per_block": 4, "blocks_per_cu": 1, "tiles_per_grab": 1,
                        "chunk_tiles": 0})
    try:
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        outs = []
        torch.cuda.synchronize()
        for rep in range(3):
            for s in (s1, s2):
                with torch.cuda.stream(s):
                    o = gpu_ctx.alloc_out(p.n, SS, b.device)
                    gpu_ctx.filter_persistent(b, SS, out=o, stream=s)
                    m = gpu_ctx.alloc_out(p.n, SS, b.device)
                    gpu_ctx.filter_magnet(b, out=m, stream=s)
                    outs.append((o, m))
        torch.cuda.synchronize()
        for o, m in outs:
            assert_parity(results(o, p.n), want, "persistent, two streams")
            got = results(m, p.n)[SS]
            assert np.array_equal(got[0], want_mg[0]) and np.array_equal(got[1], want_mg[1])
    finally:
        gpu_ctx.set_layout(None)
    gpu_ctx.check()
