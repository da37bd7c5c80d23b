"""The benchmark workloads at their full sizes, in the launch configurations the
benchmark times, checked on sampled pairs against the oracle one by one and on
whole-batch properties (accept exactly when the count is at most E, SneakySnake's
count saturated at E+1, and the launch variants agreeing with each other on
every pair).

- 10M pairs of 250 bp at E = 0, 5, 10, 25: SneakySnake, GateKeeper and Shouji
  on one map, and SneakySnake alone on the compacting engine;
- 50M pairs of mixed lengths in the persistent launch with the autotuned
  layout, the fixed per-tile layout and the learned local pipeline;
- 200M pairs streamed from pinned host memory in 8M-pair chunks, plain and
  learned;
- the rows beyond the path on the 10M x 250 bp pairs: SneakySnake on
  partitioned mazes (t = 5, 10, 25, 50) and in the hardware form (t = 8,
  y = 3), MAGNET, and verification of SneakySnake's survivors (identical to
  verifying every pair).
"""
import numpy as np
import pytest
import torch

import oracle
import pairgen
import paper_1910_03936_amd as paf
from gpu_util import results

pytestmark = pytest.mark.gpu

SS, ALL = paf.SNEAKYSNAKE, paf.ALL_FILTERS


def check_properties(got: dict, E):
    E = np.asarray(E).astype(np.uint16)
    for f, (acc, cnt) in got.items():
        if f == SS:   # GateKeeper and Shouji report their popcounts unsaturated
            assert np.all(cnt <= E + np.uint16(1)), f"filter {f}: count above E+1"
        assert np.array_equal(acc == 1, cnt <= E), f"filter {f}: accept bit disagrees with the count"


def check_sample(got: dict, s: pairgen.Pairs, ids: np.ndarray, E, filters: int):
    want = oracle.filter_batch(s.reads, s.refs, s.len, E, filters)
    ix = ids.astype(np.int64)
    for f in want:
        ga, gc = got[f][0][ix], got[f][1][ix]
        bad = np.nonzero((ga != want[f][0]) | (gc != want[f][1]))[0]
        assert bad.size == 0, (f"filter {f}: {bad.size} sampled mismatches, first pair ids {ix[bad[:5]]}: "
                               f"gpu {ga[bad[:5]]}/{gc[bad[:5]]} oracle {want[f][0][bad[:5]]}/{want[f][1][bad[:5]]}")


@pytest.fixture(scope="module")
def fixed250(gpu_ctx):
    from paper_1910_03936_amd.batches import device_batch
    w = pairgen.FIXED_250BP
    b = device_batch(gpu_ctx, w, w.n_pairs, per_pair=False)
    ids = pairgen.sample_ids(w.n_pairs, 5000)
    return b, ids, pairgen.generate_ids(w, ids)


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_full_size_fixed_250bp_all_filters(gpu_ctx, fixed250, E):
    b, ids, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    got = results(gpu_ctx.filter(b, ALL), n)
    check_properties(got, E)
    check_sample(got, s, ids, np.full(s.n, E), ALL)
    # SneakySnake alone runs the compacting engine: same decisions as on the shared map
    alone = results(gpu_ctx.filter(b, SS), n)
    assert np.array_equal(alone[SS][0], got[SS][0]) and np.array_equal(alone[SS][1], got[SS][1])
    gpu_ctx.check()


def test_full_size_uneven_50M(gpu_ctx):
    from paper_1910_03936_amd.batches import device_batch
    w = pairgen.UNEVEN_MIX
    n = w.n_pairs
    b = device_batch(gpu_ctx, w, n)
    _, Es = pairgen.lengths(w, 0, n)
    gpu_ctx.set_layout({"lanes_per_pair": 1, "waves_per_block": 4, "blocks_per_cu": 4, "tiles_per_grab": 2,
                        "chunk_tiles": 0})
    fixed = results(gpu_ctx.filter_persistent(b, SS), n)
    gpu_ctx.set_layout(None)
    tuned_layout, _, _ = gpu_ctx.autotune(b, SS)
    tuned = results(gpu_ctx.filter_persistent(b, SS), n)
    check_properties(tuned, Es)
    ids = pairgen.sample_ids(n, 20000)
    s = pairgen.generate_ids(w, ids)
    check_sample(tuned, s, ids, s.E, SS)
    for a, bb in zip(fixed[SS], tuned[SS]):
        assert np.array_equal(a, bb), f"fixed layout and autotuned {tuned_layout} disagree"
    # The learned local pipeline (model levels, then chunks ordered by level)
    # with the initial weights: the decisions never depend on the model.
    gpu_ctx.mlp_set_params(pairgen.init_mlp_params())
    learned = results(gpu_ctx.filter_bucketed_local(b), n)
    for a, bb in zip(learned[SS], tuned[SS]):
        assert np.array_equal(a, bb), "learned pipeline disagrees with the plain launch"
    gpu_ctx.check()
    gpu_ctx.set_layout(None)


def test_full_size_stream_200M(gpu_ctx):
    from paper_1910_03936_amd.hostbatch import host_batch
    w = pairgen.STREAM_MIX
    n = w.n_pairs
    hb = host_batch(w, n)
    gpu_ctx.mlp_set_params(pairgen.init_mlp_params())
    out = {}
    for learned in (False, True):
        o, st = paf.stream_filter(gpu_ctx, hb, 8_000_000, SS, learned)
        gpu_ctx.check()
        assert st["chunks"] == 25
        out[learned] = results(o, n)
    del hb
    assert np.array_equal(out[False][SS][0], out[True][SS][0])
    assert np.array_equal(out[False][SS][1], out[True][SS][1])
    _, Es = pairgen.lengths(w, 0, n)
    check_properties(out[True], Es)
    ids = pairgen.sample_ids(n, 20000)
    s = pairgen.generate_ids(w, ids)
    check_sample(out[True], s, ids, s.E, SS)


def _sampled(got_acc, got_cnt, ids, want_acc, want_cnt, label):
    ix = ids.astype(np.int64)
    bad = np.nonzero((got_acc[ix] != want_acc) | (got_cnt[ix] != want_cnt))[0]
    assert bad.size == 0, (f"{label}: {bad.size} sampled mismatches, first pair ids {ix[bad[:5]]}: "
                           f"gpu {got_acc[ix][bad[:5]]}/{got_cnt[ix][bad[:5]]} oracle {want_acc[bad[:5]]}/"
                           f"{want_cnt[bad[:5]]}")


@pytest.mark.parametrize("E", [5, 10, 25])
def test_full_size_partitioned_and_hardware_form(gpu_ctx, fixed250, E):
    b, ids, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    whole = results(gpu_ctx.filter(b, SS), n)[SS][1].astype(np.int64)
    prev = None
    for t, y in ((5, 0), (10, 0), (25, 0), (50, 0), (8, 3)):
        acc, cnt = results(gpu_ctx.filter_partitioned(b, t, y), n)[SS]
        check_properties({SS: (acc, cnt)}, E)
        if y == 0:
            wa, wc = oracle.sneakysnake_t_batch(s.reads, s.refs, s.len, E, t)
            # no sub-maze count exceeds the whole maze's
            assert np.all(cnt.astype(np.int64) <= whole)
        else:
            wa, wc = oracle.sneakysnake_fpga_batch(s.reads, s.refs, s.len, E, t, y)
        _sampled(acc, cnt, ids, wa, wc, f"E={E} t={t} y={y}")
        if t == 10:
            # t = 5 refines t = 10: never more obstacles
            assert np.all(prev <= cnt)
        prev = cnt
    gpu_ctx.check()


@pytest.mark.parametrize("E", [5, 10])
def test_full_size_magnet(gpu_ctx, fixed250, E):
    b, ids, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    acc, cnt = results(gpu_ctx.filter_magnet(b), n)[SS]
    check_properties({SS: (acc, cnt)}, E)
    wa, wc = oracle.magnet_batch(s.reads, s.refs, s.len, E)
    _sampled(acc, cnt, ids, wa, wc, f"MAGNET E={E}")
    gpu_ctx.check()


@pytest.mark.parametrize("E", [5, 10, 25])
def test_full_size_verify_survivors(gpu_ctx, fixed250, E):
    b, ids, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    out = gpu_ctx.filter(b, SS)
    d_sel = gpu_ctx.verify(b, out[SS][0])
    d_all = gpu_ctx.verify(b)
    torch.cuda.synchronize()
    assert torch.equal(d_sel, d_all), "verifying the survivors differs from verifying every pair"
    d = paf.counts_u16(d_all).cpu().numpy().astype(np.uint16)
    assert np.all(d <= E + 1)
    want = oracle.banded_batch(s.reads, s.refs, s.len, np.full(s.n, E))
    bad = np.nonzero(d[ids.astype(np.int64)] != want)[0]
    assert bad.size == 0, f"E={E}: {bad.size} sampled distances differ from the oracle"
    # A pair within E edits always survives SneakySnake.
    acc = paf.accept_bits_to_bool(out[SS][0], n).cpu().numpy()
    assert np.all(acc[d <= E])
    gpu_ctx.check()
