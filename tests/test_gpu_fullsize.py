"""The benchmark workloads at their full sizes, in the launch configurations the
benchmark times, checked against the oracle element by element.

- SneakySnake on every pair: 10M pairs of 250 bp at E = 0, 5, 10, 25 (the
  compacting engine alone, the shared map with all three stages, and at
  E >= 8 the whole-map kernel of the persistent launch with all stages), 50M
  pairs of mixed lengths in the persistent launch (fixed and autotuned
  layouts, learned local pipeline), and 200M pairs streamed from pinned host
  memory in 8M-pair chunks (plain and learned);
- the other decision stages on the deterministic subsample of every 16th
  pair (pair id % 16 == 0): GateKeeper and Shouji at every E, SneakySnake-t
  (t = 5, 10, 25, 50) and the hardware form (t = 8, y = 3), MAGNET and
  verification of SneakySnake's survivors;
- whole-batch properties everywhere (accept exactly when count <= E,
  SneakySnake's count at most E+1) and agreement of the launch variants on
  every pair.

The oracle regenerates the pairs chunk by chunk from their ids (the
generator is a pure function of seed and pair id), so no batch sits in host
memory whole."""
import numpy as np
import pytest
import torch

import oracle
import pairgen
import paper_1910_03936_amd as paf
from gpu_util import results

pytestmark = pytest.mark.gpu

SS, GK, SH, ALL = paf.SNEAKYSNAKE, paf.GATEKEEPER, paf.SHOUJI, paf.ALL_FILTERS
CHUNK = 2_000_000
SUB = 16          # the subsample: every 16th pair


def check_properties(got: dict, E):
    E = np.asarray(E).astype(np.uint16)
    for f, (acc, cnt) in got.items():
        if f == SS:   # GateKeeper and Shouji report their popcounts unsaturated
            assert np.all(cnt <= E + np.uint16(1)), f"filter {f}: count above E+1"
        assert np.array_equal(acc == 1, cnt <= E), f"filter {f}: accept bit disagrees with the count"


def _mismatch(label, ids, ga, gc, wa, wc):
    bad = np.nonzero((ga != wa) | (gc != wc))[0]
    assert bad.size == 0, (f"{label}: {bad.size} mismatches, first pair ids {ids[bad[:5]]}: gpu "
                           f"{ga[bad[:5]]}/{gc[bad[:5]]} oracle {wa[bad[:5]]}/{wc[bad[:5]]}")


def every_pair_snake(w: pairgen.Workload, n: int, got: dict, label: str):
    """SneakySnake of every pair [0, n) of workload w against the oracle.
    got: {E or None (the workload's own per-pair thresholds): [(name, accept
    uint8[n], count uint16[n]), ...]}; the pairs are generated once per chunk
    for all of them."""
    for a in range(0, n, CHUNK):
        q = pairgen.generate(w, a, min(CHUNK, n - a))
        ids = np.arange(a, a + q.n)
        for E, outs in got.items():
            wa, wc = oracle.filter_batch(q.reads, q.refs, q.len, q.E if E is None else E, SS)[SS]
            for name, acc, cnt in outs:
                _mismatch(f"{label} {name} E={E}", ids, acc[a:a + q.n], cnt[a:a + q.n], wa, wc)


@pytest.fixture(scope="module")
def fixed250(gpu_ctx):
    from paper_1910_03936_amd.batches import device_batch
    w = pairgen.FIXED_250BP
    b = device_batch(gpu_ctx, w, w.n_pairs, per_pair=False)
    sub = np.arange(0, w.n_pairs, SUB, dtype=np.uint64)
    return b, sub, pairgen.generate_ids(w, sub)


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_full_size_fixed_250bp(gpu_ctx, fixed250, E):
    b, sub, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    shared = results(gpu_ctx.filter(b, ALL), n)
    check_properties(shared, E)
    alone = results(gpu_ctx.filter(b, SS), n)[SS]
    # The learned pipeline (levels, then the undecided pairs of each chunk in
    # level order) with the initial weights: the decisions never depend on
    # the model.
    gpu_ctx.mlp_set_params(pairgen.init_mlp_params())
    learned = results(gpu_ctx.filter_bucketed_local(b), n)[SS]
    outs = [("compacting engine", alone[0], alone[1]), ("all stages in one call", shared[SS][0], shared[SS][1]),
            ("learned pipeline", learned[0], learned[1])]
    if E >= 8:
        # the whole-map kernel's SneakySnake (persistent launch, all stages)
        whole = results(gpu_ctx.filter_persistent(b, ALL), n)
        for f in (SS, GK, SH):
            assert np.array_equal(whole[f][0], shared[f][0]) and np.array_equal(whole[f][1], shared[f][1]), \
                f"E={E}: persistent whole-map launch and paf_filter disagree on filter {f}"
        outs.append(("whole-map kernel", whole[SS][0], whole[SS][1]))
    gpu_ctx.check()
    every_pair_snake(pairgen.FIXED_250BP.with_E(E), n, {E: outs}, "10M x 250 bp")
    # GateKeeper and Shouji on every 16th pair
    want = oracle.filter_batch(s.reads, s.refs, s.len, np.full(s.n, E), GK | SH)
    ix = sub.astype(np.int64)
    for f in (GK, SH):
        _mismatch(f"filter {f} E={E}", ix, shared[f][0][ix], shared[f][1][ix], want[f][0], want[f][1])


def test_full_size_uneven_50M(gpu_ctx):
    from paper_1910_03936_amd.batches import device_batch
    w = pairgen.UNEVEN_MIX
    n = w.n_pairs
    b = device_batch(gpu_ctx, w, n)
    _, Es = pairgen.lengths(w, 0, n)
    gpu_ctx.set_layout({"lanes_per_pair": 1, "waves_per_block": 4, "blocks_per_cu": 4, "tiles_per_grab": 2,
                        "chunk_tiles": 0})
    fixed = results(gpu_ctx.filter_persistent(b, SS), n)[SS]
    gpu_ctx.set_layout(None)
    tuned_layout, _, _ = gpu_ctx.autotune(b, SS)
    tuned = results(gpu_ctx.filter_persistent(b, SS), n)
    check_properties(tuned, Es)
    # The learned local pipeline (model levels, then the undecided pairs of
    # each chunk ordered by level) with the initial weights: the decisions
    # never depend on the model.
    gpu_ctx.mlp_set_params(pairgen.init_mlp_params())
    learned = results(gpu_ctx.filter_bucketed_local(b), n)[SS]
    gpu_ctx.check()
    gpu_ctx.set_layout(None)
    del b
    torch.cuda.empty_cache()
    every_pair_snake(w, n, {None: [("fixed layout", *fixed), (f"autotuned {tuned_layout}", *tuned[SS]),
                                   ("learned local", *learned)]}, "50M uneven")


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
        out[learned] = results(o, n)[SS]
    del hb
    _, Es = pairgen.lengths(w, 0, n)
    check_properties({SS: out[True]}, Es)
    every_pair_snake(w, n, {None: [("plain", *out[False]), ("learned", *out[True])]}, "200M streamed")


@pytest.mark.parametrize("E", [5, 10, 25])
def test_full_size_partitioned_and_hardware_form(gpu_ctx, fixed250, E):
    b, sub, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    ix = sub.astype(np.int64)
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
        _mismatch(f"E={E} t={t} y={y}", ix, acc[ix], cnt[ix], wa, wc)
        if t == 10:
            # t = 5 refines t = 10: never more obstacles
            assert np.all(prev <= cnt)
        prev = cnt
    gpu_ctx.check()


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_full_size_magnet(gpu_ctx, fixed250, E):
    b, sub, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    acc, cnt = results(gpu_ctx.filter_magnet(b), n)[SS]
    check_properties({SS: (acc, cnt)}, E)
    wa, wc = oracle.magnet_batch(s.reads, s.refs, s.len, E)
    ix = sub.astype(np.int64)
    _mismatch(f"MAGNET E={E}", ix, acc[ix], cnt[ix], wa, wc)
    gpu_ctx.check()


@pytest.mark.parametrize("E", [5, 10, 25])
def test_full_size_verify_survivors(gpu_ctx, fixed250, E):
    b, sub, s = fixed250
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
    ix = sub.astype(np.int64)
    bad = np.nonzero(d[ix] != want)[0]
    assert bad.size == 0, f"E={E}: {bad.size} subsampled distances differ from the oracle, ids {ix[bad[:5]]}"
    # A pair within E edits always survives SneakySnake.
    acc = paf.accept_bits_to_bool(out[SS][0], n).cpu().numpy()
    assert np.all(acc[d <= E])
    gpu_ctx.check()


@pytest.mark.parametrize("E", [0, 5, 10, 25])
def test_full_size_accuracy(gpu_ctx, fixed250, E):
    """Confusion counts (Sec. 3.1.2) of every filter against the exact
    verdict: on every pair from the GPU's banded distances (SneakySnake never
    rejects a correct pair), and on the subsample the GPU's counts equal the
    ones the oracle's filters and banded distance give."""
    from paper_1910_03936_amd.accuracy import confusion
    b, sub, s = fixed250
    b.uniform_E = E
    b.max_E = E
    n = b.n_pairs
    dist = paf.counts_u16(gpu_ctx.verify(b)).cpu().numpy()
    gpu = {"sneakysnake": results(gpu_ctx.filter(b, SS), n)[SS][0]}
    shared = results(gpu_ctx.filter(b, GK | SH), n)
    gpu["gatekeeper"], gpu["shouji"] = shared[GK][0], shared[SH][0]
    for t in (5, 10, 25, 50):
        gpu[f"sneakysnake-{t}"] = results(gpu_ctx.filter_partitioned(b, t), n)[SS][0]
    gpu["hardware t=8 y=3"] = results(gpu_ctx.filter_partitioned(b, 8, 3), n)[SS][0]
    gpu["magnet"] = results(gpu_ctx.filter_magnet(b), n)[SS][0]
    gpu_ctx.check()
    whole = confusion(gpu["sneakysnake"], dist, E)
    assert whole["FR"] == 0 and whole["FRR"] == 0.0, f"E={E}: SneakySnake rejected {whole['FR']} correct pairs"
    # the subsample, from the oracle alone
    Es = np.full(s.n, E)
    correct = oracle.banded_batch(s.reads, s.refs, s.len, Es).astype(np.int64) <= E
    ref = {"sneakysnake": oracle.filter_batch(s.reads, s.refs, s.len, Es, SS)[SS][0]}
    o2 = oracle.filter_batch(s.reads, s.refs, s.len, Es, GK | SH)
    ref["gatekeeper"], ref["shouji"] = o2[GK][0], o2[SH][0]
    for t in (5, 10, 25, 50):
        ref[f"sneakysnake-{t}"] = oracle.sneakysnake_t_batch(s.reads, s.refs, s.len, E, t)[0]
    ref["hardware t=8 y=3"] = oracle.sneakysnake_fpga_batch(s.reads, s.refs, s.len, E, 8, 3)[0]
    ref["magnet"] = oracle.magnet_batch(s.reads, s.refs, s.len, E)[0]
    ix = sub.astype(np.int64)
    for name, acc in gpu.items():
        got = confusion(acc[ix], dist[ix], E)
        a = ref[name].astype(bool)
        want = (int(np.sum(a & correct)), int(np.sum(~a & correct)), int(np.sum(a & ~correct)),
                int(np.sum(~a & ~correct)))
        assert (got["TA"], got["FR"], got["FA"], got["TR"]) == want, f"E={E} {name}: {got} vs oracle {want}"
        if name.startswith("sneakysnake") or name.startswith("hardware"):
            assert got["FR"] == 0, f"E={E} {name} rejected a correct pair"
