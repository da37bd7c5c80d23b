"""Checkpoint and resume: the autotune cache and the cost model (with its
optimizer state) saved to a file and loaded into a new context, and a stream
resumed from a chunk index.  Outputs of the restored context are compared
element by element with those of the one that was saved, and the resumed
stream with an uninterrupted one."""
import numpy as np
import pytest
import torch

import pairgen
import paper_1910_03936_amd as paf
from tests.gpu_util import results

pytestmark = pytest.mark.gpu

SS = paf.SNEAKYSNAKE


def _uneven_batch(ctx, n):
    from paper_1910_03936_amd import costmodel
    return costmodel.pack_workload(ctx, pairgen.UNEVEN_MIX, 0, n, torch.device("cuda", 0))


def test_autotune_cache_round_trip(gpu_ctx, tmp_path):
    n = 200_000
    b = _uneven_batch(gpu_ctx, n)
    gpu_ctx.set_layout(None)
    layout, _, _ = gpu_ctx.autotune(b, SS)
    tuned = gpu_ctx.tuned_export()
    assert any(e["layout"] == layout and e["filters"] == SS for e in tuned)
    want = results(gpu_ctx.filter_persistent(b, SS), n)
    path = str(tmp_path / "state.npz")
    gpu_ctx.save_state(path, model=False)

    ctx2 = paf.Context(0)
    try:
        assert ctx2.tuned_export() == []
        assert ctx2.load_state(path) == {"tuned": len(tuned), "model": False}
        assert sorted(map(str, ctx2.tuned_export())) == sorted(map(str, tuned))
        got = results(ctx2.filter_persistent(b, SS), n)
        for k in (0, 1):
            assert np.array_equal(got[SS][k], want[SS][k])
        ctx2.check()
    finally:
        ctx2.close()


def test_tuned_import_rejects_bad_entries(gpu_ctx):
    ctx2 = paf.Context(0)
    try:
        good = {"max_words": 8, "max_E": 10, "filters": SS,
                "layout": {"lanes_per_pair": 1, "waves_per_block": 2, "blocks_per_cu": 0, "tiles_per_grab": 1,
                           "chunk_tiles": 6, "first_pass_windows": 2, "pass_windows": 3}}
        bad = [dict(good, max_words=17), dict(good, max_E=9), dict(good, filters=8), dict(good, filters=0),
               dict(good, layout=dict(good["layout"], waves_per_block=3)),
               dict(good, layout=dict(good["layout"], lanes_per_pair=2), max_E=8),
               dict(good, layout=dict(good["layout"], lanes_per_pair=2), filters=3)]
        for e in bad:
            with pytest.raises(paf.PafError) as ei:
                ctx2.tuned_import([good, e])
            assert ei.value.status == 1
            assert ctx2.tuned_export() == []     # nothing added when one entry is bad
        ctx2.tuned_import([good])
        assert ctx2.tuned_export() == [good]
    finally:
        ctx2.close()


def test_model_state_round_trip_resumes_training(gpu_ctx, tmp_path):
    """Training resumed from a saved state takes exactly the steps the
    uninterrupted context takes (same weights, moments and step count)."""
    b = _uneven_batch(gpu_ctx, 4096)
    feats = gpu_ctx.features(b)
    t = torch.arange(4096, device="cuda", dtype=torch.float32) % 23
    ctx1 = paf.Context(0)
    ctx2 = paf.Context(0)
    try:
        ctx1.mlp_set_params(pairgen.init_mlp_params(pairgen.SEED_BASE + 3))
        for _ in range(3):
            ctx1.mlp_train_step(feats, t, lr=1e-3)
        path = str(tmp_path / "model.npz")
        ctx1.save_state(path)
        assert ctx2.load_state(path) == {"tuned": 0, "model": True}
        s1, s2 = ctx1.mlp_get_state(), ctx2.mlp_get_state()
        assert s2["step"] == s1["step"] == 3
        for k in ("params", "adam_m", "adam_v"):
            assert np.array_equal(s1[k], s2[k])
        for _ in range(2):
            ctx1.mlp_train_step(feats, t, lr=1e-3)
            ctx2.mlp_train_step(feats, t, lr=1e-3)
        torch.cuda.synchronize()
        s1, s2 = ctx1.mlp_get_state(), ctx2.mlp_get_state()
        assert s1["step"] == s2["step"] == 5
        for k in ("params", "adam_m", "adam_v"):
            assert np.array_equal(s1[k], s2[k]), k
        # set_params alone clears the moments and the step count; the
        # predictions of the two contexts' models are still equal.
        ctx2.mlp_set_params(s1["params"])
        assert ctx2.mlp_get_state()["step"] == 0
        assert torch.equal(ctx1.mlp_predict(b), ctx2.mlp_predict(b))
    finally:
        ctx1.close()
        ctx2.close()


def test_model_state_rejects_bad_values(gpu_ctx, tmp_path):
    ctx2 = paf.Context(0)
    try:
        p = pairgen.init_mlp_params(pairgen.SEED_BASE + 4).astype(np.float32)
        z = np.zeros_like(p)
        for st in ({"params": np.where(np.arange(p.size) == 7, np.nan, p), "adam_m": z, "adam_v": z, "step": 1},
                   {"params": p, "adam_m": z, "adam_v": -np.ones_like(p), "step": 1},
                   {"params": p, "adam_m": np.full_like(p, np.inf), "adam_v": z, "step": 1}):
            with pytest.raises(paf.PafError) as ei:
                ctx2.mlp_set_state(st)
            assert ei.value.status == 1
        with pytest.raises(paf.PafError) as ei:
            ctx2.mlp_get_state()
        assert ei.value.status == 5          # still no model
        bad = str(tmp_path / "bad.npz")
        np.savez(bad, format=np.array([1, 1], dtype=np.uint32), tuned=np.zeros((0, 10), np.uint32))
        with pytest.raises(ValueError):
            ctx2.load_state(bad)
    finally:
        ctx2.close()


def test_stream_resumes_from_chunk_index(gpu_ctx):
    from paper_1910_03936_amd.hostbatch import host_batch
    n, chunk = 50_003, 8192
    hb = host_batch(pairgen.STREAM_MIX, n, chunk=20_000)
    full, st = paf.stream_filter(gpu_ctx, hb, chunk_pairs=chunk, filters=paf.ALL_FILTERS)
    assert st["chunks"] == 7
    for done in (0, 1, 3, 6):
        first = done * chunk
        # The outputs of a stream stopped after `done` chunks: later pairs unset.
        part = {f: (a.clone().pin_memory(), c.clone().pin_memory()) for f, (a, c) in full.items()}
        for a, c in part.values():
            a[first // 32:] = 0
            c[first:] = 0
        out, st = paf.stream_filter(gpu_ctx, hb, chunk_pairs=chunk, filters=paf.ALL_FILTERS,
                                    first_pair=first, out=part)
        assert out is part
        assert st["chunks"] == 7 - done
        for f in full:
            assert torch.equal(part[f][0], full[f][0]) and torch.equal(part[f][1], full[f][1]), (done, f)
    gpu_ctx.check()
    with pytest.raises(ValueError):
        paf.stream_filter(gpu_ctx, hb, chunk_pairs=chunk, first_pair=100)
