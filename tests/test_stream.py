"""Streaming filter from pinned host memory: decisions equal the oracle's for
every pair, in plain and learned mode, including a ragged last chunk."""
import numpy as np
import pytest
import torch

import oracle
import pairgen
import paper_1910_03936_amd as paf

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("learned", [False, True])
def test_stream_matches_oracle(gpu_ctx, learned):
    from paper_1910_03936_amd.hostbatch import host_batch
    w = pairgen.STREAM_MIX
    n = 50_003
    hb = host_batch(w, n, chunk=20_000)
    if learned:
        gpu_ctx.mlp_set_params(pairgen.init_mlp_params())
    out, stats = paf.stream_filter(gpu_ctx, hb, chunk_pairs=16_384, filters=paf.ALL_FILTERS, learned=learned)
    gpu_ctx.check()
    assert stats["chunks"] == 4
    p = pairgen.generate(w, 0, n)
    want = oracle.filter_batch(p.reads, p.refs, p.len, p.E, paf.ALL_FILTERS)
    for f, (bits, cnt) in out.items():
        acc = paf.accept_bits_to_bool(bits, n).numpy().astype(np.uint8)
        assert np.array_equal(acc, want[f][0])
        assert np.array_equal(paf.counts_u16(cnt).numpy(), want[f][1].astype(np.int64))


def test_stream_rejects_bad_chunk(gpu_ctx):
    from paper_1910_03936_amd.hostbatch import host_batch
    hb = host_batch(pairgen.STREAM_MIX, 100)
    with pytest.raises(paf.PafError):
        paf.stream_filter(gpu_ctx, hb, chunk_pairs=100)
