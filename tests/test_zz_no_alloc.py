"""The entry point that allocates nothing, paf_filter_magnet_noalloc, called
through the C ABI and checked bit for bit against paf_filter_magnet (same
pairs, same outputs), on two calls in a row with the second batch smaller
than the first, plus its size limit (rejected on the host)."""
import ctypes

import numpy as np
import pytest
import torch

import pairgen
import paper_1910_03936_amd as paf
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

SS = paf.SNEAKYSNAKE


def _call(ctx, name, b, n):
    out = ctx.alloc_out(n, SS, b.device)
    cb, co = b.c(), ctx._out(out)
    st = getattr(ctx.lib, name)(ctx.h, ctypes.byref(cb), ctypes.byref(co), None)
    return st, out


def test_magnet_noalloc_matches_magnet(gpu_ctx):
    cases = ((pairgen.UNEVEN_MIX, 300_001, True), (pairgen.FIXED_250BP.with_E(10), 70_017, False))
    for i, (w, n, per_pair) in enumerate(cases):
        p = pairgen.generate(w, 5 + i, n)
        b = to_device(p, gpu_ctx, per_pair=per_pair, offsets=per_pair)
        st, got = _call(gpu_ctx, "paf_filter_magnet_noalloc", b, n)
        assert st == 0, gpu_ctx.lib.paf_last_error()
        st2, want = _call(gpu_ctx, "paf_filter_magnet", b, n)
        assert st2 == 0, gpu_ctx.lib.paf_last_error()
        torch.cuda.synchronize()
        gpu_ctx.check()
        for k in (0, 1):
            assert torch.equal(got[SS][k], want[SS][k]), f"case {i}: output {k} differs from paf_filter_magnet"
        assert int(paf.counts_u16(got[SS][1]).max()) <= int(p.E.max()) + 1


def test_magnet_noalloc_takes_no_device_memory(gpu_ctx):
    p = pairgen.generate(pairgen.FIXED_250BP.with_E(5), 9, 50_000)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    outs = [gpu_ctx.alloc_out(p.n, SS, b.device) for _ in range(3)]
    torch.cuda.synchronize()
    st, _ = _call(gpu_ctx, "paf_filter_magnet_noalloc", b, p.n)   # first use of the kernels
    assert st == 0
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for o in outs:
        cb, co = b.c(), gpu_ctx._out(o)
        assert gpu_ctx.lib.paf_filter_magnet_noalloc(gpu_ctx.h, ctypes.byref(cb), ctypes.byref(co), None) == 0
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for o in outs[1:]:
        assert torch.equal(o[SS][0], outs[0][SS][0]) and torch.equal(o[SS][1], outs[0][SS][1])


def test_magnet_noalloc_rejects_batches_above_its_workspace(gpu_ctx):
    p = pairgen.generate(pairgen.FIXED_250BP.with_E(5), 3, 64)
    b = to_device(p, gpu_ctx, per_pair=False, offsets=False)
    cb = b.c()
    cb.n_pairs = paf.MAGNET_NOALLOC_MAX_PAIRS + 1     # rejected on the host, nothing launched
    out = gpu_ctx.alloc_out(64, SS, b.device)
    co = gpu_ctx._out(out)
    assert gpu_ctx.lib.paf_filter_magnet_noalloc(gpu_ctx.h, ctypes.byref(cb), ctypes.byref(co), None) == 2
    assert b"static workspace" in gpu_ctx.lib.paf_last_error()
