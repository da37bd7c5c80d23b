"""Device-resident batches of the synthetic workloads, built chunk by chunk
(generation on the host, encoding by the library's GPU encoder) so that large
batches never sit in host memory whole."""
from __future__ import annotations

import numpy as np
import torch

import pairgen

from . import Batch, Context, _check, words_for


def device_batch(ctx: Context, w: pairgen.Workload, n: int, first: int = 0, chunk: int = 2_000_000,
                 per_pair: bool = True) -> Batch:
    """Pairs [first, first + n) of w on the GPU.  per_pair: lengths, thresholds
    and word offsets per pair, pairs stored back to back; otherwise (uniform
    length and E only) a fixed stride of words."""
    dev = torch.device("cuda", ctx.device)
    lens, Es = pairgen.lengths(w, first, n)
    if not per_pair:
        assert len(set(w.lens)) == 1 and w.fixed_E >= 0
        m = w.lens[0]
        stride = words_for(m)
        rd = torch.empty(n * stride, dtype=torch.int64, device=dev)
        rf = torch.empty(n * stride, dtype=torch.int64, device=dev)
        for a in range(0, n, chunk):
            q = pairgen.generate(w, first + a, min(chunk, n - a))
            rd[a * stride:(a + q.n) * stride] = ctx.pack(torch.from_numpy(q.reads).to(dev), uniform_len=m,
                                                         stride_words=stride)
            rf[a * stride:(a + q.n) * stride] = ctx.pack(torch.from_numpy(q.refs).to(dev), uniform_len=m,
                                                         stride_words=stride)
        torch.cuda.synchronize()
        return Batch(rd, rf, n, stride, uniform_len=m, uniform_E=w.fixed_E, max_len=m, max_E=w.fixed_E)
    words = (lens.astype(np.int64) + 31) // 32
    off = np.zeros(n + 1, np.int64)
    np.cumsum(words, out=off[1:])
    total = int(off[-1])
    rd = torch.zeros(max(total, 1), dtype=torch.int64, device=dev)
    rf = torch.zeros(max(total, 1), dtype=torch.int64, device=dev)
    off_d = torch.from_numpy(off[:n]).to(dev)
    len_d = torch.from_numpy(lens.astype(np.int16)).to(dev)
    E_d = torch.from_numpy(Es).to(dev)
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        q = pairgen.generate(w, first + a, m)
        o = off_d[a:a + m]
        ln = len_d[a:a + m]
        for codes, dst in ((q.reads, rd), (q.refs, rf)):
            c = torch.from_numpy(codes).to(dev)
            # the encoder writes each pair at its absolute word offset
            _check(ctx.lib.paf_pack(ctx.h, c.data_ptr(), q.stride, ln.data_ptr(), 0, o.data_ptr(), 0, m,
                                    dst.data_ptr(), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    ctx.check()
    return Batch(rd, rf, n, 0, off_d, len_d, E_d, 0, 0, int(lens.max()), int(Es.max()))
