"""Pairs in pinned host memory for the streaming filter (paf_stream_filter).

The synthetic workload is generated chunk by chunk and encoded on the host by
the library's host encoder (paf_pack_host) straight into page-locked buffers,
pairs stored back to back."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

import pairgen

from . import HostBatch, _check, load_library


def host_batch(w: pairgen.Workload, n: int, first: int = 0, chunk: int = 4_000_000,
               threads: int = 16) -> HostBatch:
    lib = load_library()
    lens, Es = pairgen.lengths(w, first, n)
    words = (lens.astype(np.int64) + 31) // 32
    off = np.zeros(n + 1, np.int64)
    np.cumsum(words, out=off[1:])
    total = int(off[-1])
    reads = torch.empty(max(total, 1), dtype=torch.int64, pin_memory=True)
    refs = torch.empty(max(total, 1), dtype=torch.int64, pin_memory=True)
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        q = pairgen.generate(w, first + a, m)
        o = np.ascontiguousarray(off[a:a + m].astype(np.uint64))
        for codes, dst in ((q.reads, reads), (q.refs, refs)):
            _check(lib.paf_pack_host(codes.ctypes.data_as(ctypes.c_void_p), q.stride,
                                     q.len.ctypes.data_as(ctypes.c_void_p), 0,
                                     o.ctypes.data_as(ctypes.c_void_p), 0, m,
                                     ctypes.c_void_p(dst.data_ptr()), threads))
    ln = torch.from_numpy(lens.astype(np.int16)).pin_memory()
    E = torch.from_numpy(Es).pin_memory()
    return HostBatch(reads, refs, ln, E, int(lens.max()), int(Es.max()))
