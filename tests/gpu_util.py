"""Helpers shared by the GPU tests: move generated pairs to the device, run the
library through its binding, and compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import pairgen
import paper_1910_03936_amd as paf


def to_device(p: pairgen.Pairs, ctx: paf.Context, per_pair: bool, offsets: bool,
              max_len: int | None = None, max_E: int | None = None) -> paf.Batch:
    """Upload codes and pack them on the GPU with the library's encoder."""
    dev = torch.device("cuda", 0)
    rd = torch.from_numpy(p.reads).to(dev)
    rf = torch.from_numpy(p.refs).to(dev)
    ml = int(max_len if max_len is not None else p.len.max())
    me = int(max_E if max_E is not None else p.E.max())
    if per_pair:
        ln = torch.from_numpy(p.len.astype(np.int16)).to(dev)
        E = torch.from_numpy(p.E.astype(np.uint8)).to(dev)
        return ctx.pack_pairs(rd, rf, lens=ln, Es=E, max_len=ml, max_E=me, offsets=offsets)
    assert len(set(p.len.tolist())) == 1 and len(set(p.E.tolist())) == 1
    return ctx.pack_pairs(rd, rf, uniform_len=int(p.len[0]), uniform_E=int(p.E[0]),
                          max_len=ml, max_E=me)


def results(out: dict, n: int) -> dict:
    torch.cuda.synchronize()
    r = {}
    for f, (bits, cnt) in out.items():
        r[f] = (paf.accept_bits_to_bool(bits, n).cpu().numpy().astype(np.uint8),
                paf.counts_u16(cnt).cpu().numpy().astype(np.uint16))
    return r


def assert_parity(got: dict, want: dict, label: str = ""):
    for f in want:
        ga, gc = got[f]
        wa, wc = want[f]
        bad = np.nonzero((ga != wa) | (gc != wc))[0]
        assert bad.size == 0, (f"{label} filter {f}: {bad.size} mismatches, first at {bad[:5]}: "
                               f"gpu acc/cnt {ga[bad[:5]]}/{gc[bad[:5]]} oracle {wa[bad[:5]]}/{wc[bad[:5]]}")


def oracle_for(p: pairgen.Pairs, filters: int) -> dict:
    return oracle.filter_batch(p.reads, p.refs, p.len, p.E, filters)
