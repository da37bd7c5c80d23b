"""Learned cost model: training-set construction and training.

Host orchestration only: generation of the synthetic training pairs (the seeded
generator), packing, features, labels and every training step run through
libpaf.  The label of a pair is SneakySnake's obstacle count computed by the
library's own filter at the largest supported threshold (E = 31, so counts
run 0..32): it says how many obstacles the snake meets over the whole maze,
hence how far it gets before it stops at a smaller threshold E.  The model
never decides anything; it only orders the work.
"""
from __future__ import annotations

import torch

import pairgen

from . import SNEAKYSNAKE, Batch, Context

LABEL_E = 31


def pack_workload(ctx: Context, w: pairgen.Workload, first: int, n: int, dev=None,
                  chunk: int = 1_000_000) -> Batch:
    """Pairs [first, first + n) of w, packed on the GPU with per-pair lengths,
    thresholds and word offsets."""
    from .batches import device_batch
    return device_batch(ctx, w, n, first=first, chunk=chunk, per_pair=True)


def labels_for(ctx: Context, b: Batch) -> torch.Tensor:
    """SneakySnake counts at E = 31 (uint16 values in an int16 tensor)."""
    lab = Batch(b.reads, b.refs, b.n_pairs, b.stride_words, b.word_offset, b.len, None, 0, LABEL_E,
                b.max_len, LABEL_E)
    out = ctx.filter(lab, SNEAKYSNAKE)
    return out[SNEAKYSNAKE][1]


def training_set(ctx: Context, w: pairgen.Workload, n: int, first: int = 0):
    """Features [n][64] fp32 and labels [n] of pairs [first, first + n) of w."""
    dev = torch.device("cuda", ctx.device)
    b = pack_workload(ctx, w, first, n, dev)
    feats = ctx.features(b)
    labels = labels_for(ctx, b)
    torch.cuda.synchronize()
    ctx.check()
    return feats, labels


def train(ctx: Context, w: pairgen.Workload, n: int = 2_000_000, epochs: int = 4, batch: int = 4096,
          lr: float = 1e-3, seed: int = 7):
    """Train the context's cost model from the seeded initial weights on n
    pairs drawn like workload w (with its own seed).  Returns per-epoch mean
    losses."""
    tw = w.with_seed(w.seed + 1000 + seed)
    feats, labels = training_set(ctx, tw, n)
    g = torch.Generator().manual_seed(seed)
    order = torch.randperm(n, generator=g).to(feats.device)
    feats = feats[order].contiguous()
    labels = labels[order].contiguous()
    ctx.mlp_set_params(pairgen.init_mlp_params(pairgen.SEED_BASE + 17 + seed))
    return ctx.mlp_train(feats, labels, epochs, batch, lr)
