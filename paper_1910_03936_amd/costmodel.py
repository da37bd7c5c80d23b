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
    lab = Batch(b.reads, b.refs, b.n_pairs, b.stride_words, b.word_offset, b.len, None,
                b.uniform_len if b.len is None else 0, LABEL_E, b.max_len or b.uniform_len, LABEL_E)
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


def evaluate(ctx: Context, w: pairgen.Workload, n: int = 200_000, seed_offset: int = 2000) -> dict:
    """The trained model's error on n held-out pairs drawn like workload w with
    a seed used neither for training nor by the benchmark batch: predictions
    of the fused inference kernel (paf_mlp_predict) against the labels (the
    filter's counts at E = 31).  Beside the model: the error of predicting
    the held-out set's mean label, and of predicting each (length, E) class's
    mean label (the trivial length x E key)."""
    hw = w.with_seed(w.seed + seed_offset)
    b = pack_workload(ctx, hw, 0, n)
    y = ctx.mlp_predict(b).double()
    lab = labels_for(ctx, b).to(torch.int64).double()
    torch.cuda.synchronize()
    ctx.check()
    err = y - lab
    cls = (b.len.to(torch.int64) & 0xFFFF) * 64 + b.E.to(torch.int64)
    uniq, inv = torch.unique(cls, return_inverse=True)
    sums = torch.zeros(uniq.numel(), dtype=torch.float64, device=lab.device).index_add_(0, inv, lab)
    cnts = torch.zeros(uniq.numel(), dtype=torch.float64, device=lab.device).index_add_(0, inv, torch.ones_like(lab))
    cls_mean = (sums / cnts)[inv]
    return {"pairs": n, "mse": float((err ** 2).mean()), "mae": float(err.abs().mean()),
            "label_mean": float(lab.mean()),
            "mse_of_mean": float(((lab - lab.mean()) ** 2).mean()),
            "mae_of_mean": float((lab - lab.mean()).abs().mean()),
            "mse_of_length_E_class_mean": float(((lab - cls_mean) ** 2).mean()),
            "mae_of_length_E_class_mean": float((lab - cls_mean).abs().mean())}


def oracle_key(ctx: Context, b: Batch) -> torch.Tensor:
    """The in-chunk level key (paf_cost_levels' encoding: 15 - min(15, y / 2))
    computed from the true labels instead of the model: the best any
    prediction of the label could do (an ablation bound, not a pipeline)."""
    lab = labels_for(ctx, b).to(torch.int64)
    return (15 - torch.clamp(lab // 2, max=15)).to(torch.uint8)


def length_e_key(b: Batch) -> torch.Tensor:
    """A trivial key from the pair's length and threshold alone (longest and
    largest E first): 15 - the (length, E) rank on the 16 levels."""
    dev = b.reads.device
    if b.len is None:
        return torch.full((b.n_pairs,), 15, dtype=torch.uint8, device=dev)
    m = (b.len.to(torch.int64) & 0xFFFF)
    e = b.E.to(torch.int64) if b.E is not None else torch.full_like(m, b.uniform_E)
    work = m * (e + 1)                      # columns x obstacles the snake may cross
    lv = torch.clamp(work * 16 // (int(work.max()) + 1), max=15)
    return (15 - lv).to(torch.uint8)
