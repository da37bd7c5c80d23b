"""Filtering accuracy (Ch. 3, Sec. 3.1.2): confusion counts of a filter's
decisions against the exact verdict of read alignment.

A mapping (pair) is correct when its edit distance is at most E, i.e. when an
optimal aligner accepts it; `dist` is min(edit distance, E+1) per pair, as
paf_verify computes it (the banded distance equals the true one whenever it
is at most E).  Then, per filter:
  TA / FR: correct pairs the filter accepts / rejects,
  FA / TR: incorrect pairs the filter accepts / rejects,
  FAR = FA / incorrect, TRR = TR / incorrect, TAR = TA / correct,
  FRR = FR / correct.
Host-side reporting over the library's outputs; no part of the filter."""
from __future__ import annotations

import numpy as np


def confusion(accept, dist, E) -> dict:
    accept = np.asarray(accept).astype(bool)
    correct = np.asarray(dist).astype(np.int64) <= np.asarray(E).astype(np.int64)
    ta = int(np.count_nonzero(accept & correct))
    fr = int(np.count_nonzero(~accept & correct))
    fa = int(np.count_nonzero(accept & ~correct))
    tr = int(np.count_nonzero(~accept & ~correct))
    nc, ni = ta + fr, fa + tr
    return {"TA": ta, "FR": fr, "FA": fa, "TR": tr, "correct": nc, "incorrect": ni,
            "FAR": fa / ni if ni else 0.0, "FRR": fr / nc if nc else 0.0,
            "TAR": ta / nc if nc else 1.0, "TRR": tr / ni if ni else 1.0}
