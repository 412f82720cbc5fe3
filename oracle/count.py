"""Work counters and rank log of the oracle (test infrastructure only)."""
from __future__ import annotations

from collections import defaultdict

import numpy as np


class Counter:
    """Algorithmic FP64 flop counts by category plus a log of every
    recompression (site, sizes, input width, kept rank, tau and the singular
    values just around the cut).

    Each log entry carries a `key` that names the recompression independently
    of the order in which an implementation runs them:
      ("S", lo, hi, i)          i-th recompression of the sum S~ at the node
                                covering rows/cols [lo, hi) (Alg. hQR, S~)
      ("A12", lo, hi)           the new upper block of R at that node
      ("update", lo, hi, r, c)  the -_H update at node [lo, hi) of the block whose
                                first row / column are r / c
      ("T", lo, hi, i)          i-th recompression of the sum T~12 at the node
    """

    def __init__(self):
        self.flops = defaultdict(float)
        self.truncs = []

    def add(self, cat: str, f: float):
        self.flops[cat] += float(f)

    def log_trunc(self, site, mL, mR, w, k, tau, s, key=None):
        s = np.asarray(s)
        self.truncs.append(dict(
            site=site, key=tuple(key) if key is not None else None,
            mL=int(mL), mR=int(mR), w=int(w), k=int(k), tau=float(tau),
            sk=float(s[k - 1]) if k >= 1 and s.size >= k else float("inf"),
            sk1=float(s[k]) if s.size > k else 0.0))

    @property
    def total(self) -> float:
        return float(sum(self.flops.values()))
