"""Work counters and rank log of the oracle (test infrastructure only)."""
from __future__ import annotations

from collections import defaultdict

import numpy as np


class Counter:
    """Algorithmic FP64 flop counts by category plus a log of every
    recompression (site, sizes, input width, kept rank, tau and the singular
    values just around the cut)."""

    def __init__(self):
        self.flops = defaultdict(float)
        self.truncs = []

    def add(self, cat: str, f: float):
        self.flops[cat] += float(f)

    def log_trunc(self, site, mL, mR, w, k, tau, s):
        s = np.asarray(s)
        self.truncs.append(dict(
            site=site, mL=int(mL), mR=int(mR), w=int(w), k=int(k), tau=float(tau),
            sk=float(s[k - 1]) if k >= 1 and s.size >= k else float("inf"),
            sk1=float(s[k]) if s.size > k else 0.0))

    @property
    def total(self) -> float:
        return float(sum(self.flops.values()))
