"""Served HODLR QR / solve requests with continuous batching on one GPU.

Requests (QR of a device-resident HODLR matrix, or a solve with the factor of
an earlier QR request) arrive over time.  One host thread runs the loop: at
every step it takes the requests that have arrived and are admissible, runs
all their factorisations as one `hodlr_qr_batched` call (the library groups
them by shape and runs each group as one launch sequence), then their solves;
requests arriving meanwhile join the next step.  Factors stay resident for
later solves; resident factors beyond the device-memory budget are evicted
least recently used, sparing those a pending solve needs, and a solve whose
factor was evicted factorises its matrix again first (counted in
`refactored`).  `batching=False` serves one request per step in arrival order
(the plain loop it is compared with).

Every library call is issued from the calling thread, one after the other.
Each factorisation in a batch computes exactly what it computes alone: the
library's kernels never mix the jobs of two factorisations (tested in
tests/test_serve.py on the GPU, and in tests/test_gpu_parity.py for the batched
call itself).

The loop takes a backend with `qr_batch(keys)`, `solve(factor, nrhs, seed)`,
`footprint(key)` and `release(factor)`, so it is exercised on the CPU with a
stand-in backend; `GpuBackend` binds it to the library.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    kind: str               # "qr" or "solve"
    key: int                # qr: matrix index; solve: index of the qr request whose factor it uses
    nrhs: int = 0
    seed: int = 0
    start: float = -1.0
    done: float = -1.0
    result: object = None


def poisson_requests(count: int, rate: float, n_matrices: int, seed: int, p_qr: float = 0.5,
                     max_nrhs: int = 64) -> list:
    """`count` requests with Exp(1/rate) gaps; each is a QR of a uniformly chosen
    matrix with probability p_qr, otherwise (when a QR was issued before) a
    solve with the factor of a uniformly chosen earlier QR request and
    nrhs ~ U{1..max_nrhs}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out, qrs = [], []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        if not qrs or rng.random() < p_qr:
            out.append(Request(rid, t, "qr", int(rng.integers(n_matrices))))
            qrs.append(rid)
        else:
            out.append(Request(rid, t, "solve", int(qrs[rng.integers(len(qrs))]),
                               int(rng.integers(1, max_nrhs + 1)), int(rng.integers(1 << 30))))
    return out


class Scheduler:
    """Continuous batching from one host thread.  A step admits the arrived QR
    requests in arrival order while their factors fit the budget next to the
    resident ones (at most `max_batch` of them; one always, so the loop makes
    progress), plus the arrived solves whose factor is resident, is formed in
    this step, or was evicted (then its matrix is factorised again in this
    step).  keep_results: leave each request's factor or solution in its
    `result` (otherwise only the loop holds factors, so evicting frees them)."""

    def __init__(self, backend, budget: float, max_batch: int = 64, batching: bool = True,
                 keep_results: bool = False):
        self.b, self.budget, self.max_batch, self.batching = backend, budget, max_batch, batching
        self.keep = keep_results
        self.resident = collections.OrderedDict()  # qr rid -> bytes (LRU order)
        self.factors = {}                          # qr rid -> factor handle
        self.evicted = set()                       # qr rids whose factors were released
        self.qr_matrix = {}                        # qr rid -> matrix index
        self.evictions = 0
        self.refactored = 0
        self.steps = 0
        self.max_qr_batch = 0

    def _resident_bytes(self):
        return sum(self.resident.values())

    def _make_room(self, need, keep):
        """Evict least recently used factors outside `keep` until `need` more
        bytes fit; returns whether they do."""
        for victim in list(self.resident):
            if self._resident_bytes() + need <= self.budget:
                break
            if victim in keep:
                continue
            del self.resident[victim]
            self.b.release(self.factors.pop(victim))
            self.evicted.add(victim)
            self.evictions += 1
        return self._resident_bytes() + need <= self.budget

    def _plan(self, pending):
        """The requests of the next step: (qr requests, refactored qr rids, solves)."""
        if not self.batching:
            r = pending[0]
            if r.kind == "qr":
                return [r], [], []
            if r.key in self.factors:
                return [], [], [r]
            if r.key in self.evicted:
                return [], [r.key], [r]
            return [], [], []  # its factorisation has not run yet (cannot happen in FIFO order)
        wanted = {p.key for p in pending if p.kind == "solve"}
        qrs, refs, need = [], [], 0.0
        for r in pending:
            if r.kind != "qr" or len(qrs) + len(refs) >= self.max_batch:
                continue
            fp = self.b.footprint(r.key)
            if self._make_room(need + fp, wanted) or not (qrs or refs):
                qrs.append(r)
                need += fp
        batch_qr = {r.rid for r in qrs}
        solves = []
        for r in pending:
            if r.kind != "solve":
                continue
            if r.key in self.factors or r.key in batch_qr or r.key in refs:
                solves.append(r)
            elif r.key in self.evicted and len(qrs) + len(refs) < self.max_batch:
                fp = self.b.footprint(self.qr_matrix[r.key])
                if self._make_room(need + fp, wanted) or not (qrs or refs):
                    refs.append(r.key)
                    need += fp
                    solves.append(r)
        return qrs, refs, solves

    def run(self, requests, time_scale: float = 1.0):
        """Serve the requests at their arrival times (times time_scale); returns
        them with start/done times (seconds) and results filled in."""
        order = sorted(requests, key=lambda r: r.arrival)
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        pending = []
        i = 0
        while i < len(order) or pending:
            while i < len(order) and order[i].arrival * time_scale <= clock():
                r = order[i]
                if r.kind == "qr":
                    self.qr_matrix[r.rid] = r.key
                pending.append(r)
                i += 1
            if not pending:
                time.sleep(max(0.0, order[i].arrival * time_scale - clock()))
                continue
            qrs, refs, solves = self._plan(pending)
            if not (qrs or refs or solves):  # a solve waiting for its factor's step
                time.sleep(max(0.0, order[i].arrival * time_scale - clock()) if i < len(order) else 0.0)
                continue
            self.steps += 1
            start = clock()
            keys = [r.key for r in qrs] + [self.qr_matrix[f] for f in refs]
            if keys:
                self.max_qr_batch = max(self.max_qr_batch, len(keys))
                made = self.b.qr_batch(keys)
                done = clock()
                for rid, key, F in zip([r.rid for r in qrs] + refs, keys, made):
                    self.factors[rid] = F
                    self.resident[rid] = self.b.footprint(key)
                    self.evicted.discard(rid)
                self.refactored += len(refs)
                for r, F in zip(qrs, made):
                    r.start, r.done = start, done
                    r.result = F if self.keep else None
                del made
            for r in solves:
                self.resident.move_to_end(r.key)
                r.start = start
                x = self.b.solve(self.factors[r.key], r.nrhs, r.seed)
                r.done = clock()
                r.result = x if self.keep else None
            served = {id(r) for r in qrs} | {id(r) for r in solves}
            pending = [r for r in pending if id(r) not in served]
        return requests


def summarize(requests) -> dict:
    lat = np.array([r.done - r.arrival for r in requests])
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    return {"requests": len(requests), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_rps": len(requests) / span}


class GpuBackend:
    """The library behind the loop: inputs resident on the device, calls on the
    current stream, each returning when its work is done."""

    def __init__(self, H, matrices, eps: float):
        import torch
        self.H, self.torch, self.eps = H, torch, eps
        self.A = matrices
        self._fp = [self._estimate(A) for A in matrices]

    @staticmethod
    def _estimate(A):
        # factors of the same partition and capacity (leaves twice, blocks three
        # times, n x cap temporaries) plus the schedule's workspace, as a bound
        return 64.0 * A.n * (A.rank_cap * (A.levels + 16) + 512)

    def footprint(self, key):
        return self._fp[key]

    def qr_batch(self, keys):
        Fs = self.H.hodlr_qr_batched([self.A[k] for k in keys], self.eps)
        self.torch.cuda.synchronize()
        return Fs

    def solve(self, F, nrhs, seed):
        torch = self.torch
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        B = torch.randn((nrhs, F.n), generator=g, dtype=torch.float64, device="cuda").t()
        X = self.H.hodlr_solve(F, B)
        torch.cuda.synchronize()
        return X

    def release(self, F):
        del F
