"""Served HODLR QR / solve requests with continuous batching on one GPU.

A request stream (arrival times, kinds) is fed to a pool of `slots` workers,
each owning its own HIP stream: a request that arrives while others are on the
GPU starts as soon as a slot is free and its device-memory footprint fits the
budget, so the launch sequences of several factorisations overlap on the
device.  QR requests factorise a device-resident HODLR matrix with hodlr_qr and
keep the factors resident; solve requests run hodlr_solve with a resident
factor.  Resident factors beyond the budget are evicted least recently used.

Every request computes exactly what it computes alone: the library's kernels
never mix the jobs of two factorisations, so results are bitwise independent of
what else runs (tested in tests/test_serve.py).

The scheduling logic takes a backend with `qr(rid, key, stream)`, `solve(fkey,
nrhs, seed, stream)`, `footprint(key)`, `release(fkey)` and `stream(i)`, so it
can be exercised on the CPU with a stand-in backend; `GpuBackend` binds it to
the library.  A solve whose factor was evicted before it arrived factorises the
matrix again first (counted in `refactored`).
"""
from __future__ import annotations

import collections
import dataclasses
import threading
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
    """Continuous-batching loop: `slots` workers, admission by footprint
    against `budget` bytes, LRU eviction of resident factors that no pending
    solve needs.  A factor is used by one request at a time (handles are not
    shared between streams)."""

    def __init__(self, backend, slots: int, budget: float):
        self.b, self.slots, self.budget = backend, slots, budget
        self.lock = threading.Condition()
        self.resident = collections.OrderedDict()  # qr rid -> bytes (LRU order)
        self.busy = set()                          # factors in use by a running solve
        self.inflight = 0.0
        self.pending = collections.deque()
        self.finished = False
        self.evictions = 0
        self.refactored = 0
        self.evicted = set()   # qr rids whose factors were released
        self.qr_matrix = {}    # qr rid -> matrix index

    def _resident_bytes(self):
        return sum(self.resident.values())

    def _admit_qr(self, r):
        """Called with the lock held: may QR request r start now?  Evicts least
        recently used factors that neither a running nor a pending solve needs."""
        need = self.b.footprint(r.key)
        if self._resident_bytes() + self.inflight + need > self.budget:
            wanted = {p.key for p in self.pending if p.kind == "solve"} | self.busy
            for victim in list(self.resident):
                if self._resident_bytes() + self.inflight + need <= self.budget:
                    break
                if victim in wanted:
                    continue
                del self.resident[victim]
                self.b.release(victim)
                self.evicted.add(victim)
                self.evictions += 1
        return self._resident_bytes() + self.inflight + need <= self.budget or self.inflight == 0.0

    def _next(self):
        """Called with the lock held: the first pending request that can start."""
        for i, r in enumerate(self.pending):
            if r.kind == "solve":
                if r.key in self.evicted and r.key not in self.busy:
                    ok = self._admit_qr(Request(-1, 0.0, "qr", self.qr_matrix[r.key]))
                else:
                    ok = r.key in self.resident and r.key not in self.busy
            else:
                ok = self._admit_qr(r)
            if ok:
                del self.pending[i]
                return r
        return None

    def _worker(self, stream):
        while True:
            with self.lock:
                r = self._next()
                while r is None:
                    if self.finished and not self.pending:
                        return
                    self.lock.wait(0.001)
                    r = self._next()
                refactor = r.kind == "solve" and r.key in self.evicted
                if r.kind == "qr":
                    self.inflight += self.b.footprint(r.key)
                else:
                    self.busy.add(r.key)
                    if refactor:
                        self.evicted.discard(r.key)
                        self.refactored += 1
                        self.inflight += self.b.footprint(self.qr_matrix[r.key])
                    else:
                        self.resident.move_to_end(r.key)
            r.start = time.perf_counter() - self.t0
            if r.kind == "qr":
                r.result = self.b.qr(r.rid, r.key, stream)
            else:
                if refactor:
                    self.b.qr(r.key, self.qr_matrix[r.key], stream)
                r.result = self.b.solve(r.key, r.nrhs, r.seed, stream)
            r.done = time.perf_counter() - self.t0
            with self.lock:
                if r.kind == "qr":
                    self.inflight -= self.b.footprint(r.key)
                    self.resident[r.rid] = self.b.footprint(r.key)
                else:
                    if refactor:
                        fp = self.b.footprint(self.qr_matrix[r.key])
                        self.inflight -= fp
                        self.resident[r.key] = fp
                    self.busy.discard(r.key)
                self.lock.notify_all()

    def run(self, requests, time_scale: float = 1.0):
        """Release the requests at their arrival times (times time_scale) and
        serve them; returns them with start/done times filled in (seconds)."""
        self.t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(self.b.stream(i),)) for i in range(self.slots)]
        for w in workers:
            w.start()
        for r in requests:
            r.arrival *= time_scale
            delay = r.arrival - (time.perf_counter() - self.t0)
            if delay > 0:
                time.sleep(delay)
            with self.lock:
                if r.kind == "qr":
                    self.qr_matrix[r.rid] = r.key
                self.pending.append(r)
                self.lock.notify_all()
        with self.lock:
            self.finished = True
            self.lock.notify_all()
        for w in workers:
            w.join()
        return requests


def summarize(requests) -> dict:
    lat = np.array([r.done - r.arrival for r in requests])
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    return {"requests": len(requests), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_rps": len(requests) / span}


class GpuBackend:
    """The library behind the scheduler: inputs resident on the device, one HIP
    stream per worker slot, factors kept per QR request."""

    def __init__(self, H, matrices, eps: float, slots: int):
        import torch
        self.H, self.torch, self.eps = H, torch, eps
        self.A = matrices
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.factors = {}
        self.flock = threading.Lock()
        self._fp = [self._estimate(A) for A in matrices]

    @staticmethod
    def _estimate(A):
        # factors of the same partition and capacity (leaves twice, blocks three
        # times, n x cap temporaries) plus the schedule's workspace, as a bound
        return 64.0 * A.n * (A.rank_cap * (A.levels + 16) + 512)

    def stream(self, i):
        return self.streams[i]

    def footprint(self, key):
        return self._fp[key]

    def qr(self, rid, key, stream):
        F = self.H.hodlr_qr(self.A[key], self.eps, stream=stream)
        with self.flock:
            self.factors[rid] = F
        return F

    def solve(self, fkey, nrhs, seed, stream):
        torch = self.torch
        with self.flock:
            F = self.factors[fkey]
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        with torch.cuda.stream(stream):
            B = torch.randn((nrhs, F.n), generator=g, dtype=torch.float64, device="cuda").t()
            X = self.H.hodlr_solve(F, B, stream=stream)
        stream.synchronize()
        return X

    def release(self, fkey):
        with self.flock:
            self.factors.pop(fkey, None)
