"""Served HODLR QR / solve requests with continuous batching on one GPU.

Requests (QR of a device-resident HODLR matrix, or a solve with the factor of
an earlier QR request) arrive over time.  One host thread runs the loop: at
every step it takes the requests that have arrived and are admissible and
  1. queues the solves whose factors are already resident on a second stream,
  2. runs all the step's factorisations as one `hodlr_qr_batched` call (every
     shape in one merged launch sequence) on the main stream, while those
     solves run beside it,
  3. queues the solves with factors made in this step behind them,
  4. waits for both streams;
requests arriving meanwhile join the next step.  Admission is by device
memory: a factor's footprint is the library's own count of the bytes it
holds (`hodlr_qr_info.device_bytes`).  Factors stay resident for later
solves; resident factors beyond the budget are evicted least recently used,
sparing those a pending solve needs (and only when the eviction lets the
request in), and a solve whose factor was evicted factorises its matrix again
first (counted in `refactored`).  `batching=False` serves one request per
step in arrival order (the plain loop it is compared with), under the same
budget.

Every library call is issued from the calling thread, one after the other.
Each factorisation in a batch computes exactly what it computes alone: the
library's kernels never mix the jobs of two factorisations (tested in
tests/test_serve.py on the GPU, and in tests/test_gpu_parity.py for the batched
call itself).

The loop takes a backend with `qr_batch(keys)`, `solve_async(factor, nrhs,
seed, side)`, `sync()`, `footprint(key)` and `release(factor)`, so it is
exercised on the CPU with a stand-in backend; `GpuBackend` binds it to the
library.
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
                     max_nrhs: int = 64, pools=None) -> list:
    """`count` requests with Exp(1/rate) gaps; each is a QR of a uniformly chosen
    matrix with probability p_qr, otherwise (when a QR was issued before) a
    solve with the factor of a uniformly chosen earlier QR request and
    nrhs ~ U{1..max_nrhs}.  pools: lists of matrix indices (one per generator);
    a QR request then picks a pool uniformly and a matrix of it uniformly."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out, qrs = [], []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        if not qrs or rng.random() < p_qr:
            if pools:
                pool = pools[int(rng.integers(len(pools)))]
                key = int(pool[int(rng.integers(len(pool)))])
            else:
                key = int(rng.integers(n_matrices))
            out.append(Request(rid, t, "qr", key))
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
        self.overlapped = 0  # solves that ran beside a step's factorisations

    def _resident_bytes(self):
        return sum(self.resident.values())

    def _make_room(self, need, keep, force=False):
        """Evict least recently used factors outside `keep` until `need` more
        bytes fit; returns whether they do.  Nothing is evicted unless the
        evictions make the room (or `force`: the request goes in regardless)."""
        if self._resident_bytes() + need <= self.budget:
            return True
        spare = sum(b for rid, b in self.resident.items() if rid not in keep)
        if self._resident_bytes() - spare + need > self.budget and not force:
            return False
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
            wanted = {p.key for p in pending if p.kind == "solve"}
            if r.kind == "qr":
                self._make_room(self.b.footprint(r.key), wanted, force=True)
                return [r], [], []
            if r.key in self.factors:
                return [], [], [r]
            if r.key in self.evicted:
                self._make_room(self.b.footprint(self.qr_matrix[r.key]), wanted, force=True)
                return [], [r.key], [r]
            return [], [], []  # its factorisation has not run yet (cannot happen in FIFO order)
        wanted = {p.key for p in pending if p.kind == "solve"}
        qrs, refs, need = [], [], 0.0
        for r in pending:
            if r.kind != "qr" or len(qrs) + len(refs) >= self.max_batch:
                continue
            fp = self.b.footprint(r.key)
            if self._make_room(need + fp, wanted, force=not (qrs or refs)):
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
                if self._make_room(need + fp, wanted, force=not (qrs or refs)):
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
            # solves with factors resident before this step run beside its QRs
            early = [r for r in solves if r.key in self.factors]
            late = [r for r in solves if r.key not in self.factors]
            outs = {}
            for r in early:
                self.resident.move_to_end(r.key)
                r.start = start
                outs[id(r)] = self.b.solve_async(self.factors[r.key], r.nrhs, r.seed, True)
            self.overlapped += len(early) if keys else 0
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
            for r in late:
                self.resident.move_to_end(r.key)
                r.start = start
                outs[id(r)] = self.b.solve_async(self.factors[r.key], r.nrhs, r.seed, False)
            self.b.sync()
            end = clock()
            for r in solves:
                r.done = end
                r.result = outs[id(r)] if self.keep else None
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
    """The library behind the loop: inputs resident on the device; QRs on the
    current stream, solves queued on it or on a second stream.  Footprints are
    the library's device_bytes of each matrix's factors, measured once by
    factorising every matrix (which also warms the kernels and the
    allocator)."""

    def __init__(self, H, matrices, eps: float):
        import torch
        self.H, self.torch, self.eps = H, torch, eps
        self.A = matrices
        self.side = torch.cuda.Stream()
        self._fp = []
        for i in range(0, len(matrices), 16):
            Fs = self.qr_batch(list(range(i, min(i + 16, len(matrices)))))
            self._fp += [float(H.hodlr_qr_info(F)["device_bytes"]) for F in Fs]
            del Fs

    def footprint(self, key):
        return self._fp[key]

    def qr_batch(self, keys):
        Fs = self.H.hodlr_qr_batched([self.A[k] for k in keys], self.eps)
        self.torch.cuda.synchronize()
        return Fs

    def solve_async(self, F, nrhs, seed, side=False):
        torch = self.torch
        st = self.side if side else torch.cuda.current_stream()
        if side:
            st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            g = torch.Generator(device="cuda")
            g.manual_seed(seed)
            B = torch.randn((nrhs, F.n), generator=g, dtype=torch.float64, device="cuda").t()
            return self.H.hodlr_solve(F, B, stream=st)

    def solve(self, F, nrhs, seed):
        X = self.solve_async(F, nrhs, seed)
        self.torch.cuda.synchronize()
        return X

    def sync(self):
        self.torch.cuda.synchronize()

    def release(self, F):
        del F
