"""The served request loop: scheduling logic on the CPU with a stand-in
backend, and on the GPU the bitwise alone-vs-in-the-mix property."""
import time

import numpy as np
import pytest

from paper_1809_10585_amd import serve


class FakeBackend:
    """Sleeps instead of computing (a batch of b factorisations costs
    qr_s (1 + (b - 1) / 4)); factors are (matrix, serial) tuples."""

    def __init__(self, sizes, qr_s=0.004, solve_s=0.001):
        self.sizes, self.qr_s, self.solve_s = sizes, qr_s, solve_s
        self.made = 0
        self.live = set()
        self.released = []
        self.batches = []
        self.queued = 0
        self.sides = []

    def footprint(self, key):
        return float(self.sizes[key])

    def qr_batch(self, keys):
        self.batches.append(len(keys))
        time.sleep(self.qr_s * (1.0 + 0.25 * (len(keys) - 1)))
        out = []
        for k in keys:
            F = (k, self.made)
            self.made += 1
            self.live.add(F)
            out.append(F)
        return out

    def solve_async(self, F, nrhs, seed, side=False):
        assert F in self.live, "solve with a released factor"
        self.queued += 1
        self.sides.append(side)
        time.sleep(self.solve_s)
        return ("X", F, nrhs, seed)

    def sync(self):
        self.queued = 0

    def release(self, F):
        self.live.remove(F)
        self.released.append(F)


def test_poisson_requests_shape():
    reqs = serve.poisson_requests(200, rate=100.0, n_matrices=5, seed=4)
    assert [r.rid for r in reqs] == list(range(200))
    t = [r.arrival for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert abs(np.mean(np.diff([0.0] + t)) - 0.01) < 0.004
    qrs = {r.rid for r in reqs if r.kind == "qr"}
    for r in reqs:
        if r.kind == "solve":
            assert r.key in qrs and r.key < r.rid and 1 <= r.nrhs <= 64


def test_scheduler_serves_everything_and_batches():
    reqs = serve.poisson_requests(120, rate=2000.0, n_matrices=4, seed=1)
    b = FakeBackend([1.0, 1.0, 1.0, 1.0])
    sch = serve.Scheduler(b, budget=1e9, keep_results=True)
    out = sch.run(reqs)
    assert all(r.done >= r.start >= r.arrival for r in out)
    assert sch.max_qr_batch > 1 and sch.steps < len(reqs)
    mat = {r.rid: r.key for r in out if r.kind == "qr"}
    for r in out:
        if r.kind == "qr":
            assert r.result[0] == r.key
        else:  # the factor of the QR request it names (never evicted here)
            assert r.result[1] == out[r.key].result
            assert r.result[1][0] == mat[r.key]
    s = serve.summarize(out)
    assert s["requests"] == 120 and s["p99_ms"] >= s["p50_ms"] > 0


def test_scheduler_budget_evicts_and_refactors():
    # room for two factors: older ones are evicted; later solves on them refactor
    reqs = serve.poisson_requests(150, rate=3000.0, n_matrices=6, seed=2, p_qr=0.5)
    b = FakeBackend([1.0] * 6, qr_s=0.002, solve_s=0.0005)
    sch = serve.Scheduler(b, budget=2.5, keep_results=True)
    out = sch.run(reqs)
    assert all(r.done > 0 for r in out)
    assert sch.evictions > 0 and sch.refactored > 0
    assert len(sch.resident) <= 2 and len(b.live) == len(sch.factors) <= 2
    for r in out:
        if r.kind == "solve":  # solved with a factor of the right matrix
            assert r.result[1][0] == out[r.key].key


def test_plain_loop_is_fifo_one_request_per_step():
    reqs = serve.poisson_requests(60, rate=5000.0, n_matrices=3, seed=3)
    b = FakeBackend([1.0] * 3)
    sch = serve.Scheduler(b, budget=1e9, batching=False)
    out = sch.run(reqs)
    starts = [r.start for r in sorted(out, key=lambda r: r.arrival)]
    assert starts == sorted(starts)
    assert sch.max_qr_batch == 1 and sch.steps == len(reqs)
    assert max(b.batches) == 1


def test_batching_beats_plain_under_load():
    reqs = lambda: serve.poisson_requests(80, rate=3000.0, n_matrices=4, seed=5)
    served = serve.summarize(serve.Scheduler(FakeBackend([1.0] * 4), budget=1e9).run(reqs()))
    plain = serve.summarize(serve.Scheduler(FakeBackend([1.0] * 4), budget=1e9, batching=False).run(reqs()))
    assert served["p99_ms"] < plain["p99_ms"]


def test_solves_overlap_the_factorisations():
    """Solves whose factors were resident before a step are queued on the
    second stream ahead of the step's factorisations."""
    reqs = serve.poisson_requests(200, rate=4000.0, n_matrices=4, seed=6)
    b = FakeBackend([1.0] * 4)
    sch = serve.Scheduler(b, budget=1e9)
    sch.run(reqs)
    assert sch.overlapped > 0 and any(b.sides) and not all(b.sides)


def test_no_eviction_without_admission():
    """A request that cannot fit even after evicting every evictable factor
    evicts nothing (unless it is forced in as the step's only request)."""
    b = FakeBackend([1.0] * 4)
    sch = serve.Scheduler(b, budget=2.5)
    for rid in (1, 2):
        F = b.qr_batch([rid])[0]
        sch.factors[rid], sch.resident[rid] = F, 1.0
    assert not sch._make_room(2.0, keep={1})
    assert list(sch.resident) == [1, 2] and sch.evictions == 0
    assert sch._make_room(1.5, keep={1}) and list(sch.resident) == [1] and sch.evictions == 1
    assert not sch._make_room(3.0, keep={1}, force=True) and list(sch.resident) == [1]


def test_plain_loop_keeps_the_budget():
    reqs = serve.poisson_requests(120, rate=3000.0, n_matrices=6, seed=7, p_qr=0.6)
    b = FakeBackend([1.0] * 6, qr_s=0.001, solve_s=0.0002)
    sch = serve.Scheduler(b, budget=2.5, batching=False, keep_results=True)
    out = sch.run(reqs)
    assert all(r.done > 0 for r in out)
    assert sch.evictions > 0 and len(sch.resident) <= 2
    for r in out:
        if r.kind == "solve":
            assert r.result[1][0] == out[r.key].key


def test_request_pools():
    pools = [[0, 1, 2], [3, 4]]
    reqs = serve.poisson_requests(400, rate=100.0, n_matrices=5, seed=8, pools=pools)
    keys = [r.key for r in reqs if r.kind == "qr"]
    share = np.mean([k >= 3 for k in keys])
    assert set(keys) == {0, 1, 2, 3, 4} and 0.4 < share < 0.6


@pytest.mark.gpu
def test_served_results_equal_alone_bitwise():
    """Factors and solutions of a served run (requests batched with others)
    equal those of each request run alone."""
    import torch
    import hodlr_gen as G
    import paper_1809_10585_amd as H
    assert torch.cuda.is_available()
    ns = [1024, 1500, 2048, 3000]
    mats = [H.hodlr_build(G.gaussian_hodlr(n, 256, 2 + i % 3, seed=40 + i), rank_cap=32)
            for i, n in enumerate(ns)]
    reqs = serve.poisson_requests(24, rate=400.0, n_matrices=len(mats), seed=9)
    be = serve.GpuBackend(H, mats, 1e-10)
    print("serving", len(reqs), "requests", flush=True)
    sch = serve.Scheduler(be, budget=1e12, keep_results=True)
    mixed = sch.run(reqs)
    print("served in", sch.steps, "steps, largest batch", sch.max_qr_batch, flush=True)
    assert sch.max_qr_batch > 1
    for r in mixed:
        if r.kind == "qr":
            F = H.hodlr_qr(mats[r.key], 1e-10)
            X = np.random.default_rng(r.rid).standard_normal((F.n, 3))
            a = H.hodlr_qr_matmul(r.result, "R", H.colmajor(X)).cpu().numpy()
            b = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
            assert np.array_equal(a, b)
        else:
            F = H.hodlr_qr(mats[mixed[r.key].key], 1e-10)
            x = be.solve(F, r.nrhs, r.seed)
            assert np.array_equal(r.result.cpu().numpy(), x.cpu().numpy())
