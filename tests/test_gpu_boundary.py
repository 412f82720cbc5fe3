"""The C ABI's memory, stream and view contract on the GPU (needs an MI355X):
device memory from the installed allocator (PyTorch's caching allocator
through hodlr_set_allocator), stream-ordered apply-Q / solve / products that
may run on one handle from several streams at once, borrowed factor views
(hodlr_qr_factor) and the device-flag check (hodlr_check)."""
import numpy as np
import pytest

import hodlr_gen as G
from helpers import leaf_sizes

pytestmark = pytest.mark.gpu

EPS = 1e-10


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1809_10585_amd as H
    H.load()
    return H


@pytest.fixture(scope="module")
def fac(H):
    inp = G.expkernel_hodlr(8192, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    F = H.hodlr_qr(A, EPS, anorm=0.186 * 8192)
    return inp, A, F


def test_memory_comes_from_the_torch_allocator(H):
    """hodlr_qr's factors are blocks of torch's caching allocator: torch's
    allocated-bytes counter grows by the factors' size and falls back when the
    handle is released."""
    import torch
    torch.cuda.synchronize()
    inp = G.expkernel_hodlr(4096, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    F = H.hodlr_qr(A, EPS, anorm=0.186 * 4096)
    torch.cuda.synchronize()
    grew = torch.cuda.memory_allocated() - before
    dev = H.hodlr_qr_info(F)["device_bytes"]
    print(f"torch allocated +{grew} bytes, factors hold {dev}")
    assert grew >= dev
    del F
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before


def test_without_the_torch_allocator(H):
    """hodlr_set_allocator(NULL, NULL): hipMalloc / hipMallocAsync again, same bits."""
    import torch
    inp = G.gaussian_hodlr(1024, 128, 4, seed=7)
    X = np.random.default_rng(1).standard_normal((inp.n, 5))
    A = H.hodlr_build(inp, rank_cap=32)
    F = H.hodlr_qr(A, EPS)
    ref = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
    H.use_torch_allocator(False)
    try:
        A2 = H.hodlr_build(inp, rank_cap=32)
        F2 = H.hodlr_qr(A2, EPS)
        out = H.hodlr_apply_q(F2, H.colmajor(X)).cpu().numpy()
        sol = H.hodlr_solve(F2, H.colmajor(X)).cpu().numpy()
        torch.cuda.synchronize()
        del F2, A2
    finally:
        H.use_torch_allocator(True)
    assert np.array_equal(out, ref)
    assert np.isfinite(sol).all()


def test_calls_are_stream_ordered_and_concurrent(H, fac):
    """apply_q, solve and the products queued on two streams at once on the
    same handle, without waiting in between, give the bits of the same calls
    run one after another (each call has its own temporaries)."""
    import torch
    inp, A, F = fac
    rng = np.random.default_rng(3)
    Xs = [rng.standard_normal((inp.n, s)) for s in (3, 70, 1, 16)]
    seq = []
    for X in Xs:
        seq.append((H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy(),
                    H.hodlr_solve(F, H.colmajor(X)).cpu().numpy(),
                    H.hodlr_qr_matmul(F, "R", H.colmajor(X), trans=True).cpu().numpy()))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ins = [(H.colmajor(X), H.colmajor(X), H.colmajor(X)) for X in Xs]
    torch.cuda.synchronize()
    outs = []
    for i, (a, b, c) in enumerate(ins):
        st = s1 if i % 2 == 0 else s2
        with torch.cuda.stream(st):
            a = H.hodlr_apply_q(F, a, stream=st)
            b = H.hodlr_solve(F, b, stream=st)
            z = H.hodlr_qr_matmul(F, "R", c, trans=True, stream=st)
            outs.append((a, b, z))
    torch.cuda.synchronize()
    for (a, b, z), (ra, rb, rz) in zip(outs, seq):
        assert np.array_equal(a.cpu().numpy(), ra)
        assert np.array_equal(b.cpu().numpy(), rb)
        assert np.array_equal(z.cpu().numpy(), rz)


def test_factor_views(H, fac):
    """hodlr_qr_factor: Y, T, R as borrowed HODLR matrices, usable with
    hodlr_matmul and hodlr_export exactly like hodlr_qr_matmul / _export."""
    inp, A, F = fac
    X = np.random.default_rng(4).standard_normal((inp.n, 6))
    ls = leaf_sizes(inp)
    for w in "YTR":
        V = H.hodlr_qr_factor(F, w)
        for tr in (False, True):
            a = H.hodlr_matmul(V, H.colmajor(X), trans=tr).cpu().numpy()
            b = H.hodlr_qr_matmul(F, w, H.colmajor(X), trans=tr).cpu().numpy()
            assert np.array_equal(a, b), (w, tr)
        ea, eb = H.hodlr_export(V, ls), H.hodlr_qr_export(F, w, ls)
        for key in ea:
            assert np.array_equal(ea[key], eb[key]), (w, key)
    with pytest.raises(H.HodlrError):
        H.hodlr_qr(H.hodlr_qr_factor(F, "R"), EPS)


def test_check_reports_device_flags(H):
    inp = G.config(0)
    F = H.hodlr_qr(H.hodlr_build(inp, rank_cap=64), EPS)
    H.hodlr_check(F)
    with pytest.raises(H.HodlrError) as e:
        H.hodlr_qr(H.hodlr_build(inp, rank_cap=8), EPS)
    assert e.value.status == -4


def test_ranklog_shape(H, fac):
    inp, A, F = fac
    log = H.hodlr_qr_ranklog(F)
    info = H.hodlr_qr_info(F)
    assert log.shape == (info["n_truncations"], 7)
    assert ((log[:, 6] >= 0) & (log[:, 6] <= log[:, 5])).all()
    assert set(np.unique(log[:, 0])) <= {0, 1, 2, 3, 4}


def test_allocation_failure_is_reported(H):
    """A caller's allocator that refuses once a small budget is spent: hodlr_qr
    returns HODLR_ENOMEM (releasing what it had taken) instead of failing
    later, and the library works again with the normal allocator."""
    import ctypes as C
    import torch
    from paper_1809_10585_amd import _lib
    inp = G.expkernel_hodlr(4096, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    state = {"used": 0, "live": {}, "budget": 4 << 20}
    raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc
    raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete

    def alloc(size, stream, ctx):
        if state["used"] + size > state["budget"]:
            return None
        p = int(raw_alloc(int(size), int(stream or 0)))
        state["used"] += size
        state["live"][p] = size
        return p

    def release(ptr, stream, ctx):
        state["used"] -= state["live"].pop(int(ptr))
        raw_delete(int(ptr))

    H.set_allocator(_lib.ALLOC_FN(alloc), _lib.RELEASE_FN(release))
    try:
        with pytest.raises(H.HodlrError) as e:
            H.hodlr_qr(A, EPS, anorm=0.186 * 4096)
        assert e.value.status == -2
        torch.cuda.synchronize()
        assert state["used"] == 0 and not state["live"]
    finally:
        H.use_torch_allocator(True)
    F = H.hodlr_qr(A, EPS, anorm=0.186 * 4096)
    H.hodlr_check(F)
