"""The allocation-free apply-Q entry point (hodlr_apply_q_noalloc) against
hodlr_apply_q, through the C ABI: two calls in a row on the same device, the
second with a smaller factor and fewer columns, and a factor too large for the
static scratch refused on the host.  The bar: relative difference <= 1e-13 (the
same kernels; the columns per pass can differ, which changes the rounding
order of the projections)."""
import ctypes as C

import numpy as np
import pytest

import hodlr_gen as G

pytestmark = pytest.mark.gpu

EPS = 1e-10


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1809_10585_amd as H
    lib = H.load()
    f = lib.hodlr_apply_q_noalloc
    f.restype = C.c_int32
    f.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
    return H


def _noalloc(H, F, X, trans):
    import torch
    lib = H.load()
    st = torch.cuda.current_stream()
    ld = X.stride(1) if X.shape[1] > 1 else X.shape[0]
    rc = lib.hodlr_apply_q_noalloc(F.handle, 1 if trans else 0, X.shape[1], C.c_void_p(X.data_ptr()), ld,
                                   C.c_void_p(int(st.cuda_stream)))
    return rc


def _case(H, n, leaf, k, cap, nrhs, seed):
    inp = G.gaussian_hodlr(n, leaf, k, seed=seed) if k else G.expkernel_hodlr(n, leaf, 2)
    A = H.hodlr_build(inp, rank_cap=cap)
    F = H.hodlr_qr(A, EPS)
    X = np.random.default_rng(seed).standard_normal((n, nrhs))
    return F, X


def test_noalloc_matches_apply_q_two_calls(H):
    for (n, leaf, k, cap, nrhs, seed) in [(8192, 256, 0, 16, 70, 1), (2048, 256, 3, 32, 3, 2)]:
        F, X = _case(H, n, leaf, k, cap, nrhs, seed)
        for trans in (False, True):
            ref = H.hodlr_apply_q(F, H.colmajor(X), trans=trans).cpu().numpy()
            Xg = H.colmajor(X)
            assert _noalloc(H, F, Xg, trans) == 0, H.load().hodlr_last_error()
            out = Xg.cpu().numpy()
            err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
            print(f"n={n} nrhs={nrhs} trans={trans}: rel.diff {err:.2e}")
            assert err <= 1e-13


def test_noalloc_refuses_oversize(H):
    """n = 65536 with rank capacity 64: the projections alone need 2 x 511 x 64 x 64
    doubles (33.5 MB), more than the 32 MiB scratch."""
    F, X = _case(H, 65536, 256, 0, 64, 2, 3)
    Xg = H.colmajor(X)
    rc = _noalloc(H, F, Xg, False)
    assert rc == -1
    assert b"scratch" in H.load().hodlr_last_error()
    assert np.array_equal(Xg.cpu().numpy(), X)  # untouched
