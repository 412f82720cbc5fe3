"""Rectangular HODLR matrices (Sec. 6) on the device: products with A and A^T
and the |A|_2 estimate against the rectangular oracle (needs an MI355X)."""
import numpy as np
import pytest

import hodlr_gen as G
from oracle import rect as RR

pytestmark = pytest.mark.gpu

SHAPES = [  # m, n, n_min, rank, row partition override
    (40, 20, 5, 2, None),
    (61, 37, 6, 2, None),
    (48, 32, 8, 2, [0, 8, 20, 28, 48]),
    (2000, 1000, 63, 3, None),
    (40000, 20000, 250, 2, None),  # products over >= 32768 output rows (64-row tiles)
]


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1809_10585_amd as H
    H.load()
    return H


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("m,n,nmin,k,roff", SHAPES)
def test_rect_products_against_oracle(H, m, n, nmin, k, roff):
    inp = G.rect_gaussian_hodlr(m, n, nmin, k, seed=7, row_off=roff)
    A = H.hodlr_build_rect(inp, rank_cap=16)
    root = RR.rfrom_input(inp)
    rng = np.random.default_rng(8)
    for s in (1, 3, 9, 20):
        print(f"m={m} n={n} s={s}", flush=True)
        X = rng.standard_normal((n, s))
        Yv = rng.standard_normal((m, s))
        AX = H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy()
        AtY = H.hodlr_matmul(A, H.colmajor(Yv), trans=True).cpu().numpy()
        assert AX.shape == (m, s) and AtY.shape == (n, s)
        assert _rel(AX, RR.rhmat(root, X)) <= 1e-13
        assert _rel(AtY, RR.rhmatT(root, Yv)) <= 1e-13


@pytest.mark.parametrize("m,n,nmin", [(61, 37, 6), (2000, 1000, 63)])
def test_rect_norm_estimate(H, m, n, nmin):
    inp = G.rect_gaussian_hodlr(m, n, nmin, 2, seed=9)
    A = H.hodlr_build_rect(inp, rank_cap=16)
    ref = RR.rnorm2_est(RR.rfrom_input(inp))
    assert H.hodlr_norm2_est(A) == pytest.approx(ref, rel=1e-12)
    true = np.linalg.norm(inp.to_dense(), 2)
    assert 0.99 * true <= ref <= true * (1 + 1e-12)  # a power-iteration estimate from below
