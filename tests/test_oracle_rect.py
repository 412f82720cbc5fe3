"""Pins of the rectangular-HODLR oracle (oracle/rect.py, Sec. 6): the dense
permuted Householder QR against LAPACK, the HODLR algorithm at eps = 0 against
it, the square special case against Algorithm hQR, backward bounds at
eps = 1e-10, least squares against LAPACK, and the ranks and memory of
Table 5's random rectangular example."""
import os

import numpy as np
import pytest

import hodlr_gen as G
import oracle as O
from oracle import rect as RR

HERE = os.path.dirname(__file__)

SHAPES = [  # m, n, n_min, rank, row partition override (None: proportional)
    (24, 12, 12, 2, None),            # one leaf: a dense tall QR
    (40, 20, 5, 2, None),             # depth 2, m_j = 2 n_j
    (61, 37, 6, 2, None),             # ragged leaves, uneven split
    (100, 64, 8, 3, None),            # depth 3
    (48, 32, 8, 2, [0, 8, 20, 28, 48]),  # some leaves square (m_j = n_j), one 20 x 8
]


def _inp(m, n, nmin, k, roff, seed=3):
    return G.rect_gaussian_hodlr(m, n, nmin, k, seed=seed, row_off=roff)


def test_perm_house_qr_matches_lapack():
    """Column c reflected onto row piv[c]: LAPACK dgeqrf of the rows in pivot
    order, rows put back (R, the Householder vectors and tau)."""
    H = _inp(61, 37, 6, 2, None)
    A, piv = H.to_dense(), H.pivot_rows()
    Y, T, R = RR.perm_house_qr(A, piv)
    order = np.concatenate([piv, np.setdiff1d(np.arange(A.shape[0]), piv)])
    h, tau = np.linalg.qr(A[order], mode="raw")
    h = h.T
    n = A.shape[1]
    assert np.allclose(R[order][:n], np.triu(h[:n]), rtol=0, atol=1e-13 * np.abs(A).max())
    assert np.allclose(Y[order], np.tril(h, -1)[:, :n] + np.eye(A.shape[0], n), atol=1e-13)
    assert np.allclose(np.diag(T), tau, atol=1e-15)
    free = np.setdiff1d(np.arange(A.shape[0]), piv)
    assert np.all(R[free] == 0.0)
    for c in range(n):  # unit at its pivot, zero on the pivots of earlier columns
        assert Y[piv[c], c] == 1.0 and np.all(Y[piv[:c], c] == 0.0)


@pytest.mark.parametrize("m,n,nmin,k,roff", SHAPES)
def test_eps0_equals_dense_permuted_qr(m, n, nmin, k, roff):
    H = _inp(m, n, nmin, k, roff)
    A = H.to_dense()
    F = RR.rhqr(H, 0.0)
    Y, T, R, Q = RR.rect_dense_factors(F)
    Yd, Td, Rd = RR.perm_house_qr(A, H.pivot_rows())
    assert np.abs(Y - Yd).max() <= 1e-12
    assert np.abs(T - Td).max() <= 1e-12
    assert np.abs(R - Rd).max() <= 1e-12 * np.abs(A).max()
    assert np.array_equal(F.piv, H.pivot_rows())


def test_square_partition_is_algorithm_hqr():
    """With m_j = n_j for every leaf there are no free rows: the factors and
    every recompression equal Algorithm hQR's (square oracle) at eps = 1e-10."""
    n = 96
    R = G.rect_gaussian_hodlr(n, n, 12, 3, seed=8)
    S = G.HodlrInput(n=n, levels=R.levels, leaf_off=R.col_off, leaves=R.leaves, blocks=R.blocks)
    Fr = RR.rhqr(R, 1e-10)
    Fs = O.hqr(S, 1e-10)
    assert Fr.anorm == pytest.approx(Fs.anorm, rel=1e-14)
    Yr, Tr, Rr, _ = RR.rect_dense_factors(Fr)
    Ys, Ts, Rs, _ = O.dense_factors(Fs)
    assert np.abs(Yr - Ys).max() <= 1e-12 and np.abs(Tr - Ts).max() <= 1e-12
    assert np.abs(Rr - Rs).max() <= 1e-12 * np.abs(Rs).max()
    assert [t["k"] for t in Fr.counter.truncs] == [t["k"] for t in Fs.counter.truncs]


@pytest.mark.parametrize("m,n,nmin,k", [(2000, 1000, 63, 1), (1200, 700, 50, 4)])
def test_backward_bounds(m, n, nmin, k):
    H = G.rect_gaussian_hodlr(m, n, nmin, k, seed=5, shift=0.0 if k == 1 else 4.0)
    F = RR.rhqr(H, 1e-10)
    acc = RR.rect_accuracy(F, H.to_dense())
    assert acc["e_orth"] <= 1e-9 and acc["e_acc_rel"] <= 1e-9, acc


def test_exact_rank_is_lossless():
    """Blocks of exact rank stay exact: eps = 1e-10 gives the eps = 0 factors
    up to the truncated noise."""
    H = _inp(100, 64, 8, 3, None)
    A = H.to_dense()
    Y0, T0, R0, _ = RR.rect_dense_factors(RR.rhqr(H, 0.0))
    Y1, T1, R1, _ = RR.rect_dense_factors(RR.rhqr(H, 1e-10))
    sc = np.abs(A).max()
    assert np.abs(R1 - R0).max() <= 1e-9 * sc and np.abs(Y1 - Y0).max() <= 1e-9


def test_least_squares_matches_lapack():
    H = _inp(100, 64, 8, 3, None)
    A = H.to_dense()
    b = np.random.default_rng(1).standard_normal((100, 3))
    x = RR.rect_lstsq(RR.rhqr(H, 0.0), b)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()


def _golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "rect_table5.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def _mem(M):
    if M.is_leaf:
        return M.D.size
    s = _mem(M.c1) + _mem(M.c2)
    for b in (M.A12, M.A21):
        if b is not None:
            s += b.L.shape[0] * b.k + b.R.shape[1] * b.k
    return s


def test_table5_random_rectangular_ranks_and_memory():
    """Table 5, random rectangular example (8000 x 4000, rank one, n_min 250,
    eps 1e-10; random Gaussian diagonal blocks and rank-one factors stand in for
    the unstated distribution): maximal ranks of Y, T, R as printed, memory of
    Y and T and of R relative to A within 0.1 of the printed ratios."""
    g = _golden()
    H = G.rect_gaussian_hodlr(int(g["m"]), int(g["n"]), int(g["n_min"]), int(g["rank"]), seed=5, shift=0.0)
    F = RR.rhqr(H, 1e-10)
    assert RR.rmax_ranks(F.Y) == g["max_rank_Y"]
    assert RR.rmax_ranks(F.T) == g["max_rank_T"]
    assert RR.rmax_ranks(F.R) == g["max_rank_R"]
    A = RR.rfrom_input(H)
    assert abs((_mem(F.Y) + _mem(F.T)) / _mem(A) - g["memory_Y_and_T"]) <= 0.1
    assert abs(_mem(F.R) / _mem(A) - g["memory_R"]) <= 0.1
