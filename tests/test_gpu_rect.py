"""Rectangular HODLR matrices (Sec. 6) on the device: products with A and A^T
and the |A|_2 estimate against the rectangular oracle (needs an MI355X)."""
import numpy as np
import pytest

import hodlr_gen as G
import oracle as O
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


QR_SHAPES = [  # m, n, n_min, rank, row partition override, rank_cap
    (40, 20, 5, 2, None, 16),
    (61, 37, 6, 2, None, 16),
    (48, 32, 8, 2, [0, 8, 20, 28, 48], 16),  # square and tall leaves mixed
    (100, 64, 8, 3, None, 32),
]


def _dense_factors(H, F, m, n):
    Y = H.hodlr_qr_matmul(F, "Y", H.colmajor(np.eye(n))).cpu().numpy()
    T = H.hodlr_qr_matmul(F, "T", H.colmajor(np.eye(n))).cpu().numpy()
    Rp = H.hodlr_qr_matmul(F, "R", H.colmajor(np.eye(n))).cpu().numpy()
    return Y, T, Rp


@pytest.mark.parametrize("m,n,nmin,k,roff,cap", QR_SHAPES)
def test_rect_qr_lossless_equals_permuted_householder(H, m, n, nmin, k, roff, cap):
    """eps = 0: Y, T and R on its pivot rows equal the dense permuted
    Householder QR (column c reflected onto its pivot row), entrywise."""
    inp = G.rect_gaussian_hodlr(m, n, nmin, k, seed=3, row_off=roff)
    A = inp.to_dense()
    piv = inp.pivot_rows()
    F = H.hodlr_qr(H.hodlr_build_rect(inp, rank_cap=cap), 0.0, anorm=1.0)
    Y, T, Rp = _dense_factors(H, F, m, n)
    Yd, Td, Rd = RR.perm_house_qr(A, piv)
    print(f"m={m} n={n}: Y {np.abs(Y - Yd).max():.2e} T {np.abs(T - Td).max():.2e} "
          f"R {np.abs(Rp - Rd[piv]).max():.2e}", flush=True)
    assert np.abs(Y - Yd).max() <= 1e-12
    assert np.abs(T - Td).max() <= 1e-12
    assert np.abs(Rp - Rd[piv]).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("m,n,nmin,k,seed", [(2000, 1000, 63, 3, 11), (1200, 700, 50, 4, 12),
                                             (3000, 1024, 128, 2, 13)])
def test_rect_qr_against_oracle(H, m, n, nmin, k, seed):
    """eps = 1e-10 (the oracle's |A|_2 on both sides): R on its pivot rows and Q
    applied to a random block against the rectangular oracle, the backward
    error of A = Q R and Q's orthogonality on it, the maximal ranks, and least
    squares against LAPACK."""
    inp = G.rect_gaussian_hodlr(m, n, nmin, k, seed=seed)
    root = RR.rfrom_input(inp)
    an = RR.rnorm2_est(root)
    ref = RR.rhqr(root, 1e-10, anorm=an)
    A = H.hodlr_build_rect(inp, rank_cap=64)  # T's ranks reach 36 and 44
    F = H.hodlr_qr(A, 1e-10, anorm=an)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 8))
    Xm = rng.standard_normal((m, 8))
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    rR = _rel(RX, O.hmat(RR.pivot_r(ref.R), X))
    QX = H.hodlr_apply_q(F, H.colmajor(Xm)).cpu().numpy()
    rQ = float(np.linalg.norm(QX - RR.rect_apply_q(ref, Xm)) / np.linalg.norm(Xm))
    print(f"m={m} n={n}: relR {rR:.2e} relQ {rQ:.2e}", flush=True)
    assert rR <= 1e-8 and rQ <= 1e-8
    # backward: A X = Q (R X), R X placed on the pivot rows
    RXm = np.zeros((m, 8))
    RXm[inp.pivot_rows()] = RX
    QRX = H.hodlr_apply_q(F, H.colmajor(RXm)).cpu().numpy()
    AX = H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy()
    assert np.linalg.norm(AX - QRX) / (an * np.linalg.norm(X)) <= 10 * 1e-10
    QtQ = H.hodlr_apply_q(F, H.colmajor(QX), trans=True).cpu().numpy()
    assert np.linalg.norm(QtQ - Xm) / np.linalg.norm(Xm) <= 10 * 1e-10
    info = H.hodlr_qr_info(F)
    assert info["max_rank_r"] == RR.rmax_ranks(ref.R)
    assert info["max_rank_y"] == RR.rmax_ranks(ref.Y)
    assert info["max_rank_t"] == RR.rmax_ranks(ref.T)
    if m <= 2000:
        b = rng.standard_normal((m, 3))
        x = H.hodlr_lstsq(F, H.colmajor(b)).cpu().numpy()
        xd = np.linalg.lstsq(inp.to_dense(), b, rcond=None)[0]
        assert np.abs(x - xd).max() <= 1e-7 * np.abs(xd).max()


def test_rect_qr_table5_example(H):
    """Table 5, random rectangular example: 8000 x 4000, rank-one blocks, n_min
    250, eps 1e-10 (Gaussian stand-in, as in the oracle's pin): the device
    factors have the printed maximal ranks of Y, T and R (8, 12, 8), and meet
    the backward and orthogonality bounds on a random block."""
    inp = G.rect_gaussian_hodlr(8000, 4000, 250, 1, seed=5, shift=0.0)
    A = H.hodlr_build_rect(inp, rank_cap=32)
    an = RR.rnorm2_est(RR.rfrom_input(inp))
    F = H.hodlr_qr(A, 1e-10, anorm=an)
    info = H.hodlr_qr_info(F)
    print("ranks Y, T, R:", info["max_rank_y"], info["max_rank_t"], info["max_rank_r"], flush=True)
    assert (info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]) == (8, 12, 8)
    X = np.random.default_rng(5).standard_normal((4000, 8))
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    RXm = np.zeros((8000, 8))
    RXm[inp.pivot_rows()] = RX
    QRX = H.hodlr_apply_q(F, H.colmajor(RXm)).cpu().numpy()
    AX = H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy()
    assert np.linalg.norm(AX - QRX) / (an * np.linalg.norm(X)) <= 10 * 1e-10


SITE = {1: "S", 2: "A12", 3: "update", 4: "T", 5: "E"}


def _device_log(H, F):
    out = {}
    for r in H.hodlr_qr_ranklog(F):
        site = int(r[0])
        if site == 0:  # the up-front orthogonalisation (the oracle does it lazily)
            continue
        key = (SITE[site], int(r[1]), int(r[2]))
        if site in (1, 4):
            key += (int(r[3]),)
        elif site == 3:
            key += (int(r[3]), int(r[4]))
        out[key] = (int(r[5]), int(r[6]))
    return out


def _oracle_log(ref):
    """The oracle's keys (site, rows, columns, ...) on the device's naming: the
    node by its column range."""
    out = {}
    for t in ref.counter.truncs:
        k = t["key"]
        out[(k[0], k[3], k[4]) + tuple(k[5:])] = (t["w"], t["k"])
    return out


@pytest.mark.parametrize("m,n,nmin,k,seed", [(2000, 1000, 63, 3, 11), (3000, 1024, 128, 2, 13)])
def test_rect_rank_log(H, m, n, nmin, k, seed):
    """Every recompression of the rectangular factorisation, E groups included,
    takes the oracle's decision (input width and kept rank)."""
    inp = G.rect_gaussian_hodlr(m, n, nmin, k, seed=seed)
    root = RR.rfrom_input(inp)
    an = RR.rnorm2_est(root)
    ref = RR.rhqr(root, 1e-10, anorm=an)
    F = H.hodlr_qr(H.hodlr_build_rect(inp, rank_cap=64), 1e-10, anorm=an)
    dev, ora = _device_log(H, F), _oracle_log(ref)
    assert set(dev) == set(ora)
    assert sum(1 for key in ora if key[0] == "E") > 0
    bad = [(key, dev[key], ora[key]) for key in ora if dev[key] != ora[key]]
    assert not bad, bad[:5]
