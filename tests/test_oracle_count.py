"""Pins of the oracle's work counter and rank log (Sec. 4.1 cost estimates,
Table 1 operation costs, the accumulation order of the sums S~ and T~12).

The counter is pinned to values that do not come from the counter itself:
operation counts of the Householder loop counted one multiply/add at a time,
hand-evaluated closed forms (Householder QR 2mn^2 - 2n^3/3, GEMM 2mkn, the
recompression's parts), a hand count of a 4 x 4 HODLR product, and the
O(k^2 n log^2 n) growth law of the whole factorisation (Sec. 4.1, overall
complexity), fitted over n = 2^10 .. 2^15.
"""
import math

import numpy as np
import pytest

import hodlr_gen as G
import oracle as O
from oracle.count import Counter
from oracle.dense import qr_flops, trunc_flops


def _count_householder_loop(m, n):
    """Multiplies and adds of the column-by-column Householder QR of an m x n
    matrix (reflector of each column, applied to the later columns; Q not
    formed), counted operation by operation."""
    f = 0
    for j in range(min(m, n)):
        h = m - j                      # length of the column below the diagonal
        f += 2 * h                     # |x|^2
        f += h - 1                     # scale x2 by 1/(alpha - rho)
        f += (n - j - 1) * (2 * h)     # y^T A(:, c) for each later column
        f += (n - j - 1) * (2 * h)     # A(:, c) -= (gamma * dot) * y
    return f


def _count_t_recurrence(m, n):
    """Multiplies and adds of the forward T recurrence T[:j, j] =
    -gamma_j T[:j, :j] (Y[:, :j]^T y_j): Y^T y (j dot products of length
    m - j) and the triangular product (j(j+1)/2 multiply-adds)."""
    f = 0
    for j in range(n):
        f += 2 * j * (m - j)
        f += j * (j + 1)
    return f


@pytest.mark.parametrize("m,n", [(1000, 200), (600, 600), (296, 256), (5000, 40)])
def test_qr_flops_against_loop_count(m, n):
    bf = _count_householder_loop(m, n)
    assert abs(qr_flops(m, n) - bf) / bf <= 2.0 / n + 0.01


def test_qr_flops_wide_and_hand_values():
    # 2 m n^2 - 2 n^3 / 3 evaluated by hand
    assert qr_flops(1000, 10) == pytest.approx(199333.33333333333, rel=1e-12)
    assert qr_flops(800, 10) == pytest.approx(159333.33333333333, rel=1e-12)
    # wide (m < n): the QR stops after m columns: 2 n m^2 - 2 m^3 / 3
    assert qr_flops(5, 8) == pytest.approx(316.66666666666667, rel=1e-12)
    bf = _count_householder_loop(50, 400)
    assert abs(qr_flops(50, 400) - bf) / bf <= 0.05


def test_trunc_flops_hand_values():
    """T_tau of width w kept at rank k (Sec. 2.1.1): two economy QRs, the w x w
    product of the R factors, a nominal 21 p^3 SVD, the left factor Q1 U_k
    (reflectors applied to k columns: 4 m p k) and the right factor R (R1^T U_k)
    (2 m w k).  Values evaluated by hand:
      (1000, 800, w=10, k=4): 199333.33 + 159333.33 + 2000 + 21000 + 160000 + 64000
      (5, 100, w=8, k=3), p1 = 5 < w: 316.67 + 12458.67 + 640 + 10752 + 300 + 4800"""
    assert trunc_flops(1000, 800, 10, 4) == pytest.approx(605666.6666666667, rel=1e-12)
    assert trunc_flops(5, 100, 8, 3) == pytest.approx(29267.33333333333, rel=1e-12)


def test_trunc_counter_records_its_cost():
    rng = np.random.default_rng(0)
    L, R = rng.standard_normal((300, 6)), rng.standard_normal((6, 200))
    c = Counter()
    _, Rk = O.trunc(L, R, 1e-12, c, "x")
    assert c.flops["trunc"] == pytest.approx(trunc_flops(300, 200, 6, Rk.shape[0]), rel=1e-15)
    assert c.truncs[0]["w"] == 6 and c.truncs[0]["k"] == 6


@pytest.mark.parametrize("m,n", [(296, 256), (64, 64), (1000, 100)])
def test_house_qr_counter_against_loop_count(m, n):
    """The leaf QR's credited cost (QR 2mn^2 - 2n^3/3 plus T mn^2 - n^3/3,
    Sec. 4.1) against the two loops counted operation by operation."""
    c = Counter()
    O.house_qr(np.random.default_rng(1).standard_normal((m, n)), c)
    bf = _count_householder_loop(m, n) + _count_t_recurrence(m, n)
    assert abs(c.flops["leaf_qr"] - bf) / bf <= 2.0 / n + 0.01


def test_hmat_counter_hand_count():
    """4 x 4 HODLR of level 1 (two 2 x 2 leaves, rank-1 blocks) times 3
    columns: leaves 2 * (2*2*2*3) = 48, each block V^T X (2*1*2*3) then
    U (V^T X) (2*2*1*3): 2 * 24 = 48; total 96.  Triangular operands count
    half of each leaf product: 24 + 48 = 72."""
    inp = G.gaussian_hodlr(4, 2, 1, seed=0)
    M = O.from_input(inp)
    X = np.ones((4, 3))
    c = Counter()
    O.hmat(M, X, c)
    assert c.flops["hmat"] == 96.0
    c = Counter()
    O.hmatT(M, X, c, tri=True)
    assert c.flops["hmat"] == 72.0


def test_counter_scaling_law():
    """Sec. 4.1: hQR costs O(k^2 n log^2 n) for fixed leaf size and ranks; the
    leaf QRs alone are O(n).  On the exponential-kernel matrices (ranks stay at
    1..3) the oracle's counter over n = 2^10 .. 2^15 (leaf 256):
      * leaf QRs double with n (ratio 2.0 .. 2.1 per doubling: one more leaf
        per leaf, stacked heights grow only with the depth);
      * products, recompressions, -_H leaf updates and the small dense
        products grow like n L or n L^2: their mean ratio over the last three
        doublings lies between those of n L and n L^2 (a block counted as
        dense, or an n^2 term anywhere, pushes it towards 4);
      * the total is fitted by a n + b n L + c n L^2 (L = log2(n / 256)) to
        within 6 % at every size."""
    ns = [1 << e for e in range(10, 16)]
    tot, cats = [], []
    for n in ns:
        inp = G.expkernel_hodlr(n, 256, 2)
        F = O.hqr(inp, 1e-10, anorm=0.186 * n)
        tot.append(F.counter.total)
        cats.append(dict(F.counter.flops))
    r = np.array([cats[i + 1]["leaf_qr"] / cats[i]["leaf_qr"] for i in range(len(ns) - 1)])
    assert np.all((r >= 2.0) & (r <= 2.1)), r
    # a term n L^p grows by 2 ((L + 1) / L)^p per doubling; products and leaf
    # updates are n L (+ a small n L^2 part), recompressions and the small dense
    # products n L^2 (their ranks grow slowly with L on this family)
    lv = [math.log2(n / 256) for n in ns]
    steps = range(len(ns) - 4, len(ns) - 1)
    p1 = np.mean([2.0 * (lv[i + 1] / lv[i]) for i in steps])
    p2 = np.mean([2.0 * (lv[i + 1] / lv[i]) ** 2 for i in steps])
    for c, hi in (("hmat", p2), ("update", p2), ("trunc", 1.15 * p2), ("dense", 1.15 * p2)):
        g = np.mean([cats[i + 1][c] / cats[i][c] for i in steps])
        assert 0.95 * p1 <= g <= hi, (c, g, p1, p2)
    tot = np.array(tot)
    L = np.array([math.log2(n / 256) for n in ns])
    nn = np.array(ns, dtype=float)
    A = np.stack([nn, nn * L, nn * L * L], axis=1)
    coef, *_ = np.linalg.lstsq(A / tot[:, None], np.ones(len(ns)), rcond=None)
    fit = A @ coef
    assert np.all(np.abs(fit - tot) / tot <= 0.06), (fit / tot)


def _groups_at(inp, lo, hi):
    """Number of row groups of the sum S~ at node [lo, hi): the lower block of
    the parent when the node is a left child, plus one per further ancestor
    whose left subtree holds the node (eq. defH, the stacked C)."""
    v, q = 1, 0
    anc = []
    while True:
        a, b = inp.node_range(v)
        if (a, b) == (lo, hi):
            break
        mid = inp.node_range(2 * v)[1]
        if hi <= mid:
            anc.append(v)
            v = 2 * v
        else:
            v = 2 * v + 1
    return len(anc)


def test_rank_log_follows_the_chunked_order():
    """The sums S~ and T~12 are accumulated one term at a time, each addition
    followed by a recompression (the remedy of Sec. 4.2 against rank growth):
    at every node the S~ chain has 1 + q recompressions (the first one of the
    two A-terms, then one per row group), and each one after the first is
    wider than the rank the previous one kept (its input is that result plus
    a new term).  A single stacked recompression, or a chain that restarts
    from the terms, fails this."""
    inp = G.config(0)
    F = O.hqr(inp, 1e-10)
    chains = {}
    for t in F.counter.truncs:
        if t["key"] and t["key"][0] in ("S", "T"):
            chains.setdefault(t["key"][:3], []).append(t)
    nodes = [inp.node_range(v) for v in inp.internal_nodes()]
    for lo, hi in nodes:
        q = _groups_at(inp, lo, hi)
        s = chains[("S", lo, hi)]
        assert [t["key"][3] for t in s] == list(range(1 + q))
        for prev, cur in zip(s, s[1:]):
            assert cur["w"] > prev["k"]
        tt = chains[("T", lo, hi)]
        assert [t["key"][3] for t in tt] == list(range(max(1, q)))
        for prev, cur in zip(tt, tt[1:]):
            assert cur["w"] > prev["k"]
    # every -_H update names a block of the trailing part (right subtree) of its node
    mids = {inp.node_range(v): inp.node_range(2 * v)[1] for v in inp.internal_nodes()}
    n_upd = 0
    for t in F.counter.truncs:
        if t["key"] and t["key"][0] == "update":
            _, lo, hi, r, c = t["key"]
            assert mids[(lo, hi)] <= r < hi and mids[(lo, hi)] <= c < hi
            n_upd += 1
    # one per block of each right subtree: 2 * (internal nodes of the subtree)
    assert n_upd == sum(2 * ((1 << (inp.levels - (v.bit_length() - 1) - 1)) - 1)
                        for v in inp.internal_nodes())
