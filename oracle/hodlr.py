"""HODLR matrices for the oracle: a plain recursive tree with dense leaves and
factorized off-diagonal blocks (Sec. 2.1, eq. toplevelpartitioning,
eq. factoroffdiagonal), the HODLR times dense product (Table 1, matrix-vector
multiplication, applied column block at once), the low-rank update -_H
(Table 1, matrix low-rank update), and conversion to dense.

Blocks use the paper's orientation A_off = A_L A_R with A_L (n_L x k) and
A_R (k x n_R).  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .count import Counter
from .dense import trunc


class LowRank:
    """A_off = L @ R.  `orth` records whether L has orthonormal columns
    (true for every output of T_tau, Sec. 2.1.1 "In passing ... left-orthogonal")."""

    __slots__ = ("L", "R", "orth")

    def __init__(self, L, R, orth=False):
        self.L = np.asarray(L, dtype=np.float64)
        self.R = np.asarray(R, dtype=np.float64)
        self.orth = orth
        assert self.L.shape[1] == self.R.shape[0]

    @property
    def k(self):
        return self.L.shape[1]

    def dense(self):
        return self.L @ self.R


class HNode:
    """Node of a HODLR tree covering rows/cols [lo, hi).  A leaf holds D; an
    internal node holds children c1, c2 and the blocks A12 (rows of c1, cols of
    c2) and A21 (rows of c2, cols of c1); a block may be None (zero)."""

    __slots__ = ("lo", "hi", "D", "c1", "c2", "A12", "A21")

    def __init__(self, lo, hi, D=None, c1=None, c2=None, A12=None, A21=None):
        self.lo, self.hi = lo, hi
        self.D, self.c1, self.c2, self.A12, self.A21 = D, c1, c2, A12, A21

    @property
    def m(self):
        return self.hi - self.lo

    @property
    def is_leaf(self):
        return self.c1 is None

    def leaves(self):
        if self.is_leaf:
            return [self]
        return self.c1.leaves() + self.c2.leaves()


def from_input(H) -> HNode:
    """Build the oracle tree from a hodlr_gen.HodlrInput (copies the data)."""

    def rec(v, depth):
        lo, hi = H.node_range(v)
        if depth == H.levels:
            return HNode(lo, hi, D=np.array(H.leaves[v - (1 << H.levels)], dtype=np.float64))
        c1, c2 = rec(2 * v, depth + 1), rec(2 * v + 1, depth + 1)
        U, V = H.blocks[(v, "up")]
        A12 = LowRank(np.array(U), np.array(V).T)
        U, V = H.blocks[(v, "lo")]
        A21 = LowRank(np.array(U), np.array(V).T)
        return HNode(lo, hi, c1=c1, c2=c2, A12=A12, A21=A21)

    return rec(1, 0)


def to_dense(M: HNode) -> np.ndarray:
    if M.is_leaf:
        return np.array(M.D)
    m1 = M.c1.m
    out = np.zeros((M.m, M.m))
    out[:m1, :m1] = to_dense(M.c1)
    out[m1:, m1:] = to_dense(M.c2)
    if M.A12 is not None:
        out[:m1, m1:] = M.A12.dense()
    if M.A21 is not None:
        out[m1:, :m1] = M.A21.dense()
    return out


def _gemm_flops(m, k, n):
    return 2.0 * m * k * n


def hmat(M: HNode, X: np.ndarray, cnt: Counter | None = None, tri: bool = False) -> np.ndarray:
    """M @ X for a HODLR M and a dense X (m x s), by the recursion
    [M11 M12; M21 M22] [X1; X2] = [M11 X1 + M12 X2; M21 X1 + M22 X2]; a low-rank
    block is applied as L (R X).  `tri` only halves the leaf flop count."""
    X = np.asarray(X, dtype=np.float64)
    s = X.shape[1]
    if M.is_leaf:
        if cnt is not None:
            cnt.add("hmat", _gemm_flops(M.m, M.m, s) * (0.5 if tri else 1.0))
        return M.D @ X
    m1 = M.c1.m
    X1, X2 = X[:m1], X[m1:]
    Z1 = hmat(M.c1, X1, cnt, tri)
    Z2 = hmat(M.c2, X2, cnt, tri)
    if M.A12 is not None and M.A12.k:
        Z1 = Z1 + M.A12.L @ (M.A12.R @ X2)
        if cnt is not None:
            cnt.add("hmat", _gemm_flops(M.A12.k, X2.shape[0], s) + _gemm_flops(m1, M.A12.k, s))
    if M.A21 is not None and M.A21.k:
        Z2 = Z2 + M.A21.L @ (M.A21.R @ X1)
        if cnt is not None:
            cnt.add("hmat", _gemm_flops(M.A21.k, m1, s) + _gemm_flops(X2.shape[0], M.A21.k, s))
    return np.vstack([Z1, Z2])


def hmatT(M: HNode, X: np.ndarray, cnt: Counter | None = None, tri: bool = False) -> np.ndarray:
    """M^T @ X: [M11 M12; M21 M22]^T [X1; X2] = [M11^T X1 + M21^T X2; M12^T X1 + M22^T X2]."""
    X = np.asarray(X, dtype=np.float64)
    s = X.shape[1]
    if M.is_leaf:
        if cnt is not None:
            cnt.add("hmat", _gemm_flops(M.m, M.m, s) * (0.5 if tri else 1.0))
        return M.D.T @ X
    m1 = M.c1.m
    X1, X2 = X[:m1], X[m1:]
    Z1 = hmatT(M.c1, X1, cnt, tri)
    Z2 = hmatT(M.c2, X2, cnt, tri)
    if M.A12 is not None and M.A12.k:
        Z2 = Z2 + M.A12.R.T @ (M.A12.L.T @ X1)
        if cnt is not None:
            cnt.add("hmat", _gemm_flops(M.A12.k, m1, s) + _gemm_flops(X2.shape[0], M.A12.k, s))
    if M.A21 is not None and M.A21.k:
        Z1 = Z1 + M.A21.R.T @ (M.A21.L.T @ X2)
        if cnt is not None:
            cnt.add("hmat", _gemm_flops(M.A21.k, X2.shape[0], s) + _gemm_flops(m1, M.A21.k, s))
    return np.vstack([Z1, Z2])


def lowrank_update(M: HNode, U: np.ndarray, Vr: np.ndarray, tau: float,
                   cnt: Counter | None = None, key=()) -> HNode:
    """M -_H U Vr (Table 1, matrix low-rank update, with the sign of Alg. 2
    line compute_update): every off-diagonal block b with rows I and columns J
    becomes T_tau([b_L | U(I,:)] [b_R; -Vr(:,J)]) and every leaf becomes
    D - U(I,:) Vr(:,I).  U is m x r, Vr is r x m.  Returns a new tree.  Each
    recompression is logged with key `key + (first row, first column)` of its
    block."""
    r = U.shape[1]

    def rec(N: HNode, off: int) -> HNode:
        a, b = N.lo - off, N.hi - off
        if N.is_leaf:
            D = N.D - U[a:b] @ Vr[:, a:b]
            if cnt is not None:
                cnt.add("update", _gemm_flops(N.m, r, N.m))
            return HNode(N.lo, N.hi, D=D)
        mid = N.c1.hi - off
        c1, c2 = rec(N.c1, off), rec(N.c2, off)
        A12 = N.A12
        L12, R12 = trunc(np.hstack([A12.L, U[a:mid]]), np.vstack([A12.R, -Vr[:, mid:b]]), tau,
                         cnt, "update", tuple(key) + (N.lo, N.c1.hi))
        L21, R21 = trunc(np.hstack([N.A21.L, U[mid:b]]), np.vstack([N.A21.R, -Vr[:, a:mid]]), tau,
                         cnt, "update", tuple(key) + (N.c1.hi, N.lo))
        return HNode(N.lo, N.hi, c1=c1, c2=c2, A12=LowRank(L12, R12, True),
                     A21=LowRank(L21, R21, True))

    return rec(M, M.lo)


def norm2_est(M: HNode, iters: int = 50) -> float:
    """Estimate of |M|_2 by power iteration on M^T M from x0 = 1/sqrt(n),
    returning |M x| for the last normalised iterate.  (The paper uses
    eps*|A|_2 in Alg. 2 without saying how |A|_2 is obtained; this fixed
    iteration is the reading shared by the oracle and the GPU library.)"""
    n = M.m
    x = np.full((n, 1), 1.0 / np.sqrt(n))
    for _ in range(iters):
        z = hmatT(M, hmat(M, x))
        nz = float(np.linalg.norm(z))
        if nz == 0.0:
            return 0.0
        x = z / nz
    return float(np.linalg.norm(hmat(M, x)))
