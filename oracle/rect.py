"""hQR for rectangular HODLR matrices (Kressner & Susnjara, Sec. 6): a permuted
QR decomposition A = Q R, Q = I - Y T Y^T, of an m x n HODLR matrix whose
leaves are m_j x n_j with m_j >= n_j.

Block column j is reduced so that its triangular factor sits in the first n_j
rows of leaf j (its "pivot rows"); every other row of the block column becomes
zero.  Y and R keep A's rectangular HODLR format (R is zero outside the pivot
rows, Y is unit at the pivot rows and zero on the pivot rows of earlier
columns), and T is an n x n upper triangular HODLR matrix on the column
partition.  The section only sketches the algorithm; this module writes it out
as Algorithm hQR (the square oracle, oracle/hqr.py) with these changes, each
a reading of the sketch:

  * a leaf's stacked column [D_j; B_R; C] is reduced by the plain Householder
    QR with D_j (m_j x n_j) on top, so column i of the leaf reflects onto the
    leaf's row i and the rows n_j..m_j of D_j are rows like those of B_R and C;
  * at a node, the updated upper block A^_12 = A12 - Y_A11 S splits by rows:
    its pivot rows are final (the upper block of R, recompressed on those rows
    alone), its other rows ("free rows" of the first child) are still
    unreduced in the second block column: they are compressed to
    E = E_L E_R (E_L orthonormal, a T_tau at eps |A|_2) and E_R joins the
    second block column's row groups, after the groups inherited from above
    (Sec. 6: the low-rank parts of the unreduced block column are compressed
    first);
  * the reflectors' rows on E are E_L Y~_E: they form the upper block of Y at
    the node (Y inherits the structure of the second block column), and
    T~12 gains the term Y_A11^T E_L Y~_E, first in the sum (rows top down);
  * the square case (all m_j = n_j) has no free rows and is Algorithm hQR.

At eps = 0 every recompression is exact and the factors equal the dense
permuted Householder QR (`perm_house_qr`): the columns in order, column c
reflected onto its pivot row over all rows not yet used as pivots.

Test infrastructure only: the GPU library never imports, links or runs this.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .count import Counter
from .dense import chunked_trunc, house_qr, qr_flops, trunc
from .hodlr import HNode, LowRank, hmat, hmatT
from .hqr import backsolve


class RNode:
    """Node of a rectangular HODLR tree: rows [rlo, rhi), columns [clo, chi).
    A leaf holds the dense D (m x n); an internal node holds children c1, c2,
    A12 (rows of c1 x columns of c2) and A21 (rows of c2 x columns of c1)."""

    __slots__ = ("rlo", "rhi", "clo", "chi", "D", "c1", "c2", "A12", "A21")

    def __init__(self, rlo, rhi, clo, chi, D=None, c1=None, c2=None, A12=None, A21=None):
        self.rlo, self.rhi, self.clo, self.chi = rlo, rhi, clo, chi
        self.D, self.c1, self.c2, self.A12, self.A21 = D, c1, c2, A12, A21

    @property
    def m(self):
        return self.rhi - self.rlo

    @property
    def n(self):
        return self.chi - self.clo

    @property
    def is_leaf(self):
        return self.c1 is None


def rfrom_input(H) -> RNode:
    """The oracle tree of a hodlr_gen.RectHodlrInput (copies the data)."""

    def rec(v, depth):
        (rlo, rhi), (clo, chi) = H.node_rows(v), H.node_cols(v)
        if depth == H.levels:
            return RNode(rlo, rhi, clo, chi, D=np.array(H.leaves[v - (1 << H.levels)], dtype=np.float64))
        c1, c2 = rec(2 * v, depth + 1), rec(2 * v + 1, depth + 1)
        U, V = H.blocks[(v, "up")]
        A12 = LowRank(np.array(U), np.array(V).T)
        U, V = H.blocks[(v, "lo")]
        A21 = LowRank(np.array(U), np.array(V).T)
        return RNode(rlo, rhi, clo, chi, c1=c1, c2=c2, A12=A12, A21=A21)

    return rec(1, 0)


def rto_dense(M: RNode) -> np.ndarray:
    if M.is_leaf:
        return np.array(M.D)
    m1, n1 = M.c1.m, M.c1.n
    out = np.zeros((M.m, M.n))
    out[:m1, :n1] = rto_dense(M.c1)
    out[m1:, n1:] = rto_dense(M.c2)
    if M.A12 is not None:
        out[:m1, n1:] = M.A12.dense()
    if M.A21 is not None:
        out[m1:, :n1] = M.A21.dense()
    return out


def rhmat(M: RNode, X: np.ndarray, cnt: Counter | None = None) -> np.ndarray:
    """M @ X (X: n x s) by [M11 M12; M21 M22] [X1; X2], blocks as L (R X)."""
    X = np.asarray(X, dtype=np.float64)
    s = X.shape[1]
    if M.is_leaf:
        if cnt is not None:
            cnt.add("hmat", 2.0 * M.m * M.n * s)
        return M.D @ X
    n1 = M.c1.n
    X1, X2 = X[:n1], X[n1:]
    Z1 = rhmat(M.c1, X1, cnt)
    Z2 = rhmat(M.c2, X2, cnt)
    for blk, Xb, Z, rows in ((M.A12, X2, 1, M.c1.m), (M.A21, X1, 2, M.c2.m)):
        if blk is not None and blk.k:
            add = blk.L @ (blk.R @ Xb)
            if Z == 1:
                Z1 = Z1 + add
            else:
                Z2 = Z2 + add
            if cnt is not None:
                cnt.add("hmat", 2.0 * blk.k * Xb.shape[0] * s + 2.0 * rows * blk.k * s)
    return np.vstack([Z1, Z2])


def rhmatT(M: RNode, X: np.ndarray, cnt: Counter | None = None) -> np.ndarray:
    """M^T @ X (X: m x s): [M11^T X1 + M21^T X2; M12^T X1 + M22^T X2]."""
    X = np.asarray(X, dtype=np.float64)
    s = X.shape[1]
    if M.is_leaf:
        if cnt is not None:
            cnt.add("hmat", 2.0 * M.m * M.n * s)
        return M.D.T @ X
    m1 = M.c1.m
    X1, X2 = X[:m1], X[m1:]
    Z1 = rhmatT(M.c1, X1, cnt)
    Z2 = rhmatT(M.c2, X2, cnt)
    if M.A12 is not None and M.A12.k:
        Z2 = Z2 + M.A12.R.T @ (M.A12.L.T @ X1)
        if cnt is not None:
            cnt.add("hmat", 2.0 * M.A12.k * m1 * s + 2.0 * M.c2.n * M.A12.k * s)
    if M.A21 is not None and M.A21.k:
        Z1 = Z1 + M.A21.R.T @ (M.A21.L.T @ X2)
        if cnt is not None:
            cnt.add("hmat", 2.0 * M.A21.k * X2.shape[0] * s + 2.0 * M.c1.n * M.A21.k * s)
    return np.vstack([Z1, Z2])


def rlowrank_update(M: RNode, U: np.ndarray, Vr: np.ndarray, tau: float,
                    cnt: Counter | None = None, key=()) -> RNode:
    """M -_H U Vr for a rectangular HODLR M (U: m x r, Vr: r x n): every block
    with rows I and columns J becomes T_tau([b_L | U(I,:)] [b_R; -Vr(:,J)]),
    every leaf D - U(I,:) Vr(:,J).  Returns a new tree; recompressions are
    logged with key `key + (first row, first column)` of the block."""
    r = U.shape[1]

    def rec(N: RNode) -> RNode:
        a, b = N.rlo - M.rlo, N.rhi - M.rlo
        c, d = N.clo - M.clo, N.chi - M.clo
        if N.is_leaf:
            if cnt is not None:
                cnt.add("update", 2.0 * N.m * r * N.n)
            return RNode(N.rlo, N.rhi, N.clo, N.chi, D=N.D - U[a:b] @ Vr[:, c:d])
        rm, cm = N.c1.rhi - M.rlo, N.c1.chi - M.clo
        c1, c2 = rec(N.c1), rec(N.c2)
        L12, R12 = trunc(np.hstack([N.A12.L, U[a:rm]]), np.vstack([N.A12.R, -Vr[:, cm:d]]), tau,
                         cnt, "update", tuple(key) + (N.rlo, N.c1.chi))
        L21, R21 = trunc(np.hstack([N.A21.L, U[rm:b]]), np.vstack([N.A21.R, -Vr[:, c:cm]]), tau,
                         cnt, "update", tuple(key) + (N.c1.rhi, N.clo))
        return RNode(N.rlo, N.rhi, N.clo, N.chi, c1=c1, c2=c2, A12=LowRank(L12, R12, True),
                     A21=LowRank(L21, R21, True))

    return rec(M)


def pivot_mask(M: RNode) -> np.ndarray:
    """Rows of M (relative) that receive a triangular factor: the first n_j rows
    of every leaf."""
    if M.is_leaf:
        mask = np.zeros(M.m, dtype=bool)
        mask[:M.n] = True
        return mask
    return np.concatenate([pivot_mask(M.c1), pivot_mask(M.c2)])


def rnorm2_est(M: RNode, iters: int = 50) -> float:
    """|M|_2 by power iteration on M^T M from x0 = 1/sqrt(n), as norm2_est."""
    x = np.full((M.n, 1), 1.0 / np.sqrt(M.n))
    for _ in range(iters):
        z = rhmatT(M, rhmat(M, x))
        nz = float(np.linalg.norm(z))
        if nz == 0.0:
            return 0.0
        x = z / nz
    return float(np.linalg.norm(rhmat(M, x)))


@dataclass
class RectQRFactors:
    """Q = I - Y T Y^T (m x m) and R (m x n, zero outside the pivot rows)."""
    Y: RNode
    T: HNode
    R: RNode
    piv: np.ndarray
    anorm: float
    eps: float
    tauA: float
    tauT: float
    counter: Counter = field(default_factory=Counter)


@dataclass
class _Out:
    YA: RNode
    T: HNode
    R: RNode
    B: LowRank | None
    YtB: np.ndarray | None
    YC: list


class _Ctx:
    def __init__(self, tauA, tauT, cnt):
        self.tauA, self.tauT, self.cnt = tauA, tauT, cnt


def _embed(L: np.ndarray, mask: np.ndarray) -> np.ndarray:
    out = np.zeros((mask.size, L.shape[1]))
    out[mask] = L
    return out


def _node(At: RNode, B: LowRank | None, C: list, ctx: _Ctx) -> _Out:
    cnt = ctx.cnt
    # left-orthogonalise B (B_L orthonormal; its reflector rows are B_L Y~_B)
    if B is not None and not B.orth:
        Q, Rb = np.linalg.qr(B.L)
        cnt.add("orth", 2 * qr_flops(*B.L.shape) + 2.0 * Rb.shape[0] * Rb.shape[1] * B.R.shape[1])
        B = LowRank(Q, Rb @ B.R, True)
    BR = B.R if B is not None else None

    if At.is_leaf:
        # the stacked column [D; B_R; C] with D (m x n, m >= n) on top
        m, n = At.m, At.n
        parts = [At.D] + ([BR] if B is not None else []) + list(C)
        Y, T, R = house_qr(np.vstack(parts), cnt)
        pos = m
        YtB = None
        if B is not None:
            YtB = Y[pos:pos + B.k]
            pos += B.k
        YC = []
        for c in C:
            YC.append(Y[pos:pos + c.shape[0]])
            pos += c.shape[0]
        Rl = np.zeros((m, n))
        Rl[:n] = R
        return _Out(RNode(At.rlo, At.rhi, At.clo, At.chi, D=Y[:m]), HNode(At.clo, At.chi, D=T),
                    RNode(At.rlo, At.rhi, At.clo, At.chi, D=Rl), B, YtB, YC)

    n1 = At.c1.n
    A12, A21, A22 = At.A12, At.A21, At.c2
    key = (At.rlo, At.rhi, At.clo, At.chi)
    groups = ([BR] if B is not None else []) + list(C)
    G1 = [g[:, :n1] for g in groups]
    G2 = [g[:, n1:] for g in groups]

    # first block column
    left = _node(At.c1, A21, G1, ctx)
    YA11, T1, R1 = left.YA, left.T, left.R
    BL, YtB21, Y1 = left.B.L, left.YtB, left.YC

    # S~ = Y_A11^T A12 + Y_A21^T A22 + sum over row groups, then S = T1^T S~
    terms = [(rhmatT(YA11, A12.L, cnt), A12.R), (YtB21.T, rhmatT(A22, BL, cnt).T)]
    for Yg1, Cg2 in zip(Y1, G2):
        terms.append((Yg1.T, Cg2))
    SL, SR = chunked_trunc(terms, ctx.tauA, cnt, "S", ("S",) + key)
    SL = hmatT(T1, SL, cnt, tri=True)

    # A^12 = A12 - Y_A11 S: pivot rows -> upper block of R, free rows -> E
    piv = pivot_mask(At.c1)
    Lcat = np.hstack([A12.L, -rhmat(YA11, SL, cnt)])
    Rcat = np.vstack([A12.R, SR])
    Lp, Rp = trunc(Lcat[piv], Rcat, ctx.tauA, cnt, "A12", ("A12",) + key)
    has_e = not piv.all()
    if has_e:
        Lf, Rf = trunc(Lcat[~piv], Rcat, ctx.tauA, cnt, "E", ("E",) + key)

    # A^22 = A22 -_H Y_A21 S, and the row groups
    W = YtB21 @ SL
    cnt.add("dense", 2.0 * W.shape[0] * YtB21.shape[1] * W.shape[1])
    A22h = rlowrank_update(A22, BL, W @ SR, ctx.tauA, cnt, ("update",) + key)
    cnt.add("dense", 2.0 * W.shape[0] * W.shape[1] * SR.shape[1])
    G2h = []
    for Yg1, Cg2 in zip(Y1, G2):
        G2h.append(Cg2 - (Yg1 @ SL) @ SR)
        cnt.add("dense", 2.0 * Yg1.shape[0] * Yg1.shape[1] * SL.shape[1]
                + 2.0 * Yg1.shape[0] * SL.shape[1] * SR.shape[1])

    # second block column: the inherited groups, then E_R
    right = _node(A22h, None, G2h + ([Rf] if has_e else []), ctx)
    YA22, T2, R2 = right.YA, right.T, right.R
    Y2 = right.YC[:len(G2h)]
    YE = right.YC[len(G2h)] if has_e else None

    # T~12 = Y_1^T Y_2 over all rows (c1 rows: Y_A11^T E_L Y~_E), T12 = -T1 T~12 T2
    tterms = []
    if has_e:
        tterms.append((rhmatT(YA11, _embed(Lf, ~piv), cnt), YE))
    tterms.append((YtB21.T, rhmatT(YA22, BL, cnt).T))
    for Yg1, Yg2 in zip(Y1, Y2):
        tterms.append((Yg1.T, Yg2))
    TL, TR = chunked_trunc(tterms, ctx.tauT, cnt, "T", ("T",) + key)
    T12 = LowRank(-hmat(T1, TL, cnt, tri=True), hmatT(T2, TR.T, cnt, tri=True).T)

    YA = RNode(At.rlo, At.rhi, At.clo, At.chi, c1=YA11, c2=YA22, A21=LowRank(BL, YtB21),
               A12=LowRank(_embed(Lf, ~piv), YE) if has_e else None)
    T = HNode(At.clo, At.chi, c1=T1, c2=T2, A12=T12)
    R = RNode(At.rlo, At.rhi, At.clo, At.chi, c1=R1, c2=R2, A12=LowRank(_embed(Lp, piv), Rp))
    Ycat = [np.hstack([a, b]) for a, b in zip(Y1, Y2)]
    YtB, YC = (Ycat[0], Ycat[1:]) if B is not None else (None, Ycat)
    return _Out(YA, T, R, B, YtB, YC)


def rhqr(A, eps: float, anorm: float | None = None) -> RectQRFactors:
    """Permuted QR A ~= (I - Y T Y^T) R of a rectangular HODLR matrix
    (hodlr_gen.RectHodlrInput or RNode), thresholds eps |A|_2 and eps."""
    root = A if isinstance(A, RNode) else rfrom_input(A)
    if anorm is None:
        anorm = rnorm2_est(root)
    cnt = Counter()
    ctx = _Ctx(eps * anorm, eps, cnt)
    out = _node(root, None, [], ctx)
    piv = np.flatnonzero(pivot_mask(root))
    return RectQRFactors(out.YA, out.T, out.R, piv, float(anorm), eps, ctx.tauA, ctx.tauT, cnt)


# --------------------------------------------------------------------------
# using the factors

def rect_apply_q(F: RectQRFactors, X: np.ndarray, trans: bool = False) -> np.ndarray:
    """Q X or Q^T X for X (m x s), Q = I - Y T Y^T."""
    X = np.asarray(X, dtype=np.float64)
    W = rhmatT(F.Y, X)
    W = hmatT(F.T, W) if trans else hmat(F.T, W)
    return X - rhmat(F.Y, W)


def rect_rmat(F: RectQRFactors, X: np.ndarray) -> np.ndarray:
    return rhmat(F.R, X)


def pivot_r(R: RNode) -> HNode:
    """R restricted to its pivot rows: an n x n upper triangular HODLR matrix on
    the column partition (the triangular factor in column order)."""
    if R.is_leaf:
        return HNode(R.clo, R.chi, D=np.array(R.D[:R.n]))
    c1, c2 = pivot_r(R.c1), pivot_r(R.c2)
    A12 = None
    if R.A12 is not None:
        A12 = LowRank(R.A12.L[pivot_mask(R.c1)], R.A12.R)
    return HNode(R.clo, R.chi, c1=c1, c2=c2, A12=A12)


def rect_lstsq(F: RectQRFactors, B: np.ndarray) -> np.ndarray:
    """Least-squares solution x = argmin |A x - b|: R_p^{-1} (Q^T b)(pivot rows)."""
    C = rect_apply_q(F, B, trans=True)
    return backsolve(pivot_r(F.R), C[F.piv])


def rect_dense_factors(F: RectQRFactors):
    Y, R = rto_dense(F.Y), rto_dense(F.R)
    from .hodlr import to_dense
    T = to_dense(F.T)
    Q = np.eye(Y.shape[0]) - Y @ T @ Y.T
    return Y, T, R, Q


def rect_accuracy(F: RectQRFactors, A_dense: np.ndarray) -> dict:
    """e_orth = |Q^T Q - I|_2, e_acc = |Q R - A|_2 (eq. accuracy)."""
    _, _, R, Q = rect_dense_factors(F)
    m = A_dense.shape[0]
    e_orth = float(np.linalg.norm(Q.T @ Q - np.eye(m), 2))
    e_acc = float(np.linalg.norm(Q @ R - A_dense, 2))
    return dict(e_orth=e_orth, e_acc=e_acc, e_acc_rel=e_acc / float(np.linalg.norm(A_dense, 2)))


def perm_house_qr(A: np.ndarray, piv: np.ndarray):
    """Dense permuted Householder QR: column c reflected onto row piv[c] over the
    rows not yet used as pivots, i.e. the Householder QR of the rows ordered
    [piv; the remaining rows] with the rows put back.  Returns Y (m x n, unit
    at piv[c] in column c), T (n x n) and R (m x n, zero outside piv)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    rest = np.setdiff1d(np.arange(m), piv)
    order = np.concatenate([np.asarray(piv, dtype=np.int64), rest])
    Ys, T, Rs = house_qr(A[order])
    Y = np.zeros((m, n))
    Y[order] = Ys
    R = np.zeros((m, n))
    R[order[:n]] = Rs
    return Y, T, R


def rmax_ranks(M) -> int:
    if M.is_leaf:
        return 0
    rk = lambda b: b.k if b is not None else 0
    sub = rmax_ranks(M.c1), rmax_ranks(M.c2)
    return max(max(sub), rk(M.A12), rk(M.A21))
