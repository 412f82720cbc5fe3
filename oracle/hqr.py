"""hQR: recursive Householder QR of a HODLR matrix (Kressner & Susnjara,
Sec. 4, Algorithm hQR), written step by step in the paper's notation.

Each call works on H = [A~; B; C] (eq. defH) with B = B_L B_R factorized and C
a stack of dense row groups, and returns Y (eq. defY), T and R.  The step
numbers in the comments refer to the algorithm's own labels:
  left_orthogonal       - make B_L orthonormal (Sec. 2.1)
  compute_lowest_level  - dense Householder QR of H~ = [A~; B_R; C] at a leaf
  computeQR_first_blcol - recursion on the first block column
  compute_Stilde        - S~ = T_{eps|A|}(Y_A11^T A12 + Y_A21^T A22 + Y_BR1^T B_R2 + Y_C1^T C2)
  compute_S             - S = T1^T S~
  compute_update        - second block column update, eq. (update2ndblockH)
  computeQR_second_blcol- recursion on the updated second block column
  compute_T, compute_T2 - T~12 = T_eps(Y_A21^T Y_A22 + Y_BR1^T Y_BR2 + Y_C1^T Y_C2),
                          T12 = -T1 T~12 T2
followed by the assembly of Y_A, T, R and Y_B = B_L Y~_B (postprocessing).

Readings where the paper is silent (shared with the GPU library):
  * |A|_2 in eps*|A|_2 comes from `norm2_est` unless the caller passes it;
  * the -_H update of compute_update truncates at eps*|A|_2 as well;
  * compute_T truncates at the unscaled eps, as written;
  * the sums of compute_Stilde and compute_T are accumulated term by term
    (Y_A11^T A12, Y_A21^T A22, Y_BR1^T B_R2, then one term per row group of
    C, nearest group first), each addition followed by a recompression
    (`chunked_trunc`), which is the paper's remedy against rank growth;
  * C is kept as a list of row groups, B_R's rows first, so that each group
    is one term of that sum.

Test infrastructure only: the GPU library never imports, links or runs this.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .count import Counter
from .dense import chunked_trunc, house_qr, qr_flops, trunc
from .hodlr import (HNode, LowRank, from_input, hmat, hmatT, lowrank_update,
                    norm2_est, to_dense)


@dataclass
class QRFactors:
    """Q = I - Y T Y^T and R, all level-l HODLR matrices on A's partition."""
    Y: HNode
    T: HNode
    R: HNode
    anorm: float
    eps: float
    tauA: float
    tauT: float
    counter: Counter = field(default_factory=Counter)


@dataclass
class _Out:
    YA: HNode
    T: HNode
    R: HNode
    B: LowRank | None      # B after left-orthogonalisation (B_L orthonormal)
    YtB: np.ndarray | None  # Y~_B (r1 x m);  Y_B = B_L Y~_B
    YC: list                # one (k_g x m) array per row group of C


class _Ctx:
    def __init__(self, tauA, tauT, cnt):
        self.tauA, self.tauT, self.cnt = tauA, tauT, cnt


def _node(At: HNode, B: LowRank | None, C: list, ctx: _Ctx) -> _Out:
    cnt = ctx.cnt
    # left_orthogonal: economy QR B_L = Q R, B_L <- Q, B_R <- R B_R
    if B is not None and not B.orth:
        Q, Rb = np.linalg.qr(B.L)
        cnt.add("orth", 2 * qr_flops(*B.L.shape) + 2.0 * Rb.shape[0] * Rb.shape[1] * B.R.shape[1])
        B = LowRank(Q, Rb @ B.R, True)
    BR = B.R if B is not None else None

    if At.is_leaf:
        # compute_lowest_level: dense QR of H~ = [A~; B_R; C]
        m = At.m
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
        return _Out(HNode(At.lo, At.hi, D=Y[:m]), HNode(At.lo, At.hi, D=T),
                    HNode(At.lo, At.hi, D=R), B, YtB, YC)

    m1 = At.c1.m
    A12, A21, A22 = At.A12, At.A21, At.c2
    groups = ([BR] if B is not None else []) + list(C)   # rows of [B_R; C]
    G1 = [g[:, :m1] for g in groups]
    G2 = [g[:, m1:] for g in groups]

    # computeQR_first_blcol: hQR(A11, A21, [B_R1; C1])
    left = _node(At.c1, A21, G1, ctx)
    YA11, T1, R1 = left.YA, left.T, left.R
    BL = left.B.L                 # orthonormal left factor of A21
    YtB21 = left.YtB              # Y_A21 = BL @ YtB21
    Y1 = left.YC                  # [Y_BR1] + Y_C1 groups (same order as G1)

    # compute_Stilde
    terms = [(hmatT(YA11, A12.L, cnt, tri=True), A12.R),
             (YtB21.T, hmatT(A22, BL, cnt).T)]
    for Yg1, Cg2 in zip(Y1, G2):
        terms.append((Yg1.T, Cg2))
    SL, SR = chunked_trunc(terms, ctx.tauA, cnt, "S", ("S", At.lo, At.hi))

    # compute_S: S = T1^T S~  (S = SL @ SR)
    SL = hmatT(T1, SL, cnt, tri=True)

    # compute_update, eq. (update2ndblockH)
    L12, R12 = trunc(np.hstack([A12.L, -hmat(YA11, SL, cnt, tri=True)]),
                     np.vstack([A12.R, SR]), ctx.tauA, cnt, "A12", ("A12", At.lo, At.hi))
    W = YtB21 @ SL                                   # Y_A21 S = BL (W SR)
    cnt.add("dense", 2.0 * W.shape[0] * YtB21.shape[1] * W.shape[1])
    A22h = lowrank_update(A22, BL, W @ SR, ctx.tauA, cnt, ("update", At.lo, At.hi))
    cnt.add("dense", 2.0 * W.shape[0] * W.shape[1] * SR.shape[1])
    G2h = []
    for Yg1, Cg2 in zip(Y1, G2):
        G2h.append(Cg2 - (Yg1 @ SL) @ SR)            # B_R2 - Y_BR1 S,  C2 - Y_C1 S
        cnt.add("dense", 2.0 * Yg1.shape[0] * Yg1.shape[1] * SL.shape[1]
                + 2.0 * Yg1.shape[0] * SL.shape[1] * SR.shape[1])

    # computeQR_second_blcol: hQR(A22^, [], [B^_R2; C^2])
    right = _node(A22h, None, G2h, ctx)
    YA22, T2, R2 = right.YA, right.T, right.R
    Y2 = right.YC

    # compute_T: T~12 = T_eps(Y_A21^T Y_A22 + Y_BR1^T Y_BR2 + Y_C1^T Y_C2)
    tterms = [(YtB21.T, hmatT(YA22, BL, cnt, tri=True).T)]
    for Yg1, Yg2 in zip(Y1, Y2):
        tterms.append((Yg1.T, Yg2))
    TL, TR = chunked_trunc(tterms, ctx.tauT, cnt, "T", ("T", At.lo, At.hi))

    # compute_T2: T12 = -T1 T~12 T2 = (-T1 TL)(TR T2)
    T12 = LowRank(-hmat(T1, TL, cnt, tri=True), hmatT(T2, TR.T, cnt, tri=True).T)

    # assembly of Y_A, T, R; postprocessing Y~_B = [Y_BR1 Y_BR2], Y_C = [Y_C1 Y_C2]
    YA = HNode(At.lo, At.hi, c1=YA11, c2=YA22, A21=LowRank(BL, YtB21))
    T = HNode(At.lo, At.hi, c1=T1, c2=T2, A12=T12)
    R = HNode(At.lo, At.hi, c1=R1, c2=R2, A12=LowRank(L12, R12, True))
    Ycat = [np.hstack([a, b]) for a, b in zip(Y1, Y2)]
    YtB, YC = (Ycat[0], Ycat[1:]) if B is not None else (None, Ycat)
    return _Out(YA, T, R, B, YtB, YC)


def hqr(A, eps: float, anorm: float | None = None) -> QRFactors:
    """QR decomposition A ~= (I - Y T Y^T) R of a square HODLR matrix.

    A: hodlr_gen.HodlrInput or an oracle HNode.  eps: truncation tolerance.
    anorm: |A|_2 used for tau_A = eps*|A|_2 (estimated by `norm2_est` when None).
    """
    root = A if isinstance(A, HNode) else from_input(A)
    if anorm is None:
        anorm = norm2_est(root)
    cnt = Counter()
    ctx = _Ctx(eps * anorm, eps, cnt)
    out = _node(root, None, [], ctx)
    return QRFactors(out.YA, out.T, out.R, float(anorm), eps, ctx.tauA, ctx.tauT, cnt)


# --------------------------------------------------------------------------
# using the factors

def apply_q(F: QRFactors, X: np.ndarray, trans: bool = False) -> np.ndarray:
    """Q X = X - Y (T (Y^T X)), or Q^T X = X - Y (T^T (Y^T X))  (eq. compactwy)."""
    X = np.asarray(X, dtype=np.float64)
    W = hmatT(F.Y, X)
    W = hmatT(F.T, W) if trans else hmat(F.T, W)
    return X - hmat(F.Y, W)


def rmat(F: QRFactors, X: np.ndarray, trans: bool = False) -> np.ndarray:
    return hmatT(F.R, X) if trans else hmat(F.R, X)


def backsolve(R: HNode, C: np.ndarray) -> np.ndarray:
    """R^{-1} C for an upper triangular HODLR R: x2 = R22^{-1} c2,
    x1 = R11^{-1} (c1 - R12 x2); dense triangular solves at the leaves."""
    import scipy.linalg
    C = np.asarray(C, dtype=np.float64)
    if R.is_leaf:
        return scipy.linalg.solve_triangular(R.D, C, lower=False)
    m1 = R.c1.m
    X2 = backsolve(R.c2, C[m1:])
    C1 = C[:m1]
    if R.A12 is not None and R.A12.k:
        C1 = C1 - R.A12.L @ (R.A12.R @ X2)
    X1 = backsolve(R.c1, C1)
    return np.vstack([X1, X2])


def solve(F: QRFactors, B: np.ndarray) -> np.ndarray:
    """x = R^{-1} Q^T b, the least-squares / linear-system solution from A = QR."""
    return backsolve(F.R, apply_q(F, B, trans=True))


def dense_factors(F: QRFactors):
    """(Y, T, R, Q) as dense arrays (small n only)."""
    Y, T, R = to_dense(F.Y), to_dense(F.T), to_dense(F.R)
    Q = np.eye(Y.shape[0]) - Y @ T @ Y.T
    return Y, T, R, Q


def accuracy(F: QRFactors, A_dense: np.ndarray) -> dict:
    """e_orth = |Q^T Q - I|_2 and e_acc = |Q R - A|_2 (eq. accuracy), plus the
    residual relative to |A|_2."""
    _, _, R, Q = dense_factors(F)
    n = A_dense.shape[0]
    e_orth = float(np.linalg.norm(Q.T @ Q - np.eye(n), 2))
    e_acc = float(np.linalg.norm(Q @ R - A_dense, 2))
    return dict(e_orth=e_orth, e_acc=e_acc, e_acc_rel=e_acc / float(np.linalg.norm(A_dense, 2)))


def max_ranks(M: HNode) -> int:
    if M.is_leaf:
        return 0
    k = max(max_ranks(M.c1), max_ranks(M.c2))
    for b in (M.A12, M.A21):
        if b is not None:
            k = max(k, b.k)
    return k
