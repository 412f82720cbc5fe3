"""Dense FP64 building blocks of the oracle: Householder reflector, Householder
QR with compact WY factor, and the low-rank recompression T_eps.

Test infrastructure only: the GPU library never imports, links or runs this.
"""
from __future__ import annotations

import math

import numpy as np

from .count import Counter


def house(x: np.ndarray):
    """Householder reflector I - gamma*y*y^T mapping x to rho*e1 (Sec. 3, the n = 1
    case of the recursive QR).

    Sign convention (the paper leaves it to its textbook reference): write
    x = [alpha; x2].  If |x2| = 0 the reflector is the identity: gamma = 0,
    y = e1, rho = alpha.  Otherwise rho = -sign(alpha)*|x|_2 with sign(0) = +1,
    gamma = (rho - alpha)/rho (so gamma lies in [1, 2]) and
    y = [1; x2/(alpha - rho)].  Returns (y, gamma, rho).
    """
    x = np.asarray(x, dtype=np.float64)
    alpha = float(x[0])
    x2 = x[1:]
    s = float(np.sqrt(np.dot(x2, x2))) if x2.size else 0.0
    y = np.zeros_like(x)
    y[0] = 1.0
    if s == 0.0:
        return y, 0.0, alpha
    rho = -math.copysign(math.hypot(alpha, s), alpha if alpha != 0.0 else 1.0)
    gamma = (rho - alpha) / rho
    y[1:] = x2 / (alpha - rho)
    return y, gamma, rho


def house_qr(H: np.ndarray, cnt: Counter | None = None):
    """Householder QR of an m x n matrix (m >= n) with its compact WY factor:
    H = Q [R; 0], Q = I - Y T Y^T (eq. compactwy), Y unit lower trapezoidal,
    T upper triangular, R upper triangular.

    The paper allows any Householder QR at the leaves (Alg. 1 "for example");
    with a fixed sign convention Y, T and R are unique, so this uses the plain
    column-by-column loop: reflect column j, apply the reflector to the
    trailing columns, and extend T column by column
    (T[:j, j] = -gamma_j T[:j, :j] (Y[:, :j]^T y_j), T[j, j] = gamma_j), which is
    eq. (recqrcombined) with a one-column second block.
    """
    A = np.array(H, dtype=np.float64, copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("house_qr needs m >= n")
    Y = np.zeros((m, n))
    T = np.zeros((n, n))
    for j in range(n):
        y, g, rho = house(A[j:, j])
        A[j, j] = rho
        A[j + 1:, j] = 0.0
        if j + 1 < n and g != 0.0:
            A[j:, j + 1:] -= g * np.outer(y, y @ A[j:, j + 1:])
        Y[j:, j] = y
        T[j, j] = g
        if j > 0:
            T[:j, j] = -g * (T[:j, :j] @ (Y[j:, :j].T @ y))
    R = np.triu(A[:n, :])
    if cnt is not None:
        cnt.add("leaf_qr", 2.0 * m * n * n - 2.0 / 3.0 * n ** 3 + m * n * n - n ** 3 / 3.0)
    return Y, T, R


def trunc(L: np.ndarray, R: np.ndarray, tau: float, cnt: Counter | None = None,
          site: str = "", key=None):
    """Recompression T_tau of a low-rank product L @ R (Sec. 2.1.1,
    "Recompression"): economy QRs L = Q1 R1 and R^T = Q2 R2, SVD
    R1 R2^T = U S V^T, keep the k singular values with sigma_i > tau (the
    smallest k with sigma_{k+1} <= tau), and return L' = Q1 U_k (orthonormal
    columns) and R' = S_k V_k^T Q2^T.

    Paper orientation: L is m_L x w, R is w x m_R.  A width-0 input returns
    empty factors.  `cnt` receives the flop count and a rank-log entry (with
    `key`, the recompression's name in the log).
    """
    mL, w = L.shape
    mR = R.shape[1]
    assert R.shape[0] == w
    if w == 0:
        if cnt is not None:
            cnt.log_trunc(site, mL, mR, 0, 0, tau, np.zeros(0), key)
        return np.zeros((mL, 0)), np.zeros((0, mR))
    Q1, R1 = np.linalg.qr(L)            # LAPACK Householder QR (dgeqrf/dorgqr)
    Q2, R2 = np.linalg.qr(R.T)
    U, s, Vt = np.linalg.svd(R1 @ R2.T, full_matrices=False)
    k = int(np.sum(s > tau))
    Lk = Q1 @ U[:, :k]
    Rk = (s[:k, None] * Vt[:k]) @ Q2.T
    if cnt is not None:
        cnt.add("trunc", trunc_flops(mL, mR, w, k))
        cnt.log_trunc(site, mL, mR, w, k, tau, s, key)
    return Lk, Rk


def qr_flops(m: int, n: int) -> float:
    """Householder QR of an m x n matrix without forming Q."""
    p = min(m, n)
    return 2.0 * m * n * p - 2.0 / 3.0 * p ** 3 if m >= n else 2.0 * n * m * m - 2.0 / 3.0 * m ** 3


def trunc_flops(mL: int, mR: int, w: int, k: int) -> float:
    """Counting convention for one recompression of width w kept at rank k:
    two Householder QRs, the w x w product, a nominal 21 w^3 SVD, and the two
    output products (explicit Q1 times U_k, and the right factor)."""
    p1, p2 = min(mL, w), min(mR, w)
    return (qr_flops(mL, w) + qr_flops(mR, w) + 2.0 * p1 * p2 * w + 21.0 * max(p1, p2) ** 3
            + 4.0 * mL * p1 * k + 2.0 * mR * w * k)


def chunked_trunc(terms, tau: float, cnt: Counter | None = None, site: str = "", key=()):
    """Sum of low-rank terms with rank control (Sec. 4.2, cost of lines
    compute_Stilde/compute_S): the terms are added one at a time and every
    addition is followed immediately by T_tau, so the width of each
    recompression stays at (current rank + rank of one term).  A single term
    is recompressed once.  terms: list of (L_t, R_t) with L_t @ R_t the term.
    The i-th recompression is logged with key `key + (i,)`.
    """
    L, R = terms[0]
    if len(terms) == 1:
        return trunc(L, R, tau, cnt, site, tuple(key) + (0,))
    for i, (Lt, Rt) in enumerate(terms[1:]):
        L, R = trunc(np.hstack([L, Lt]), np.vstack([R, Rt]), tau, cnt, site, tuple(key) + (i,))
    return L, R
