"""Pins of the oracle's dense building blocks (CPU only).

house / house_qr: hand-derived fixtures (tests/golden), LAPACK dgeqrf through
numpy.linalg.qr(mode='raw') (same reflector convention), and the WY identities.
trunc: the closed-form error of eq. (localapproximationerror), exact-rank
inputs, and the strict sigma > tau rule.
"""
import os

import numpy as np
import pytest

import oracle as O


def _golden_house(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "householder.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            x, rho, g, y = [p.strip() for p in line.split("|")]
            rows.append((np.array(x.split(), float), float(rho), float(g), np.array(y.split(), float)))
    return rows


def test_house_golden(golden_dir):
    rows = _golden_house(golden_dir)
    assert len(rows) >= 6
    for x, rho, g, y in rows:
        yy, gg, rr = O.house(x)
        assert rr == pytest.approx(rho, abs=1e-15)
        assert gg == pytest.approx(g, abs=1e-15)
        np.testing.assert_allclose(yy, y, atol=1e-15)
        # the reflector really maps x to rho*e1
        out = x - gg * yy * (yy @ x)
        e = np.zeros_like(x)
        e[0] = rho
        np.testing.assert_allclose(out, e, atol=1e-14)


def _parse_mat(s):
    return np.array([[float(v) for v in r.split()] for r in s.split(";")])


def test_house_qr_golden(golden_dir):
    mats = {}
    with open(os.path.join(golden_dir, "qr3x2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, rest = line.split(None, 1)
            mats[key] = _parse_mat(rest)
    Y, T, R = O.house_qr(mats["A"])
    np.testing.assert_allclose(R, mats["R"], atol=1e-15)
    np.testing.assert_allclose(Y, mats["Y"], atol=1e-15)
    np.testing.assert_allclose(T, mats["T"], atol=1e-15)


@pytest.mark.parametrize("m,n,seed", [(5, 5, 0), (9, 4, 1), (40, 17, 2), (130, 64, 3), (7, 1, 4)])
def test_house_qr_matches_lapack(m, n, seed):
    """numpy.linalg.qr(mode='raw') returns LAPACK dgeqrf's h (transposed) and tau,
    which use the same reflector convention."""
    A = np.random.default_rng(seed).standard_normal((m, n))
    Y, T, R = O.house_qr(A)
    h, tau = np.linalg.qr(A, mode="raw")
    h = h.T
    np.testing.assert_allclose(R, np.triu(h[:n]), rtol=0, atol=1e-12 * np.abs(R).max())
    np.testing.assert_allclose(np.tril(Y, -1), np.tril(h, -1)[:, :n], atol=1e-12)
    np.testing.assert_allclose(np.diag(T), tau, atol=1e-14)


@pytest.mark.parametrize("m,n,seed", [(12, 12, 5), (50, 20, 6), (33, 33, 7)])
def test_wy_identities(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    A[:, 3] = 0.0            # a zero column gives gamma = 0
    Y, T, R = O.house_qr(A)
    Q = np.eye(m) - Y @ T @ Y.T
    np.testing.assert_allclose(Q.T @ Q, np.eye(m), atol=1e-13)
    np.testing.assert_allclose(Q[:, :n] @ R, A, atol=1e-13)
    # Y unit lower trapezoidal, T upper with diag in {0} U [1, 2]
    assert np.allclose(np.triu(Y, 1), 0) and np.allclose(np.diag(Y), 1)
    assert np.allclose(np.tril(T, -1), 0)
    d = np.diag(T)
    assert np.all((d == 0) | ((d >= 1 - 1e-15) & (d <= 2 + 1e-15)))
    assert d[3] == 0.0 or abs(R[3, 3]) > 0
    # T + T^T = T^T (Y^T Y) T  (orthogonality of I - Y T Y^T written through T)
    np.testing.assert_allclose(T + T.T, T.T @ (Y.T @ Y) @ T, atol=1e-12)


def test_house_qr_upper_triangular_input_is_identity():
    A = np.triu(np.random.default_rng(8).standard_normal((6, 6)))
    Y, T, R = O.house_qr(A)
    assert np.all(T == 0)
    assert np.array_equal(Y, np.eye(6))
    assert np.array_equal(R, A)


def _orth(m, k, rng):
    q, _ = np.linalg.qr(rng.standard_normal((m, k)))
    return q


@pytest.mark.parametrize("mL,mR", [(40, 30), (9, 50), (64, 64)])
def test_trunc_closed_form_error(mL, mR):
    """L R = Qa diag(s) Qb^T: T_tau keeps #{s > tau} terms and its 2-norm error is
    the first dropped singular value (eq. localapproximationerror)."""
    rng = np.random.default_rng(mL + mR)
    s = np.array([10.0, 1.0, 1e-3, 1e-7, 1e-12, 0.0])
    w = len(s)
    L = _orth(mL, w, rng) * s
    R = _orth(mR, w, rng).T
    for tau, k in [(1e-9, 4), (1e-4, 3), (0.5, 2), (20.0, 0)]:
        Lk, Rk = O.trunc(L, R, tau)
        assert Lk.shape[1] == k
        err = np.linalg.norm(L @ R - Lk @ Rk, 2)
        sk1 = s[k] if k < w else 0.0
        assert abs(err - sk1) <= 1e-13 * s[0]
        if k:
            np.testing.assert_allclose(Lk.T @ Lk, np.eye(k), atol=1e-13)


def test_trunc_exact_rank_loses_nothing():
    rng = np.random.default_rng(11)
    L = rng.standard_normal((200, 5))
    R = rng.standard_normal((5, 150))
    Lw = np.hstack([L, L[:, :2] * 3.0])      # width 7, rank 5
    Rw = np.vstack([R, R[:2] * 0.0 + rng.standard_normal((2, 150))])
    M = Lw @ Rw
    Lk, Rk = O.trunc(Lw, Rw, 1e-10 * np.linalg.norm(M, 2))
    assert Lk.shape[1] == 5
    assert np.linalg.norm(M - Lk @ Rk, 2) <= 1e-13 * np.linalg.norm(M, 2)


def test_trunc_strict_threshold_and_empty():
    L = np.zeros((6, 3))
    L[0, 0], L[1, 1], L[2, 2] = 2.0, 1.0, 0.5
    R = np.eye(3, 5)
    Lk, Rk = O.trunc(L, R, 0.5)          # sigma == tau is dropped
    assert Lk.shape == (6, 2) and Rk.shape == (2, 5)
    Lk, Rk = O.trunc(np.zeros((4, 0)), np.zeros((0, 3)), 1.0)
    assert Lk.shape == (4, 0) and Rk.shape == (0, 3)
    Lk, Rk = O.trunc(np.zeros((4, 2)), np.ones((2, 3)), 0.0)   # zero product keeps nothing
    assert Lk.shape[1] == 0


def test_trunc_wide_block():
    """w larger than the number of rows: the economy QR is capped at m."""
    rng = np.random.default_rng(12)
    L = rng.standard_normal((3, 8))
    R = rng.standard_normal((8, 20))
    Lk, Rk = O.trunc(L, R, 1e-12)
    assert Lk.shape[1] == 3
    np.testing.assert_allclose(Lk @ Rk, L @ R, atol=1e-12)


def test_chunked_trunc_error_bound():
    rng = np.random.default_rng(13)
    terms = [(rng.standard_normal((60, 4)), rng.standard_normal((4, 50))) for _ in range(5)]
    exact = sum(a @ b for a, b in terms)
    tau = 1e-3
    L, R = O.chunked_trunc(terms, tau)
    assert np.linalg.norm(exact - L @ R, 2) <= len(terms) * tau
    L0, R0 = O.chunked_trunc(terms, 0.0)
    np.testing.assert_allclose(L0 @ R0, exact, atol=1e-11)
