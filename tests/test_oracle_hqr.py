"""Pins of the oracle's HODLR arithmetic and of hQR itself (CPU only).

* HODLR products against dense products (brute force).
* -_H against the dense update, within (levels) * tau per block.
* hQR with eps = 0 against the dense Householder QR of the assembled matrix
  and against LAPACK: the compressed block column of Sec. 4.1 produces the same
  reflectors as the full one, so with no truncation loss hQR *is* Householder QR.
* eps = 1e-10: backward bounds |A - QR|/|A| <= 10 eps, |I - Q^T Q| <= 10 eps.
* special cases: level 0, zero off-diagonal ranks, upper triangular A, identity.
* invariants of Y, T, R; apply_q and solve against dense algebra.
"""
import numpy as np
import pytest

import hodlr_gen as G
import oracle as O


def _rand_hodlr(n, leaf, k, seed, shift=4.0):
    return G.gaussian_hodlr(n, leaf, k, seed, shift=shift)


@pytest.mark.parametrize("n,leaf,k,seed", [(33, 4, 2, 0), (64, 8, 3, 1), (100, 7, 5, 2), (9, 16, 1, 3)])
def test_hmat_against_dense(n, leaf, k, seed):
    H = _rand_hodlr(n, leaf, k, seed)
    A = H.to_dense()
    M = O.from_input(H)
    X = np.random.default_rng(seed).standard_normal((n, 3))
    np.testing.assert_allclose(O.hmat(M, X), A @ X, atol=1e-12)
    np.testing.assert_allclose(O.hmatT(M, X), A.T @ X, atol=1e-12)
    np.testing.assert_allclose(O.to_dense(M), A, atol=0)


def test_lowrank_update_against_dense():
    H = _rand_hodlr(96, 8, 3, 4)
    A = H.to_dense()
    M = O.from_input(H)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((96, 2))
    Vr = rng.standard_normal((2, 96))
    tau = 1e-6
    N = O.lowrank_update(M, U, Vr, tau)
    err = np.linalg.norm(O.to_dense(N) - (A - U @ Vr), 2)
    assert err <= H.levels * tau * 2
    # lossless at tau = 0
    N0 = O.lowrank_update(M, U, Vr, 0.0)
    np.testing.assert_allclose(O.to_dense(N0), A - U @ Vr, atol=1e-12)


PARTS = [(8, 4, 1, 0), (16, 4, 2, 1), (37, 5, 3, 2), (64, 8, 4, 3), (50, 6, 2, 4), (128, 16, 5, 5),
         (23, 3, 1, 6), (64, 64, 4, 7)]


@pytest.mark.parametrize("n,leaf,k,seed", PARTS)
def test_hqr_lossless_equals_dense_householder(n, leaf, k, seed):
    H = _rand_hodlr(n, leaf, k, seed)
    A = H.to_dense()
    F = O.hqr(H, 0.0, anorm=1.0)
    Y, T, R, Q = O.dense_factors(F)
    Yd, Td, Rd = O.house_qr(A)
    scale = np.abs(A).max()
    np.testing.assert_allclose(R, Rd, atol=1e-12 * scale)
    np.testing.assert_allclose(Y, Yd, atol=1e-12)
    np.testing.assert_allclose(T, Td, atol=1e-12)
    # and against LAPACK directly
    h, tau = np.linalg.qr(A, mode="raw")
    np.testing.assert_allclose(np.diag(T), tau, atol=1e-12)
    np.testing.assert_allclose(R, np.triu(h.T), atol=1e-12 * scale)


@pytest.mark.parametrize("n,leaf,k,seed", [(256, 32, 6, 10), (300, 40, 8, 11), (512, 64, 8, 0)])
def test_hqr_backward_bounds(n, leaf, k, seed):
    eps = 1e-10
    H = _rand_hodlr(n, leaf, k, seed)
    A = H.to_dense()
    F = O.hqr(H, eps)
    acc = O.accuracy(F, A)
    assert acc["e_acc_rel"] <= 10 * eps
    assert acc["e_orth"] <= 10 * eps
    # forward closeness to dense Householder QR for these well-conditioned inputs
    _, _, R, _ = O.dense_factors(F)
    _, _, Rd = O.house_qr(A)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(R - Rd) / np.linalg.norm(Rd) <= 10 * kappa * eps


def test_hqr_eps_controls_error():
    """Errors shrink roughly in proportion to eps (Example 3's behaviour)."""
    H = G.cauchy_hodlr(512, 64, seed=5, eps=1e-14)
    A = H.to_dense()
    errs = []
    for eps in (1e-4, 1e-7, 1e-10):
        F = O.hqr(H, eps)
        errs.append(O.accuracy(F, A)["e_acc_rel"])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] <= 1e-9


def test_special_level_zero_is_dense_qr():
    H = _rand_hodlr(40, 64, 3, 20)
    assert H.levels == 0
    F = O.hqr(H, 1e-10)
    Y, T, R, _ = O.dense_factors(F)
    Yd, Td, Rd = O.house_qr(H.to_dense())
    np.testing.assert_array_equal(R, Rd)
    np.testing.assert_array_equal(T, Td)


def test_special_zero_ranks_block_diagonal():
    H = _rand_hodlr(64, 8, 0, 21)
    F = O.hqr(H, 1e-10)
    assert O.max_ranks(F.Y) == 0 and O.max_ranks(F.R) == 0 and O.max_ranks(F.T) == 0
    for leafA, leafR in zip(O.from_input(H).leaves(), F.R.leaves()):
        _, _, Rd = O.house_qr(leafA.D)
        np.testing.assert_allclose(leafR.D, Rd, atol=1e-14)


def test_special_upper_triangular_input():
    """An upper triangular HODLR matrix (zero lower blocks, triangular leaves)
    needs no reflection at all: every gamma is 0, Y = I, T = 0 and R = A."""
    H = _rand_hodlr(64, 8, 3, 22)
    H.leaves = [np.triu(D) for D in H.leaves]
    for v in H.internal_nodes():
        U, V = H.blocks[(v, "lo")]
        H.blocks[(v, "lo")] = (U[:, :0], V[:, :0])
    A = H.to_dense()
    F = O.hqr(H, 1e-10)
    Y, T, R, _ = O.dense_factors(F)
    np.testing.assert_array_equal(T, 0 * T)
    np.testing.assert_array_equal(Y, np.eye(64))
    np.testing.assert_allclose(R, A, atol=1e-14)


def test_special_identity():
    H = G.gaussian_hodlr(32, 4, 0, 23, shift=0.0)
    H.leaves = [np.eye(D.shape[0]) for D in H.leaves]
    F = O.hqr(H, 1e-10)
    Y, T, R, Q = O.dense_factors(F)
    np.testing.assert_array_equal(R, np.eye(32))
    np.testing.assert_array_equal(Q, np.eye(32))


def test_invariants():
    eps = 1e-10
    H = _rand_hodlr(200, 25, 4, 24)
    A = H.to_dense()
    F = O.hqr(H, eps)
    Y, T, R, Q = O.dense_factors(F)
    assert np.allclose(np.triu(Y, 1), 0) and np.allclose(np.diag(Y), 1)
    assert np.allclose(np.tril(T, -1), 0) and np.allclose(np.tril(R, -1), 0)
    d = np.diag(T)
    assert np.all((d == 0) | ((d >= 1 - 1e-12) & (d <= 2 + 1e-12)))
    # Q^T A is upper triangular up to the truncation level
    assert np.abs(np.tril(Q.T @ A, -1)).max() <= 50 * eps * np.linalg.norm(A, 2)
    # no off-diagonal rank of Y exceeds the rank of the corresponding block of R + A's
    assert O.max_ranks(F.Y) <= 200


def test_apply_q_and_solve():
    H = _rand_hodlr(160, 20, 4, 25)
    A = H.to_dense()
    F = O.hqr(H, 1e-12)
    _, _, R, Q = O.dense_factors(F)
    X = np.random.default_rng(26).standard_normal((160, 5))
    np.testing.assert_allclose(O.apply_q(F, X), Q @ X, atol=1e-12)
    np.testing.assert_allclose(O.apply_q(F, X, trans=True), Q.T @ X, atol=1e-12)
    np.testing.assert_allclose(O.rmat(F, X), R @ X, atol=1e-11)
    x = O.solve(F, X)
    np.testing.assert_allclose(A @ x, X, atol=1e-9)
    np.testing.assert_allclose(x, np.linalg.solve(A, X), atol=1e-9)


def test_norm2_est():
    # dominant singular value with a large gap: the estimate is exact to roundoff
    H = G.gaussian_hodlr(64, 8, 1, 27, shift=0.0)
    H.leaves = [np.diag(np.linspace(0.1, 0.5, D.shape[0])) for D in H.leaves]
    H.leaves[2][0, 0] = 10.0
    for v in H.internal_nodes():
        U, V = H.blocks[(v, "up")]
        H.blocks[(v, "up")] = (U * 1e-3, V)
    A = H.to_dense()
    est = O.norm2_est(O.from_input(H))
    assert est == pytest.approx(np.linalg.norm(A, 2), rel=1e-12)
    # in general a lower bound that is close for these inputs
    H = G.config(0)
    A = H.to_dense()
    est = O.norm2_est(O.from_input(H))
    true = np.linalg.norm(A, 2)
    assert est <= true * (1 + 1e-13) and est >= 0.95 * true


def test_counter_and_rank_log():
    H = G.config(0)
    F = O.hqr(H, 1e-10)
    c = F.counter
    assert c.total > 0 and c.flops["leaf_qr"] > 0
    sites = {t["site"] for t in c.truncs}
    assert {"S", "A12", "T", "update"} <= sites
    for t in c.truncs:
        assert t["k"] <= t["w"]
        if t["k"]:
            assert t["sk"] > t["tau"]
        assert t["sk1"] <= t["tau"]
