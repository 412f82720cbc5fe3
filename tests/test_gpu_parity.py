"""GPU parity of the HIP hQR library against the CPU oracle (needs an MI355X).

Every call goes through the C ABI (libhodlr.so) via the ctypes binding; the
oracle runs on the host on the same seeded inputs.

Tolerances (written where they are used):
  * lossless runs (eps = 0) reproduce dense Householder QR entrywise to
    1e-12 relative: only rounding order differs;
  * well-conditioned inputs (Gaussian HODLR, kappa ~ 1e3..1e5): relative
    difference of R X and of Q X to the oracle <= 1e-8 (eps = 1e-10);
  * ill-conditioned inputs (exponential kernel, Cauchy): the same forward
    comparison is bounded by 10x the oracle's own noise floor (oracle of A vs
    oracle of A perturbed at roundoff level) or 1e-8, whichever is larger,
    plus the backward bounds |A - QR|/|A| <= 10 eps and |I - Q^T Q| <= 10 eps.
"""
import numpy as np
import pytest

import hodlr_gen as G
import oracle as O
from helpers import dense_from_export, leaf_sizes

pytestmark = pytest.mark.gpu

EPS = 1e-10


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1809_10585_amd as H
    H.load()
    return H


def _rel(a, b, scale=None):
    return float(np.linalg.norm(a - b) / (np.linalg.norm(b) if scale is None else scale))


def _factor_dense(H, F, inp):
    ls = leaf_sizes(inp)
    return {w: dense_from_export(H.hodlr_qr_export(F, w, ls), inp.leaf_off, inp.levels) for w in "YTR"}


def test_build_export_roundtrip(H):
    inp = G.gaussian_hodlr(300, 40, 5, seed=3)
    A = H.hodlr_build(inp, rank_cap=8)
    ex = H.hodlr_export(A, leaf_sizes(inp))
    np.testing.assert_array_equal(dense_from_export(ex, inp.leaf_off, inp.levels), inp.to_dense())


@pytest.mark.parametrize("n,leaf,k", [(64, 8, 3), (300, 40, 5), (1000, 100, 7), (700, 256, 4)])
def test_matmul_against_dense(H, n, leaf, k):
    inp = G.gaussian_hodlr(n, leaf, k, seed=n)
    A = H.hodlr_build(inp, rank_cap=16)
    Ad = inp.to_dense()
    X = np.random.default_rng(1).standard_normal((n, 9))
    np.testing.assert_allclose(H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy(), Ad @ X, atol=1e-12 * n)
    np.testing.assert_allclose(H.hodlr_matmul(A, H.colmajor(X), trans=True).cpu().numpy(), Ad.T @ X,
                               atol=1e-12 * n)
    X = np.random.default_rng(2).standard_normal((n, 70))  # more columns than one pass
    np.testing.assert_allclose(H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy(), Ad @ X, atol=1e-12 * n)


def test_matmul_long_launch_against_oracle(H):
    """Products over at least 32768 rows take the 64-row tiles (and, for A^T X
    with at most 4 columns, the transposed leaf tiles staged in LDS); checked
    against the oracle's HODLR products on a ragged partition."""
    from oracle import hodlr as OH
    inp = G.gaussian_hodlr(33001, 256, 3, seed=31)
    A = H.hodlr_build(inp, rank_cap=8)
    M = OH.from_input(inp)
    for s_cols in (1, 3, 9):
        X = np.random.default_rng(s_cols).standard_normal((inp.n, s_cols))
        print(f"n=33001 s={s_cols}", flush=True)
        for trans, ref in ((False, OH.hmat(M, X)), (True, OH.hmatT(M, X))):
            Z = H.hodlr_matmul(A, H.colmajor(X), trans=trans).cpu().numpy()
            err = np.abs(Z - ref).max() / np.abs(ref).max()
            assert err <= 1e-13, (s_cols, trans, err)


def test_factor_products_long_launch_adjoint(H):
    """Y, T and R (unit lower, upper, upper leaves) over 33001 rows: the
    transposed products (64-row tiles staged through LDS) are the adjoints of
    the direct ones, <M X1, X2> = <X1, M^T X2>."""
    inp = G.gaussian_hodlr(33001, 256, 2, seed=32)  # oracle ranks of Y, T, R: 16, 16, 31
    A = H.hodlr_build(inp, rank_cap=48)
    F = H.hodlr_qr(A, EPS)
    rng = np.random.default_rng(5)
    for s_cols in (1, 4, 9):
        X1 = rng.standard_normal((inp.n, s_cols))
        X2 = rng.standard_normal((inp.n, s_cols))
        for which in "YTR":
            print(f"n=33001 {which} s={s_cols}", flush=True)
            MX1 = H.hodlr_qr_matmul(F, which, H.colmajor(X1)).cpu().numpy()
            MtX2 = H.hodlr_qr_matmul(F, which, H.colmajor(X2), trans=True).cpu().numpy()
            a, b = np.sum(MX1 * X2), np.sum(X1 * MtX2)
            scale = np.linalg.norm(MX1) * np.linalg.norm(X2) + np.linalg.norm(MtX2) * np.linalg.norm(X1)
            assert abs(a - b) <= 1e-13 * scale, (which, s_cols, a, b)


def test_norm2_est_matches_oracle(H):
    inp = G.config(0)
    A = H.hodlr_build(inp, rank_cap=8)
    est = H.hodlr_norm2_est(A, 50)
    assert est == pytest.approx(O.norm2_est(O.from_input(inp)), rel=1e-12)


PARTS = [(64, 64, 3, 0), (64, 32, 3, 1), (64, 8, 3, 2), (100, 13, 4, 3), (257, 33, 5, 4), (512, 64, 6, 5)]


@pytest.mark.parametrize("n,leaf,k,seed", PARTS)
def test_lossless_equals_dense_householder(H, n, leaf, k, seed):
    """eps = 0: hQR is exactly Householder QR of the assembled matrix."""
    inp = G.gaussian_hodlr(n, leaf, k, seed)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, 0.0, anorm=1.0)
    d = _factor_dense(H, F, inp)
    Yd, Td, Rd = O.house_qr(inp.to_dense())
    assert _rel(d["R"], Rd) <= 1e-12
    assert np.abs(d["Y"] - Yd).max() <= 1e-12
    assert np.abs(d["T"] - Td).max() <= 1e-12


def test_config0_parity(H):
    inp = G.config(0)
    ref = O.hqr(inp, EPS)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, EPS, anorm=ref.anorm)
    X = np.random.default_rng(1000).standard_normal((inp.n, 16))
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    QX = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
    assert _rel(RX, O.rmat(ref, X)) <= 1e-8
    assert _rel(QX, O.apply_q(ref, X), np.linalg.norm(X)) <= 1e-8
    # backward bounds on the dense factors
    d = _factor_dense(H, F, inp)
    Q = np.eye(inp.n) - d["Y"] @ d["T"] @ d["Y"].T
    Ad = inp.to_dense()
    assert np.linalg.norm(Q @ d["R"] - Ad, 2) / np.linalg.norm(Ad, 2) <= 10 * EPS
    assert np.linalg.norm(Q.T @ Q - np.eye(inp.n), 2) <= 10 * EPS
    # same rank structure as the oracle
    info = H.hodlr_qr_info(F)
    assert (info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]) == (
        O.max_ranks(ref.Y), O.max_ranks(ref.T), O.max_ranks(ref.R))
    assert info["n_truncations"] >= len([t for t in ref.counter.truncs if t["site"] != "orth"]) - 0


def test_config0_anorm_on_device(H):
    """anorm <= 0: the library estimates |A|_2 itself, as the oracle does."""
    inp = G.config(0)
    ref = O.hqr(inp, EPS)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, EPS)
    info = H.hodlr_qr_info(F)
    assert info["anorm"] == pytest.approx(ref.anorm, rel=1e-12)
    assert info["tau_a"] == pytest.approx(EPS * ref.anorm, rel=1e-12)
    X = np.random.default_rng(7).standard_normal((inp.n, 4))
    assert _rel(H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X)) <= 1e-8


@pytest.mark.parametrize("n,leaf", [(512, 64), (16384, 256)])
def test_launch_modes_agree_bitwise(H, n, leaf):
    """Two streams (default), one stream and graph replay give the same bits."""
    inp = G.config(0) if n == 512 else G.expkernel_hodlr(n, leaf, 2)
    A = H.hodlr_build(inp, rank_cap=64 if n == 512 else 16)
    X = np.random.default_rng(3).standard_normal((inp.n, 8))
    outs = []
    for flags in (0, H.HODLR_QR_ONE_STREAM, H.HODLR_QR_GRAPH, 0):
        F = H.hodlr_qr(A, EPS, anorm=17.6, flags=flags)
        outs.append((H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(),
                     H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()))
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0]) and np.array_equal(outs[0][1], o[1])


def test_flop_count_matches_oracle(H):
    inp = G.config(0)
    ref = O.hqr(inp, EPS)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, EPS, anorm=ref.anorm)
    info = H.hodlr_qr_info(F)
    # the library left-orthogonalises every lower block up front, the oracle
    # only the blocks that reach line left_orthogonal unorthonormalised
    other = ref.counter.total - ref.counter.flops["orth"]
    assert other <= info["flops"] <= other + 4 * ref.counter.flops["orth"] + 2e7


def test_apply_q_transpose_and_solve(H):
    inp = G.gaussian_hodlr(1024, 128, 6, seed=9)
    ref = O.hqr(inp, 1e-12)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, 1e-12, anorm=ref.anorm)
    X = np.random.default_rng(4).standard_normal((inp.n, 70))
    QtX = H.hodlr_apply_q(F, H.colmajor(X), trans=True).cpu().numpy()
    assert _rel(QtX, O.apply_q(ref, X, trans=True), np.linalg.norm(X)) <= 1e-9
    B = H.hodlr_solve(F, H.colmajor(X)).cpu().numpy()
    Ad = inp.to_dense()
    assert np.linalg.norm(Ad @ B - X) / np.linalg.norm(X) <= 1e-9
    assert _rel(B, O.solve(ref, X)) <= 1e-8


def _noise_floor(inp, eps, anorm, X):
    a = O.hqr(inp, eps, anorm=anorm)
    b = O.hqr(G.perturb(inp, 11), eps, anorm=anorm)
    return a, (_rel(O.rmat(a, X), O.rmat(b, X)), _rel(O.apply_q(a, X), O.apply_q(b, X), np.linalg.norm(X)))


@pytest.mark.parametrize("n", [4096, 16384])
def test_expkernel_parity(H, n):
    inp = G.expkernel_hodlr(n, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    anorm = H.hodlr_norm2_est(A, 50)
    X = np.random.default_rng(1002).standard_normal((n, 16))
    ref, (fr, fq) = _noise_floor(inp, EPS, anorm, X)
    F = H.hodlr_qr(A, EPS, anorm=anorm)
    rR = _rel(H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
    rQ = _rel(H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
    print(f"n={n}: relR {rR:.2e} (floor {fr:.2e})  relQ {rQ:.2e} (floor {fq:.2e})")
    assert rR <= max(1e-8, 10 * fr)
    assert rQ <= max(1e-8, 10 * fq)
    info = H.hodlr_qr_info(F)
    assert (info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]) == (
        O.max_ranks(ref.Y), O.max_ranks(ref.T), O.max_ranks(ref.R))


def test_expkernel_full_size_sampled(H):
    """n = 65536 (the benchmark matrix): products with a random block against
    the oracle, and the backward residual A X - Q (R X) through HODLR products."""
    n = 65536
    inp = G.expkernel_hodlr(n, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    F = H.hodlr_qr(A, EPS)
    info = H.hodlr_qr_info(F)
    X = np.random.default_rng(1002).standard_normal((n, 4))
    ref, (fr, fq) = _noise_floor(inp, EPS, info["anorm"], X)
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    RXo = O.rmat(ref, X)
    QX = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
    QXo = O.apply_q(ref, X)
    rR, rQ = _rel(RX, RXo), _rel(QX, QXo, np.linalg.norm(X))
    print(f"n=65536: relR {rR:.2e} (floor {fr:.2e})  relQ {rQ:.2e} (floor {fq:.2e})")
    assert rR <= max(1e-8, 10 * fr) and rQ <= max(1e-8, 10 * fq)
    # backward: |A X - Q R X| / (|A| |X|) <= 10 eps
    AX = H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy()
    QRX = H.hodlr_apply_q(F, H.colmajor(RX)).cpu().numpy()
    assert np.linalg.norm(AX - QRX) / (info["anorm"] * np.linalg.norm(X)) <= 10 * EPS
    # orthogonality on the sample: |Q^T Q X - X| / |X|
    QtQX = H.hodlr_apply_q(F, H.colmajor(QX), trans=True).cpu().numpy()
    assert np.linalg.norm(QtQX - X) / np.linalg.norm(X) <= 10 * EPS


def test_cauchy_backward_and_floor(H):
    inp = G.cauchy_hodlr(2048, 256, seed=1)
    A = H.hodlr_build(inp, rank_cap=64)
    anorm = H.hodlr_norm2_est(A, 50)
    X = np.random.default_rng(1001).standard_normal((inp.n, 16))
    ref, (fr, fq) = _noise_floor(inp, EPS, anorm, X)
    F = H.hodlr_qr(A, EPS, anorm=anorm)
    d = _factor_dense(H, F, inp)
    Q = np.eye(inp.n) - d["Y"] @ d["T"] @ d["Y"].T
    Ad = inp.to_dense()
    assert np.linalg.norm(Q @ d["R"] - Ad, 2) / np.linalg.norm(Ad, 2) <= 10 * EPS
    assert np.linalg.norm(Q.T @ Q - np.eye(inp.n), 2) <= 10 * EPS
    rQ = _rel(Q @ X, O.apply_q(ref, X), np.linalg.norm(X))
    print(f"cauchy n=2048: relQ {rQ:.2e} (floor {fq:.2e})")
    assert rQ <= max(1e-8, 10 * fq)


def test_special_cases(H):
    # zero off-diagonal ranks: block diagonal factors
    inp = G.gaussian_hodlr(256, 32, 0, seed=21)
    F = H.hodlr_qr(H.hodlr_build(inp, rank_cap=8), EPS)
    info = H.hodlr_qr_info(F)
    assert info["max_rank_y"] == info["max_rank_t"] == info["max_rank_r"] == 0
    # upper triangular HODLR: Y = I, T = 0, R = A exactly
    inp = G.gaussian_hodlr(128, 16, 3, seed=22)
    inp.leaves = [np.triu(D) for D in inp.leaves]
    for v in inp.internal_nodes():
        U, V = inp.blocks[(v, "lo")]
        inp.blocks[(v, "lo")] = (U[:, :0], V[:, :0])
    F = H.hodlr_qr(H.hodlr_build(inp, rank_cap=8), EPS)
    d = _factor_dense(H, F, inp)
    assert np.array_equal(d["Y"], np.eye(128)) and not d["T"].any()
    np.testing.assert_allclose(d["R"], inp.to_dense(), atol=1e-14)
    # level 0: one dense leaf
    inp = G.gaussian_hodlr(200, 256, 0, seed=23)
    F = H.hodlr_qr(H.hodlr_build(inp, rank_cap=4), EPS)
    d = _factor_dense(H, F, inp)
    _, _, Rd = O.house_qr(inp.to_dense())
    np.testing.assert_allclose(d["R"], Rd, atol=1e-12)


def test_capacity_error_is_reported(H):
    inp = G.config(0)
    A = H.hodlr_build(inp, rank_cap=8)
    with pytest.raises(H.HodlrError) as e:
        H.hodlr_qr(A, EPS)
    assert e.value.status == -4


def test_repeat_runs_are_deterministic(H):
    inp = G.expkernel_hodlr(4096, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    X = H.colmajor(np.random.default_rng(5).standard_normal((4096, 4)))
    a = H.hodlr_apply_q(H.hodlr_qr(A, EPS), X.clone()).cpu().numpy()
    b = H.hodlr_apply_q(H.hodlr_qr(A, EPS), X.clone()).cpu().numpy()
    assert np.array_equal(a, b)


def _batch_inputs():
    """A small batch of two shapes: three n=1024 and two n=2048 Gaussian HODLR
    matrices (leaf 256) of different ranks."""
    specs = [(1024, 1, 30), (2048, 3, 31), (1024, 4, 32), (2048, 2, 33), (1024, 2, 34)]
    return [G.gaussian_hodlr(n, 256, k, seed=sd) for n, k, sd in specs]


def test_batched_equals_one_at_a_time_bitwise(H):
    """Each factorisation of a batch gives the bits hodlr_qr gives alone."""
    inps = _batch_inputs()
    As = [H.hodlr_build(inp, rank_cap=32) for inp in inps]
    Fb = H.hodlr_qr_batched(As, EPS)
    for inp, A, Fi in zip(inps, As, Fb):
        X = np.random.default_rng(5).standard_normal((inp.n, 4))
        F1 = H.hodlr_qr(A, EPS)
        for which in "YTR":
            a = H.hodlr_qr_matmul(Fi, which, H.colmajor(X)).cpu().numpy()
            b = H.hodlr_qr_matmul(F1, which, H.colmajor(X)).cpu().numpy()
            assert np.array_equal(a, b), which
        assert H.hodlr_qr_info(Fi)["anorm"] == H.hodlr_qr_info(F1)["anorm"]


def test_batched_parity_with_oracle(H):
    """Batched factors against the oracle (same thresholds), well-conditioned inputs."""
    inps = _batch_inputs()
    As = [H.hodlr_build(inp, rank_cap=32) for inp in inps]
    anorms = [H.hodlr_norm2_est(A, 50) for A in As]
    Fb = H.hodlr_qr_batched(As, EPS, anorm=anorms)
    for inp, Fi, an in list(zip(inps, Fb, anorms))[:3]:
        ref = O.hqr(inp, EPS, anorm=an)
        X = np.random.default_rng(6).standard_normal((inp.n, 8))
        rR = _rel(H.hodlr_qr_matmul(Fi, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
        rQ = _rel(H.hodlr_apply_q(Fi, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
        assert rR <= 1e-8 and rQ <= 1e-8, (inp.n, rR, rQ)


# Recompressions run in k_tr_small when both factors have at most four 256-row
# chunks (narrow: w <= 8 inside one block; wide: one block per chunk and the
# forming step in the block that ran the SVD), otherwise in k_tr_qr + k_tr_form.
# n, leaf, k, rank_cap: 2048/256/2/16 has narrow jobs of 1, 2 and 4 even chunks;
# 2048/256/5/32 wide jobs of several chunks (R ranks up to 30); 1500/200/3/32
# uneven chunk splits (blocks of 750 and 375 rows).
RECOMP_CASES = [(2048, 256, 2, 16, 40), (2048, 256, 5, 32, 41), (1500, 200, 3, 32, 42)]


@pytest.mark.parametrize("n,leaf,k,cap,seed", RECOMP_CASES)
def test_recompression_kernel_paths(H, n, leaf, k, cap, seed):
    inp = G.gaussian_hodlr(n, leaf, k, seed=seed)
    A = H.hodlr_build(inp, rank_cap=cap)
    anorm = H.hodlr_norm2_est(A, 50)
    F = H.hodlr_qr(A, EPS, anorm=anorm)
    ref = O.hqr(inp, EPS, anorm=anorm)
    X = np.random.default_rng(seed).standard_normal((n, 8))
    rR = _rel(H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
    rQ = _rel(H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
    assert rR <= 1e-8 and rQ <= 1e-8, (n, rR, rQ)
    # the factorisation itself: |A X - Q R X| / (|A| |X|) and |Q^T Q X - X| / |X|
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    AX = H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy()
    QRX = H.hodlr_apply_q(F, H.colmajor(RX)).cpu().numpy()
    assert np.linalg.norm(AX - QRX) / (anorm * np.linalg.norm(X)) <= 10 * EPS
    QX = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
    QtQX = H.hodlr_apply_q(F, H.colmajor(QX), trans=True).cpu().numpy()
    assert np.linalg.norm(QtQX - X) / np.linalg.norm(X) <= 10 * EPS


def test_batched_time_runs(H):
    inps = _batch_inputs()[:2]
    As = [H.hodlr_build(inp, rank_cap=32) for inp in inps]
    ms = H.hodlr_qr_batched_time(As, EPS, warmup=1, reps=2)
    assert ms.shape == (2,) and (ms > 0).all()
