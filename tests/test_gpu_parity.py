"""GPU parity of the HIP hQR library against the CPU oracle (needs an MI355X).

Every call goes through the C ABI (libhodlr.so) via the ctypes binding; the
oracle runs on the host on the same seeded inputs.  Every parity test gives
both sides the oracle's |A|_2 estimate (power iteration, reading C1), so the
truncation thresholds never come from the device; the device's own estimate is
checked against the oracle's separately.

Tolerances (written where they are used):
  * lossless runs (eps = 0) reproduce dense Householder QR entrywise to
    1e-12 relative: only rounding order differs;
  * well-conditioned inputs (Gaussian HODLR, kappa ~ 1e3..1e5): relative
    difference of R X and of Q X to the oracle <= 1e-8 (eps = 1e-10);
  * ill-conditioned inputs (exponential kernel, Cauchy): the same forward
    comparison is bounded by 10x the oracle's own noise floor (oracle of A vs
    oracle of A perturbed at roundoff level) or 1e-8, whichever is larger,
    plus the backward bounds |A - QR|/|A| <= 10 eps and |I - Q^T Q| <= 10 eps;
  * the rank of every recompression equals the oracle's, decision by decision,
    except at a near tie |sigma - tau| <= 1e-8 tau or where the oracle itself
    takes the device's decision on the roundoff-perturbed noise-floor input
    (then the singular value is rounding noise; the runs diverge from there).
"""
import numpy as np
import pytest

import hodlr_gen as G
import oracle as O
from helpers import dense_from_export, leaf_sizes

pytestmark = pytest.mark.gpu

EPS = 1e-10
_ANORM = {}


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


def oracle_anorm(inp, key=None):
    """The oracle's |A|_2 estimate (50 power-iteration steps, reading C1)."""
    if key is not None and key in _ANORM:
        return _ANORM[key]
    a = O.norm2_est(O.from_input(inp))
    if key is not None:
        _ANORM[key] = a
    return a


SITE = {1: "S", 2: "A12", 3: "update", 4: "T"}


def ranklog_check(H, F, ref, alt=(), tie=1e-8):
    """Decision-by-decision comparison of the device's rank log with the
    oracle's (Counter.truncs): the same recompressions (the up-front
    orthogonalisation of the lower blocks excluded, the oracle does it lazily,
    reading C10) with the same input width and kept rank, in the oracle's
    (sequential) order.

    `alt` are oracle runs on A perturbed at roundoff level (the noise-floor
    inputs).  On an ill-conditioned A a singular value near tau can be below
    the method's own rounding noise; the oracle runs then take different
    decisions there, and every one of them is correct.  The device is compared
    with every run that has agreed with it so far; a decision passes when one
    of those runs takes it.  When none does, the decision may still differ by
    one where rounding decides it: at a near tie, |sigma - tau| <= max(tie *
    tau, 3 * spread), spread being how far that singular value moves between
    the runs, or where the oracle runs themselves keep different ranks at this
    recompression.  The runs diverge from there and the comparison stops.
    Returns (decisions compared, 1 if stopped at such a divergence)."""
    dev = {}
    for r in H.hodlr_qr_ranklog(F):
        site = int(r[0])
        if site == 0:
            continue
        key = (SITE[site], int(r[1]), int(r[2]))
        if site in (1, 4):
            key += (int(r[3]),)
        elif site == 3:
            key += (int(r[3]), int(r[4]))
        dev[key] = (int(r[5]), int(r[6]))
    ora = [t for t in ref.counter.truncs if t["key"] is not None]
    assert set(dev) == {t["key"] for t in ora}, "different sets of recompressions"
    runs = [{t["key"]: t for t in c.counter.truncs if t["key"] is not None} for c in [ref] + list(alt)]
    live = list(range(len(runs)))
    n = 0
    for t in ora:
        key = t["key"]
        wk = dev[key]
        agree = [i for i in live if (runs[i][key]["w"], runs[i][key]["k"]) == wk]
        if agree:
            if agree != live:
                print(f"rank decision {key}: device {wk}, taken by oracle run(s) {agree} of {live} "
                      f"(sigma_k / sigma_k+1 {t['sk']:.3e} / {t['sk1']:.3e}, tau {t['tau']:.3e})")
            live = agree
            n += 1
            continue
        w, k = wk
        near = len({r[key]["k"] for r in runs}) > 1  # the oracle runs disagree here
        for i in live:
            c = runs[i][key]
            if c["w"] != w or abs(k - c["k"]) != 1:
                continue
            field = "sk1" if k > c["k"] else "sk"
            vals = [r[key][field] for r in runs if r[key]["k"] == c["k"] and r[key]["w"] == w]
            spread = max(vals) - min(vals)
            if abs(c[field] - c["tau"]) <= max(tie * c["tau"], 3.0 * spread):
                near = True
        assert near, (key, "rank differs from every oracle run away from a near tie", wk,
                      [(runs[i][key]["w"], runs[i][key]["k"], runs[i][key]["sk"], runs[i][key]["sk1"]) for i in live],
                      t["tau"])
        print(f"rank decision {key}: device {wk} at a near tie; comparison stops after {n} decisions")
        return n, 1
    return n, 0


def _spectral(apply, n, iters=30, seed=0):
    """|M|_2 estimate of a symmetric positive semidefinite M by block power
    iteration (two seeded columns); apply(X) returns M X (host arrays)."""
    X = np.random.default_rng(seed).standard_normal((n, 2))
    X /= np.linalg.norm(X, axis=0)
    est = 0.0
    for _ in range(iters):
        Y = apply(X)
        nrm = np.linalg.norm(Y, axis=0)
        est = float(nrm.max())
        if est == 0.0:
            return 0.0
        X = Y / np.where(nrm > 0, nrm, 1.0)
    return est


def orth_error(H, F, n):
    """|I - Q^T Q|_2 estimate: E = Q^T Q - I is symmetric, power iteration on E^2."""
    def E(X):
        Q = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
        return H.hodlr_apply_q(F, H.colmajor(Q), trans=True).cpu().numpy() - X
    return np.sqrt(_spectral(lambda X: E(E(X)), n))


def backward_error(H, A, F, n):
    """|A - QR|_2 estimate: power iteration on B^T B, B = A - Q R."""
    def B(X):
        RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
        return H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy() - H.hodlr_apply_q(F, H.colmajor(RX)).cpu().numpy()

    def Bt(Y):
        QtY = H.hodlr_apply_q(F, H.colmajor(Y), trans=True).cpu().numpy()
        return (H.hodlr_matmul(A, H.colmajor(Y), trans=True).cpu().numpy()
                - H.hodlr_qr_matmul(F, "R", H.colmajor(QtY), trans=True).cpu().numpy())
    return np.sqrt(_spectral(lambda X: Bt(B(X)), n))


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


def test_factor_products_long_launch_against_oracle(H):
    """The factors Y (unit lower leaves), T and R (upper leaves) over 33001 rows
    (64-row product tiles, transposed leaf tiles through LDS) against the
    oracle's factors of the same matrix, same thresholds: Y X, Y^T X, T X,
    T^T X, R X, R^T X on 1, 4 and 9 columns within 1e-8 (a well-conditioned
    Gaussian matrix: the forward bound of the scope applies), and the same
    rank decisions."""
    from oracle import hodlr as OH
    inp = G.gaussian_hodlr(33001, 256, 2, seed=32)
    an = oracle_anorm(inp)
    ref = O.hqr(inp, EPS, anorm=an)
    A = H.hodlr_build(inp, rank_cap=48)
    F = H.hodlr_qr(A, EPS, anorm=an)
    print("ranks Y, T, R:", O.max_ranks(ref.Y), O.max_ranks(ref.T), O.max_ranks(ref.R), flush=True)
    n_cmp, tie = ranklog_check(H, F, ref)
    assert tie == 0 and n_cmp > 1000
    rng = np.random.default_rng(5)
    for s_cols in (1, 4, 9):
        X = rng.standard_normal((inp.n, s_cols))
        for which, M in (("Y", ref.Y), ("T", ref.T), ("R", ref.R)):
            print(f"n=33001 {which} s={s_cols}", flush=True)
            for trans in (False, True):
                Z = H.hodlr_qr_matmul(F, which, H.colmajor(X), trans=trans).cpu().numpy()
                Zo = OH.hmatT(M, X) if trans else OH.hmat(M, X)
                assert _rel(Z, Zo) <= 1e-8, (which, trans, s_cols, _rel(Z, Zo))


@pytest.mark.parametrize("n", [512, 4096, 16384, 65536])
def test_norm2_est_matches_oracle(H, n):
    """Reading C1 on both sides: the device's 50-step power iteration equals
    the oracle's to 1e-12."""
    inp = G.config(0) if n == 512 else G.expkernel_hodlr(n, 256, 2)
    A = H.hodlr_build(inp, rank_cap=64 if n == 512 else 16)
    est = H.hodlr_norm2_est(A, 50)
    assert est == pytest.approx(oracle_anorm(inp, ("exp", n) if n > 512 else "cfg0"), rel=1e-12)


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
    an = oracle_anorm(inp, "cfg0")
    ref = O.hqr(inp, EPS, anorm=an)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, EPS, anorm=an)
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
    # the same rank decisions, one by one
    n_cmp, tie = ranklog_check(H, F, ref)
    assert tie == 0 and n_cmp == len([t for t in ref.counter.truncs if t["key"] is not None])
    info = H.hodlr_qr_info(F)
    assert (info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]) == (
        O.max_ranks(ref.Y), O.max_ranks(ref.T), O.max_ranks(ref.R))


def test_config0_anorm_on_device(H):
    """anorm <= 0: the library estimates |A|_2 itself, as the oracle does."""
    inp = G.config(0)
    ref = O.hqr(inp, EPS)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, EPS)
    info = H.hodlr_qr_info(F)
    assert info["anorm"] == pytest.approx(ref.anorm, rel=1e-12)
    assert info["tau_a"] == pytest.approx(EPS * ref.anorm, rel=1e-12)
    assert info["norm_flops"] > 0
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
    an = oracle_anorm(inp, "cfg0")
    ref = O.hqr(inp, EPS, anorm=an)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, EPS, anorm=an)
    info = H.hodlr_qr_info(F)
    assert info["norm_flops"] == 0.0
    # the library left-orthogonalises every lower block up front, the oracle
    # only the blocks that reach the left_orthogonal step unorthonormalised
    other = ref.counter.total - ref.counter.flops["orth"]
    assert other <= info["flops"] <= other + 4 * ref.counter.flops["orth"] + 2e7


def test_apply_q_transpose_and_solve(H):
    inp = G.gaussian_hodlr(1024, 128, 6, seed=9)
    an = oracle_anorm(inp)
    ref = O.hqr(inp, 1e-12, anorm=an)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, 1e-12, anorm=an)
    X = np.random.default_rng(4).standard_normal((inp.n, 70))
    QtX = H.hodlr_apply_q(F, H.colmajor(X), trans=True).cpu().numpy()
    assert _rel(QtX, O.apply_q(ref, X, trans=True), np.linalg.norm(X)) <= 1e-9
    B = H.hodlr_solve(F, H.colmajor(X)).cpu().numpy()
    Ad = inp.to_dense()
    assert np.linalg.norm(Ad @ B - X) / np.linalg.norm(X) <= 1e-9
    assert _rel(B, O.solve(ref, X)) <= 1e-8


def _noise_floor(inp, eps, anorm, X, extra=()):
    """The oracle on A, and on A perturbed at roundoff level (seed 11, plus the
    `extra` seeds): forward noise floor of R X and Q X, and the perturbed runs."""
    a = O.hqr(inp, eps, anorm=anorm)
    b = O.hqr(G.perturb(inp, 11), eps, anorm=anorm)
    NOISE_RUNS[id(a)] = [b] + [O.hqr(G.perturb(inp, sd), eps, anorm=anorm) for sd in extra]
    return a, (_rel(O.rmat(a, X), O.rmat(b, X)), _rel(O.apply_q(a, X), O.apply_q(b, X), np.linalg.norm(X)))


NOISE_RUNS = {}


@pytest.mark.parametrize("n", [4096, 16384])
def test_expkernel_parity(H, n):
    inp = G.expkernel_hodlr(n, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    an = oracle_anorm(inp, ("exp", n))
    assert H.hodlr_norm2_est(A, 50) == pytest.approx(an, rel=1e-12)
    X = np.random.default_rng(1002).standard_normal((n, 16))
    ref, (fr, fq) = _noise_floor(inp, EPS, an, X, extra=(12, 13))
    F = H.hodlr_qr(A, EPS, anorm=an)
    rR = _rel(H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
    rQ = _rel(H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
    print(f"n={n}: relR {rR:.2e} (floor {fr:.2e})  relQ {rQ:.2e} (floor {fq:.2e})")
    assert rR <= max(1e-8, 10 * fr)
    assert rQ <= max(1e-8, 10 * fq)
    n_cmp, stop = ranklog_check(H, F, ref, alt=NOISE_RUNS[id(ref)])
    print(f"n={n}: {n_cmp} rank decisions equal before any divergence (stopped: {stop})")
    assert n_cmp > 0
    info = H.hodlr_qr_info(F)
    assert (info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]) == (
        O.max_ranks(ref.Y), O.max_ranks(ref.T), O.max_ranks(ref.R))


def test_expkernel_full_size(H):
    """n = 65536 (the benchmark matrix, the benchmark's launch configuration),
    the oracle's |A|_2 on both sides: products with a random block against the
    oracle within 10x its noise floor; |A - QR|_2 / |A|_2 and |I - Q^T Q|_2 by
    30-step power iterations through the device's products (estimates, lower
    bounds of the 2-norms) within 10 eps; every rank decision equal; the work
    counters within 1 %."""
    n = 65536
    inp = G.expkernel_hodlr(n, 256, 2)
    A = H.hodlr_build(inp, rank_cap=16)
    an = oracle_anorm(inp, ("exp", n))
    assert H.hodlr_norm2_est(A, 50) == pytest.approx(an, rel=1e-12)
    F = H.hodlr_qr(A, EPS, anorm=an)
    X = np.random.default_rng(1002).standard_normal((n, 16))
    ref, (fr, fq) = _noise_floor(inp, EPS, an, X, extra=(12, 13))
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    QX = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
    rR, rQ = _rel(RX, O.rmat(ref, X)), _rel(QX, O.apply_q(ref, X), np.linalg.norm(X))
    print(f"n=65536: relR {rR:.2e} (floor {fr:.2e})  relQ {rQ:.2e} (floor {fq:.2e})", flush=True)
    assert rR <= max(1e-8, 10 * fr) and rQ <= max(1e-8, 10 * fq)
    e_orth = orth_error(H, F, n)
    e_acc = backward_error(H, A, F, n) / an
    print(f"n=65536: |I - Q^T Q|_2 ~ {e_orth:.2e}, |A - QR|_2/|A|_2 ~ {e_acc:.2e}", flush=True)
    assert e_orth <= 10 * EPS and e_acc <= 10 * EPS
    n_cmp, stop = ranklog_check(H, F, ref, alt=NOISE_RUNS[id(ref)])
    print(f"n=65536: {n_cmp} rank decisions equal before any divergence (stopped: {stop})", flush=True)
    assert n_cmp > 0
    info = H.hodlr_qr_info(F)
    assert info["flops"] == pytest.approx(ref.counter.total, rel=0.01)


def test_config1_cauchy(H):
    """Config 1 (Sec. 5, Ex. 2 stand-in): Cauchy matrix n = 8192, leaf 256,
    depth 5, compressed at 1e-10 |A|_2, kappa ~ 1e22.  Backward bounds by power
    iteration within 10 eps, forward R X and Q X within 10x the oracle's noise
    floor, and the rank log decision by decision."""
    inp = G.config(1)
    A = H.hodlr_build(inp, rank_cap=64)
    an = oracle_anorm(inp)
    assert H.hodlr_norm2_est(A, 50) == pytest.approx(an, rel=1e-12)
    X = np.random.default_rng(1001).standard_normal((inp.n, 16))
    ref, (fr, fq) = _noise_floor(inp, EPS, an, X, extra=(12, 13))
    F = H.hodlr_qr(A, EPS, anorm=an)
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    QX = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
    rR, rQ = _rel(RX, O.rmat(ref, X)), _rel(QX, O.apply_q(ref, X), np.linalg.norm(X))
    print(f"config 1: relR {rR:.2e} (floor {fr:.2e})  relQ {rQ:.2e} (floor {fq:.2e})", flush=True)
    assert rR <= max(1e-8, 10 * fr) and rQ <= max(1e-8, 10 * fq)
    e_orth = orth_error(H, F, inp.n)
    e_acc = backward_error(H, A, F, inp.n) / an
    print(f"config 1: |I - Q^T Q|_2 ~ {e_orth:.2e}, |A - QR|_2/|A|_2 ~ {e_acc:.2e}", flush=True)
    assert e_orth <= 10 * EPS and e_acc <= 10 * EPS
    n_cmp, stop = ranklog_check(H, F, ref, alt=NOISE_RUNS[id(ref)])
    print(f"config 1: {n_cmp} rank decisions equal before any divergence (stopped: {stop})", flush=True)
    assert n_cmp > 0
    # kappa ~ 1e22: Y and T are not determined at this precision (the oracle's own
    # relQ between A and its roundoff perturbation is O(1)), so most later rank
    # decisions are rounding noise; the device's rank profile must lie within
    # the range of the oracle runs'
    info = H.hodlr_qr_info(F)
    for fld, attr in (("max_rank_y", "Y"), ("max_rank_t", "T"), ("max_rank_r", "R")):
        vals = [O.max_ranks(getattr(r, attr)) for r in [ref] + NOISE_RUNS[id(ref)]]
        print(f"config 1: {fld} device {info[fld]}, oracle runs {vals}")
        assert 0.8 * min(vals) <= info[fld] <= 1.2 * max(vals)


def test_cauchy_backward_and_floor(H):
    inp = G.cauchy_hodlr(2048, 256, seed=1)
    A = H.hodlr_build(inp, rank_cap=64)
    an = oracle_anorm(inp)
    X = np.random.default_rng(1001).standard_normal((inp.n, 16))
    # four oracle runs, as for the other ill-conditioned inputs: with one
    # perturbed run the rank check cannot see that the runs themselves split
    # at the T-lane recompressions of the top node (rank 20 or 21 at sigma
    # within a few tau of each other)
    ref, (fr, fq) = _noise_floor(inp, EPS, an, X, extra=(12, 13))
    F = H.hodlr_qr(A, EPS, anorm=an)
    d = _factor_dense(H, F, inp)
    Q = np.eye(inp.n) - d["Y"] @ d["T"] @ d["Y"].T
    Ad = inp.to_dense()
    assert np.linalg.norm(Q @ d["R"] - Ad, 2) / np.linalg.norm(Ad, 2) <= 10 * EPS
    assert np.linalg.norm(Q.T @ Q - np.eye(inp.n), 2) <= 10 * EPS
    rQ = _rel(Q @ X, O.apply_q(ref, X), np.linalg.norm(X))
    rR = _rel(d["R"] @ X, O.rmat(ref, X))
    print(f"cauchy n=2048: relR {rR:.2e} (floor {fr:.2e}) relQ {rQ:.2e} (floor {fq:.2e})")
    assert rQ <= max(1e-8, 10 * fq) and rR <= max(1e-8, 10 * fr)
    ranklog_check(H, F, ref, alt=NOISE_RUNS[id(ref)])


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


@pytest.mark.parametrize("mode", ["merged", "by_shape", "merged_graph", "by_shape_one_stream"])
def test_batched_equals_one_at_a_time_bitwise(H, mode):
    """Each factorisation of a batch gives the bits hodlr_qr gives alone:
    shapes merged into one launch sequence (the default), shape groups one
    after another (two streams, or one), and the merged sequence captured and
    replayed as a HIP graph."""
    flags = {"merged": 0, "by_shape": H.HODLR_QR_BY_SHAPE, "merged_graph": H.HODLR_QR_GRAPH,
             "by_shape_one_stream": H.HODLR_QR_BY_SHAPE | H.HODLR_QR_ONE_STREAM}[mode]
    inps = _batch_inputs()
    As = [H.hodlr_build(inp, rank_cap=32) for inp in inps]
    Fb = H.hodlr_qr_batched(As, EPS, flags=flags)
    for inp, A, Fi in zip(inps, As, Fb):
        X = np.random.default_rng(5).standard_normal((inp.n, 4))
        F1 = H.hodlr_qr(A, EPS)
        for which in "YTR":
            a = H.hodlr_qr_matmul(Fi, which, H.colmajor(X)).cpu().numpy()
            b = H.hodlr_qr_matmul(F1, which, H.colmajor(X)).cpu().numpy()
            assert np.array_equal(a, b), which
        i1, ib = H.hodlr_qr_info(F1), H.hodlr_qr_info(Fi)
        assert ib["anorm"] == i1["anorm"]
        assert ib["n_truncations"] == i1["n_truncations"]
        assert np.array_equal(H.hodlr_qr_ranklog(Fi), H.hodlr_qr_ranklog(F1))


@pytest.mark.parametrize("mode", ["merged", "merged_graph"])
def test_batched_chains_bitwise(H, mode):
    """At rank capacity 16 the recompression chains run one block per chain
    (k_tr_chain); merged across shapes, and captured as a HIP graph, each
    factorisation still gives the bits hodlr_qr gives alone."""
    flags = {"merged": 0, "merged_graph": H.HODLR_QR_GRAPH}[mode]
    inps = [G.gaussian_hodlr(n, 256, k, seed=sd) for n, k, sd in [(1024, 1, 70), (2048, 2, 71), (1024, 2, 72)]]
    As = [H.hodlr_build(inp, rank_cap=16) for inp in inps]
    assert H.hodlr_qr_profile(As[1], EPS)["tr_chain"]["count"] > 0
    Fb = H.hodlr_qr_batched(As, EPS, flags=flags)
    for inp, A, Fi in zip(inps, As, Fb):
        X = np.random.default_rng(6).standard_normal((inp.n, 4))
        F1 = H.hodlr_qr(A, EPS)
        for which in "YTR":
            a = H.hodlr_qr_matmul(Fi, which, H.colmajor(X)).cpu().numpy()
            b = H.hodlr_qr_matmul(F1, which, H.colmajor(X)).cpu().numpy()
            assert np.array_equal(a, b), which
        assert np.array_equal(H.hodlr_qr_ranklog(Fi), H.hodlr_qr_ranklog(F1))


def test_batched_graph_replays(H):
    """The merged batch schedule kept (HODLR_QR_KEEP) and captured as one HIP
    graph, then replayed by hodlr_qr_refactor several times with eager work and
    synchronisations between the replays, alternating between two sets of
    inputs of the same shapes: every replay leaves exactly the factors that
    hodlr_qr computes for those inputs alone."""
    import torch
    shapes = [(1024, 1), (2048, 3), (1024, 4)]
    sets = [[G.gaussian_hodlr(n, 256, k, seed=60 + 10 * r + i) for i, (n, k) in enumerate(shapes)]
            for r in range(2)]
    As = [[H.hodlr_build(inp, rank_cap=32) for inp in s] for s in sets]
    X = [np.random.default_rng(8).standard_normal((n, 3)) for n, _ in shapes]
    ref = [[(H.hodlr_qr_matmul(F, "R", H.colmajor(x)).cpu().numpy(), H.hodlr_apply_q(F, H.colmajor(x)).cpu().numpy())
            for F, x in zip([H.hodlr_qr(A, EPS) for A in a], X)] for a in As]
    Fk = H.hodlr_qr_batched(As[0], EPS, flags=H.HODLR_QR_GRAPH | H.HODLR_QR_KEEP)
    for rep in range(5):
        r = rep % 2
        if rep > 0:
            H.hodlr_qr_refactor(Fk, As[r], flags=H.HODLR_QR_GRAPH)
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum().item()  # eager work between
        torch.cuda.synchronize()
        for i, (F, x) in enumerate(zip(Fk, X)):
            assert np.array_equal(H.hodlr_qr_matmul(F, "R", H.colmajor(x)).cpu().numpy(), ref[r][i][0]), (rep, i, junk)
            assert np.array_equal(H.hodlr_apply_q(F, H.colmajor(x)).cpu().numpy(), ref[r][i][1]), (rep, i)


def test_refactor_rules(H):
    """A kept single factorisation refactorised with new values (direct
    launches) matches hodlr_qr; a batch member alone, a factorisation that kept
    nothing, or a matrix of another shape is refused."""
    a, b = G.gaussian_hodlr(1024, 128, 3, seed=70), G.gaussian_hodlr(1024, 128, 3, seed=71)
    Aa, Ab = H.hodlr_build(a, rank_cap=32), H.hodlr_build(b, rank_cap=32)
    F = H.hodlr_qr(Aa, EPS, flags=H.HODLR_QR_KEEP)
    H.hodlr_qr_refactor([F], [Ab])
    X = H.colmajor(np.random.default_rng(9).standard_normal((1024, 2)))
    assert np.array_equal(H.hodlr_qr_matmul(F, "R", X).cpu().numpy(),
                          H.hodlr_qr_matmul(H.hodlr_qr(Ab, EPS), "R", X).cpu().numpy())
    assert H.hodlr_qr_info(F)["anorm"] == H.hodlr_qr_info(H.hodlr_qr(Ab, EPS))["anorm"]
    Fb = H.hodlr_qr_batched([Aa, Ab], EPS, flags=H.HODLR_QR_KEEP)
    with pytest.raises(H.HodlrError):
        H.hodlr_qr_refactor(Fb[:1], [Aa])
    with pytest.raises(H.HodlrError):
        H.hodlr_qr_refactor([H.hodlr_qr(Aa, EPS)], [Ab])
    Ac = H.hodlr_build(G.gaussian_hodlr(2048, 128, 3, seed=72), rank_cap=32)
    with pytest.raises(H.HodlrError):
        H.hodlr_qr_refactor([F], [Ac])


def test_batched_parity_with_oracle(H):
    """Every matrix of a batch against the oracle (the oracle's thresholds on
    both sides), well-conditioned inputs: forward bound and rank decisions."""
    inps = _batch_inputs()
    As = [H.hodlr_build(inp, rank_cap=32) for inp in inps]
    anorms = [oracle_anorm(inp) for inp in inps]
    Fb = H.hodlr_qr_batched(As, EPS, anorm=anorms)
    for inp, Fi, an in zip(inps, Fb, anorms):
        ref = O.hqr(inp, EPS, anorm=an)
        X = np.random.default_rng(6).standard_normal((inp.n, 8))
        rR = _rel(H.hodlr_qr_matmul(Fi, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
        rQ = _rel(H.hodlr_apply_q(Fi, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
        assert rR <= 1e-8 and rQ <= 1e-8, (inp.n, rR, rQ)
        assert ranklog_check(H, Fi, ref)[1] == 0


def test_batched_workload_sample_vs_oracle(H):
    """Matrices of the batched benchmark's recipe (d ~ U{2..4} here so the oracle
    finishes in seconds; k ~ U{4..min(32, 32/d)}, rank capacity 64), factorised
    as one merged batch of several shapes: each against the oracle (forward
    bound, backward bound, rank decisions)."""
    inps = G.batched_set(count=8, seed=21, dmin=2, dmax=4, kmin=4, kmax=32, rank_budget=64)
    print("batch:", [inp.name for inp in inps])
    As = [H.hodlr_build(inp, rank_cap=64) for inp in inps]
    anorms = [oracle_anorm(inp) for inp in inps]
    Fb = H.hodlr_qr_batched(As, EPS, anorm=anorms)
    for inp, A, Fi, an in zip(inps, As, Fb, anorms):
        ref = O.hqr(inp, EPS, anorm=an)
        X = np.random.default_rng(7).standard_normal((inp.n, 8))
        RX = H.hodlr_qr_matmul(Fi, "R", H.colmajor(X)).cpu().numpy()
        rR = _rel(RX, O.rmat(ref, X))
        rQ = _rel(H.hodlr_apply_q(Fi, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
        assert rR <= 1e-8 and rQ <= 1e-8, (inp.name, rR, rQ)
        AX = H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy()
        QRX = H.hodlr_apply_q(Fi, H.colmajor(RX)).cpu().numpy()
        assert np.linalg.norm(AX - QRX) / (an * np.linalg.norm(X)) <= 10 * EPS
        assert ranklog_check(H, Fi, ref)[1] == 0
        assert H.hodlr_qr_info(Fi)["max_rank_r"] == O.max_ranks(ref.R)


# Recompressions run in k_tr_small when both factors have at most four 256-row
# chunks (narrow: w <= 8 inside one block; wide: one block per chunk and the
# forming step in the block that ran the SVD), otherwise in k_tr_qr + k_tr_form.
# n, leaf, k, rank_cap:
#  * 2048/256/2/16: narrow jobs of 1, 2 and 4 even chunks;
#  * 2048/256/5/32: wide jobs of several chunks (R ranks up to 30);
#  * 1500/200/3/32: uneven chunk splits (blocks of 750 and 375 rows);
#  * 2048/256/10/64: rank capacity 64, the widest tier (widths 65..90, R ranks 60);
#  * 2048/512/8/32: leaves of 512 rows: stacked leaf columns of up to 528 rows
#    (the 9-rows-per-lane panel, strips staged in two row chunks).
RECOMP_CASES = [(2048, 256, 2, 16, 40), (2048, 256, 5, 32, 41), (1500, 200, 3, 32, 42),
                (2048, 256, 10, 64, 55), (2048, 512, 8, 32, 53)]


@pytest.mark.parametrize("n,leaf,k,cap,seed", RECOMP_CASES)
def test_recompression_and_leaf_paths(H, n, leaf, k, cap, seed):
    inp = G.gaussian_hodlr(n, leaf, k, seed=seed)
    A = H.hodlr_build(inp, rank_cap=cap)
    an = oracle_anorm(inp)
    F = H.hodlr_qr(A, EPS, anorm=an)
    ref = O.hqr(inp, EPS, anorm=an)
    widths = [t["w"] for t in ref.counter.truncs]
    print(f"n={n} leaf={leaf} k={k}: widest recompression {max(widths)}, ranks R {O.max_ranks(ref.R)}")
    X = np.random.default_rng(seed).standard_normal((n, 8))
    RX = H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy()
    QX = H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy()
    rR = _rel(RX, O.rmat(ref, X))
    rQ = _rel(QX, O.apply_q(ref, X), np.linalg.norm(X))
    assert rR <= 1e-8 and rQ <= 1e-8, (n, rR, rQ)
    n_cmp, tie = ranklog_check(H, F, ref)
    assert tie == 0
    # the factorisation itself: |A X - Q R X| / (|A| |X|) and |Q^T Q X - X| / |X|
    AX = H.hodlr_matmul(A, H.colmajor(X)).cpu().numpy()
    QRX = H.hodlr_apply_q(F, H.colmajor(RX)).cpu().numpy()
    assert np.linalg.norm(AX - QRX) / (an * np.linalg.norm(X)) <= 10 * EPS
    QtQX = H.hodlr_apply_q(F, H.colmajor(QX), trans=True).cpu().numpy()
    assert np.linalg.norm(QtQX - X) / np.linalg.norm(X) <= 10 * EPS


# Chains of recompressions (the term-by-term S~ and T~12 sums) run in one block
# per chain when the rank capacity is at most 16: narrow steps (w <= 8, the
# exp kernel, whose parity test_expkernel_parity checks) and wider ones whose
# chunks the block runs one after another (Gaussian rank 2: widths up to 24).
def test_recompression_chains(H):
    inp = G.expkernel_hodlr(4096, 256, seed=2)
    prof = H.hodlr_qr_profile(H.hodlr_build(inp, rank_cap=16), EPS, anorm=oracle_anorm(inp, ("exp", 4096)))
    assert prof["tr_chain"]["count"] > 0 and "tr_small" in prof, prof.keys()
    n, seed = 4096, 11
    inp = G.gaussian_hodlr(n, 256, 2, seed=seed)
    A = H.hodlr_build(inp, rank_cap=16)
    an = oracle_anorm(inp)
    prof = H.hodlr_qr_profile(A, EPS, anorm=an)
    assert prof["tr_chain"]["count"] > 0, prof.keys()
    F = H.hodlr_qr(A, EPS, anorm=an)
    ref = O.hqr(inp, EPS, anorm=an)
    widths = [t["w"] for t in ref.counter.truncs]
    print(f"gaussian n={n}: {prof['tr_chain']['count']} chain launches, widest recompression {max(widths)}")
    assert max(widths) > 8
    X = np.random.default_rng(seed).standard_normal((n, 6))
    rR = _rel(H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
    rQ = _rel(H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
    assert rR <= 1e-8 and rQ <= 1e-8, (rR, rQ)
    assert ranklog_check(H, F, ref)[1] == 0


# Wide recompressions over the lane shapes of the one-sided Jacobi (lanes per
# column pair x rows per lane: 32 x 1 for widths 17..32, 16 x 3..4 up to 64,
# 8 x 10..16 up to 128): Gaussian HODLR matrices whose ranks put recompressions
# in each class up to 81..96 (k = 3: widths 18..27; 7: up to 63; 8: 24..72;
# 10: 70 and 90), against the oracle decision by decision.  (Rank 11 reaches
# width 99 but an intermediate rank then exceeds the capacity 64.)
@pytest.mark.parametrize("k,seed", [(3, 61), (7, 67), (8, 66), (10, 64)])
def test_wide_recompression_width_classes(H, k, seed):
    n = 2048
    inp = G.gaussian_hodlr(n, 256, k, seed=seed)
    an = oracle_anorm(inp)
    F = H.hodlr_qr(H.hodlr_build(inp, rank_cap=64), EPS, anorm=an)
    ref = O.hqr(inp, EPS, anorm=an)
    widths = sorted({t["w"] for t in ref.counter.truncs})
    print(f"k={k}: recompression widths {widths[0]}..{widths[-1]}, "
          f"{sum(1 for w in widths if w > 16)} distinct widths above 16")
    X = np.random.default_rng(seed).standard_normal((n, 6))
    rR = _rel(H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
    rQ = _rel(H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
    assert rR <= 1e-8 and rQ <= 1e-8, (rR, rQ)
    assert ranklog_check(H, F, ref)[1] == 0


def test_batched_time_runs(H):
    inps = _batch_inputs()[:2]
    As = [H.hodlr_build(inp, rank_cap=32) for inp in inps]
    ms = H.hodlr_qr_batched_time(As, EPS, warmup=1, reps=2)
    assert ms.shape == (2,) and (ms > 0).all()


@pytest.mark.parametrize("rt,chunks", [(4096, 1), (1 << 30, 2), (32768, 4)])
def test_launch_shape_candidates_keep_parity(H, rt, chunks):
    """Every candidate launch shape of the autotuner computes the same
    factorisation (oracle parity and identical rank decisions)."""
    inp = G.gaussian_hodlr(2048, 256, 5, seed=41)
    an = oracle_anorm(inp)
    ref = O.hqr(inp, EPS, anorm=an)
    H.set_tuning(rt, chunks)
    try:
        F = H.hodlr_qr(H.hodlr_build(inp, rank_cap=32), EPS, anorm=an)
    finally:
        H.set_tuning()
    X = np.random.default_rng(41).standard_normal((inp.n, 8))
    rR = _rel(H.hodlr_qr_matmul(F, "R", H.colmajor(X)).cpu().numpy(), O.rmat(ref, X))
    rQ = _rel(H.hodlr_apply_q(F, H.colmajor(X)).cpu().numpy(), O.apply_q(ref, X), np.linalg.norm(X))
    assert rR <= 1e-8 and rQ <= 1e-8, (rR, rQ)
    assert ranklog_check(H, F, ref)[1] == 0
