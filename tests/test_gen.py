"""Seeded input generators: shapes, determinism, exact ranks (CPU only)."""
import numpy as np
import pytest

import hodlr_gen as G


def test_partition_rules():
    lv, off = G.partition(512, 64)
    assert lv == 3 and list(np.diff(off)) == [64] * 8
    lv, off = G.partition(65536, 256)
    assert lv == 8 and len(off) == 257 and np.all(np.diff(off) == 256)
    lv, off = G.partition(1000, 256)
    assert lv == 2 and off[-1] == 1000 and np.diff(off).max() <= 256
    lv, off = G.partition(100, 256)
    assert lv == 0 and list(off) == [0, 100]
    lv, off = G.partition(1031, 100)
    assert off[-1] == 1031 and np.all(np.diff(off) > 50) and np.all(np.diff(off) <= 100)


def test_config0_shape_and_determinism():
    a, b = G.config(0), G.config(0)
    assert a.n == 512 and a.levels == 3 and len(a.leaves) == 8
    assert all(k == 8 for k in a.ranks().values())
    pa, pb = a.pack(), b.pack()
    for key in pa:
        assert np.array_equal(np.asarray(pa[key]), np.asarray(pb[key]))
    A = a.to_dense()
    # diagonal shift 4I and N(0,1) leaves
    assert abs(np.mean(np.diag(A)) - 4.0) < 0.3


def test_expkernel_blocks_are_exact():
    H = G.expkernel_hodlr(2048, 256, seed=2)
    t = np.sort(np.random.default_rng(2).random(2048))
    A = np.exp(-np.abs(t[:, None] - t[None, :]) / 0.1) + 1e-8 * np.eye(2048)
    np.testing.assert_allclose(H.to_dense(), A, rtol=0, atol=1e-15)
    assert all(k == 1 for k in H.ranks().values())


def test_cauchy_compression_accuracy():
    H = G.cauchy_hodlr(1024, 128, seed=1)
    rng = np.random.default_rng(1)
    x = np.sort(rng.random(1024))
    y = x + 1e-3 * (0.5 + rng.random(1024))
    A = 1.0 / (x[:, None] - y[None, :])
    err = np.linalg.norm(H.to_dense() - A, 2)
    assert err <= H.levels * 1e-10 * np.linalg.norm(A, 2) * 1.5
    ks = list(H.ranks().values())
    assert 5 <= max(ks) <= 60


def test_pack_layout():
    H = G.gaussian_hodlr(100, 16, 3, 7)
    p = H.pack()
    assert p["leaf_off"][-1] == 100
    nblocks = 2 * ((1 << H.levels) - 1)
    assert len(p["ranks"]) == nblocks == len(p["u_off"]) == len(p["v_off"])
    # first block is the root's upper block, column-major
    U, V = H.blocks[(1, "up")]
    k = U.shape[1]
    np.testing.assert_array_equal(p["U"][: U.size].reshape(U.shape, order="F"), U)
    assert p["ranks"][0] == k


def test_perturb_is_roundoff_close():
    H = G.config(0)
    P = G.perturb(H, 3)
    d = np.linalg.norm(P.to_dense() - H.to_dense(), 2) / np.linalg.norm(H.to_dense(), 2)
    assert 0 < d < 1e-14


def test_batched_set_draws():
    s1 = G.batched_set(count=6, seed=3)
    s2 = G.batched_set(count=6, seed=3)
    assert [a.n for a in s1] == [b.n for b in s2]
    assert all(a.n in (1024, 2048, 4096, 8192, 16384) for a in s1)
    assert np.array_equal(s1[0].leaves[0], s2[0].leaves[0])
    for a in s1:
        ks = {U.shape[1] for (U, V) in a.blocks.values()}
        assert len(ks) == 1 and 1 <= ks.pop() <= 4
