"""The paper's accuracy example (Sec. 5, Cauchy matrices A_1..A_3 of order
2000, leaf 250): the generator on the CPU, and hQR on the device against the
magnitudes the paper reports (e_orth, e_acc of eq. accuracy at eps = 1e-10)."""
import numpy as np
import pytest

import hodlr_gen as G

# kappa_2(A_i) the paper reports for its draw of the +-2e-2 perturbations
PAPER_KAPPA = {1: 4.8e5, 2: 1.3e8, 3: 2.9e12}


def test_cauchy_example_matrices():
    """Same construction as the paper: conditioning grows from A_1 to A_3 by the
    paper's orders of magnitude (the paper does not give its draw of the +-2e-2
    moves; ours puts kappa within 30x of the paper's values: 6x, 12x, 5x), the
    HODLR approximation has maximal off-diagonal rank about 20 (the paper: 20;
    18 to 20 for our draw) and is within levels * eps |A|_2 of the dense matrix
    (local truncation bound of Sec. 2)."""
    kap = {}
    for i in (1, 2, 3):
        H = G.cauchy_example(i)
        s = np.linalg.svd(H.dense, compute_uv=False)
        kap[i] = s[0] / s[-1]
        assert PAPER_KAPPA[i] / 30 <= kap[i] <= PAPER_KAPPA[i] * 30, (i, kap[i])
        assert 16 <= max(U.shape[1] for U, V in H.blocks.values()) <= 22
        err = np.linalg.norm(H.to_dense() - H.dense, 2)
        assert err <= H.levels * 1e-10 * s[0]
    assert kap[1] < kap[2] < kap[3]


@pytest.mark.gpu
@pytest.mark.parametrize("which", [1, 2, 3])
def test_cauchy_example_accuracy(which):
    """e_orth = |Q^T Q - I|_2 and e_acc = |QR - A|_2 of the device path at
    eps = 1e-10 within 10x of the largest value the paper reports for the three
    matrices (e_orth <= 3.6e-10, e_acc <= 1.1e-8)."""
    import torch
    import paper_1809_10585_amd as H
    assert torch.cuda.is_available()
    inp = G.cauchy_example(which)
    A = H.hodlr_build(inp, rank_cap=64)
    F = H.hodlr_qr(A, 1e-10)
    n = inp.n
    I = np.eye(n)
    Q = H.hodlr_apply_q(F, H.colmajor(I)).cpu().numpy()
    R = H.hodlr_qr_matmul(F, "R", H.colmajor(I)).cpu().numpy()
    e_orth = np.linalg.norm(Q.T @ Q - I, 2)
    e_acc = np.linalg.norm(Q @ R - inp.to_dense(), 2)
    print(f"A{which}: e_orth {e_orth:.2e}  e_acc {e_acc:.2e}")
    assert e_orth <= 3.6e-9 and e_acc <= 1.1e-7
    assert np.allclose(np.tril(R, -1), 0.0)
