"""CPU oracle for the HODLR QR decomposition (Kressner & Susnjara, "Fast QR
decomposition of HODLR matrices").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy
implementation that follows the paper step by step.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it; the GPU
library never imports, links or calls it and shares no code with it.

Pins (see tests/test_oracle_*.py): the Householder QR against LAPACK's dgeqrf
and hand-derived fixtures; T_tau against the closed-form truncation error of
eq. (localapproximationerror); the HODLR products against dense products;
hQR at eps = 0 against the dense Householder QR of the assembled matrix
(the compressed block column gives the same reflectors, Sec. 4.1
postprocessing); the backward bounds at eps = 1e-10; special cases.  The
rectangular extension (Sec. 6, rect.py): its dense permuted Householder QR
against LAPACK, the HODLR algorithm at eps = 0 against it, the square case
against hQR, and Table 5's ranks and memory.
"""
from .count import Counter
from .dense import chunked_trunc, house, house_qr, trunc, trunc_flops
from .hodlr import HNode, LowRank, from_input, hmat, hmatT, lowrank_update, norm2_est, to_dense
from .hqr import (QRFactors, accuracy, apply_q, backsolve, dense_factors, hqr, max_ranks, rmat,
                  solve)
from .rect import (RNode, RectQRFactors, perm_house_qr, rect_accuracy, rect_apply_q, rect_dense_factors,
                   rect_lstsq, rect_rmat, rfrom_input, rhmat, rhmatT, rhqr, rmax_ranks, rto_dense)

__all__ = [
    "Counter", "house", "house_qr", "trunc", "trunc_flops", "chunked_trunc", "HNode", "LowRank",
    "from_input", "hmat", "hmatT", "lowrank_update", "norm2_est", "to_dense", "QRFactors",
    "hqr", "apply_q", "rmat", "backsolve", "solve", "dense_factors", "accuracy", "max_ranks",
    "RNode", "RectQRFactors", "rfrom_input", "rto_dense", "rhmat", "rhmatT", "rhqr", "rect_apply_q",
    "rect_rmat", "rect_lstsq", "rect_dense_factors", "rect_accuracy", "perm_house_qr", "rmax_ranks",
]
