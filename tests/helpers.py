"""Test-side helpers: dense reconstruction of exported HODLR layouts."""
import numpy as np


def node_range(leaf_off, levels, v):
    depth = v.bit_length() - 1
    span = 1 << (levels - depth)
    first = (v - (1 << depth)) * span
    return int(leaf_off[first]), int(leaf_off[first + span])


def dense_from_export(ex, leaf_off, levels):
    """Assemble the dense matrix from a hodlr_export / hodlr_qr_export dict."""
    n = int(leaf_off[-1])
    A = np.zeros((n, n))
    pos = 0
    for j in range(1 << levels):
        a, b = int(leaf_off[j]), int(leaf_off[j + 1])
        m = b - a
        A[a:b, a:b] = ex["leaves"][pos:pos + m * m].reshape((m, m), order="F")
        pos += m * m
    bi = 0
    for d in range(levels):
        for v in range(1 << d, 2 << d):
            lo, hi = node_range(leaf_off, levels, v)
            mid = node_range(leaf_off, levels, 2 * v)[1]
            for kind in ("up", "lo"):
                rows, cols = (mid - lo, hi - mid) if kind == "up" else (hi - mid, mid - lo)
                k = int(ex["ranks"][bi])
                if k:
                    U = ex["U"][ex["u_off"][bi]:ex["u_off"][bi] + rows * k].reshape((rows, k), order="F")
                    V = ex["V"][ex["v_off"][bi]:ex["v_off"][bi] + cols * k].reshape((cols, k), order="F")
                    if kind == "up":
                        A[lo:mid, mid:hi] = U @ V.T
                    else:
                        A[mid:hi, lo:mid] = U @ V.T
                bi += 1
    return A


def leaf_sizes(H):
    return [int(x) for x in np.diff(H.leaf_off)]
