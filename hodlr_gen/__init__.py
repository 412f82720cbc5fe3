"""Seeded synthetic HODLR inputs shared by the oracle, the tests and the benchmark.

This module only *constructs* inputs: it holds none of the factorisation's
arithmetic (no Householder QR, no recompression, no hQR step).  Both the CPU
oracle and the GPU library consume exactly the arrays produced here.

HODLR format (Kressner & Susnjara, Sec. 2.1, eq. (toplevelpartitioning) and
eq. (integerpart)): a level-l matrix is split recursively into 2x2 blocks; the
off-diagonal blocks are stored as factors A_off = U V^T (eq.
(factoroffdiagonal), written here with V = A_R^T) and the diagonal blocks of
the last level ("leaves") are dense.

Partition rule when n is not n_min * 2^l (the paper only asks for leaves
"nearly equal" to n_min): l = max(0, ceil(log2(n / n_min))) and every node of
order m is split into m1 = floor(m/2) and m2 = m - m1.

Node numbering: heap order, root = 1, children of v are 2v and 2v+1; the
nodes of depth d are 2^d .. 2^(d+1)-1; leaf j is node 2^l + j.  For an
internal node v with children L (rows/cols I_L) and R (I_R):
  block (v, 'up') = A(I_L, I_R) = U V^T,  U: |I_L| x k,  V: |I_R| x k
  block (v, 'lo') = A(I_R, I_L) = U V^T,  U: |I_R| x k,  V: |I_L| x k
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "HodlrInput", "partition", "gaussian_hodlr", "cauchy_hodlr", "expkernel_hodlr",
    "config", "perturb", "CONFIG_EPS", "RectHodlrInput", "rect_partition", "rect_gaussian_hodlr",
]

# truncation tolerance of every workload (the paper's default eps, Sec. 5)
CONFIG_EPS = 1e-10


def partition(n: int, n_min: int) -> tuple[int, np.ndarray]:
    """Return (levels, leaf offsets) for the balanced partition of n."""
    if n <= 0 or n_min <= 0:
        raise ValueError("n and n_min must be positive")
    levels = 0 if n <= n_min else int(math.ceil(math.log2(n / n_min)))
    sizes = [n]
    for _ in range(levels):
        nxt = []
        for m in sizes:
            m1 = m // 2
            nxt += [m1, m - m1]
        sizes = nxt
    if min(sizes) < 1:
        raise ValueError("partition produced an empty leaf")
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return levels, off


@dataclass
class HodlrInput:
    """A HODLR matrix in the library's input layout.

    leaves[j]: dense (n_j x n_j) diagonal block of leaf j.
    blocks[(v, 'up'|'lo')] = (U, V): factors of the off-diagonal blocks of
    internal node v (heap numbering), block = U @ V.T.
    """
    n: int
    levels: int
    leaf_off: np.ndarray
    leaves: list
    blocks: dict = field(default_factory=dict)
    name: str = ""

    # ---- structural helpers (no arithmetic) -------------------------------
    def node_range(self, v: int) -> tuple[int, int]:
        depth = v.bit_length() - 1
        span = 1 << (self.levels - depth)
        first = (v - (1 << depth)) * span
        return int(self.leaf_off[first]), int(self.leaf_off[first + span])

    def internal_nodes(self):
        """Internal nodes in level order (depth 0..levels-1, left to right)."""
        for d in range(self.levels):
            for v in range(1 << d, 1 << (d + 1)):
                yield v

    def ranks(self) -> dict:
        return {key: uv[0].shape[1] for key, uv in self.blocks.items()}

    def to_dense(self) -> np.ndarray:
        """Assemble the full matrix (only for small n; used by tests)."""
        A = np.zeros((self.n, self.n))
        for j, D in enumerate(self.leaves):
            a, b = int(self.leaf_off[j]), int(self.leaf_off[j + 1])
            A[a:b, a:b] = D
        for v in self.internal_nodes():
            lo, hi = self.node_range(v)
            mid = self.node_range(2 * v)[1]
            U, V = self.blocks[(v, "up")]
            A[lo:mid, mid:hi] = U @ V.T
            U, V = self.blocks[(v, "lo")]
            A[mid:hi, lo:mid] = U @ V.T
        return A

    def pack(self) -> dict:
        """Flatten into the C-ABI layout (column-major arrays, block order:
        internal nodes in level order, 'up' then 'lo' for each node)."""
        leaf_data_off = [0]
        for D in self.leaves:
            leaf_data_off.append(leaf_data_off[-1] + D.size)
        leaves = np.concatenate([np.asarray(D, dtype=np.float64).ravel(order="F")
                                 for D in self.leaves]) if self.leaves else np.zeros(0)
        Us, Vs, ranks, u_off, v_off = [], [], [], [0], [0]
        for v in self.internal_nodes():
            for kind in ("up", "lo"):
                U, V = self.blocks[(v, kind)]
                Us.append(np.asarray(U, dtype=np.float64).ravel(order="F"))
                Vs.append(np.asarray(V, dtype=np.float64).ravel(order="F"))
                ranks.append(U.shape[1])
                u_off.append(u_off[-1] + U.size)
                v_off.append(v_off[-1] + V.size)
        cat = (lambda xs: np.concatenate(xs) if xs else np.zeros(0))
        return dict(
            n=self.n, levels=self.levels,
            leaf_off=np.ascontiguousarray(self.leaf_off, dtype=np.int64),
            leaves=np.ascontiguousarray(leaves, dtype=np.float64),
            leaf_data_off=np.asarray(leaf_data_off[:-1], dtype=np.int64),
            U=np.ascontiguousarray(cat(Us), dtype=np.float64),
            V=np.ascontiguousarray(cat(Vs), dtype=np.float64),
            ranks=np.asarray(ranks, dtype=np.int32),
            u_off=np.asarray(u_off[:-1], dtype=np.int64),
            v_off=np.asarray(v_off[:-1], dtype=np.int64),
        )


def _preorder(levels: int):
    """Internal nodes in depth-first pre-order (root, left subtree, right)."""
    out = []

    def rec(v, d):
        if d == levels:
            return
        out.append(v)
        rec(2 * v, d + 1)
        rec(2 * v + 1, d + 1)
    rec(1, 0)
    return out


def gaussian_hodlr(n: int, n_min: int, rank, seed, shift: float = 4.0,
                   rng: np.random.Generator | None = None, name: str = "") -> HodlrInput:
    """Random HODLR matrix in the style of the paper's Example 1 (random dense
    diagonal blocks, random low-rank off-diagonal blocks).

    Draw order: all leaves first (leaf_j = G_j + shift*I, G_j ~ N(0,1)), then the
    off-diagonal blocks in depth-first pre-order; at each node the upper block
    (U then V) and then the lower block (U then V).  U ~ N(0,1)/sqrt(rows),
    V ~ N(0,1)/sqrt(cols).  `rank` is an int or a callable (v, kind, rows,
    cols) -> int; ranks are clipped to min(rows, cols).
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    levels, off = partition(n, n_min)
    leaves = []
    for j in range(len(off) - 1):
        m = int(off[j + 1] - off[j])
        leaves.append(rng.standard_normal((m, m)) + shift * np.eye(m))
    H = HodlrInput(n=n, levels=levels, leaf_off=off, leaves=leaves,
                   name=name or f"gaussian(n={n},leaf={n_min})")
    for v in _preorder(levels):
        lo, hi = H.node_range(v)
        mid = H.node_range(2 * v)[1]
        for kind, rows, cols in (("up", mid - lo, hi - mid), ("lo", hi - mid, mid - lo)):
            k = rank(v, kind, rows, cols) if callable(rank) else int(rank)
            k = max(0, min(k, rows, cols))
            U = rng.standard_normal((rows, k)) / math.sqrt(rows)
            V = rng.standard_normal((cols, k)) / math.sqrt(cols)
            H.blocks[(v, kind)] = (U, V)
    return H


def expkernel_hodlr(n: int, n_min: int = 256, seed=2, ell: float = 0.1,
                    nugget: float = 1e-8) -> HodlrInput:
    """Exponential-kernel matrix A_ij = exp(-|t_i - t_j| / ell) + nugget*delta_ij,
    t = sorted U[0,1] samples.

    With sorted t every off-diagonal block is exactly rank one: for the lower
    block (rows I after columns J) and the split point t_c = t[first row of I],
    A_ij = u_i v_j with u_i = exp(-(t_i - t_c)/ell), v_j = exp(-(t_c - t_j)/ell).
    The factors are stored as U = u/|u|, V = v*|u|; the upper block is the
    transpose of the lower one (A is symmetric).  A dense SVD of the 32768^2
    top-level blocks is unnecessary: this closed form is the exact truncated
    SVD of each block (rank one, singular value |u||v|).
    """
    rng = np.random.default_rng(seed)
    t = np.sort(rng.random(n))
    levels, off = partition(n, n_min)
    leaves = []
    for j in range(len(off) - 1):
        a, b = int(off[j]), int(off[j + 1])
        tt = t[a:b]
        leaves.append(np.exp(-np.abs(tt[:, None] - tt[None, :]) / ell) + nugget * np.eye(b - a))
    H = HodlrInput(n=n, levels=levels, leaf_off=off, leaves=leaves,
                   name=f"expkernel(n={n},leaf={n_min})")
    for v in H.internal_nodes():
        lo, hi = H.node_range(v)
        mid = H.node_range(2 * v)[1]
        tc = t[mid]
        u = np.exp(-(t[mid:hi] - tc) / ell)
        w = np.exp(-(tc - t[lo:mid]) / ell)
        nu = np.linalg.norm(u)
        U = (u / nu)[:, None]
        V = (w * nu)[:, None]
        H.blocks[(v, "lo")] = (U, V)
        H.blocks[(v, "up")] = (V.copy(), U.copy())
    return H


def _cauchy_block(x, y):
    return 1.0 / (x[:, None] - y[None, :])


def cauchy_hodlr(n: int, n_min: int = 256, seed=1, eps: float = 1e-10,
                 sketch: int = 96) -> HodlrInput:
    """Cauchy matrix A_ij = 1/(x_i - y_j), x = sorted U[0,1], y = x + 1e-3*(0.5+U[0,1]),
    compressed to HODLR by truncated SVD of every off-diagonal block, keeping
    the singular values > eps*|A|_2 (U = U_k, V = V_k Sigma_k).

    The SVD of each block is computed from a seeded randomized range finder
    (Gaussian sketch of `sketch` columns, two power passes with
    re-orthonormalisation) followed by the exact SVD of the projected block;
    for these blocks, whose singular values decay geometrically, the sketch
    captures every singular value above the threshold to working accuracy.
    |A|_2 is estimated by 40 power iterations on the dense matrix, assembled
    one row panel at a time.
    """
    rng = np.random.default_rng(seed)
    x = np.sort(rng.random(n))
    y = x + 1e-3 * (0.5 + rng.random(n))
    levels, off = partition(n, n_min)
    # |A|_2 by power iteration on A^T A (dense panels; deterministic start)
    z = np.ones(n) / math.sqrt(n)
    panel = 2048
    nrm = 0.0
    for _ in range(40):
        Az = np.concatenate([_cauchy_block(x[i:i + panel], y) @ z for i in range(0, n, panel)])
        w = np.zeros(n)
        for i in range(0, n, panel):
            w += _cauchy_block(x[i:i + panel], y).T @ Az[i:i + panel]
        nrm = math.sqrt(np.linalg.norm(w))
        z = w / np.linalg.norm(w)
    Az = np.concatenate([_cauchy_block(x[i:i + panel], y) @ z for i in range(0, n, panel)])
    anorm = float(np.linalg.norm(Az))
    del nrm
    thr = eps * anorm
    leaves = []
    for j in range(len(off) - 1):
        a, b = int(off[j]), int(off[j + 1])
        leaves.append(_cauchy_block(x[a:b], y[a:b]))
    H = HodlrInput(n=n, levels=levels, leaf_off=off, leaves=leaves,
                   name=f"cauchy(n={n},leaf={n_min})")
    srng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    for v in H.internal_nodes():
        lo, hi = H.node_range(v)
        mid = H.node_range(2 * v)[1]
        for kind, ri, cj in (("up", (lo, mid), (mid, hi)), ("lo", (mid, hi), (lo, mid))):
            B = _cauchy_block(x[ri[0]:ri[1]], y[cj[0]:cj[1]])
            rows, cols = B.shape
            p = min(sketch, rows, cols)
            Om = srng.standard_normal((cols, p))
            Q, _ = np.linalg.qr(B @ Om)
            for _ in range(2):
                Q, _ = np.linalg.qr(B.T @ Q)
                Q, _ = np.linalg.qr(B @ Q)
            Ub, s, Vt = np.linalg.svd(Q.T @ B, full_matrices=False)
            k = int(np.sum(s > thr))
            U = Q @ Ub[:, :k]
            V = Vt[:k].T * s[:k]
            H.blocks[(v, kind)] = (np.ascontiguousarray(U), np.ascontiguousarray(V))
    H.anorm_generator = anorm
    return H


# Intervals of Sec. 5, Example "Accuracy for Cauchy matrices": x from I_x,
# y from I_y(i) for the matrices A_1, A_2, A_3 (closer intervals: worse conditioned).
CAUCHY_EXAMPLE_IX = (-1.25, 998.25)
CAUCHY_EXAMPLE_IY = {1: (-0.7, 998.9), 2: (-0.45, 999.15), 3: (-0.15, 999.45)}


def cauchy_example(which: int, n: int = 2000, n_min: int = 250, eps: float = 1e-10,
                   seed: int = 11) -> HodlrInput:
    """The Cauchy matrices A_1..A_3 of the paper's accuracy example (Sec. 5):
    A_ij = 1/(x_i - y_j) with x, y n equally spaced points of I_x, I_y(which),
    each moved by +-2e-2 (sign drawn uniformly, x's signs first, then y's),
    compressed to HODLR (leaf n_min) by the truncated SVD of every off-diagonal
    block, keeping singular values > eps |A|_2 (U = U_k, V = V_k Sigma_k).  n is
    small enough for dense SVDs; `dense` holds the uncompressed matrix."""
    rng = np.random.default_rng(seed)
    x = np.linspace(*CAUCHY_EXAMPLE_IX, n) + 2e-2 * rng.choice([-1.0, 1.0], n)
    y = np.linspace(*CAUCHY_EXAMPLE_IY[which], n) + 2e-2 * rng.choice([-1.0, 1.0], n)
    A = _cauchy_block(x, y)
    anorm = float(np.linalg.norm(A, 2))
    thr = eps * anorm
    levels, off = partition(n, n_min)
    leaves = [A[int(off[j]):int(off[j + 1]), int(off[j]):int(off[j + 1])].copy() for j in range(len(off) - 1)]
    H = HodlrInput(n=n, levels=levels, leaf_off=off, leaves=leaves,
                   name=f"cauchy_example(A{which},n={n},leaf={n_min},eps={eps:g})")
    for v in H.internal_nodes():
        lo, hi = H.node_range(v)
        mid = H.node_range(2 * v)[1]
        for kind, ri, cj in (("up", (lo, mid), (mid, hi)), ("lo", (mid, hi), (lo, mid))):
            Ub, sv, Vt = np.linalg.svd(A[ri[0]:ri[1], cj[0]:cj[1]], full_matrices=False)
            k = int(np.sum(sv > thr))
            H.blocks[(v, kind)] = (np.ascontiguousarray(Ub[:, :k]), np.ascontiguousarray(Vt[:k].T * sv[:k]))
    H.anorm_generator = anorm
    H.dense = A
    return H


def batched_set(count: int = 256, seed: int = 3, dmin: int = 2, dmax: int = 6, kmin: int = 1,
                kmax: int = 4, n_min: int = 256, rank_budget: int | None = None) -> list:
    """The batch of independent matrices of the batched workload: for each of
    `count` matrices in turn, d ~ U{dmin..dmax} and k ~ U{kmin..kmax'} are
    drawn, then a Gaussian HODLR matrix (gaussian_hodlr, shift 4I) of order
    n_min * 2^d with exact off-diagonal rank k, all from one stream seeded
    with `seed`.  kmax' = kmax, or with a rank budget
    max(kmin, min(kmax, rank_budget // (2 d))): the top block of R has rank
    about 2 d k for these matrices, so the budget bounds R's ranks."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = int(rng.integers(dmin, dmax + 1))
        top = kmax if rank_budget is None else max(kmin, min(kmax, rank_budget // (2 * d)))
        k = int(rng.integers(kmin, top + 1))
        out.append(gaussian_hodlr(n_min * 2 ** d, n_min, k, seed=None, rng=rng,
                                  name=f"batched(d={d},k={k})"))
    return out


def config(i: int, **kw) -> HodlrInput:
    """The benchmark workloads, seeded as documented:
    0: Gaussian, n=512, leaf 64, rank 8, shift 4I, seed 0.
    1: Cauchy, n=8192, leaf 256, seed 1 (compressed at 1e-10 |A|_2).
    2: exponential kernel, n=65536, leaf 256, seed 2 (rank-one blocks).
    `n` may be overridden to get a smaller instance of the same family."""
    if i == 0:
        return gaussian_hodlr(kw.get("n", 512), kw.get("leaf", 64), kw.get("rank", 8),
                              seed=kw.get("seed", 0), name="config0")
    if i == 1:
        return cauchy_hodlr(kw.get("n", 8192), kw.get("leaf", 256), seed=kw.get("seed", 1))
    if i == 2:
        return expkernel_hodlr(kw.get("n", 65536), kw.get("leaf", 256), seed=kw.get("seed", 2))
    raise ValueError(f"unknown config {i}")


def perturb(H: HodlrInput, seed: int, rel: float = 2.0 ** -53) -> HodlrInput:
    """Copy of H with every stored entry x replaced by x*(1 + rel*xi), xi ~ N(0,1):
    a HODLR matrix at roundoff distance from H, used to measure the noise floor
    of forward comparisons on ill-conditioned inputs."""
    rng = np.random.default_rng(seed)
    leaves = [D * (1.0 + rel * rng.standard_normal(D.shape)) for D in H.leaves]
    G = HodlrInput(n=H.n, levels=H.levels, leaf_off=H.leaf_off.copy(), leaves=leaves,
                   name=H.name + "+perturbed")
    for key in sorted(H.blocks):
        U, V = H.blocks[key]
        G.blocks[key] = (U * (1.0 + rel * rng.standard_normal(U.shape)),
                         V * (1.0 + rel * rng.standard_normal(V.shape)))
    return G


# ---------------------------------------------------------------- rectangular
def rect_partition(m: int, n: int, n_min: int) -> tuple[int, np.ndarray, np.ndarray]:
    """(levels, row offsets, column offsets) of an m x n rectangular HODLR
    matrix (Sec. 6, two integer partitions with m_j >= n_j): the columns are
    split as partition(n, n_min) and row boundary j is floor(m c_j / n) for
    column boundary c_j, so m_j >= n_j for every leaf when m >= n."""
    if m < n:
        raise ValueError("a rectangular HODLR matrix here has m >= n")
    levels, col_off = partition(n, n_min)
    row_off = (np.int64(m) * col_off) // np.int64(n)
    return levels, row_off.astype(np.int64), col_off


@dataclass
class RectHodlrInput:
    """A rectangular HODLR matrix (Sec. 6): leaf j is the dense m_j x n_j
    diagonal block (rows row_off[j]:row_off[j+1], columns col_off[j]:...);
    blocks[(v, 'up')] = (U, V) is the block rows(2v) x cols(2v+1) = U V^T and
    blocks[(v, 'lo')] the block rows(2v+1) x cols(2v)."""
    m: int
    n: int
    levels: int
    row_off: np.ndarray
    col_off: np.ndarray
    leaves: list
    blocks: dict = field(default_factory=dict)
    name: str = ""

    def _range(self, off, v):
        depth = v.bit_length() - 1
        span = 1 << (self.levels - depth)
        first = (v - (1 << depth)) * span
        return int(off[first]), int(off[first + span])

    def node_rows(self, v: int) -> tuple[int, int]:
        return self._range(self.row_off, v)

    def node_cols(self, v: int) -> tuple[int, int]:
        return self._range(self.col_off, v)

    def internal_nodes(self):
        for d in range(self.levels):
            for v in range(1 << d, 1 << (d + 1)):
                yield v

    def pivot_rows(self) -> np.ndarray:
        """Row index that column c is reduced onto: the first n_j rows of each
        leaf's row block, in column order (structure only)."""
        out = []
        for j in range(len(self.col_off) - 1):
            nj = int(self.col_off[j + 1] - self.col_off[j])
            out += list(range(int(self.row_off[j]), int(self.row_off[j]) + nj))
        return np.asarray(out, dtype=np.int64)

    def pack(self) -> dict:
        """Flatten into the C-ABI layout of hodlr_build_rect (column-major; leaf j
        m_j x n_j; blocks in level order, 'up' then 'lo' for each node)."""
        leaf_data_off = [0]
        for D in self.leaves:
            leaf_data_off.append(leaf_data_off[-1] + D.size)
        leaves = np.concatenate([np.asarray(D, dtype=np.float64).ravel(order="F") for D in self.leaves])
        Us, Vs, ranks, u_off, v_off = [], [], [], [0], [0]
        for v in self.internal_nodes():
            for kind in ("up", "lo"):
                U, V = self.blocks[(v, kind)]
                Us.append(np.asarray(U, dtype=np.float64).ravel(order="F"))
                Vs.append(np.asarray(V, dtype=np.float64).ravel(order="F"))
                ranks.append(U.shape[1])
                u_off.append(u_off[-1] + U.size)
                v_off.append(v_off[-1] + V.size)
        cat = (lambda xs: np.concatenate(xs) if xs else np.zeros(0))
        return dict(
            m=self.m, n=self.n, levels=self.levels,
            row_off=np.ascontiguousarray(self.row_off, dtype=np.int64),
            col_off=np.ascontiguousarray(self.col_off, dtype=np.int64),
            leaves=np.ascontiguousarray(leaves, dtype=np.float64),
            leaf_data_off=np.asarray(leaf_data_off[:-1], dtype=np.int64),
            U=np.ascontiguousarray(cat(Us), dtype=np.float64),
            V=np.ascontiguousarray(cat(Vs), dtype=np.float64),
            ranks=np.asarray(ranks, dtype=np.int32),
            u_off=np.asarray(u_off[:-1], dtype=np.int64),
            v_off=np.asarray(v_off[:-1], dtype=np.int64),
        )

    def to_dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        for j, D in enumerate(self.leaves):
            A[self.row_off[j]:self.row_off[j + 1], self.col_off[j]:self.col_off[j + 1]] = D
        for v in self.internal_nodes():
            r1, c1, r2, c2 = self.node_rows(2 * v), self.node_cols(2 * v), self.node_rows(2 * v + 1), \
                self.node_cols(2 * v + 1)
            U, V = self.blocks[(v, "up")]
            A[r1[0]:r1[1], c2[0]:c2[1]] = U @ V.T
            U, V = self.blocks[(v, "lo")]
            A[r2[0]:r2[1], c1[0]:c1[1]] = U @ V.T
        return A


def rect_gaussian_hodlr(m: int, n: int, n_min: int, rank: int, seed=0, shift: float = 4.0,
                        row_off=None, rng=None, name: str | None = None) -> RectHodlrInput:
    """Rectangular Gaussian HODLR matrix: leaves i.i.d. N(0,1) with shift*I added
    to their top n_j x n_j part, off-diagonal blocks U V^T of exact rank `rank`
    with U, V i.i.d. N(0,1)/sqrt(rows), N(0,1)/sqrt(cols).  row_off overrides
    the row partition (it must keep m_j >= n_j)."""
    levels, roff, coff = rect_partition(m, n, n_min)
    if row_off is not None:
        roff = np.asarray(row_off, dtype=np.int64)
        if roff[0] != 0 or roff[-1] != m or len(roff) != len(coff) or np.any(np.diff(roff) < np.diff(coff)):
            raise ValueError("row partition must run from 0 to m with m_j >= n_j")
    rng = rng if rng is not None else np.random.default_rng(seed)
    leaves = []
    for j in range(len(coff) - 1):
        mj, nj = int(roff[j + 1] - roff[j]), int(coff[j + 1] - coff[j])
        D = rng.standard_normal((mj, nj))
        D[:nj, :nj] += shift * np.eye(nj)
        leaves.append(D)
    H = RectHodlrInput(m=m, n=n, levels=levels, row_off=roff, col_off=coff, leaves=leaves,
                       name=name or f"rect_gaussian(m={m},n={n},leaf={n_min},k={rank})")
    for v in H.internal_nodes():
        for kind, rv, cv in (("up", 2 * v, 2 * v + 1), ("lo", 2 * v + 1, 2 * v)):
            r, c = H.node_rows(rv), H.node_cols(cv)
            mr, nc = r[1] - r[0], c[1] - c[0]
            H.blocks[(v, kind)] = (rng.standard_normal((mr, rank)) / math.sqrt(mr),
                                   rng.standard_normal((nc, rank)) / math.sqrt(nc))
    return H
