"""MI355X (gfx950) HODLR QR decomposition: Python binding of libhodlr.so.

The functions carry the names of the C ABI (include/hodlr.h) and only marshal
arguments: the factorisation, the products, apply-Q and solve all run in the
library's HIP kernels.  Dense operands are torch float64 tensors on the GPU,
laid out column-major: an n x nrhs operand is a tensor of shape (n, nrhs) with
strides (1, ld) -- use `colmajor` to make one.  Nothing here falls back to the
CPU; a missing library raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

import os

from . import _lib
from ._lib import (HODLR_CHECK_ESTIMATE, HODLR_CHECK_PLANT, HODLR_QR_BY_SHAPE, HODLR_QR_GRAPH,
                   HODLR_QR_KEEP, HODLR_QR_ONE_STREAM, HodlrError, QRInfo)

__all__ = [
    "hodlr_build", "hodlr_qr", "hodlr_apply_q", "hodlr_solve", "hodlr_matmul", "hodlr_qr_matmul",
    "hodlr_qr_factor", "hodlr_check", "hodlr_qr_ranklog", "hodlr_plan_check", "hodlr_norm2_est",
    "hodlr_qr_info", "hodlr_export", "hodlr_qr_export", "hodlr_qr_time", "hodlr_qr_profile",
    "hodlr_qr_batched", "hodlr_qr_batched_time", "use_torch_allocator", "HodlrMatrix", "QRFactors",
    "HodlrError", "colmajor", "HODLR_QR_GRAPH", "HODLR_QR_ONE_STREAM", "HODLR_QR_BY_SHAPE", "HODLR_QR_KEEP", "hodlr_qr_refactor", "hodlr_build_rect", "hodlr_lstsq", "tuning", "set_tuning", "HODLR_CHECK_ESTIMATE", "set_allocator",
    "HODLR_CHECK_PLANT", "load",
]

_alloc_hook = None   # the allocator installed in the library: None (not yet), False (hipMalloc), a hook
_torch_hook = None   # PyTorch's caching allocator as a pair of ctypes callbacks (made once)
_keepalive = []      # every callback pair ever installed: handles made under an allocator call
                     # its release function when they are freed, so none may be collected


def set_allocator(alloc, release):
    """Install a pair of ctypes callbacks (_lib.ALLOC_FN, _lib.RELEASE_FN) as the
    library's allocator (hodlr_set_allocator); they are kept alive for the rest
    of the process."""
    global _alloc_hook
    _keepalive.append((alloc, release))
    _lib.check(_lib.load().hodlr_set_allocator(alloc, release, None))
    _alloc_hook = (alloc, release)


def use_torch_allocator(enable: bool = True):
    """Route the library's device memory through PyTorch's caching allocator
    (hodlr_set_allocator): handles and per-call temporaries are then blocks of
    torch's pool on the stream of the call.  Installed by the first call that
    touches the device unless HODLR_TORCH_ALLOCATOR=0; enable=False restores
    hipMalloc / hipMallocAsync."""
    global _alloc_hook, _torch_hook
    lib = _lib.load()
    if not enable:
        _lib.check(lib.hodlr_set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None))
        _alloc_hook = False
        return
    if _torch_hook is not None:
        set_allocator(*_torch_hook)
        return
    import torch

    raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc  # on the current device
    raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete

    def _alloc(size, stream, ctx):
        try:
            return int(raw_alloc(int(size), int(stream or 0)))
        except Exception:
            return None

    def _release(ptr, stream, ctx):
        try:
            raw_delete(int(ptr))
        except Exception:
            pass

    _torch_hook = (_lib.ALLOC_FN(_alloc), _lib.RELEASE_FN(_release))
    set_allocator(*_torch_hook)


def load(path: str = _lib.LIB_PATH):
    return _lib.load(path)


def _device():
    """First call that touches the device: install torch's allocator once."""
    if _alloc_hook is None and os.environ.get("HODLR_TORCH_ALLOCATOR", "1") != "0":
        use_torch_allocator(True)
    return _lib.load()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def colmajor(a, device="cuda"):
    """torch float64 tensor (n, k) with column-major strides (1, n) from an array."""
    import torch
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    t = torch.from_numpy(np.ascontiguousarray(a.T)).to(device)
    return t.t()


def _operand(X, n):
    import torch
    if not isinstance(X, torch.Tensor) or X.dtype != torch.float64 or not X.is_cuda:
        raise HodlrError(-1, "operand must be a float64 CUDA (HIP) tensor")
    if X.dim() == 1:
        X = X[:, None]
    if X.shape[0] != n:
        raise HodlrError(-1, f"operand has {X.shape[0]} rows, expected {n}")
    if X.shape[1] > 1 and X.stride(0) != 1:
        raise HodlrError(-1, "operand must be column-major (strides (1, ld)); see colmajor()")
    ld = X.stride(1) if X.shape[1] > 1 else n
    return X, max(ld, n)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class HodlrMatrix:
    """Owning wrapper of a hodlr_t handle (or a borrowed factor view, which
    keeps its QRFactors alive and is never freed)."""

    def __init__(self, handle, n, levels, rank_cap, owner=None, m=None):
        self.handle, self.n, self.levels, self.rank_cap = handle, n, levels, rank_cap
        self.m = n if m is None else m  # rows (a rectangular matrix has m >= n)
        self.owner = owner

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h and lib is not None and getattr(self, "owner", None) is None:
            lib.hodlr_free(h)
        self.handle = None


class QRFactors:
    """Owning wrapper of a hodlr_qr_t handle (factors Y, T, R)."""

    def __init__(self, handle, A):
        self.handle, self.n, self.levels, self.rank_cap = handle, A.n, A.levels, A.rank_cap
        self.m = getattr(A, "m", A.n)  # rows of A (and of Q, Y)

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h and lib is not None:
            lib.hodlr_qr_free(h)
            self.handle = None


def hodlr_build(H, rank_cap: int = 64, stream=None) -> HodlrMatrix:
    """Copy a HODLR matrix (hodlr_gen.HodlrInput or its .pack() dict) to the GPU."""
    lib = _device()
    p = H.pack() if hasattr(H, "pack") else H
    h = C.c_void_p()
    _lib.check(lib.hodlr_build(
        int(p["n"]), int(p["levels"]), _ptr(p["leaf_off"], C.c_int64), _ptr(p["leaves"], C.c_double),
        _ptr(p["leaf_data_off"], C.c_int64), _ptr(p["U"], C.c_double), _ptr(p["u_off"], C.c_int64),
        _ptr(p["V"], C.c_double), _ptr(p["v_off"], C.c_int64), _ptr(p["ranks"], C.c_int32),
        int(rank_cap), _stream(stream), C.byref(h)))
    return HodlrMatrix(h, int(p["n"]), int(p["levels"]), int(rank_cap))


def hodlr_build_rect(H, rank_cap: int = 64, stream=None) -> HodlrMatrix:
    """Copy a rectangular HODLR matrix (hodlr_gen.RectHodlrInput or its .pack()
    dict) to the GPU."""
    lib = _device()
    p = H.pack() if hasattr(H, "pack") else H
    h = C.c_void_p()
    _lib.check(lib.hodlr_build_rect(
        int(p["m"]), int(p["n"]), int(p["levels"]), _ptr(p["row_off"], C.c_int64), _ptr(p["col_off"], C.c_int64),
        _ptr(p["leaves"], C.c_double), _ptr(p["leaf_data_off"], C.c_int64), _ptr(p["U"], C.c_double),
        _ptr(p["u_off"], C.c_int64), _ptr(p["V"], C.c_double), _ptr(p["v_off"], C.c_int64),
        _ptr(p["ranks"], C.c_int32), int(rank_cap), _stream(stream), C.byref(h)))
    return HodlrMatrix(h, int(p["n"]), int(p["levels"]), int(rank_cap), m=int(p["m"]))


def hodlr_qr(A: HodlrMatrix, eps: float, anorm: float = 0.0, flags: int = 0, stream=None) -> QRFactors:
    lib = _device()
    h = C.c_void_p()
    _lib.check(lib.hodlr_qr(A.handle, float(eps), float(anorm), int(flags), _stream(stream), C.byref(h)))
    return QRFactors(h, A)


def _handles(As):
    arr = (C.c_void_p * len(As))(*[A.handle for A in As])
    return C.cast(arr, C.POINTER(C.c_void_p)), arr


def _anorms(anorm, count):
    if anorm is None:
        return None, None
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(anorm, dtype=np.float64), (count,)))
    return _ptr(a, C.c_double), a


def hodlr_qr_batched(As, eps: float, anorm=None, flags: int = 0, stream=None) -> list:
    """hodlr_qr of every matrix of As in shared launches; anorm: None, a value
    or one value per matrix (<= 0: estimate)."""
    lib = _device()
    hp, keep = _handles(As)
    ap, akeep = _anorms(anorm, len(As))
    out = (C.c_void_p * len(As))()
    _lib.check(lib.hodlr_qr_batched(hp, len(As), float(eps), ap, int(flags), _stream(stream),
                                    C.cast(out, C.POINTER(C.c_void_p))))
    return [QRFactors(C.c_void_p(out[i]), A) for i, A in enumerate(As)]


def hodlr_qr_refactor(Fs, As, flags: int = 0, stream=None) -> None:
    """Factorise As into the kept factorisations Fs (made with HODLR_QR_KEEP),
    replaying their schedules; Fs[i] then holds the factors of As[i]."""
    Fs = list(Fs)
    fp = (C.c_void_p * len(Fs))(*[F.handle for F in Fs])
    hp, keep = _handles(As)
    _lib.check(load().hodlr_qr_refactor(C.cast(fp, C.POINTER(C.c_void_p)), hp, len(Fs), int(flags),
                                        _stream(stream)))


def tuning(n: int, rank_cap: int) -> dict:
    """The launch shapes schedules of order n and rank_cap get (table or override)."""
    t = _lib.Tuning()
    _lib.check(load().hodlr_tuning(int(n), int(rank_cap), C.byref(t)))
    return {"mm_rt64_rows": t.mm_rt64_rows, "tr_small_chunks": t.tr_small_chunks}


def set_tuning(mm_rt64_rows=None, tr_small_chunks=None) -> None:
    """Override the launch-shape table for schedules built from now on; with
    no arguments, go back to the table."""
    if mm_rt64_rows is None and tr_small_chunks is None:
        _lib.check(load().hodlr_set_tuning(None))
        return
    cur = tuning(1 << 16, 16)
    t = _lib.Tuning(int(cur["mm_rt64_rows"] if mm_rt64_rows is None else mm_rt64_rows),
                    int(cur["tr_small_chunks"] if tr_small_chunks is None else tr_small_chunks))
    _lib.check(load().hodlr_set_tuning(C.byref(t)))


def hodlr_qr_batched_time(As, eps: float, anorm=None, flags: int = 0, warmup: int = 1, reps: int = 3,
                          stream=None):
    """Per-run wall times (ms) of factorising the whole batch."""
    hp, keep = _handles(As)
    ap, akeep = _anorms(anorm, len(As))
    ms = np.zeros(reps)
    _lib.check(load().hodlr_qr_batched_time(hp, len(As), float(eps), ap, int(flags), int(warmup), int(reps),
                                            _stream(stream), _ptr(ms, C.c_double)))
    return ms


def hodlr_apply_q(F: QRFactors, X, trans: bool = False, stream=None):
    """X <- Q X (or Q^T X) in place (X: m rows)."""
    X, ld = _operand(X, F.m)
    _lib.check(load().hodlr_apply_q(F.handle, 1 if trans else 0, X.shape[1], C.c_void_p(X.data_ptr()), ld,
                                    _stream(stream)))
    return X


def hodlr_solve(F: QRFactors, B, stream=None):
    """B <- R^{-1} Q^T B in place (solution of A x = b per column)."""
    B, ld = _operand(B, F.n)
    _lib.check(load().hodlr_solve(F.handle, B.shape[1], C.c_void_p(B.data_ptr()), ld, _stream(stream)))
    return B


def hodlr_lstsq(F: QRFactors, B, stream=None):
    """Least-squares solutions argmin |A x - b| per column of B (m rows; B is
    overwritten with Q^T B); returns X (n rows)."""
    B, ldb = _operand(B, F.m)
    X = _new_like(B, F.n)
    _lib.check(load().hodlr_lstsq(F.handle, B.shape[1], C.c_void_p(B.data_ptr()), ldb, C.c_void_p(X.data_ptr()),
                                  F.n, _stream(stream)))
    return X


def _new_like(X, rows=None):
    import torch
    rows = X.shape[0] if rows is None else rows
    return torch.empty((X.shape[1], rows), dtype=torch.float64, device=X.device).t()


def hodlr_matmul(A: HodlrMatrix, X, trans: bool = False, stream=None):
    """Z = A X (X: n rows, Z: m rows) or A^T X (X: m rows, Z: n rows)."""
    xr, zr = (A.m, A.n) if trans else (A.n, A.m)
    X, ldx = _operand(X, xr)
    Z = _new_like(X, zr)
    _lib.check(load().hodlr_matmul(A.handle, 1 if trans else 0, X.shape[1], C.c_void_p(X.data_ptr()), ldx,
                                   C.c_void_p(Z.data_ptr()), zr, _stream(stream)))
    return Z


def hodlr_qr_matmul(F: QRFactors, which: str, X, trans: bool = False, stream=None):
    """Z = op(M) X for M = Y (m x n), T (n x n) or R on its pivot rows (n x n)."""
    rows = F.m if which[:1] == "Y" else F.n
    xr, zr = (rows, F.n) if trans else (F.n, rows)
    X, ldx = _operand(X, xr)
    Z = _new_like(X, zr)
    _lib.check(load().hodlr_qr_matmul(F.handle, which.encode()[:1], 1 if trans else 0, X.shape[1],
                                      C.c_void_p(X.data_ptr()), ldx, C.c_void_p(Z.data_ptr()), zr,
                                      _stream(stream)))
    return Z


def hodlr_qr_factor(F: QRFactors, which: str) -> HodlrMatrix:
    """Borrowed view of the factor 'Y', 'T' or 'R' of F as a HODLR matrix
    (usable with hodlr_matmul and hodlr_export; keeps F alive)."""
    v = C.c_void_p()
    _lib.check(load().hodlr_qr_factor(F.handle, which.encode()[:1], C.byref(v)))
    return HodlrMatrix(v, F.n, F.levels, F.rank_cap, owner=F, m=F.m if which[:1] == "Y" else F.n)


def hodlr_check(F: QRFactors, stream=None):
    """Wait for the stream; raise HodlrError if the device flagged a capacity overflow."""
    _lib.check(load().hodlr_check(F.handle, _stream(stream)))


def hodlr_qr_ranklog(F: QRFactors):
    """Every recompression's decision: int32 array (count, 7) of
    (site, a, b, c, d, w, k); see include/hodlr.h."""
    lib = load()
    cnt = C.c_int64()
    _lib.check(lib.hodlr_qr_ranklog(F.handle, None, 0, C.byref(cnt)))
    out = np.zeros((max(cnt.value, 1), 7), dtype=np.int32)
    _lib.check(lib.hodlr_qr_ranklog(F.handle, _ptr(out, C.c_int32), cnt.value, C.byref(cnt)))
    return out[:cnt.value]


def hodlr_plan_check(H, rank_cap: int, count: int = 1, flags: int = 0) -> dict:
    """Hazard check of the factorisation schedule on H's partition (no device
    needed); H: hodlr_gen.HodlrInput or (n, levels, leaf_off), or a list of
    them: the merged launch sequence of a batch with `count` matrices of each
    partition."""
    shapes = H if isinstance(H, (list, tuple)) and not isinstance(H[0], (int, np.integer)) else [H]
    ns, lv, offs = [], [], []
    for S in shapes:
        if hasattr(S, "leaf_off"):
            n, levels, off = S.n, S.levels, S.leaf_off
        else:
            n, levels, off = S
        ns.append(int(n))
        lv.append(int(levels))
        offs.append(np.asarray(off, dtype=np.int64))
    ns = np.asarray(ns, dtype=np.int64)
    lv = np.asarray(lv, dtype=np.int32)
    off = np.ascontiguousarray(np.concatenate(offs))
    stats = np.zeros(5, dtype=np.int64)
    msg = C.create_string_buffer(512)
    _lib.check(load().hodlr_plan_check_set(len(shapes), _ptr(ns, C.c_int64), _ptr(lv, C.c_int32),
                                           _ptr(off, C.c_int64), int(rank_cap), int(count), int(flags),
                                           _ptr(stats, C.c_int64), msg, 512))
    return {"launches": int(stats[0]), "launches_stream1": int(stats[1]), "pairs": int(stats[2]),
            "conflicts": int(stats[3]), "intra_conflicts": int(stats[4]), "first": msg.value.decode()}


def hodlr_norm2_est(A: HodlrMatrix, iters: int = 50, stream=None) -> float:
    out = C.c_double()
    _lib.check(load().hodlr_norm2_est(A.handle, int(iters), _stream(stream), C.byref(out)))
    return out.value


def hodlr_qr_info(F: QRFactors) -> dict:
    info = QRInfo()
    _lib.check(load().hodlr_qr_info(F.handle, C.byref(info)))
    return info.as_dict()


def _export(call, n, levels, rank_cap, leaf_sizes):
    nb = 2 * ((1 << levels) - 1)
    leaves = np.zeros(int(sum(m * m for m in leaf_sizes)))
    cap_u = n * levels * rank_cap + 1
    U = np.zeros(cap_u)
    V = np.zeros(cap_u)
    u_off = np.zeros(max(nb, 1), dtype=np.int64)
    v_off = np.zeros(max(nb, 1), dtype=np.int64)
    ranks = np.zeros(max(nb, 1), dtype=np.int32)
    _lib.check(call(_ptr(leaves, C.c_double), _ptr(U, C.c_double), _ptr(u_off, C.c_int64),
                    _ptr(V, C.c_double), _ptr(v_off, C.c_int64), _ptr(ranks, C.c_int32)))
    return dict(leaves=leaves, U=U, V=V, u_off=u_off[:nb], v_off=v_off[:nb], ranks=ranks[:nb])


def hodlr_export(A: HodlrMatrix, leaf_sizes) -> dict:
    """Host copy of A in the hodlr_build layout (leaf_sizes: the partition)."""
    return _export(lambda *a: load().hodlr_export(A.handle, *a), A.n, A.levels, A.rank_cap, leaf_sizes)


def hodlr_qr_export(F: QRFactors, which: str, leaf_sizes) -> dict:
    """Host copy of the factor 'Y', 'T' or 'R' in the hodlr_build layout."""
    return _export(lambda *a: load().hodlr_qr_export(F.handle, which.encode()[:1], *a), F.n, F.levels,
                   F.rank_cap, leaf_sizes)


def hodlr_qr_time(A: HodlrMatrix, eps: float, anorm: float = 0.0, flags: int = 0, warmup: int = 1,
                  reps: int = 3, stream=None):
    """Per-run wall times (ms, HIP events on the stream) of `reps` factorisations."""
    ms = np.zeros(reps)
    _lib.check(load().hodlr_qr_time(A.handle, float(eps), float(anorm), int(flags), int(warmup), int(reps),
                                    _stream(stream), _ptr(ms, C.c_double)))
    return ms


def hodlr_qr_profile(A: HodlrMatrix, eps: float, anorm: float = 0.0, stream=None) -> dict:
    """Per-kernel-type totals of one factorisation run launch by launch:
    {name: {"ms": total, "count": launches, "flops": algorithmic flops}}."""
    lib = load()
    nt = lib.hodlr_op_count()
    ms = np.zeros(nt)
    cnt = np.zeros(nt, dtype=np.int64)
    fl = np.zeros(nt)
    _lib.check(lib.hodlr_qr_profile(A.handle, float(eps), float(anorm), nt, _ptr(ms, C.c_double),
                                    _ptr(cnt, C.c_int64), _ptr(fl, C.c_double), _stream(stream)))
    return {lib.hodlr_op_name(i).decode(): {"ms": float(ms[i]), "count": int(cnt[i]), "flops": float(fl[i])}
            for i in range(nt) if cnt[i] > 0}
