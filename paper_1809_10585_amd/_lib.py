"""ctypes binding of libhodlr.so (include/hodlr.h).  Argument marshalling only:
every step of the factorisation runs in the library's HIP kernels.  PyTorch
supplies device memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# HODLR_LIB_PATH selects another build of the library (the host-sanitized one)
LIB_PATH = os.environ.get("HODLR_LIB_PATH") or os.path.join(HERE, "libhodlr.so")

HODLR_OK = 0
STATUS = {0: "HODLR_OK", -1: "HODLR_EINVAL", -2: "HODLR_ENOMEM", -3: "HODLR_ENONFINITE",
          -4: "HODLR_ECAPACITY", -5: "HODLR_EDEVICE", -6: "HODLR_ENOTBUILT"}
HODLR_QR_GRAPH = 1
HODLR_QR_ONE_STREAM = 2
HODLR_QR_BY_SHAPE = 4
HODLR_QR_KEEP = 8

# every symbol include/hodlr.h declares
EXPORTS = [
    "hodlr_set_allocator", "hodlr_build", "hodlr_qr", "hodlr_apply_q", "hodlr_apply_q_noalloc",
    "hodlr_solve", "hodlr_matmul",
    "hodlr_qr_matmul", "hodlr_qr_factor", "hodlr_check", "hodlr_qr_ranklog", "hodlr_plan_check", "hodlr_plan_check_set", "hodlr_qr_refactor", "hodlr_tuning", "hodlr_set_tuning", "hodlr_build_rect", "hodlr_lstsq",
    "hodlr_norm2_est", "hodlr_qr_info", "hodlr_export", "hodlr_qr_export", "hodlr_qr_time",
    "hodlr_qr_profile", "hodlr_op_name", "hodlr_op_count", "hodlr_qr_batched", "hodlr_qr_batched_time",
    "hodlr_free", "hodlr_qr_free", "hodlr_last_error", "hodlr_version",
]
HODLR_CHECK_ESTIMATE = 0x100
HODLR_CHECK_PLANT = 0x200


class HodlrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class QRInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("levels", C.c_int32), ("rank_cap", C.c_int32),
        ("max_rank_y", C.c_int32), ("max_rank_t", C.c_int32), ("max_rank_r", C.c_int32),
        ("anorm", C.c_double), ("tau_a", C.c_double), ("tau_t", C.c_double),
        ("flops", C.c_double), ("n_truncations", C.c_int64), ("n_launches", C.c_int64),
        ("device_bytes", C.c_int64), ("norm_flops", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("mm_rt64_rows", C.c_int32), ("tr_small_chunks", C.c_int32)]


_lib = None

P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I64 = C.c_int64
I32 = C.c_int32
D = C.c_double
PD = C.POINTER(C.c_double)
PI64 = C.POINTER(C.c_int64)
PI32 = C.POINTER(C.c_int32)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def load(path: str = LIB_PATH):
    """Load libhodlr.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HodlrError(-6, f"{path} is missing; run paper_1809_10585_amd/build.py first")
    # PyTorch ships its own HIP runtime: load it first so that the library binds
    # to the same runtime instead of loading a second copy beside it
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    lib = C.CDLL(path)
    sig = {
        "hodlr_set_allocator": (I32, [ALLOC_FN, RELEASE_FN, P]),
        "hodlr_qr_factor": (I32, [P, C.c_char, PP]),
        "hodlr_check": (I32, [P, P]),
        "hodlr_qr_ranklog": (I32, [P, PI32, I64, PI64]),
        "hodlr_plan_check": (I32, [I64, I32, PI64, I32, I32, C.c_uint32, PI64, C.c_char_p, I64]),
        "hodlr_plan_check_set": (I32, [I32, PI64, PI32, PI64, I32, I32, C.c_uint32, PI64, C.c_char_p, I64]),
        "hodlr_qr_refactor": (I32, [PP, PP, I32, C.c_uint32, P]),
        "hodlr_tuning": (I32, [I64, I32, C.POINTER(Tuning)]),
        "hodlr_set_tuning": (I32, [C.POINTER(Tuning)]),
        "hodlr_build": (I32, [I64, I32, PI64, PD, PI64, PD, PI64, PD, PI64, PI32, I32, P, PP]),
        "hodlr_build_rect": (I32, [I64, I64, I32, PI64, PI64, PD, PI64, PD, PI64, PD, PI64, PI32, I32, P, PP]),
        "hodlr_lstsq": (I32, [P, I64, P, I64, P, I64, P]),
        "hodlr_qr": (I32, [P, D, D, C.c_uint32, P, PP]),
        "hodlr_apply_q": (I32, [P, I32, I64, P, I64, P]),
        "hodlr_apply_q_noalloc": (I32, [P, I32, I64, P, I64, P]),
        "hodlr_solve": (I32, [P, I64, P, I64, P]),
        "hodlr_matmul": (I32, [P, I32, I64, P, I64, P, I64, P]),
        "hodlr_qr_matmul": (I32, [P, C.c_char, I32, I64, P, I64, P, I64, P]),
        "hodlr_norm2_est": (I32, [P, I32, P, PD]),
        "hodlr_qr_info": (I32, [P, C.POINTER(QRInfo)]),
        "hodlr_export": (I32, [P, PD, PD, PI64, PD, PI64, PI32]),
        "hodlr_qr_export": (I32, [P, C.c_char, PD, PD, PI64, PD, PI64, PI32]),
        "hodlr_qr_time": (I32, [P, D, D, C.c_uint32, I32, I32, P, PD]),
        "hodlr_qr_profile": (I32, [P, D, D, I32, PD, PI64, PD, P]),
        "hodlr_qr_batched": (I32, [PP, I32, D, PD, C.c_uint32, P, PP]),
        "hodlr_qr_batched_time": (I32, [PP, I32, D, PD, C.c_uint32, I32, I32, P, PD]),
        "hodlr_op_name": (C.c_char_p, [I32]),
        "hodlr_op_count": (I32, []),
        "hodlr_free": (None, [P]),
        "hodlr_qr_free": (None, [P]),
        "hodlr_last_error": (C.c_char_p, []),
        "hodlr_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != HODLR_OK:
        raise HodlrError(status, load().hodlr_last_error().decode())
