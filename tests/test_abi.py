"""The C ABI without a GPU: the library builds, loads, exports every symbol
include/hodlr.h declares, and rejects invalid arguments on the host before
touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import hodlr_gen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hodlr.h")
LIB = os.path.join(ROOT, "paper_1809_10585_amd", "libhodlr.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1809_10585_amd import build
        build.build()
    import paper_1809_10585_amd._lib as L
    return L.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hodlr_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    import paper_1809_10585_amd._lib as L
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in hodlr.h but not exported"
    assert set(names) == set(L.EXPORTS)


def test_version_and_error_string(lib):
    assert lib.hodlr_version().startswith(b"hodlr-qr")
    assert isinstance(lib.hodlr_last_error(), bytes)
    assert lib.hodlr_op_count() >= 10
    assert lib.hodlr_op_name(0) == b"tr_qr"


def _build(lib, p, rank_cap=8, levels=None, out=True):
    h = C.c_void_p()
    P = lambda a, t: a.ctypes.data_as(C.POINTER(t))  # noqa: E731
    return lib.hodlr_build(p["n"], p["levels"] if levels is None else levels,
                           P(p["leaf_off"], C.c_int64), P(p["leaves"], C.c_double),
                           P(p["leaf_data_off"], C.c_int64), P(p["U"], C.c_double),
                           P(p["u_off"], C.c_int64), P(p["V"], C.c_double), P(p["v_off"], C.c_int64),
                           P(p["ranks"], C.c_int32), rank_cap, None, C.byref(h) if out else None)


def test_invalid_arguments_are_rejected_on_host(lib):
    p = G.gaussian_hodlr(64, 8, 3, seed=1).pack()
    # rank capacity out of range
    assert _build(lib, p, rank_cap=0) == -1
    assert _build(lib, p, rank_cap=65) == -1
    # rank larger than the capacity
    assert _build(lib, p, rank_cap=2) == -1
    assert b"rank" in lib.hodlr_last_error()
    # NULL output
    assert _build(lib, p, out=False) == -1
    # partition not ending at n
    q = dict(p)
    q["leaf_off"] = p["leaf_off"].copy()
    q["leaf_off"][-1] = 63
    assert _build(lib, q) == -1
    # empty leaf
    q["leaf_off"] = p["leaf_off"].copy()
    q["leaf_off"][1] = 0
    assert _build(lib, q) == -1
    # empty matrix (n = 0, all leaves empty)
    q = dict(p)
    q["n"] = 0
    q["leaf_off"] = np.zeros_like(p["leaf_off"])
    assert _build(lib, q) == -1
    # a leaf above the 512-row maximum
    big = G.gaussian_hodlr(1040, 520, 2, seed=2).pack()
    assert _build(lib, big, levels=1) == -1
    assert b"512" in lib.hodlr_last_error()
    # non-finite entry
    q = dict(p)
    q["leaves"] = p["leaves"].copy()
    q["leaves"][5] = np.nan
    assert _build(lib, q) == -3
    # NULL handles
    h = C.c_void_p()
    assert lib.hodlr_qr(None, 1e-10, 0.0, 0, None, C.byref(h)) == -1
    assert lib.hodlr_apply_q(None, 0, 1, None, 64, None) == -1
    assert lib.hodlr_solve(None, 1, None, 64, None) == -1
    lib.hodlr_free(None)
    lib.hodlr_qr_free(None)
    # batched: no matrices, NULL matrix, NULL output, bad eps
    out = (C.c_void_p * 2)()
    outp = C.cast(out, C.POINTER(C.c_void_p))
    assert lib.hodlr_qr_batched(None, 0, 1e-10, None, 0, None, outp) == -1
    arr = (C.c_void_p * 2)(None, None)
    assert lib.hodlr_qr_batched(C.cast(arr, C.POINTER(C.c_void_p)), 2, 1e-10, None, 0, None, outp) == -1
    assert lib.hodlr_qr_batched(C.cast(arr, C.POINTER(C.c_void_p)), 2, 1e-10, None, 0, None, None) == -1
    ms = (C.c_double * 1)()
    assert lib.hodlr_qr_batched_time(None, 1, 1e-10, None, 0, 0, 1, None, ms) == -1
    # rectangular build: a leaf with fewer rows than columns, rows not summing to m
    lv = np.zeros(64)
    for roff, m in (([0, 3, 8], 8), ([0, 4, 9], 8)):
        ro = np.asarray(roff, dtype=np.int64)
        co = np.asarray([0, 4, 8], dtype=np.int64)
        h = C.c_void_p()
        st = lib.hodlr_build_rect(m, 8, 1, ro.ctypes.data_as(C.POINTER(C.c_int64)),
                                  co.ctypes.data_as(C.POINTER(C.c_int64)), lv.ctypes.data_as(C.POINTER(C.c_double)),
                                  np.zeros(2, dtype=np.int64).ctypes.data_as(C.POINTER(C.c_int64)),
                                  lv.ctypes.data_as(C.POINTER(C.c_double)),
                                  np.zeros(2, dtype=np.int64).ctypes.data_as(C.POINTER(C.c_int64)),
                                  lv.ctypes.data_as(C.POINTER(C.c_double)),
                                  np.zeros(2, dtype=np.int64).ctypes.data_as(C.POINTER(C.c_int64)),
                                  np.zeros(2, dtype=np.int32).ctypes.data_as(C.POINTER(C.c_int32)), 4, None,
                                  C.byref(h))
        assert st == -1 and not h.value
    # refactor: no handles, NULL handle entries
    assert lib.hodlr_qr_refactor(None, None, 1, 0, None) == -1
    assert lib.hodlr_qr_refactor(C.cast(arr, C.POINTER(C.c_void_p)), C.cast(arr, C.POINTER(C.c_void_p)), 2, 0,
                                 None) == -1


def test_header_documents_every_entry_point():
    text = open(HEADER).read()
    for n in ("hodlr_build", "hodlr_qr", "hodlr_apply_q", "hodlr_solve"):
        assert text.count(n) >= 2
    assert "Algorithm hQR" in text and "eq. compactwy" in text
