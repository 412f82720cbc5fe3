"""Launch-shape table (autotuner output) and its selection, CPU only: the
library's choice for a shape is the first table row whose bounds hold, an
override replaces it until cleared, and a choice changes the schedule."""
import os
import re

import pytest

import hodlr_gen as G

TABLE = os.path.join(os.path.dirname(__file__), "..", "paper_1809_10585_amd", "csrc", "tune_table.h")


@pytest.fixture(scope="module")
def H():
    import paper_1809_10585_amd as H
    try:
        H.load()
    except H.HodlrError:
        from paper_1809_10585_amd import build
        build.build()
    yield H
    H.set_tuning()


def table_rows():
    text = open(TABLE).read()
    body = text.split("kTuneTable[] = {")[1].split("};")[0]
    rows = []
    for m in re.finditer(r"\{([^}]*)\}", body):
        vals = []
        for tok in m.group(1).split(","):
            tok = tok.strip()
            sh = re.fullmatch(r"(\d+)\s*<<\s*(\d+)", tok)
            vals.append(int(sh.group(1)) << int(sh.group(2)) if sh else int(tok))
        rows.append(vals)
    return rows


def expected(rows, n, cap):
    for n_max, cap_max, rt, ch in rows:
        if n <= n_max and cap <= cap_max:
            return {"mm_rt64_rows": rt, "tr_small_chunks": ch}
    n_max, cap_max, rt, ch = rows[-1]
    return {"mm_rt64_rows": rt, "tr_small_chunks": ch}


def test_table_lookup(H):
    rows = table_rows()
    assert rows, "empty table"
    for n_max, cap_max, rt, ch in rows:
        assert rt >= 0 and 1 <= ch <= 4
    for n in (100, 1024, 4096, 4097, 16384, 16385, 65536, 1 << 20):
        for cap in (1, 8, 16, 32, 33, 64):
            assert H.tuning(n, cap) == expected(rows, n, cap), (n, cap)


def test_override_and_reset(H):
    rows = table_rows()
    H.set_tuning(4096, 1)
    try:
        for n, cap in ((512, 64), (65536, 16)):
            assert H.tuning(n, cap) == {"mm_rt64_rows": 4096, "tr_small_chunks": 1}
    finally:
        H.set_tuning()
    assert H.tuning(65536, 16) == expected(rows, 65536, 16)
    for bad in ((4096, 0), (4096, 5), (-1, 2)):
        with pytest.raises(H.HodlrError):
            H.set_tuning(*bad)


def test_choice_changes_the_schedule(H):
    """Recompressions over 257..1024-row factors: one k_tr_small launch with
    four chunks allowed, two launches (k_tr_qr + k_tr_form) with one."""
    levels, off = G.partition(4096, 256)
    counts = {}
    for ch in (1, 4):
        H.set_tuning(32768, ch)
        try:
            r = H.hodlr_plan_check((4096, levels, off), 16, flags=H.HODLR_QR_ONE_STREAM)
        finally:
            H.set_tuning()
        assert r["conflicts"] == 0 and r["intra_conflicts"] == 0
        counts[ch] = r["launches"]
    assert counts[1] > counts[4], counts
