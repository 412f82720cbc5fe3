"""Autotuner of the schedule's launch shapes (run on an MI355X).

For each workload of the grid below every candidate (mm_rt64_rows,
tr_small_chunks) is timed with hodlr_qr_time (median of `reps` runs after one
warm-up) and the fastest is written as one row of csrc/tune_table.h, which the
library compiles in.  Rows are ordered by (rank capacity bound, n); the library
takes the first row whose bounds hold.

    python -m paper_1809_10585_amd.tune [--reps 3] [--dry-run] [--out FILE]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "tune_table.h")

RT_CANDIDATES = (4096, 32768, 1 << 30)
CHUNK_CANDIDATES = (1, 2, 4)

HEADER = """// Launch-shape table of the schedule builder, written by
// paper_1809_10585_amd/tune.py from timings of hodlr_qr on MI355X (exp-kernel
// HODLR matrices at rank capacity 16, Gaussian HODLR matrices at capacity 64;
// leaf 256, eps 1e-10).  The first row with n <= n_max and rank_cap <= cap_max
// applies; shapes beyond the last row take its values.
"""


def grid(G):
    """(row bounds, workload, rank_cap): exp-kernel matrices at rank capacity 16
    for orders up to 65536; Gaussian HODLR matrices at capacity 64 with the
    batched workload's largest ranks for their depth (k = 32 / d: 8 at n = 4096,
    5 at n = 16384)."""
    return [
        ((4096, 32), lambda: G.expkernel_hodlr(4096, 256, 2), 16),
        ((16384, 32), lambda: G.expkernel_hodlr(16384, 256, 2), 16),
        ((1 << 30, 32), lambda: G.expkernel_hodlr(65536, 256, 2), 16),
        ((4096, 1 << 30), lambda: G.gaussian_hodlr(4096, 256, 8, seed=11), 64),
        ((1 << 30, 1 << 30), lambda: G.gaussian_hodlr(16384, 256, 5, seed=12), 64),
    ]


def render(rows) -> str:
    body = "".join(f"    {{{n}, {c}, {rt}, {ch}}},  // {note}\n" for n, c, rt, ch, note in rows)
    return (HEADER + "#pragma once\n#include <cstdint>\n\nnamespace hqh {\nstruct TuneRow {\n"
            "  int64_t n_max;\n  int cap_max;\n  int mm_rt64_rows;\n  int tr_small_chunks;\n};\n"
            "constexpr TuneRow kTuneTable[] = {\n" + body + "};\n}  // namespace hqh\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--dry-run", action="store_true", help="print the table, do not write it")
    ap.add_argument("--out", default=TABLE, help="where to write the table (default: the library's)")
    args = ap.parse_args(argv)
    import numpy as np
    sys.path.insert(0, os.path.dirname(HERE))
    import hodlr_gen as G
    import paper_1809_10585_amd as H
    H.load()
    rows, report = [], []
    for (n_max, cap_max), make, cap in grid(G):
        inp = make()
        A = H.hodlr_build(inp, rank_cap=cap)
        times = {}
        for rt, ch in itertools.product(RT_CANDIDATES, CHUNK_CANDIDATES):
            H.set_tuning(rt, ch)
            ms = H.hodlr_qr_time(A, 1e-10, 0.0, 0, 1, args.reps)
            times[(rt, ch)] = float(np.median(ms))
            print(json.dumps({"n": inp.n, "cap": cap, "mm_rt64_rows": rt, "tr_small_chunks": ch,
                              "ms": round(times[(rt, ch)], 3)}), flush=True)
        H.set_tuning()
        best = min(times, key=times.get)
        base = times[(32768, 4)]
        note = f"{inp.name}: {times[best]:.2f} ms (32768/4: {base:.2f} ms)"
        rows.append((n_max, cap_max, best[0], best[1], note))
        report.append({"workload": inp.name, "cap": cap, "best": best, "ms": times[best], "default_ms": base})
    rows.sort(key=lambda r: (r[1], r[0]))
    text = render(rows)
    print(json.dumps(report))
    if args.dry_run:
        print(text)
    else:
        with open(args.out, "w") as f:
            f.write(text)
        print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
