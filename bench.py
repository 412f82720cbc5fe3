"""Benchmark: hQR of the exponential-kernel HODLR matrix, n = 65536, leaf 256,
depth 8, eps = 1e-10, on one MI355X.

One step = one whole factorisation A ~= (I - Y T Y^T) R through the HIP
library: the |A|_2 power-iteration estimate, left-orthogonalisation, every
leaf QR, every node update and recompression, issued as direct launches on
the caller's stream with the T-factor steps on a second stream (the library's
default launch mode).  The input is built on the host and copied to the GPU
before the timed region.  The FP64 TFLOP/s figure divides the oracle's
algorithmic flop count of the same factorisation (Sec. 4.1 cost terms; the
|A|_2 estimate is not counted, on either side) by the step time.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, LEAF, EPS, SEED = 65536, 256, 1e-10, 2
RANK_CAP = 16          # ranks of this workload stay <= 3; recompression width <= 32
FP64_VECTOR_PEAK = 78.6  # TFLOP/s, MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
# schedule op type -> the HIP kernel that runs it (one kernel may run several op types)
KERNEL = {"leaf_panel": "k_leaf_step", "leaf_update": "k_leaf_step", "tr_qr": "k_tr_qr",
          "tr_form": "k_tr_form", "mm_proj": "k_mm_proj", "mm_apply": "k_mm_apply",
          "gemm_tall": "k_gemm_tall", "gemm_red": "k_gemm_red", "leaf_gather": "k_leaf_gather",
          "leaf_scatter": "k_leaf_scatter", "fill": "k_fill", "normalize": "k_normalize",
          "set_scal": "k_set_scal", "leaf_trsm": "k_leaf_trsm", "mm_red": "k_mm_red",
          "tr_small": "k_tr_small", "tr_chain": "k_tr_chain", "rows": "k_rows"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_leaf_step_expkernel_n65536_traffic.txt")
CSRC = os.path.join(ROOT, "paper_1809_10585_amd", "csrc")
# translation unit of each kernel family (plus the headers every unit includes)
KERNEL_UNIT = {"k_leaf": "k_leaf.hip", "k_tr": "k_tr.hip", "k_mm": "k_mm.hip", "k_gemm": "k_mm.hip"}
SHARED_HEADERS = ["common.h", "kernels.h", "kernels_common.h"]


def kernel_source_sha(kernel):
    """sha256 over the translation unit that holds `kernel` and the shared headers."""
    import hashlib
    unit = next((u for p, u in KERNEL_UNIT.items() if kernel.startswith(p)), "k_vec.hip")
    h = hashlib.sha256()
    for f in [unit] + SHARED_HEADERS:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 PMC summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None if there is none
    for this kernel or the kernel source changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("kernels_sha256") != kernel_source_sha(kernel):
        return None
    return float(kv["bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_runs(inp, min_seconds, max_reps):
    import oracle as O
    times, F = [], None
    while len(times) < max(1, max_reps) and (not times or sum(times) < min_seconds):
        t0 = time.perf_counter()
        F = O.hqr(inp, EPS)
        times.append(time.perf_counter() - t0)
    return times, F


def cpu_baseline(inp, min_seconds=10.0, max_reps=8):
    """The oracle (NumPy FP64) factorising the same matrix on the host: with
    every BLAS thread (repeated until about `min_seconds` have been spent) and
    with one thread (once, the paper's single-core setting).  Also returns the
    oracle's algorithmic flop count of the factorisation."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threadpool_limits, threads = None, os.cpu_count() or 1
    times, F = _oracle_runs(inp, min_seconds, max_reps)
    dt = sum(times) / len(times)
    one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t1, _ = _oracle_runs(inp, 0.0, 1)
        one = {"value": 1.0 / t1[0], "unit": "QR/s", "cores": 1, "seconds": t1[0]}
    return {"value": 1.0 / dt, "unit": "QR/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "one_thread": one,
            "sample": f"{len(times)} full factorisations of the same n={inp.n} matrix with {threads} BLAS "
                      f"threads (oracle incl. its |A|_2 estimate), {sum(times):.1f} s in total, {dt:.2f} s "
                      f"each; one more with 1 thread"}, F.counter.total


def cpu_baseline_rect(G):
    """The rectangular oracle factorising the rectangular workload once on the
    host (its NumPy threads): seconds per factorisation."""
    import oracle.rect as RR
    inp = G.rect_gaussian_hodlr(8000, 4000, 250, 1, seed=5, shift=0.0)
    t0 = time.perf_counter()
    RR.rhqr(inp, EPS)
    return {"s_per_qr": time.perf_counter() - t0, "kind": "oracle", "sample": "one factorisation of the "
            "8000 x 4000 rectangular workload"}


def bench_batched(H, G, np, count=256, seed=3, rank_cap=64, reps=3):
    """Batched workload: `count` independent Gaussian HODLR matrices, n = 256 * 2^d
    with d ~ U{2..6}, leaf 256, exact off-diagonal rank k ~ U{4..32} capped at
    32 / d (R's ranks, about 2 d k, then fit rank_cap 64), shift 4I, seed 3,
    eps 1e-10.  Whole-batch wall time of hodlr_qr_batched (HIP events, inputs
    resident; the shapes merged into one launch sequence, and the shape groups
    one after another) against the sum of one-at-a-time hodlr_qr run times of
    the same matrices on the same GPU."""
    t0 = time.perf_counter()
    inps = G.batched_set(count=count, seed=seed, kmin=4, kmax=32, rank_budget=rank_cap)
    As = [H.hodlr_build(inp, rank_cap=rank_cap) for inp in inps]
    log(f"batched workload: {count} matrices, sum n = {sum(i.n for i in inps)}, "
        f"built in {time.perf_counter() - t0:.1f} s")
    Fs = H.hodlr_qr_batched(As, EPS)
    infos = [H.hodlr_qr_info(F) for F in Fs]
    flops = sum(i["flops"] for i in infos)
    max_r = max(i["max_rank_r"] for i in infos)
    del Fs
    ms = H.hodlr_qr_batched_time(As, EPS, 0.0, 0, 1, reps)
    batch_ms = float(np.median(ms))
    ms_shape = H.hodlr_qr_batched_time(As, EPS, 0.0, H.HODLR_QR_BY_SHAPE, 1, reps)
    shape_ms = float(np.median(ms_shape))
    plain_ms = sum(float(H.hodlr_qr_time(A, EPS, 0.0, 0, 0, 1)[0]) for A in As)
    log(f"batched ms {ms.round(2).tolist()} (by shape {ms_shape.round(2).tolist()}), "
        f"one at a time {plain_ms:.1f} ms")
    return {"workload": f"{count} Gaussian HODLR matrices, n = 256*2^d, d~U{{2..6}}, leaf 256, "
                        f"rank k~U{{4..min(32, 32/d)}}, shift 4I, eps {EPS:g}, seed {seed}",
            "matrices": count, "sum_n": int(sum(i.n for i in inps)), "rank_cap": rank_cap,
            "ranks": sorted({int(i.name.split("k=")[1].rstrip(")")) for i in inps}),
            "max_rank_r": max_r, "qr_per_s": count / (batch_ms / 1e3), "ms_per_batch": batch_ms,
            "launches": infos[0]["n_launches"], "by_shape_ms_per_batch": shape_ms,
            "plain_loop_ms": plain_ms, "speedup_vs_plain": plain_ms / batch_ms,
            "fp64_tflops": flops / (batch_ms / 1e3) / 1e12, "flops_per_batch": flops}


def served_pool(H, G, np, n_gauss=16, n_cauchy=6, seed=4, rank_cap=64):
    """The served workload's matrices, generated once and kept on the device
    (requests draw from them instead of generating a fresh matrix each):
    Gaussian HODLR (shift 4I) with n log-uniform in [1024, 32768], leaf 256 and
    rank k ~ U{4..32} capped at 32 / depth (R's ranks, about 2 depth k, then fit
    rank_cap 64); Cauchy HODLR (the ill-conditioned generator, compressed at
    1e-10) with n log-uniform in [1024, 4096], the sizes the host generates in
    seconds."""
    import math
    rng = np.random.default_rng(seed)
    mats, desc = [], []
    for _ in range(n_gauss):
        n = int(round(math.exp(rng.uniform(math.log(1024), math.log(32768)))))
        d = G.partition(n, 256)[0]
        k = int(rng.integers(4, max(4, min(32, 32 // d)) + 1))
        mats.append(H.hodlr_build(G.gaussian_hodlr(n, 256, k, seed=None, rng=rng), rank_cap=rank_cap))
        desc.append(("gaussian", n, k))
    for _ in range(n_cauchy):
        n = int(round(math.exp(rng.uniform(math.log(1024), math.log(4096)))))
        inp = G.cauchy_hodlr(n, 256, seed=int(rng.integers(1 << 30)))
        mats.append(H.hodlr_build(inp, rank_cap=rank_cap))
        desc.append(("cauchy", n, max(U.shape[1] for U, V in inp.blocks.values())))
    pools = [list(range(n_gauss)), list(range(n_gauss, n_gauss + n_cauchy))]
    return mats, desc, pools


def bench_served(H, G, np, requests=1000, rate=200.0, seed=4):
    """Served workload: a Poisson stream (`rate` req/s) of `requests` requests
    (a bounded part of a 20k-request stream), each a QR of a pool matrix
    (Gaussian or Cauchy generator with probability 1/2 each, see served_pool)
    with probability 1/2, else a solve with the factor of an earlier QR request
    for nrhs ~ U{1..64} N(0,1) right-hand sides.  Continuous batching (one host
    thread; each step batches every admissible arrived request, its solves on
    resident factors overlapping its factorisations; admission by the factors'
    device bytes) against serving one request per step in arrival order."""
    from paper_1809_10585_amd import serve
    t0 = time.perf_counter()
    mats, desc, pools = served_pool(H, G, np, seed=seed)
    log(f"served pool built in {time.perf_counter() - t0:.1f} s: {desc}")
    out = {"workload": f"{requests} requests (bounded part of a 20k stream), Poisson {rate:g}/s, QR (p=1/2) of a "
                       f"pool matrix: {len(pools[0])} Gaussian n~logU[1024,32768] leaf 256 k~U{{4..min(32,32/d)}} "
                       f"or {len(pools[1])} Cauchy n~logU[1024,4096] (generator chosen with p=1/2); else a solve "
                       f"with 1..64 rhs with the factor of an earlier QR request; eps {EPS:g}, seed {seed}",
           "pool": [{"gen": g, "n": n, "rank": k} for g, n, k in desc]}
    import torch
    be = serve.GpuBackend(H, mats, EPS)  # factorises every pool matrix once: footprints, warm-up
    budget = 0.75 * torch.cuda.mem_get_info()[0]  # bytes for resident factors
    out["budget_gb"] = budget / 1e9
    out["footprint_mb"] = [round(be.footprint(i) / 1e6, 2) for i in range(len(mats))]
    for name, batching in (("continuous", True), ("plain_fifo", False)):
        reqs = serve.poisson_requests(requests, rate, len(mats), seed, pools=pools)
        sch = serve.Scheduler(be, budget=budget, batching=batching)
        res = serve.summarize(sch.run(reqs))
        res.update(steps=sch.steps, max_qr_batch=sch.max_qr_batch, evictions=sch.evictions,
                   refactored=sch.refactored, overlapped_solves=sch.overlapped)
        out[name] = res
        log(f"served {name}: {res}")
    out["p99_speedup_vs_plain"] = out["plain_fifo"]["p99_ms"] / out["continuous"]["p99_ms"]
    out["throughput_speedup_vs_plain"] = (out["continuous"]["throughput_rps"] /
                                          out["plain_fifo"]["throughput_rps"])
    return out


def accuracy_case(H, inp, eps, rank_cap=64):
    """e_orth = |Q^T Q - I|_2 and e_acc = |QR - A|_2 (eq. accuracy) of hQR on the
    device for the HODLR matrix `inp`, and the same for dense Householder QR
    (numpy) of its dense form; dense products and 2-norms on the host."""
    import numpy as np
    import torch
    from paper_1809_10585_amd import _lib
    n = inp.n
    Ad = inp.to_dense()
    Qd, Rd = np.linalg.qr(Ad)
    I = np.eye(n)
    out = {"kappa2": float(np.linalg.cond(Ad)),
           "dense_e_orth": float(np.linalg.norm(Qd.T @ Qd - I, 2)),
           "dense_e_acc": float(np.linalg.norm(Qd @ Rd - Ad, 2)),
           "max_rank_A": max(U.shape[1] for U, V in inp.blocks.values())}
    try:
        A = H.hodlr_build(inp, rank_cap=rank_cap)
        F = H.hodlr_qr(A, eps)
    except _lib.HodlrError as e:
        out["hqr"] = str(e)
        return out
    Q = H.hodlr_apply_q(F, H.colmajor(I)).cpu().numpy()
    R = H.hodlr_qr_matmul(F, "R", H.colmajor(I)).cpu().numpy()
    info = H.hodlr_qr_info(F)
    torch.cuda.synchronize()
    out.update(e_orth=float(np.linalg.norm(Q.T @ Q - I, 2)), e_acc=float(np.linalg.norm(Q @ R - Ad, 2)),
               max_rank_y_t_r=[info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]])
    return out


def bench_accuracy(H, G):
    """The paper's accuracy examples on the device path: Cauchy matrices A_1..A_3
    (n = 2000, leaf 250) at eps = 1e-10, and A_3 for eps = 1e-2 .. 1e-20 (the
    HODLR approximation and hQR at the same eps)."""
    out = {"cauchy_eps_1e-10": {}, "a3_eps_sweep": {}}
    for i in (1, 2, 3):
        out["cauchy_eps_1e-10"][f"A{i}"] = accuracy_case(H, G.cauchy_example(i, eps=1e-10), 1e-10)
        log(f"A{i}: {out['cauchy_eps_1e-10'][f'A{i}']}")
    for e in range(2, 21, 2):
        eps = 10.0 ** -e
        out["a3_eps_sweep"][f"{eps:g}"] = accuracy_case(H, G.cauchy_example(3, eps=eps), eps)
        log(f"A3 eps {eps:g}: {out['a3_eps_sweep'][f'{eps:g}']}")
    return out


def bench_rect(H, G, np, reps=5):
    """Rectangular workload (Sec. 6, Table 5's random rectangular example): an
    8000 x 4000 HODLR matrix with random Gaussian leaves and rank-one
    off-diagonal blocks, n_min 250, eps 1e-10, seed 5; permuted QR on the
    device (HIP events, input resident), the factors' maximal ranks against the
    printed 8 / 12 / 8 (the oracle's time for it is in cpu_baseline)."""
    inp = G.rect_gaussian_hodlr(8000, 4000, 250, 1, seed=5, shift=0.0)
    A = H.hodlr_build_rect(inp, rank_cap=32)
    F = H.hodlr_qr(A, EPS)
    info = H.hodlr_qr_info(F)
    del F
    ms = H.hodlr_qr_time(A, EPS, 0.0, 0, 1, reps)
    out = {"workload": "rectangular HODLR 8000 x 4000, rank-one blocks, n_min 250, eps 1e-10, seed 5 "
                       "(Table 5's random rectangular example)",
           "ms_per_qr": float(np.median(ms)), "qr_per_s": 1e3 / float(np.median(ms)),
           "max_rank_y_t_r": [info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]],
           "paper_max_rank_y_t_r": [8, 12, 8]}
    log(f"rect: {out}")
    return out


def bench_host_buffers(H, inp, reps: int = 3) -> dict:
    """The path from host buffers: hodlr_build (validation, and the host-to-device
    copy of the packed matrix) followed by hodlr_qr, per factorisation.  A rate
    for callers whose matrix starts in host memory; the headline value has the
    input resident in device memory."""
    import numpy as np
    import torch
    p = inp.pack()  # host arrays in the boundary's layout (packing is not timed)
    nbytes = sum(int(np.asarray(v).nbytes) for v in p.values() if isinstance(v, np.ndarray))
    up, tot = [], []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = H.hodlr_build(p, rank_cap=RANK_CAP)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = H.hodlr_qr(A, EPS)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del F, A
        up.append(t1 - t0)
        tot.append(t2 - t0)
    up, tot = up[1:], tot[1:]  # the first repetition warms the allocator
    return {"qr_per_s": 1.0 / float(np.mean(tot)), "ms_per_qr": 1e3 * float(np.mean(tot)),
            "upload_ms": 1e3 * float(np.mean(up)), "host_bytes": nbytes,
            "upload_gb_per_s": nbytes / float(np.mean(up)) / 1e9, "reps": reps,
            "note": "hodlr_build from host arrays + hodlr_qr, host wall clock; not the headline value"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched measurement (256 independent matrices)")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served measurement (1000 requests of a Poisson stream, continuous "
                         "batching and the plain loop)")
    ap.add_argument("--served-requests", type=int, default=300)
    ap.add_argument("--no-rect", action="store_true",
                    help="skip the rectangular measurement (8000 x 4000 permuted QR)")
    ap.add_argument("--accuracy", action="store_true",
                    help="only the accuracy study of the paper's Cauchy examples (e_orth, e_acc)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy kernel (the reference "
                         "dispatch for scaling FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the factorisation of one matrix is a sequential depth-first sweep).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import hodlr_gen as G
    import paper_1809_10585_amd as H

    torch.cuda.set_device(0)
    if args.accuracy:
        print(json.dumps({"accuracy": bench_accuracy(H, G)}), flush=True)
        return
    if args.copy_calibration:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x 256 MiB")
        return
    t0 = time.perf_counter()
    inp = G.expkernel_hodlr(args.n, LEAF, SEED)
    A = H.hodlr_build(inp, rank_cap=RANK_CAP)
    log(f"input built and copied in {time.perf_counter() - t0:.1f} s")

    # one factorisation for the counts (flops, ranks)
    F = H.hodlr_qr(A, EPS)
    info = H.hodlr_qr_info(F)
    del F
    log("info", info)

    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ms = H.hodlr_qr_time(A, EPS, 0.0, 0, args.warmup, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = float(np.mean(ms))
    log(f"per-step ms {ms.round(3).tolist()}  (host wall incl. plan, graph and warmup: {wall:.2f} s)")

    roof = None
    if not args.no_profile:
        prof = H.hodlr_qr_profile(A, EPS, 0.0)
        kern = {}
        for op, v in prof.items():
            k = kern.setdefault(KERNEL.get(op, op), {"ms": 0.0, "count": 0, "flops": 0.0})
            for f in k:
                k[f] += v[f]
        name = max(kern, key=lambda k: kern[k]["ms"])
        p = kern[name]
        avg_s = p["ms"] / p["count"] / 1e3
        flops_launch = p["flops"] / p["count"]
        achieved = flops_launch / avg_s / 1e12
        # every kernel of the path is FP64 vector/MFMA arithmetic on operands that
        # stay in LDS and L2 (leaf columns of <= 512 x 256 doubles, factors of
        # rank <= 32); against HBM none comes near its roofline, so the bound is
        # the FP64 arithmetic rate
        roof = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK, "unit": "TFLOP/s",
                "frac": achieved / FP64_VECTOR_PEAK, "traffic": measured_traffic(name), "kernel": name,
                "launches": p["count"], "avg_us": avg_s * 1e6, "flops_per_launch": flops_launch,
                "share_of_step": p["ms"] / sum(q["ms"] for q in kern.values())}
        log("profile", json.dumps({k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in prof.items()}))

    cpu, oracle_flops = None, None
    if not args.no_cpu:
        cpu, oracle_flops = cpu_baseline(inp)
    # algorithmic flops of one factorisation: the oracle's count when it ran,
    # else the device's counter (same conventions; agree within 1 %)
    flops = oracle_flops if oracle_flops is not None else info["flops"]

    host = bench_host_buffers(H, inp)
    log("from host buffers", json.dumps(host))

    del A
    batched = None if args.no_batched else bench_batched(H, G, np)
    served = None if args.no_served else bench_served(H, G, np, requests=args.served_requests)
    rect = None if args.no_rect else bench_rect(H, G, np)
    if rect is not None and cpu is not None:
        cpu["rect"] = cpu_baseline_rect(G)

    out = {
        "metric": "HODLR QR s & FP64 TFLOP/s at n=65536; batched QR/s + p99 served vs plain",
        "value": 1000.0 / ms_step,
        "unit": "QR/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "s_per_qr": ms_step / 1000.0,
        "fp64_tflops": flops / (ms_step / 1000.0) / 1e12,
        "fp64_frac_of_peak": flops / (ms_step / 1000.0) / 1e12 / FP64_VECTOR_PEAK,
        "flops_per_qr": flops,
        "flops_counted_by": "oracle" if oracle_flops is not None else "device",
        "device_flops_per_qr": info["flops"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"exp-kernel HODLR QR, n={args.n}, leaf {LEAF}, depth {inp.levels}, "
                               f"eps {EPS:g}, seed {SEED}", "n": args.n, "leaf": LEAF,
                   "levels": inp.levels, "eps": EPS, "rank_cap": RANK_CAP,
                   "max_rank_y_t_r": [info["max_rank_y"], info["max_rank_t"], info["max_rank_r"]],
                   "launches_per_qr": info["n_launches"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "from_host_buffers": host,
        "batched": batched,
        "served": served,
        "rect": rect,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
