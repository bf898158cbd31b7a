"""Benchmark of the CSR SpMV / conjugate-gradient hot path on one MI355X.

One step = one Jacobi-preconditioned CG solve (FP64) of the 3-D 7-point
Poisson matrix on a 128^3 grid to a 1e-10 relative residual: the SpMV with
p.q folded in, the reductions, the fused vector updates, the Jacobi step, the
device-side stop test and the final FP64 residual check.  Inputs (matrix, b,
x0 = 0) are resident in HBM before the timed region.

Prints ONE JSON line.  `value` is the hot path's algorithmic HBM throughput
(passes x algorithmic bytes per pass / wall time of the solves); the roofline
object reports the dominant kernel (SpMV + p.q) from HIP events recorded
around each of its launches on the solve's stream; `cpu_baseline` times the
FP64 oracle on the host cores on a bounded sample of the same workload;
`forms` gives the time to tolerance of the mixed-precision and learned forms
beside plain FP64 Jacobi-PCG on their own matrices.

`workloads` adds plain CG on the 2-D Poisson 64^2 system and the cold
standalone SpMV of the other matrices and precisions; `copy_gbs` is the
measured device-copy ceiling.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--cpu-seconds 15] [--no-forms]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "SpMV GB/s (% HBM peak); CG time to 1e-10 rel. residual, learned vs plain"


def spmv_bytes(n, nnz, sv=8, sx=8):
    """Algorithmic bytes of y = A x: values + int32 columns + int32 row pointers,
    x read once, y written once."""
    return nnz * (sv + 4) + 4 * (n + 1) + n * sx + n * sx


def jpcg_pass_bytes(n, nnz):
    """FP64 Jacobi-PCG pass: SpMV + 80 n (r, q, dinv read and r written by the
    residual update; r, dinv, p, x read and p, x written by the direction
    update, which also does x += alpha p)."""
    return spmv_bytes(n, nnz) + 80 * n


# sources of the CG pass kernels (k_cg_q and the kernels around it)
CG_SOURCES = ("internal.h", "cg.hip")


def kernel_source_hash(files=None):
    """Hash of the HIP sources (all of them, or the named files of csrc/) with
    comments and blank space removed, so that a comment edit does not retire
    the counter summaries taken on the same code."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1211_1581_amd", "csrc")
    paths = sorted(glob.glob(os.path.join(csrc, "*"))) if files is None else \
        [os.path.join(csrc, f) for f in files]
    for f in paths:
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash(CG_SOURCES):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(A, b, seconds):
    """The oracle (plain FP64 C, OpenMP rows) on a bounded sample: as many
    Jacobi-PCG passes of the same system as fit in about `seconds`."""
    import oracle
    n, nnz = A.n_rows, A.nnz
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    # calibrate with a short run, then size the sample
    t = time.perf_counter()
    r = oracle.pcg(A, b, tol=0.0, maxit=3, precond="jacobi")
    dt = time.perf_counter() - t
    per = dt / max(r["iters"], 1)
    passes = int(max(5, min(425, seconds / max(per, 1e-6))))
    t = time.perf_counter()
    r = oracle.pcg(A, b, tol=0.0, maxit=passes, precond="jacobi")
    dt = time.perf_counter() - t
    gbs = r["iters"] * jpcg_pass_bytes(n, nnz) / dt / 1e9
    out = {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"{r['iters']} Jacobi-PCG passes (with set-up) of the 128^3 Poisson "
                     f"system in {dt:.1f} s; a full solve takes 425 passes",
           "est_time_to_tol_s": round(dt / r["iters"] * 425, 2)}
    out["spmv_gbs"] = cpu_spmv_rates(A)
    return out


def cpu_spmv_rates(A):
    """Oracle SpMV rate (median of 5) on all threads and on one thread, for the
    128^3 Poisson matrix and the lognormal irregular matrix (FP64)."""
    import numpy as np

    import oracle
    from paper_1211_1581_amd import inputs as I
    L, xl = I.lognormal_irregular()
    res = {}
    full = oracle.set_threads(0)
    for name, M, x in (("poisson128_f64", A, np.linspace(-1.0, 1.0, A.n_cols)),
                       ("lognormal_f64", L, xl)):
        row = {}
        for label, th in (("all_threads", full), ("one_thread", 1)):
            oracle.set_threads(th)
            ts = []
            for _ in range(5):
                t = time.perf_counter()
                oracle.spmv(M, x)
                ts.append(time.perf_counter() - t)
            row[label] = round(spmv_bytes(M.n_rows, M.nnz) / sorted(ts)[2] / 1e9, 2)
        res[name] = row
    oracle.set_threads(full)
    res["threads"] = full
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib", action="store_true",
                    help="first copy 256 MiB device-to-device once (reference dispatch for "
                         "hardware byte counters)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision (160^3) and learned (128^3) time-to-tolerance")
    ap.add_argument("--tables", action="store_true",
                    help="run the paper's own input tables instead (SpMV over the Table 1 "
                         "matrices, plain CG over the Table 2 banded systems) beside the "
                         "oracle on the host, and print that record")
    ap.add_argument("--form", choices=("mixed", "learned"), default=None,
                    help="run only this solver form beside FP64 Jacobi-PCG and print its "
                         "record (for kernel traces of one workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(how it would shard is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1211_1581_amd import inputs as I
    from paper_1211_1581_amd import spcg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.form:
        print(json.dumps(forms(args, only=args.form)), flush=True)
        return
    if args.tables:
        print(json.dumps(tables()), flush=True)
        return
    if args.calib:
        src = torch.ones(2 ** 25, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    A = I.poisson3d(128)
    xs = I.uniform_vector(A.n_rows, 1)
    b = I.rhs_from_solution(A, xs)
    n, nnz = A.n_rows, A.nnz

    torch.cuda.synchronize()
    t = time.perf_counter()
    M = spcg.CsrMatrix.from_host(A, device=dev)
    torch.cuda.synchronize()
    analysis_ms = (time.perf_counter() - t) * 1e3  # includes the host->device copy
    # the row analysis alone, on arrays already in HBM (validation, partition, long rows)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        H = spcg.CsrMatrix(M.row_ptr, M.col, M.vals)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
        H.close()
    analysis_device_ms = 1e3 * min(ts)

    bt = torch.as_tensor(b, device=dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    # HIP events bracket the SpMV of every 8th pass inside the timed solves
    # (a bracketed launch costs a few microseconds, so sampling keeps the
    # timed region within ~1 % of an uninstrumented solve)
    opts = spcg.cg_opts(tol=1e-10, maxit=20000, precond="jacobi", timing=8)
    work = spcg.CgWorkspace(M, opts)

    def step():
        x.zero_()
        return spcg.cg_solve(M, bt, x, opts=opts, work=work, want_hist=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    iters = outs[-1]["iters"]
    assert all(o["status"] == 0 for o in outs), [o["status"] for o in outs]
    passes = sum(o["iters"] for o in outs)
    value = passes * jpcg_pass_bytes(n, nnz) / (t1 - t0) / 1e9

    spmv_ms = sum(o["spmv_ms"] for o in outs)
    spmv_calls = sum(o["spmv_calls"] for o in outs)
    b_spmv = spmv_bytes(n, nnz)
    avg_us = spmv_ms * 1e3 / max(spmv_calls, 1)
    achieved = b_spmv / (avg_us * 1e-6) / 1e9
    traffic = measured_traffic("k_cg_q", "poisson128")
    matrix_mb = (nnz * 12 + 4 * (n + 1)) / 1e6

    # standalone SpMV, cold: rotate over 3 copies (651 MB > the 256 MB MALL)
    copies = [M] + [spcg.CsrMatrix.from_host(A, device=dev) for _ in range(2)]
    xt = torch.as_tensor(xs, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    for i in range(6):
        spcg.spmv_csr(copies[i % 3], xt, y)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(30)]
    for i, (e0, e1) in enumerate(evs):
        e0.record()
        spcg.spmv_csr(copies[i % 3], xt, y)
        e1.record()
    torch.cuda.synchronize()
    cold_us = float(np.median([e0.elapsed_time(e1) * 1e3 for e0, e1 in evs]))
    del copies

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D 7-point Poisson 128^3 (n=2097152, nnz=14581760, int32 CSR), "
                               "b = A x*, x* ~ U[-1,1] seed 1, x0 = 0, FP64 Jacobi-PCG to 1e-10",
                   "parallelism": "single GPU"},
        "time_to_tol_ms": round(ms_per_step, 3),
        "iters": iters,
        "true_relres": outs[-1]["true_relres"],
        "analysis_ms": round(analysis_ms, 2),
        "analysis_device_ms": round(analysis_device_ms, 3),
        "spmv_in_cg_gbs": round(achieved, 1),
        "spmv_in_cg_pct_peak": round(100 * achieved / PEAK_HBM_GBS, 1),
        "spmv_cold_gbs": round(b_spmv / (cold_us * 1e-6) / 1e9, 1),
        "spmv_cold_us": round(cold_us, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic, "kernel": "k_cg_q (SpMV q = A p with p.q partials)",
                     "bytes_per_launch": b_spmv, "avg_launch_us": round(avg_us, 2),
                     "launches": spmv_calls,
                     "note": ("A's streams (%.1f MB) fit the cache-allocating limit (%d MiB), so A stays in "
                              "the 256 MB MALL across passes; the cold HBM rate is spmv_cold_gbs"
                              % (matrix_mb, spcg.keep_bytes() >> 20)) if matrix_mb * 1e6 <= spcg.keep_bytes()
                             else "A streams from HBM with non-temporal loads"},
    }
    line["copy_gbs"] = copy_rate()
    line["read_gbs"] = read_rate()
    if not args.no_forms:
        line["workloads"] = workloads(A, xs)
        line["forms"] = forms(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(A, b, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def read_rate():
    """Streaming read of 1 GiB of FP64 (torch's sum; bytes read / time, median
    of 10): the read ceiling for kernels that, like SpMV, mostly read."""
    import numpy as np
    import torch
    a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    for _ in range(3):
        torch.sum(a, dim=0, out=out)
    ts = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.sum(a, dim=0, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a
    return round(2 ** 30 / float(np.median(ts)) / 1e9, 1)


def copy_rate():
    """Device-to-device copy of 512 MiB (read + write bytes / time, median of
    10): the streaming ceiling the SpMV rates can be read against."""
    import numpy as np
    import torch
    src = torch.ones(2 ** 26, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ts = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return round(2 * 2 ** 29 / float(np.median(ts)) / 1e9, 1)


def cold_spmv(A, x, dtype, reps=30):
    """Median duration of spmv_csr rotating over enough device copies of A
    that their total exceeds 600 MB (more than twice the 256 MB last-level
    cache), so every launch streams the matrix from HBM."""
    import numpy as np
    import torch

    from paper_1211_1581_amd import spcg
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sv = 8 if dtype == "f64" else 4
    b = spmv_bytes(A.n_rows, A.nnz, sv=sv, sx=sv)
    ncopy = max(3, -(-600_000_000 // b))
    copies = [spcg.CsrMatrix.from_host(A, dtype=tdt) for _ in range(ncopy)]
    xt = torch.as_tensor(x).to(tdt).cuda()
    y = torch.empty(A.n_rows, dtype=tdt, device="cuda")
    for i in range(2 * ncopy):
        spcg.spmv_csr(copies[i % ncopy], xt, y)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for i, (e0, e1) in enumerate(evs):
        e0.record()
        spcg.spmv_csr(copies[i % ncopy], xt, y)
        e1.record()
    torch.cuda.synchronize()
    us = float(np.median([e0.elapsed_time(e1) * 1e3 for e0, e1 in evs]))
    del copies
    gbs = b / (us * 1e-6) / 1e9
    return {"us": round(us, 2), "gbs": round(gbs, 1), "pct_peak": round(100 * gbs / PEAK_HBM_GBS, 1),
            "bytes": b, "copies": ncopy}


def workloads(A128, x128):
    """The other measured configurations: plain CG on the 2-D Poisson 64^2
    system (cache-resident, latency-bound: time and per-pass cost, no
    bandwidth figure), and the cold standalone SpMV of the 128^3 Poisson
    matrix in FP32 and of the lognormal irregular matrix in FP64 and FP32."""
    import torch

    from paper_1211_1581_amd import inputs as I
    from paper_1211_1581_amd import spcg
    out = {}
    P = I.poisson2d(64)
    b = I.rhs_from_solution(P, I.uniform_vector(P.n_rows, 0))
    M = spcg.CsrMatrix.from_host(P)
    bt = torch.as_tensor(b, device="cuda")
    opts = spcg.cg_opts(tol=1e-10, maxit=2000, precond="none")
    r = _time_solve(M, bt, opts, spcg.CgWorkspace(M, opts), reps=10)
    out["cg_poisson2d_64"] = {"workload": "2-D 5-point Poisson 64^2, plain CG to 1e-10 (one "
                                          "workgroup holds the whole loop)",
                              "ms": r["ms"], "iters": r["iters"],
                              "us_per_pass": round(1e3 * r["ms"] / max(r["iters"], 1), 2),
                              "true_relres": r["true_relres"], "status": r["status"]}
    del M, bt
    # the single-reduction (Chronopoulos-Gear) variant on the headline system
    M = spcg.CsrMatrix.from_host(A128)
    bt = torch.as_tensor(I.rhs_from_solution(A128, x128), device="cuda")
    res = {}
    for variant in ("standard", "single_reduction"):
        opts = spcg.cg_opts(tol=1e-10, maxit=20000, precond="jacobi", variant=variant)
        res[variant] = _time_solve(M, bt, opts, spcg.CgWorkspace(M, opts))
    out["jpcg_poisson128_variants"] = {
        "workload": "3-D Poisson 128^3 FP64 Jacobi-PCG to 1e-10: the two-reduction loop vs the "
                    "single-reduction (Chronopoulos-Gear) loop",
        "standard": res["standard"], "single_reduction": res["single_reduction"]}
    del M, bt
    out["spmv_cold"] = {"poisson128_f32": cold_spmv(A128, x128, "f32")}
    L, xl = I.lognormal_irregular()
    out["spmv_cold"]["lognormal_f64"] = cold_spmv(L, xl, "f64")
    out["spmv_cold"]["lognormal_f32"] = cold_spmv(L, xl, "f32")
    out["spmv_cold"]["lognormal_workload"] = ("n = 200000, lognormal row lengths (median 48, "
                                              "max 4096), nnz = 15788355, seed 2")
    return out


def tables():
    """The paper's input tables on one GPU (all cache-resident, so latency
    rather than HBM bandwidth bounds them): spmv_csr over the Table 1 square
    matrices (time per call over 200 back-to-back calls, and the median of 50
    single calls between events; GFLOP/s = 2 nnz / time per call) and plain CG
    to 1e-10 over the Table 2 banded systems (best of 5 solves), each beside
    the FP64 oracle on the host cores."""
    import numpy as np
    import torch

    import oracle
    from paper_1211_1581_amd import inputs as I
    from paper_1211_1581_amd import spcg
    out = {"table1_spmv": [], "table2_cg": [], "cpu_threads": oracle.set_threads(0)}
    for n, fill in I.TABLE1_MOD2AS:
        A, x = I.random_fill(n, fill, seed=n)
        M = spcg.CsrMatrix.from_host(A)
        xt = torch.as_tensor(x, device="cuda")
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        for _ in range(5):
            spcg.spmv_csr(M, xt, y)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(50)]
        for e0, e1 in evs:
            e0.record()
            spcg.spmv_csr(M, xt, y)
            e1.record()
        torch.cuda.synchronize()
        us_single = float(np.median([e0.elapsed_time(e1) * 1e3 for e0, e1 in evs]))
        # repeated products (the paper's loop of calls): 200 back-to-back launches
        # between two events, so the per-call event overhead is amortised
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(200):
            spcg.spmv_csr(M, xt, y)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 200
        ts = []
        for _ in range(20):
            t = time.perf_counter()
            oracle.spmv(A, x)
            ts.append(time.perf_counter() - t)
        cus = 1e6 * float(np.median(ts))
        out["table1_spmv"].append({"n": n, "fill_percent": fill, "nnz": A.nnz,
                                   "gpu_us": round(us, 2), "gpu_us_single_call": round(us_single, 2),
                                   "gpu_gflops": round(2 * A.nnz / us / 1e3, 2),
                                   "gpu_gbs": round(spmv_bytes(n, A.nnz) / us / 1e3, 1),
                                   "cpu_us": round(cus, 2),
                                   "cpu_gflops": round(2 * A.nnz / cus / 1e3, 2)})
    for n, bw in I.TABLE2_CG:
        A = I.banded_spd(n, bw)
        b = I.rhs_from_solution(A, I.uniform_vector(n, n + bw))
        M = spcg.CsrMatrix.from_host(A)
        bt = torch.as_tensor(b, device="cuda")
        opts = spcg.cg_opts(tol=1e-10, maxit=2000, precond="none")
        r = _time_solve(M, bt, opts, spcg.CgWorkspace(M, opts), reps=5)
        t = time.perf_counter()
        ro = oracle.pcg(A, b, tol=1e-10, maxit=2000, precond="none")
        cms = 1e3 * (time.perf_counter() - t)
        out["table2_cg"].append({"n": n, "bw": bw, "nnz": A.nnz, "gpu_ms": r["ms"],
                                 "iters": r["iters"],
                                 "gpu_us_per_pass": round(1e3 * r["ms"] / max(r["iters"], 1), 2),
                                 "true_relres": r["true_relres"], "status": r["status"],
                                 "cpu_ms": round(cms, 3), "cpu_iters": ro["iters"]})
    return out


def _time_solve(M, bt, opts, work, reps=3, pre=None):
    import torch

    from paper_1211_1581_amd import spcg
    x = torch.zeros_like(bt)
    best, r = None, None
    for _ in range(reps + 1):
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        if pre is not None:
            pre()
        r = spcg.cg_solve(M, bt, x, opts=opts, work=work, want_hist=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        best = dt if best is None else min(best, dt)
    return {"ms": round(1e3 * best, 2), "iters": r["iters"], "iters_fallback": r["iters_fallback"],
            "n_updates": r["n_updates"], "true_relres": r["true_relres"], "status": r["status"]}


def forms(args, only=None):
    """Time to a 1e-10 FP64 relative residual of the other solver forms, each
    beside FP64 Jacobi-PCG on the same matrix (best of 3 after a warm-up):
    mixed precision on the 160^3 finite-volume diffusion matrix (seed 3), and
    the learned factor (committed weights, prediction included) on the first
    unseen 128^3 diffusion matrix (seed 1000)."""
    out = {}
    if only != "learned":
        out["mixed_vs_jacobi"] = _mixed_form()
    if only != "mixed":
        out["learned_vs_jacobi"] = _learned_form()
    return out


def _mixed_form():
    import torch

    from paper_1211_1581_amd import inputs as I
    from paper_1211_1581_amd import spcg
    dev = torch.device("cuda:0")
    A, _, xs = I.fv_diffusion(160, 3)
    M = spcg.CsrMatrix.from_host(A, device=dev)
    bt = torch.as_tensor(I.rhs_from_solution(A, xs), device=dev)
    res = {}
    for prec in ("f64", "mixed"):
        opts = spcg.cg_opts(tol=1e-10, maxit=20000, precond="jacobi", precision=prec)
        res[prec] = _time_solve(M, bt, opts, spcg.CgWorkspace(M, opts))
    return {"workload": "FV diffusion 160^3 (n=4096000), GRF seed 3; FP64 "
                        "Jacobi-PCG vs FP32-inner / FP64 reliable-update",
            "jacobi_f64": res["f64"], "mixed": res["mixed"],
            "speedup": round(res["f64"]["ms"] / res["mixed"]["ms"], 3)}


def _learned_form():
    import torch

    from paper_1211_1581_amd import inputs as I
    from paper_1211_1581_amd import spcg, train
    dev = torch.device("cuda:0")
    A, _, xs = I.fv_diffusion(128, 1000)
    M = spcg.CsrMatrix.from_host(A, device=dev)
    bt = torch.as_tensor(I.rhs_from_solution(A, xs), device=dev)
    w, meta = train.load_weights()
    wt = torch.tensor(w, device=dev)
    g = spcg.MpnnGraph(M)
    budget = train.budget_for(128, meta.get("mean_learned_passes_48", 117.0))
    oj = spcg.cg_opts(tol=1e-10, maxit=20000, precond="jacobi")
    ol = spcg.cg_opts(tol=1e-10, maxit=20000, precond="learned", G=g.G, GT=g.GT, budget=budget)
    rj = _time_solve(M, bt, oj, spcg.CgWorkspace(M, oj))
    rl = _time_solve(M, bt, ol, spcg.CgWorkspace(M, ol), pre=lambda: g.predict(wt))
    # classical FSAI on the same pattern (set-up included), the non-learned comparator
    gf = spcg.MpnnGraph(M, ws=g.ws)
    of = spcg.cg_opts(tol=1e-10, maxit=20000, precond="learned", G=gf.G, GT=gf.GT, budget=20000)
    rf = _time_solve(M, bt, of, spcg.CgWorkspace(M, of),
                     pre=lambda: spcg.fsai_values(M, gf.G, gf.GT))
    return {"workload": "FV diffusion 128^3 (n=2097152), unseen seed 1000; "
                        "FP64 Jacobi-PCG vs learned G G^T (prediction "
                        "included, training excluded) and FSAI G G^T on the same "
                        "pattern (set-up included)",
            "jacobi_f64": rj, "learned": rl, "fsai": rf, "budget": budget,
            "speedup": round(rj["ms"] / rl["ms"], 3),
            "fsai_speedup": round(rj["ms"] / rf["ms"], 3)}


if __name__ == "__main__":
    main()
