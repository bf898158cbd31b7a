"""Benchmark of the CSR SpMV / conjugate-gradient hot path on one MI355X.

One step = one Jacobi-preconditioned CG solve (FP64) of the 3-D 7-point
Poisson matrix on a 128^3 grid to a 1e-10 relative residual: the SpMV with
p.q folded in, the reductions, the fused vector updates, the Jacobi step, the
device-side stop test and the final FP64 residual check.  Inputs (matrix, b,
x0 = 0) are resident in HBM before the timed region.

Prints ONE JSON line.  `value` is the hot path's algorithmic HBM throughput
(passes x algorithmic bytes per pass / wall time of the solves).  `roofline`
reports the product y = A x of the same matrix read from HBM (rotating device
copies that together exceed the 256 MB memory-side cache), timed by HIP events
on its stream; `roofline_in_cg` the same product inside the pass loop, where A
stays in that cache.  Every result carries its error against the FP64 oracle
(`err_vs_oracle`).  `cpu_baseline` times the oracle on the host cores (all
threads, pinned, and one thread) on a bounded sample of the same workload.
`forms` gives the time to tolerance of the mixed-precision and learned forms
beside plain FP64 Jacobi-PCG on their own matrices, the learned one also over
the 16 unseen evaluation matrices.

`workloads` adds plain CG on the 2-D Poisson 64^2 system, the single-reduction
loop, and the cold standalone SpMV of the other matrices and precisions;
`copy_gbs` and `read_gbs` are the measured streaming ceilings.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--cpu-seconds 15] [--no-forms]
                    [--no-eval16] [--no-cpu] [--spmv CASE] [--form mixed|learned] [--tables]
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
# OpenMP threads of the CPU baseline pinned one per core, packed (OpenMP reads
# these when its runtime starts, so before torch or the oracle loads it; the
# runtime then binds the main thread to the first core, so the host's CPU
# count is taken here)
os.environ.setdefault("OMP_PLACES", "cores")
os.environ.setdefault("OMP_PROC_BIND", "close")
HOST_CPUS = len(os.sched_getaffinity(0))

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


# sources of the CG pass kernels (k_cg_q and the kernels around it) and of the
# standalone product (k_spmv)
CG_SOURCES = ("internal.h", "cg.hip")
SPMV_SOURCES = ("internal.h", "csr.hip")


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


def measured_traffic(kernel, workload, sources):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel sources; else None."""
    return traffic_record(kernel, workload, sources)["bytes_per_launch"]


def traffic_record(kernel, workload, sources):
    """Which counter summary exists for the kernel and whether it applies:
    its file, the source hash it was taken on, the current hash, and its bytes
    per launch (None unless the two hashes agree)."""
    rel = os.path.join("profiles", f"traffic_{kernel}_{workload}.txt")
    path = os.path.join(ROOT, rel)
    cur = kernel_source_hash(sources)
    if not os.path.exists(path):
        return {"file": None, "taken_on_hash": None, "current_hash": cur, "bytes_per_launch": None}
    with open(path) as f:
        d = json.load(f)
    ok = d.get("source_hash") == cur
    return {"file": rel, "taken_on_hash": d.get("source_hash"), "current_hash": cur,
            "bytes_per_launch": d.get("bytes_per_launch") if ok else None,
            "bytes_per_launch_then": d.get("bytes_per_launch"),
            "ratio_to_algorithmic_then": d.get("ratio_to_algorithmic")}


def _oracle_jpcg_sample(A, b, seconds, full_passes):
    """Jacobi-PCG passes of the oracle on A x = b for about `seconds`: (passes, s)."""
    import oracle
    t = time.perf_counter()
    r = oracle.pcg(A, b, tol=0.0, maxit=3, precond="jacobi")
    per = (time.perf_counter() - t) / max(r["iters"], 1)
    passes = int(max(3, min(full_passes, seconds / max(per, 1e-6))))
    t = time.perf_counter()
    r = oracle.pcg(A, b, tol=0.0, maxit=passes, precond="jacobi")
    return r["iters"], time.perf_counter() - t


def cpu_baseline(A, b, seconds, full_passes):
    """The oracle (plain FP64 C, OpenMP rows, threads pinned one per core) on a
    bounded sample of the same workload: as many Jacobi-PCG passes of the same
    system as fit in about `seconds` on all threads, then in about a third of
    that on one thread; time to tolerance extrapolated to the full pass count."""
    import oracle
    n, nnz = A.n_rows, A.nnz
    threads = oracle.set_threads(0)
    k, dt = _oracle_jpcg_sample(A, b, seconds, full_passes)
    gbs = k * jpcg_pass_bytes(n, nnz) / dt / 1e9
    oracle.set_threads(1)
    k1, dt1 = _oracle_jpcg_sample(A, b, seconds / 3.0, full_passes)
    oracle.set_threads(threads)
    out = {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"{k} Jacobi-PCG passes (with set-up) of the 128^3 Poisson system in "
                     f"{dt:.1f} s on {threads} threads, {k1} passes in {dt1:.1f} s on one "
                     f"thread; a full solve takes {full_passes} passes",
           "est_time_to_tol_s": round(dt / k * full_passes, 2),
           "one_thread": {"value": round(k1 * jpcg_pass_bytes(n, nnz) / dt1 / 1e9, 3),
                          "est_time_to_tol_s": round(dt1 / k1 * full_passes, 2)},
           "omp": {"OMP_PLACES": os.environ.get("OMP_PLACES"),
                   "OMP_PROC_BIND": os.environ.get("OMP_PROC_BIND"),
                   "host_cpus_in_affinity": HOST_CPUS}}
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
    ap.add_argument("--no-eval16", action="store_true",
                    help="skip the learned form over the 16 unseen 128^3 matrices")
    ap.add_argument("--tables", action="store_true",
                    help="run the paper's own input tables instead (SpMV over the Table 1 "
                         "matrices, plain CG over the Table 2 banded systems) beside the "
                         "oracle on the host, and print that record")
    ap.add_argument("--form", choices=("mixed", "learned"), default=None,
                    help="run only this solver form beside FP64 Jacobi-PCG and print its "
                         "record (for kernel traces of one workload)")
    ap.add_argument("--spmv", choices=SPMV_CASES, default=None,
                    help="run only the cold standalone SpMV of this matrix and precision and "
                         "print its record (for kernel traces and counters of one product)")
    ap.add_argument("--binning", choices=("on", "off"), default="off",
                    help="row-length binning policy of the standalone products")
    ap.add_argument("--runs", choices=("on", "off"), default="off",
                    help="run-compressed column policy of the standalone products")
    ap.add_argument("--panels", choices=("auto", "on", "off"), default="auto",
                    help="column-panel policy of the standalone products (auto: the "
                         "library's default, panels for matrices of long rows spread over x)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(it would shard by rows, with a halo exchange per product and one "
              "small all-reduce per reduction)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1211_1581_amd import inputs as I
    from paper_1211_1581_amd import spcg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spcg.row_binning(args.binning)
    spcg.run_columns(args.runs)
    spcg.column_panels(args.panels)
    if args.calib and args.spmv:
        src = torch.ones(2 ** 25, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.spmv:
        print(json.dumps(spmv_case(args.spmv)), flush=True)
        return
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
    traffic_cg = measured_traffic("k_cg_q", "poisson128", CG_SOURCES)
    matrix_mb = (nnz * 12 + 4 * (n + 1)) / 1e6
    err_jpcg = oracle_errors(A, b, xs, x.cpu().numpy())

    # the standalone product of the same matrix, cold: rotating over device
    # copies whose total exceeds the 256 MB MALL, so every launch reads A from HBM
    cold = cold_spmv(A, xs, "f64", first=M)

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
        "err_vs_oracle": err_jpcg,
        "analysis_ms": round(analysis_ms, 2),
        "analysis_device_ms": round(analysis_device_ms, 3),
        "spmv_cold_gbs": cold["gbs"],
        "spmv_cold_us": cold["us"],
        "roofline": {"bound": "hbm", "achieved": cold["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(cold["gbs"] / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic("k_spmv", "poisson128", SPMV_SOURCES),
                     "kernel": "k_spmv<double> (y = A x, 128^3 Poisson, A read from HBM)",
                     "bytes_per_launch": b_spmv, "avg_launch_us": cold["us"],
                     "launches": cold["launches"],
                     "timing": ("HIP events on the launch stream around %d back-to-back launches "
                                "rotating over %d device copies of A (%.0f MB in all, more than the "
                                "256 MB MALL; streaming loads), after %d warm-up launches"
                                % (cold["launches"], cold["copies"],
                                   cold["copies"] * matrix_mb, cold["warmup"])),
                     "err_vs_oracle": cold["err_vs_oracle"],
                     # the counter summary behind `traffic` (null while the
                     # kernel sources differ from those it was taken on)
                     "traffic_source": traffic_record("k_spmv", "poisson128", SPMV_SOURCES)},
        "roofline_in_cg": {"bound": "mall", "achieved": round(achieved, 1), "unit": "GB/s",
                           "traffic": traffic_cg,
                           "traffic_source": traffic_record("k_cg_q", "poisson128", CG_SOURCES),
                           "kernel": "k_cg_q (q = A p with p.q partials, inside the Jacobi-PCG pass)",
                           "bytes_per_launch": b_spmv, "avg_launch_us": round(avg_us, 2),
                           "launches": spmv_calls,
                           "note": ("A's streams (%.1f MB) fit the cache-allocating limit (%d MiB), so "
                                    "A stays in the 256 MB MALL across passes: an algorithmic rate of "
                                    "a cache-served product, not a share of HBM peak"
                                    % (matrix_mb, spcg.keep_bytes() >> 20))
                           if matrix_mb * 1e6 <= spcg.keep_bytes()
                           else "A streams from HBM with non-temporal loads"},
    }
    line["copy_gbs"] = copy_rate()
    line["read_gbs"] = read_rate()
    if not args.no_forms:
        line["workloads"] = workloads(A, xs)
        line["forms"] = forms(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(A, b, args.cpu_seconds, iters)
    print(json.dumps(line), flush=True)


def oracle_errors(A, b, xstar, x):
    """Error of a device solution x against the FP64 oracle: ||b - A x|| / ||b||
    recomputed by the oracle, and the forward error against x*."""
    import numpy as np

    import oracle
    return {"true_relres": oracle.true_relres(A, b, x),
            "x_err": float(np.linalg.norm(x - xstar) / np.linalg.norm(xstar))}


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


def cold_spmv(A, x, dtype, launches=60, first=None):
    """Cold standalone SpMV: spmv_csr rotating over enough device copies of A
    that their total exceeds 600 MB (more than twice the 256 MB MALL), so every
    launch streams the matrix from HBM, read with the library's streaming
    (non-temporal) load policy, spcg_keep_bytes(0), the policy for products
    whose matrix is not read again soon.  `us` = the average duration of
    `launches` back-to-back launches between two HIP events on the launch
    stream (after warm-up launches); `us_bracketed` = the median of launches
    bracketed one by one (each then also carries the event and launch gaps).
    The last product is compared with the FP64 oracle (FP32: also with the
    oracle's FP64 sum of the same FP32 inputs)."""
    import numpy as np
    import torch

    import oracle
    from paper_1211_1581_amd import spcg
    keep = spcg.keep_bytes(0)
    try:
        return _cold_spmv(A, x, dtype, launches, first)
    finally:
        spcg.keep_bytes(keep)


def _cold_spmv(A, x, dtype, launches, first):
    import numpy as np
    import torch

    import oracle
    from paper_1211_1581_amd import spcg
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sv = 8 if dtype == "f64" else 4
    b = spmv_bytes(A.n_rows, A.nnz, sv=sv, sx=sv)
    ncopy = max(3, -(-600_000_000 // b))
    copies = ([first] if first is not None else []) + \
        [spcg.CsrMatrix.from_host(A, dtype=tdt) for _ in range(ncopy - (first is not None))]
    xt = torch.as_tensor(x).to(tdt).cuda()
    y = torch.empty(A.n_rows, dtype=tdt, device="cuda")
    warm = 2 * ncopy
    for i in range(warm):
        spcg.spmv_csr(copies[i % ncopy], xt, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(launches):
        spcg.spmv_csr(copies[i % ncopy], xt, y)
    e1.record()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(30)]
    for i, (f0, f1) in enumerate(evs):
        f0.record()
        spcg.spmv_csr(copies[i % ncopy], xt, y)
        f1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / launches
    us_br = float(np.median([f0.elapsed_time(f1) * 1e3 for f0, f1 in evs]))
    yh = y.cpu().numpy().astype(np.float64)
    pinfo = copies[0].panel_info() if spcg.column_panels() != "off" else None
    del copies
    if dtype == "f64":
        ref = oracle.spmv(A, x)
        err = {"rel_err": float(np.linalg.norm(yh - ref) / np.linalg.norm(ref))}
    else:
        v32 = np.asarray(A.vals, dtype=np.float32)
        x32 = np.asarray(x, dtype=np.float32)
        ref32 = oracle.spmv_f32in(A, v32, x32)
        ref = oracle.spmv(A, x)
        err = {"rel_err_same_fp32_inputs": float(np.linalg.norm(yh - ref32) / np.linalg.norm(ref32)),
               "rel_err_vs_fp64_product": float(np.linalg.norm(yh - ref) / np.linalg.norm(ref))}
    gbs = b / (us * 1e-6) / 1e9
    r = {"us": round(us, 2), "us_bracketed": round(us_br, 2), "gbs": round(gbs, 1),
         "pct_peak": round(100 * gbs / PEAK_HBM_GBS, 1), "bytes": b, "copies": ncopy,
         "launches": launches, "warmup": warm, "load_policy": "non-temporal",
         "err_vs_oracle": err}
    if pinfo is not None:
        # the panel copy the kernel streams instead of the CSR arrays: values and
        # 32-bit keys per entry (padding included); `bytes` stays the CSR figure
        r["panels"] = {"ranges": pinfo[0], "panels": pinfo[1], "entries": pinfo[2],
                       "copy_bytes": pinfo[2] * (sv + 4)}
    return r


SPMV_CASES = ("poisson128_f64", "poisson128_f32", "lognormal_f64", "lognormal_f32",
              "banded1m_f64", "banded1m_f32")


def spmv_case(name):
    """Cold standalone SpMV of one matrix (the 128^3 Poisson matrix with the
    seed-1 vector, or the lognormal irregular matrix) in one precision."""
    from paper_1211_1581_amd import inputs as I
    mat, dtype = name.split("_")
    if mat == "poisson128":
        A = I.poisson3d(128)
        x = I.uniform_vector(A.n_rows, 1)
    elif mat == "banded1m":
        # the banded shape of the paper's CG inputs at scale: 2^20 rows, bandwidth 63
        A = I.banded_spd(1 << 20, 63)
        x = I.uniform_vector(A.n_rows, 63)
    else:
        A, x = I.lognormal_irregular()
    r = cold_spmv(A, x, dtype)
    r["case"] = name
    from paper_1211_1581_amd import spcg
    r["row_binning"] = spcg.row_binning()
    r["run_columns"] = spcg.run_columns()
    r["column_panels"] = spcg.column_panels()
    return r


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
    r = _time_solve(M, bt, opts, spcg.CgWorkspace(M, opts), reps=10, check=(P, b, I.uniform_vector(P.n_rows, 0)))
    out["cg_poisson2d_64"] = {"workload": "2-D 5-point Poisson 64^2, plain CG to 1e-10 (one "
                                          "workgroup holds the whole loop)",
                              "ms": r["ms"], "iters": r["iters"],
                              "us_per_pass": round(1e3 * r["ms"] / max(r["iters"], 1), 2),
                              "true_relres": r["true_relres"], "status": r["status"],
                              "err_vs_oracle": r["err_vs_oracle"]}
    del M, bt
    # the single-reduction (Chronopoulos-Gear) variant on the headline system
    M = spcg.CsrMatrix.from_host(A128)
    b128 = I.rhs_from_solution(A128, x128)
    bt = torch.as_tensor(b128, device="cuda")
    res = {}
    for variant in ("standard", "single_reduction"):
        opts = spcg.cg_opts(tol=1e-10, maxit=20000, precond="jacobi", variant=variant)
        res[variant] = _time_solve(M, bt, opts, spcg.CgWorkspace(M, opts), check=(A128, b128, x128))
    out["jpcg_poisson128_variants"] = {
        "workload": "3-D Poisson 128^3 FP64 Jacobi-PCG to 1e-10: the two-reduction loop vs the "
                    "single-reduction (Chronopoulos-Gear) loop",
        "standard": res["standard"], "single_reduction": res["single_reduction"]}
    del M, bt
    out["spmv_cold"] = {"poisson128_f32": cold_spmv(A128, x128, "f32")}
    L, xl = I.lognormal_irregular()
    # under the library's default panel policy (auto: this matrix gets column
    # panels, reported in each row's "panels"), then with the row-block kernel
    out["spmv_cold"]["lognormal_f64"] = cold_spmv(L, xl, "f64")
    out["spmv_cold"]["lognormal_f32"] = cold_spmv(L, xl, "f32")
    old = spcg.column_panels("off")
    try:
        out["spmv_cold"]["lognormal_f64_row_blocks"] = cold_spmv(L, xl, "f64")
        out["spmv_cold"]["lognormal_f32_row_blocks"] = cold_spmv(L, xl, "f32")
    finally:
        spcg.column_panels(old)
    # the same products with row-length bins (per-bin lane groups) instead of
    # the row-block kernel
    old = spcg.row_binning("on")
    try:
        out["spmv_cold"]["lognormal_f64_row_bins"] = cold_spmv(L, xl, "f64")
        out["spmv_cold"]["lognormal_f32_row_bins"] = cold_spmv(L, xl, "f32")
    finally:
        spcg.row_binning(old)
    # and with column panels (x staged in LDS by panels, four column groups per
    # row range); an error here is recorded instead of ending the bench
    old = spcg.column_panels("on")
    try:
        for dt in ("f64", "f32"):
            try:
                out["spmv_cold"][f"lognormal_{dt}_panels"] = cold_spmv(L, xl, dt)
            except Exception as e:  # noqa: BLE001 - the line must still print
                out["spmv_cold"][f"lognormal_{dt}_panels"] = {"error": repr(e)[:300]}
    finally:
        spcg.column_panels(old)
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


def _time_solve(M, bt, opts, work, reps=3, pre=None, check=None):
    """Best of `reps` timed solves after one warm-up.  check = (A, b, x*) on the
    host: the last solution's errors against the FP64 oracle."""
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
    out = {"ms": round(1e3 * best, 2), "iters": r["iters"], "iters_fallback": r["iters_fallback"],
           "n_updates": r["n_updates"], "true_relres": r["true_relres"], "status": r["status"]}
    if check is not None:
        out["err_vs_oracle"] = oracle_errors(check[0], check[1], check[2], x.cpu().numpy())
    return out


def forms(args, only=None):
    """Time to a 1e-10 FP64 relative residual of the other solver forms, each
    beside FP64 Jacobi-PCG on the same matrix (best of 3 after a warm-up):
    mixed precision on the 160^3 finite-volume diffusion matrix (seed 3), and
    the learned factor (committed weights, prediction included) on the first
    unseen 128^3 diffusion matrix (seed 1000), then on all 16 unseen ones
    (seeds 1000-1015, best of 2)."""
    out = {}
    if only != "learned":
        out["mixed_vs_jacobi"] = _mixed_form()
    if only != "mixed":
        out["learned_vs_jacobi"] = _learned_form()
        if not getattr(args, "no_eval16", False):
            out["learned_eval_16"] = _learned_eval(range(1000, 1016))
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
    b = I.rhs_from_solution(A, xs)
    for prec in ("f64", "mixed"):
        opts = spcg.cg_opts(tol=1e-10, maxit=20000, precond="jacobi", precision=prec)
        res[prec] = _time_solve(M, bt, opts, spcg.CgWorkspace(M, opts), check=(A, b, xs))
    return {"workload": "FV diffusion 160^3 (n=4096000), GRF seed 3; FP64 "
                        "Jacobi-PCG vs FP32-inner / FP64 reliable-update",
            "jacobi_f64": res["f64"], "mixed": res["mixed"],
            "speedup": round(res["f64"]["ms"] / res["mixed"]["ms"], 3)}


def _learned_setup(N, seed):
    import torch

    from paper_1211_1581_amd import inputs as I
    from paper_1211_1581_amd import spcg
    A, _, xs = I.fv_diffusion(N, seed)
    b = I.rhs_from_solution(A, xs)
    M = spcg.CsrMatrix.from_host(A)
    return A, xs, b, M, torch.as_tensor(b, device="cuda")


def _learned_solves(A, xs, b, M, bt, w, budget, ws=None, reps=3):
    """Jacobi-PCG, the learned factor (prediction included) and FSAI (set-up
    included) on one system, each with its oracle errors."""
    from paper_1211_1581_amd import spcg
    g = spcg.MpnnGraph(M, ws=ws)
    oj = spcg.cg_opts(tol=1e-10, maxit=20000, precond="jacobi")
    ol = spcg.cg_opts(tol=1e-10, maxit=20000, precond="learned", G=g.G, GT=g.GT, budget=budget)
    chk = (A, b, xs)
    rj = _time_solve(M, bt, oj, spcg.CgWorkspace(M, oj), reps=reps, check=chk)
    rl = _time_solve(M, bt, ol, spcg.CgWorkspace(M, ol), reps=reps, pre=lambda: g.predict(w),
                     check=chk)
    # classical FSAI on the same pattern (set-up included), the non-learned comparator
    gf = spcg.MpnnGraph(M, ws=g.ws)
    of = spcg.cg_opts(tol=1e-10, maxit=20000, precond="learned", G=gf.G, GT=gf.GT, budget=20000)
    rf = _time_solve(M, bt, of, spcg.CgWorkspace(M, of), reps=reps,
                     pre=lambda: spcg.fsai_values(M, gf.G, gf.GT), check=chk)
    return rj, rl, rf, g.ws


def _learned_form():
    import torch

    from paper_1211_1581_amd import train
    A, xs, b, M, bt = _learned_setup(128, 1000)
    w, meta = train.load_weights()
    wt = torch.tensor(w, device="cuda")
    budget = train.budget_for(128, meta.get("mean_learned_passes_48", 117.0))
    rj, rl, rf, _ = _learned_solves(A, xs, b, M, bt, wt, budget)
    return {"workload": "FV diffusion 128^3 (n=2097152), unseen seed 1000; "
                        "FP64 Jacobi-PCG vs learned G G^T (prediction "
                        "included, training excluded) and FSAI G G^T on the same "
                        "pattern (set-up included)",
            "jacobi_f64": rj, "learned": rl, "fsai": rf, "budget": budget,
            "speedup": round(rj["ms"] / rl["ms"], 3),
            "fsai_speedup": round(rj["ms"] / rf["ms"], 3)}


def _learned_eval(seeds):
    """The learned factor over the unseen 128^3 evaluation matrices: per seed
    the passes and times (best of 2) of Jacobi-PCG, the learned PCG
    (prediction included) and FSAI, with the oracle's residual of each
    solution; then the means and the fallback count."""
    import numpy as np
    import torch

    from paper_1211_1581_amd import train
    w, meta = train.load_weights()
    wt = torch.tensor(w, device="cuda")
    budget = train.budget_for(128, meta.get("mean_learned_passes_48", 117.0))
    rows, ws = [], None
    for seed in seeds:
        A, xs, b, M, bt = _learned_setup(128, seed)
        rj, rl, rf, ws = _learned_solves(A, xs, b, M, bt, wt, budget, ws=ws, reps=2)
        rows.append({"seed": seed,
                     "jacobi": [rj["iters"], rj["ms"]],
                     "learned": [rl["iters"], rl["iters_fallback"], rl["ms"]],
                     "fsai": [rf["iters"], rf["ms"]],
                     "oracle_true_relres_max": max(r["err_vs_oracle"]["true_relres"]
                                                   for r in (rj, rl, rf)),
                     "status": [rj["status"], rl["status"], rf["status"]]})
        del M, bt
    mean = lambda k, i: round(float(np.mean([r[k][i] for r in rows])), 2)
    return {"workload": "FV diffusion 128^3, unseen seeds %d-%d; per seed [passes, ms] for "
                        "Jacobi and FSAI, [learned passes, fallback passes, ms] for the learned "
                        "form (prediction included)" % (seeds[0], seeds[-1]),
            "budget": budget, "rows": rows,
            "mean_passes": {"jacobi": mean("jacobi", 0), "learned": mean("learned", 0),
                            "fsai": mean("fsai", 0)},
            "mean_ms": {"jacobi": mean("jacobi", 1), "learned": mean("learned", 2),
                        "fsai": mean("fsai", 1)},
            "fallbacks": sum(1 for r in rows if r["learned"][1] > 0 or r["status"][1] == 2),
            "oracle_true_relres_max": max(r["oracle_true_relres_max"] for r in rows)}


if __name__ == "__main__":
    main()
