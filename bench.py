"""Benchmark: GSE-SEM SpMV bandwidth per segment count and stepped CG
time-to-1e-10 against plain FP64 CSR on one MI355X.

One step = the whole hot path on the 3-D 7-point variable-coefficient
diffusion operator (128^3 cells, 14.58 M non-zeros, face coefficients
log-uniform over four decades):
  * SpMV with 1, 2 and 3 segments and the FP64 CSR baseline, each over
    ``--copies`` resident copies of the matrix in rotation so that the
    working set exceeds the 256 MB Infinity Cache (cold, HBM-bound);
  * stepped GSE CG and FP64 CSR CG from x0 = 0 to relative residual 1e-10.
Inputs are synthetic (seeded generator) and resident in HBM before timing.

Prints one JSON line.  ``value`` is the GSE SpMV HBM bandwidth with one
segment (algorithmic bytes / mean kernel time from HIP events on the launch
stream); the other segment counts, the FP64 baseline and the solve times are
reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GSE-SpMV HBM GB/s (% peak) per segment count; CG time-to-1e-10 vs FP64 CSR"


def spmv_bytes(n_rows, n_cols, nnz, plane_bytes):
    """Algorithmic bytes of one SpMV: every plane byte once, row pointers,
    x once and y once."""
    return nnz * plane_bytes + (n_rows + 1) * 4 + n_cols * 8 + n_rows * 8


def kernel_name(A):
    """Name of the kernel instance the one-segment SpMV runs on this schedule."""
    if A.rv_lanes > 0:
        return f"k_spmv_rv<1, {A.rv_lanes}>"
    return f"k_spmv<1, {A.tile_nnz // 256}>"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--reps", type=int, default=10, help="SpMV launches per copy per step")
    ap.add_argument("--no-solve", action="store_true", help="SpMV only (profiling runs)")
    ap.add_argument("--cpu-baseline", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0: skip)")
    return ap.parse_args()


def cpu_baseline(A, seconds):
    """The oracle's one-segment SpMV on the same matrix, sequential C."""
    import oracle as O
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    x = np.ones(A.n_cols)
    O.gse_spmv(A.indptr, enc, 1, x)
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.gse_spmv(A.indptr, enc, 1, x)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    per = el / reps
    gbs = spmv_bytes(A.n_rows, A.n_cols, A.nnz, 6) / per / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle gse_spmv s=1 on the full {A.name} matrix, {reps} runs "
                      f"({el:.1f} s, {per * 1e3:.1f} ms each, one thread)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    import torch

    from paper_2411_04686_amd import gse as G
    from workloads import diffusion3d, rhs_from_solution

    dev = torch.device("cuda:0")
    A = diffusion3d(args.grid, args.seed)
    x_true, b = rhs_from_solution(A, args.seed)
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    mats = [G.GseMatrix(rp.clone(), ci, va, A.n_cols) for _ in range(args.copies)]
    csrs = [G.CsrMatrix(rp.clone(), ci, va, A.n_cols) for _ in range(args.copies)]
    del ci, va
    xs = torch.ones(A.n_cols, dtype=torch.float64, device=dev)
    ys = [torch.empty(A.n_rows, dtype=torch.float64, device=dev) for _ in range(args.copies)]
    stream = torch.cuda.current_stream()

    kinds = [("s1", 6), ("s2", 8), ("s3", 12), ("fp64", 12)]
    times = {k: [] for k, _ in kinds}

    def spmv_pass(record):
        for kname, _ in kinds:
            for rep in range(args.reps):
                for c in range(args.copies):
                    if record:
                        e0 = torch.cuda.Event(enable_timing=True)
                        e1 = torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                    if kname == "fp64":
                        csrs[c].spmv(xs, ys[c])
                    else:
                        mats[c].spmv(int(kname[1]), xs, ys[c])
                    if record:
                        e1.record(stream)
                        times[kname].append((e0, e1))

    solve = {}

    def solve_pass(record):
        if args.no_solve or not hasattr(G.lib(), "gse_cg"):
            return
        bd = torch.from_numpy(b).to(dev)
        p = G.gse_default_params(G.CG)
        p.max_iter = 20000
        ws = torch.empty(G.gse_solver_workspace(G.CG, A.n_rows, A.nnz, 30, p.max_iter),
                         dtype=torch.uint8, device=dev)
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
        rg = G.gse_cg(mats[0].A, bd, x, p, ws)
        x.zero_()
        r64 = G.gse_csr_cg(csrs[0].M, bd, x, p, ws)
        if record:
            solve.setdefault("gse", []).append(rg.as_dict())
            solve.setdefault("fp64", []).append(r64.as_dict())

    for _ in range(args.warmup):
        spmv_pass(False)
        solve_pass(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        spmv_pass(True)
        solve_pass(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    spmv = {}
    for kname, pb in kinds:
        ms = np.array([a.elapsed_time(c) for a, c in times[kname]])
        nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, pb)
        mean = float(ms.mean())
        spmv[kname] = {"mean_us": round(mean * 1e3, 2),
                       "median_us": round(float(np.median(ms)) * 1e3, 2),
                       "p10_us": round(float(np.percentile(ms, 10)) * 1e3, 2),
                       "p90_us": round(float(np.percentile(ms, 90)) * 1e3, 2),
                       "bytes": int(nbytes),
                       "GBps": round(nbytes / (mean * 1e-3) / 1e9, 1),
                       "frac_peak": round(nbytes / (mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out = {
        "metric": METRIC,
        "value": spmv["s1"]["GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"diffusion3d_{args.grid}^3_7pt_varcoef_4decades",
                   "n_rows": A.n_rows, "nnz": A.nnz, "copies_rotated": args.copies,
                   "x": "ones", "seed": args.seed, "tile_nnz": mats[0].A.tile_nnz,
                   "rv_lanes": mats[0].A.rv_lanes},
        "spmv": spmv,
        "roofline": {"bound": "hbm", "achieved": spmv["s1"]["GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": spmv["s1"]["frac_peak"], "traffic": None,
                     "kernel": kernel_name(mats[0].A),
                     "bytes_per_launch": spmv["s1"]["bytes"]},
    }
    if solve:
        g = solve["gse"][-1]
        f = solve["fp64"][-1]
        out["cg"] = {"gse": g, "fp64": f,
                     "speedup": round(f["time_ms"] / g["time_ms"], 3) if g["time_ms"] else None}
    if args.cpu_baseline > 0:
        out["cpu_baseline"] = cpu_baseline(A, args.cpu_baseline)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
