"""Benchmark: GSE-SEM SpMV bandwidth per segment count and stepped CG
time-to-1e-10 against plain FP64 CSR on one MI355X.

Default workload (``--workload spmv_cg``), one step = the whole hot path on
the 3-D 7-point variable-coefficient diffusion operator (128^3 cells,
14.58 M non-zeros, face coefficients log-uniform over four decades):
  * SpMV with 1, 2 and 3 segments and the FP64 CSR baseline, each over
    ``--copies`` resident copies of the matrix in rotation so that the
    working set exceeds the 256 MB Infinity Cache (cold, HBM-bound);
  * stepped GSE CG and FP64 CSR CG from x0 = 0 to relative residual 1e-10.
Inputs are synthetic (seeded generator) and resident in HBM before timing.

Prints one JSON line.  ``value`` is the GSE SpMV HBM bandwidth with one
segment: algorithmic bytes / mean time per launch, from HIP events on the
launch stream around rounds of back-to-back launches (one per copy); the
other segment counts, the FP64 baseline, a streaming-copy ceiling and the
solve times are reported beside it.  Every result states its error: each
operator's max-abs and relative error against the host FP64 CSR product
with x = 1, eta_s, and per solve the true residual and ||x - x_true|| /
||x_true||.  After the timed steps the same line carries one run of each
other configuration (``--no-legs`` skips them): the 2-D Poisson 64^2 CG,
the 1024^2 convection-diffusion GMRES(30) and the 4 M-row power-law SpMV
and CG, with the same error figures.

Other workloads (one JSON line each):
  * ``--workload gmres``: stepped GMRES(30) and FP64 GMRES(30) to 1e-10 on
    the 2-D upwind convection-diffusion operator, 1024^2 cells;
  * ``--workload serving``: a Poisson-arrival stream of 2-D / 3-D diffusion
    systems through the solver server (stepped GSE, batched) against the
    same server running FP64 CSR one request at a time; p50 / p99 latency
    and solves per second;
  * ``--workload powerlaw``: the 4 M-row power-law SPD matrix (Zipf(2) row
    lengths up to 10^4, values over six decades): SpMV per segment count on
    autotuned tiles, then stepped GSE CG and FP64 CG to 1e-10;
  * ``--workload blocks``: per-row-block shared-exponent tables on the
    layered medium 128^3 (encode, SpMV time and error; also a leg of the
    default workload).
  * ``--workload poisson``: the 2-D Poisson 64 x 64 system, stepped GSE CG
    and FP64 CG to 1e-10 (launch-bound; median over the steps).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GSE-SpMV HBM GB/s (% peak) per segment count; CG time-to-1e-10 vs FP64 CSR"
KERNEL_SOURCES = ("paper_2411_04686_amd/csrc/spmv.hip", "paper_2411_04686_amd/csrc/decode.h",
                  "paper_2411_04686_amd/csrc/gse_internal.h")


def spmv_bytes(n_rows, n_cols, nnz, plane_bytes):
    """Algorithmic bytes of one SpMV: every plane byte once, row pointers,
    x once and y once."""
    return nnz * plane_bytes + (n_rows + 1) * 4 + n_cols * 8 + n_rows * 8


def kernel_name(A):
    """Name of the kernel instance the one-segment SpMV runs on this schedule."""
    if A.rv_lanes > 0:
        return f"k_spmv_rv<1, {A.rv_lanes}{', true' if A.block_rows else ''}>"
    e = A.tile_nnz // 256
    if A.max_row_nnz <= 24:
        if A.tile_nnz == 1024 and A.nnz >= 1024:
            m = A.max_row_nnz
            if m <= 8:
                b = 3 if m <= 3 else 5 if m <= 5 else 7 if m <= 7 else 8
                if A.block_rows:
                    return f"k_spmv_rows<1, {b}, true, -1>"
                if A.idx_bits == 3 and A.idx_layout == 1:
                    # the instance with the 3-bit column-word index folded in
                    return f"k_spmv_rows<1, {b}, false, 3>"
                return f"k_spmv_rows<1, {b}, false, -1>"
            return "k_spmv_ring<1>"
        return f"k_spmv_short<1, {e}>"
    return f"k_spmv<1, {e}>"


def source_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_spmv_s1_diffusion3d_128.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    fields = dict(re.findall(r"^- (\w+): `([^`]*)`", text, re.M))
    if fields.get("kernel") != kernel or fields.get("workload") != workload:
        return None
    if fields.get("source_digest") != source_digest():
        return None
    try:
        return int(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spmv_cg",
                    choices=["spmv_cg", "gmres", "serving", "powerlaw", "poisson", "blocks",
                             "batch"])
    ap.add_argument("--pl-rows", type=int, default=4_000_000, help="powerlaw: rows")
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--reps", type=int, default=20, help="SpMV launches per copy per step")
    ap.add_argument("--no-solve", action="store_true", help="SpMV only (profiling runs)")
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="default workload: skip the Poisson, GMRES and power-law legs")
    ap.add_argument("--cpu-baseline", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0: skip)")
    ap.add_argument("--requests", type=int, default=48, help="serving: requests per load level")
    ap.add_argument("--n-hi", type=float, default=1e5, help="serving: largest request size")
    ap.add_argument("--arena-gb", type=float, default=32.0, help="serving: arena size")
    ap.add_argument("--slots", type=int, default=64, help="serving: batch slots")
    ap.add_argument("--batch-systems", type=int, default=16, help="batch: systems per batch")
    ap.add_argument("--batch-grid", type=int, default=48, help="batch: 3-D grid side per system")
    ap.add_argument("--batch-segments", type=int, default=0,
                    help="batch: 0 stepped (default), 1-3 a fixed segment count")
    ap.add_argument("--batch-kinds", default="gse,fp64",
                    help="batch: comma-separated kinds to solve (gse, fp64)")
    return ap.parse_args()


def cpu_baseline(A, seconds):
    """The oracle's one-segment SpMV on the same matrix, timed on the host's
    cores: the rows are cut into contiguous blocks that host threads run
    through the oracle's own sequential row routine (each row keeps its
    order, so the result is the single-thread one, bit for bit)."""
    import concurrent.futures as cf

    import oracle as O
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    x = np.ones(A.n_cols)
    threads = max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, A.n_rows, threads + 1).astype(np.int64)
    blocks = [np.arange(bounds[i], bounds[i + 1], dtype=np.int32) for i in range(threads)]
    y = np.empty(A.n_rows)

    def block(i):
        y[bounds[i]:bounds[i + 1]] = O.gse_spmv_rows(blocks[i], A.indptr, enc, 1, x)

    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(block, range(threads)))
        ref = O.gse_spmv(A.indptr, enc, 1, x)
        same = bool(np.array_equal(y, ref))
        reps = 0
        t0 = time.perf_counter()
        while True:
            list(ex.map(block, range(threads)))
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
    per = el / reps
    gbs = spmv_bytes(A.n_rows, A.n_cols, A.nnz, 6) / per / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle gse_spmv s=1 (row routine, {threads} host threads over contiguous "
                      f"row blocks; equal to the sequential result: {same}) on the full {A.name} "
                      f"matrix, {reps} runs ({el:.1f} s, {per * 1e3:.1f} ms each)"}


def copy_ceiling(G, torch, dev, stream):
    """Streaming copy of 512 MiB (read + write), the practical HBM ceiling."""
    n = 512 << 20
    src = torch.empty(n, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        G.gse_stream_copy(src, dst, n)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        G.gse_stream_copy(src, dst, n)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del src, dst
    return round(2 * n / (ms * 1e-3) / 1e9, 1)


def spmv_warm(torch, stream, M, C, x, y, kinds, A, reps=20):
    """One copy launched back to back: its planes (<= 217 MB here) stay in the
    256 MB Infinity Cache between launches (the warm figure beside the cold,
    rotated one)."""
    out = {}
    for kname, pb in kinds:
        def run():
            if kname == "fp64":
                C.spmv(x, y)
            else:
                M.spmv(int(kname[1]), x, y)
        for _ in range(3):
            run()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, pb)
        out[kname] = {"mean_us": round(us, 2), "GBps": round(nbytes / (us * 1e-6) / 1e9, 1)}
    return out


def copy_same_size(G, torch, dev, stream, nbytes, copies):
    """Streaming copy moving `nbytes` per launch (half read, half written),
    rotated over `copies` buffer pairs like the SpMV operands: the practical
    ceiling for one launch of that size, fill and drain included."""
    half = (nbytes // 2 + 255) // 256 * 256
    pairs = [(torch.empty(half, dtype=torch.uint8, device=dev),
              torch.empty(half, dtype=torch.uint8, device=dev)) for _ in range(copies)]
    for a, b in pairs:
        G.gse_stream_copy(a, b, half)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    rounds = 10
    e0.record(stream)
    for _ in range(rounds):
        for a, b in pairs:
            G.gse_stream_copy(a, b, half)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / (rounds * copies)
    del pairs
    return {"bytes": 2 * half, "mean_us": round(us, 2), "GBps": round(2 * half / (us * 1e-6) / 1e9, 1)}


def read_ceiling(G, torch, dev, stream, nbytes, copies):
    """Streaming reduction (eight FP64 read per one written: 89 % reads, the
    SpMV's mix) moving `nbytes` per launch, rotated over `copies` buffer
    pairs: the practical ceiling of a read-dominated launch of that size."""
    n_out = max(1, nbytes // 72)
    pairs = [(torch.rand(8 * n_out, dtype=torch.float64, device=dev),
              torch.empty(n_out, dtype=torch.float64, device=dev)) for _ in range(copies)]
    for a, b in pairs:
        G.gse_stream_reduce8(a, b, n_out)
    torch.cuda.synchronize()
    ok = bool(torch.allclose(pairs[0][1], pairs[0][0].view(-1, 8).sum(dim=1)))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    rounds = 10
    e0.record(stream)
    for _ in range(rounds):
        for a, b in pairs:
            G.gse_stream_reduce8(a, b, n_out)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / (rounds * copies)
    moved = 72 * n_out
    del pairs
    return {"bytes": moved, "read_frac": round(64 / 72, 3), "mean_us": round(us, 2),
            "GBps": round(moved / (us * 1e-6) / 1e9, 1), "checked": ok}


def progress(msg):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def base_record(args, metric, value, unit, wall, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(wall / max(args.steps, 1) * 1e3, 3),
            "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic"}


# ------------------------------------------------------------ spmv + CG ---
def run_spmv_cg(args, torch, G):
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
    copy_gbs = copy_ceiling(G, torch, dev, stream)

    kinds = [("s1", 6), ("s2", 8), ("s3", 12), ("fp64", 12)]
    times = {k: [] for k, _ in kinds}

    def spmv_pass(record):
        # HIP events on the launch stream around each round of `copies`
        # back-to-back launches (one per copy): the per-launch time is the
        # round's time over `copies`, launch gaps included.  Each kind starts
        # with one untimed round, so that no timed round opens on an idle
        # queue (after the solves' host work the first launch would otherwise
        # be timed from the event to the host's next launch call).
        for kname, _ in kinds:
            for rep in range(-1, args.reps):
                record_this = record and rep >= 0
                if record_this:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                for c in range(args.copies):
                    if kname == "fp64":
                        csrs[c].spmv(xs, ys[c])
                    else:
                        mats[c].spmv(int(kname[1]), xs, ys[c])
                if record_this:
                    e1.record(stream)
                    times[kname].append((e0, e1))

    solve = {}

    def solve_pass(record):
        if args.no_solve:
            return
        bd = torch.from_numpy(b).to(dev)
        p = G.gse_default_params(G.CG)
        p.max_iter = 20000
        ws = torch.empty(G.gse_solver_workspace(G.CG, A.n_rows, A.nnz, 30, p.max_iter),
                         dtype=torch.uint8, device=dev)
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
        # a solve's time_ms runs from its call to its return: nothing queued
        # before it may be counted in it
        torch.cuda.synchronize()
        rg = G.gse_cg(mats[0].A, bd, x, p, ws)
        if record:
            solve.setdefault("gse", []).append(solve_record(rg, x, x_true))
        x.zero_()
        torch.cuda.synchronize()
        r64 = G.gse_csr_cg(csrs[0].M, bd, x, p, ws)
        if record:
            solve.setdefault("fp64", []).append(solve_record(r64, x, x_true))

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
        ms = np.array([a.elapsed_time(c) for a, c in times[kname]]) / args.copies
        nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, pb)
        mean = float(ms.mean())
        spmv[kname] = {"mean_us": round(mean * 1e3, 2),
                       "median_us": round(float(np.median(ms)) * 1e3, 2),
                       "p10_us": round(float(np.percentile(ms, 10)) * 1e3, 2),
                       "p90_us": round(float(np.percentile(ms, 90)) * 1e3, 2),
                       "bytes": int(nbytes),
                       "GBps": round(nbytes / (mean * 1e-3) / 1e9, 1),
                       "frac_peak": round(nbytes / (mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    workload = f"diffusion3d_{args.grid}^3_7pt_varcoef_4decades"
    kname = kernel_name(mats[0].A)
    out = base_record(args, METRIC, spmv["s1"]["GBps"], "GB/s", wall)
    out["config"] = {"workload": workload, "n_rows": A.n_rows, "nnz": A.nnz,
                     "copies_rotated": args.copies, "x": "ones", "seed": args.seed,
                     "tile_nnz": mats[0].A.tile_nnz, "rv_lanes": mats[0].A.rv_lanes}
    out["spmv"] = spmv
    out["copy_ceiling_GBps"] = copy_gbs
    if not args.no_solve:  # profiling runs (--no-solve) keep to the cold launches and the copy
        out["spmv_warm"] = spmv_warm(torch, stream, mats[0], csrs[0], xs, ys[0], kinds, A)
        out["copy_same_size"] = copy_same_size(G, torch, dev, stream, spmv["s1"]["bytes"],
                                               args.copies)
        out["read_ceiling_same_size"] = read_ceiling(G, torch, dev, stream, spmv["s1"]["bytes"],
                                                     args.copies)
    out["roofline"] = {"bound": "hbm", "achieved": spmv["s1"]["GBps"], "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": spmv["s1"]["frac_peak"],
                       "traffic": measured_traffic(kname, workload), "kernel": kname,
                       "bytes_per_launch": spmv["s1"]["bytes"],
                       "mean_launch_us": spmv["s1"]["mean_us"]}
    if solve:
        g = solve["gse"][-1]
        f = solve["fp64"][-1]
        med = {k: float(np.median([r["time_ms"] for r in v])) for k, v in solve.items()}
        out["cg"] = {"gse": g, "fp64": f, "median_ms": {k: round(v, 3) for k, v in med.items()},
                     "speedup": round(med["fp64"] / med["gse"], 3) if med["gse"] else None}
    if not args.no_solve:
        out["spmv_error"] = spmv_errors(A, mats[0], csrs[0], np.ones(A.n_cols), dev, torch)
    del mats, csrs, ys
    if args.legs and not args.no_solve:
        progress("legs: FP16 / BF16 comparators and the k sweep on the 128^3 operator")
        out["lowprec_spmv"] = leg_lowprec_spmv(torch, G, A, args.copies)
        if solve:
            out["lowprec_cg"] = leg_lowprec_solve(torch, G, A, b, x_true, G.CG, solve["gse"][-1],
                                                  solve["fp64"][-1])
        out["k_sweep"] = leg_k_sweep(torch, G, A, args.copies)
        progress("legs: per-row-block tables (layered medium 128^3)")
        out["blocks"] = leg_blocks(torch, G, args.seed, args.copies, A_cg=A, b_cg=b,
                                   x_true_cg=x_true)
    if args.legs and not args.no_solve:
        # the other configurations, each once after the timed steps (their own
        # warm-up), so that every result of the path is on the one line
        progress("legs: poisson 64^2")
        out["poisson"] = leg_poisson(torch, G, args.seed, 5, 1)
        progress("legs: gmres 1024^2")
        out["gmres"] = leg_gmres(torch, G, args.seed, 1, 1)
        progress("legs: powerlaw")
        pl = leg_powerlaw(torch, G, args.seed, 1, 1, 5, args.pl_rows)
        pl.pop("wall_s")
        out["powerlaw"] = pl
        progress("legs: batched CG, 16 x 48^3")
        bt = run_batch(args, torch, G)
        out["batch"] = {"config": bt["config"], "speedup": bt.get("speedup"), **bt["batch"]}
        progress("legs: serving")
        sv = run_serving(args, torch, G)
        out["serving"] = {"config": sv["config"], **sv["serving"]}
    if args.cpu_baseline > 0:
        out["cpu_baseline"] = cpu_baseline(A, args.cpu_baseline)
    return out


# ------------------------------------------------------ error of results ---
def spmv_errors(A, M, C, x_host, dev, torch):
    """Error of each operator against the FP64 CSR product computed on the
    host (scipy, FP64) with the same x (x = 1 is the paper's SpMV protocol):
    max |y_s - y| and ||y_s - y|| / ||y||, for s = 1, 2, 3 and the GPU FP64
    CSR kernel; plus eta_s = ||A - A_s||_inf / ||A||_inf of the encoding."""
    ref = A.to_scipy() @ x_host
    nref = float(np.linalg.norm(ref))
    xd = torch.from_numpy(x_host).to(dev)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    out = {}
    for kname in ("s1", "s2", "s3", "fp64"):
        if kname == "fp64":
            C.spmv(xd, y)
        else:
            M.spmv(int(kname[1]), xd, y)
        torch.cuda.synchronize()
        d = y.cpu().numpy() - ref
        out[kname] = {"max_abs": float(np.max(np.abs(d))) if d.size else 0.0,
                      "rel": float(np.linalg.norm(d) / nref) if nref > 0 else 0.0}
    out["eta"] = [float(e) for e in M.eta]
    out["reference"] = "host FP64 CSR (scipy), x = 1"
    return out


def solution_error(x, x_true):
    return float(np.linalg.norm(x - x_true) / np.linalg.norm(x_true))


def solve_record(rep, x_dev, x_true):
    d = rep.as_dict()
    d["x_err"] = solution_error(x_dev.cpu().numpy(), x_true)
    return d


def rotated_launch_us(torch, stream, launches, reps=10):
    """Mean time per launch (us) of `launches` (one closure per resident
    copy) run back to back in rounds, HIP events around each round."""
    for f in launches:
        f()
    ev = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for f in launches:
            f()
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev])) * 1e3 / len(launches)


def host_product_errors(y_dev, ref):
    d = y_dev.cpu().numpy() - ref
    nref = float(np.linalg.norm(ref))
    with np.errstate(invalid="ignore"):
        return {"max_abs": float(np.max(np.abs(d))) if d.size else 0.0,
                "rel": float(np.linalg.norm(d) / nref) if nref > 0 else 0.0}


def leg_k_sweep(torch, G, A, copies, ks=(2, 4, 8, 16, 32, 64)):
    """The k sweep of Section IV-B: the head-only SpMV with tables of k
    shared exponents (slot index of ceil(log2 k) bits): time per launch over
    `copies` rotated copies, and max-abs / relative error against the host
    FP64 product with x = 1, eta_1 and the share of exactly represented
    exponents."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ref = A.to_scipy() @ np.ones(A.n_cols)
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    xs = torch.ones(A.n_cols, dtype=torch.float64, device=dev)
    ys = [torch.empty(A.n_rows, dtype=torch.float64, device=dev) for _ in range(copies)]
    out = {}
    for k in ks:
        mats = [G.GseMatrix(rp.clone(), ci, va, A.n_cols, num_exp=k) for _ in range(copies)]
        us = rotated_launch_us(torch, stream,
                               [lambda m=m, y=y: m.spmv(1, xs, y) for m, y in zip(mats, ys)])
        mats[0].spmv(1, xs, ys[0])
        torch.cuda.synchronize()
        nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, 6)
        out[str(k)] = {"idx_bits": mats[0].A.idx_bits, "s1_us": round(us, 2),
                       "GBps": round(nbytes / (us * 1e-6) / 1e9, 1),
                       **host_product_errors(ys[0], ref), "eta1": float(mats[0].eta[0]),
                       "exact_frac": round(float(mats[0].A.exact_frac), 4)}
        del mats
    return out


def componentwise_errors(y_dev, ref, absref):
    """Row-wise error |y - ref| / (|A| |x|) of one product: percentiles."""
    y = y_dev.cpu().numpy()
    e = np.abs(y - ref) / np.where(absref > 0, absref, 1.0)
    return {"p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99)),
            "max": float(e.max())}


def leg_blocks(torch, G, seed, copies, block_rows=4096, A_cg=None, b_cg=None, x_true_cg=None):
    """Per-row-block tables (Section III-B.1, sampling) on the layered medium
    (128^3, 16 slabs whose coefficients sit at levels spread over eight
    decades, one decade within a slab): encode time of the global table, of
    exact block tables, of tables from one drawn row per block and of one
    table from those drawn rows pooled; SpMV time
    per segment count over rotated copies (each on its default schedule);
    error against the host FP64 product with x = 1,
    norm-wise and per row; eta_s and the share of exactly represented
    exponents.  With A_cg given, also the stepped CG on that system with
    exact block tables."""
    from workloads import block_sample_rows, layered3d

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    A = layered3d(128, seed)
    S = A.to_scipy()
    ref = S @ np.ones(A.n_cols)
    absref = abs(S) @ np.ones(A.n_cols)
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    sr = torch.from_numpy(block_sample_rows(A.n_rows, block_rows, seed)).to(dev)
    xs = torch.ones(A.n_cols, dtype=torch.float64, device=dev)
    ys = [torch.empty(A.n_rows, dtype=torch.float64, device=dev) for _ in range(copies)]
    variants = {"global": {}, "blocks_exact": {"block_rows": block_rows},
                "blocks_sampled": {"block_rows": block_rows, "sample_rows": sr},
                "global_sampled": {"block_rows": block_rows, "sample_rows": sr, "pooled": True}}
    out = {"workload": "layered3d_128^3_7pt_16slabs_8+1decades", "n_rows": A.n_rows,
           "nnz": A.nnz, "block_rows": block_rows, "seed": seed, "x": "ones"}
    for name, kw in variants.items():
        mats = [G.GseMatrix(rp.clone(), ci, va, A.n_cols, **kw) for _ in range(copies)]
        M = mats[0]
        # encode time: the same call again on the first copy's buffers
        enc_ms = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kw.get("pooled"):
                G.gse_encode_sampled(M.row_ptr, ci, va, A.n_rows, A.n_cols, A.nnz, 8, block_rows,
                                     kw["sample_rows"], M.A, M.ws)
            elif kw:
                G.gse_encode_blocks(M.row_ptr, ci, va, A.n_rows, A.n_cols, A.nnz, 8, block_rows,
                                    kw.get("sample_rows"), M.A, M.ws)
            else:
                G.gse_encode(M.row_ptr, ci, va, A.n_rows, A.n_cols, A.nnz, 8, None, M.A, M.ws)
            enc_ms.append((time.perf_counter() - t0) * 1e3)
        rec = {"encode_ms": round(float(np.median(enc_ms)), 3), "eta": [float(e) for e in M.eta],
               "exact_frac": round(float(M.A.exact_frac), 4), "rv_lanes": int(M.A.rv_lanes),
               "kernel": kernel_name(M.A)}
        tables = (G.gse_block_table_entries(A.n_rows, block_rows, 8) * 2) if M.A.block_rows else 0
        for s, pb in ((1, 6), (2, 8), (3, 12)):
            us = rotated_launch_us(torch, stream,
                                   [lambda m=m, y=y, s=s: m.spmv(s, xs, y) for m, y in zip(mats, ys)])
            M.spmv(s, xs, ys[0])
            torch.cuda.synchronize()
            nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, pb) + tables
            rec[f"s{s}"] = {"mean_us": round(us, 2), "GBps": round(nbytes / (us * 1e-6) / 1e9, 1),
                            **host_product_errors(ys[0], ref),
                            "rowwise": componentwise_errors(ys[0], ref, absref)}
        out[name] = rec
        del mats
    del rp, ci, va, ys
    if A_cg is not None:
        rp = torch.from_numpy(A_cg.indptr).to(dev)
        ci = torch.from_numpy(A_cg.indices).to(dev)
        va = torch.from_numpy(A_cg.data).to(dev)
        M = G.GseMatrix(rp, ci, va, A_cg.n_cols, block_rows=block_rows)
        bd = torch.from_numpy(b_cg).to(dev)
        p = G.gse_default_params(G.CG)
        p.max_iter = 20000
        ws = torch.empty(G.gse_solver_workspace(G.CG, A_cg.n_rows, A_cg.nnz, 30, p.max_iter),
                         dtype=torch.uint8, device=dev)
        x = torch.zeros(A_cg.n_rows, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        rep = G.gse_cg(M.A, bd, x, p, ws)
        out["cg_diffusion3d_128_blocks_exact"] = {**solve_record(rep, x, x_true_cg),
                                                  "eta": [float(e) for e in M.eta],
                                                  "rv_lanes": int(M.A.rv_lanes)}
    return out


def leg_lowprec_spmv(torch, G, A, copies):
    """FP16- and BF16-SpMV (Section IV-C): time per launch over rotated
    copies, error against the host FP64 product with x = 1, eta_h and the
    number of values that overflowed to infinity."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ref = A.to_scipy() @ np.ones(A.n_cols)
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    xs = torch.ones(A.n_cols, dtype=torch.float64, device=dev)
    ys = [torch.empty(A.n_rows, dtype=torch.float64, device=dev) for _ in range(copies)]
    out = {}
    for name, fmt in (("fp16", G.LP_FP16), ("bf16", G.LP_BF16)):
        mats = [G.LpMatrix(rp.clone(), ci, va, A.n_cols, fmt=fmt) for _ in range(copies)]
        us = rotated_launch_us(torch, stream,
                               [lambda m=m, y=y: m.spmv(xs, y) for m, y in zip(mats, ys)])
        mats[0].spmv(xs, ys[0])
        torch.cuda.synchronize()
        nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, 6)
        out[name] = {"mean_us": round(us, 2), "GBps": round(nbytes / (us * 1e-6) / 1e9, 1),
                     **host_product_errors(ys[0], ref), "eta": float(mats[0].M.eta),
                     "overflow": int(mats[0].M.overflow)}
        del mats
    return out


def leg_lowprec_solve(torch, G, A, b, x_true, method, gse_rep, fp64_rep):
    """The FP16 / BF16 solver comparators (Section IV-D.3) on the same system:
    iterations, time, the residual of their own operator and the true one,
    and the Eq. 7 projection of the stepped GSE solve without conversion
    cost: (time / iterations of FP16) x iterations of GSE, against FP64."""
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    bd = torch.from_numpy(b).to(dev)
    p = G.gse_default_params(method)
    if method == G.CG:
        p.max_iter = 20000
    ws = torch.empty(G.gse_solver_workspace(method, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=dev)
    fn = G.gse_lp_gmres if method == G.GMRES else G.gse_lp_cg
    out = {}
    for name, fmt in (("fp16", G.LP_FP16), ("bf16", G.LP_BF16)):
        M = G.LpMatrix(rp, ci, va, A.n_cols, fmt=fmt)
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
        fn(M.M, bd, x, p, ws)  # warm-up (graph capture)
        x.zero_()
        torch.cuda.synchronize()
        rep = fn(M.M, bd, x, p, ws)
        xh = x.cpu().numpy()
        d = rep.as_dict()
        d["relres_fp64"] = float(np.linalg.norm(b - A.to_scipy() @ xh) / np.linalg.norm(b))
        d["x_err"] = solution_error(xh, x_true)
        d["overflow"] = int(M.M.overflow)
        out[name] = d
    f16 = out["fp16"]
    if f16["iters"] > 0 and f16["time_ms"] > 0:
        star = f16["time_ms"] / f16["iters"] * gse_rep["iters"]
        out["gse_star_eq7"] = {"time_ms": round(star, 3),
                               "speedup_vs_fp64": round(fp64_rep["time_ms"] / star, 3),
                               "speedup_gse_measured": round(fp64_rep["time_ms"] /
                                                             gse_rep["time_ms"], 3)}
    return out


# ---------------------------------------------------------------- GMRES ---
def leg_gmres(torch, G, seed, steps, warmup, N=1024):
    """Stepped GMRES(30) and FP64 GMRES(30) to 1e-10 on the 2-D upwind
    convection-diffusion operator (N^2 cells, cell Peclet 10)."""
    from workloads import convdiff2d, rhs_from_solution

    dev = torch.device("cuda:0")
    A = convdiff2d(N, seed)
    x_true, b = rhs_from_solution(A, seed)
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    C = G.CsrMatrix(rp, ci, va, A.n_cols)
    bd = torch.from_numpy(b).to(dev)
    p = G.gse_default_params(G.GMRES)
    ws = torch.empty(G.gse_solver_workspace(G.GMRES, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=dev)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
    progress("gmres: operators ready")
    for _ in range(warmup):
        x.zero_()
        G.gse_gmres(M.A, bd, x, p, ws)
        x.zero_()
        G.gse_csr_gmres(C.M, bd, x, p, ws)
    runs = {"gse": [], "fp64": []}
    res = {}
    for _ in range(steps):
        x.zero_()
        torch.cuda.synchronize()
        res["gse"] = solve_record(G.gse_gmres(M.A, bd, x, p, ws), x, x_true)
        progress(f"gmres: GSE {res['gse']}")
        x.zero_()
        torch.cuda.synchronize()
        res["fp64"] = solve_record(G.gse_csr_gmres(C.M, bd, x, p, ws), x, x_true)
        for k in runs:
            runs[k].append(res[k]["time_ms"])
    med = {k: float(np.median(v)) for k, v in runs.items()}
    errs = spmv_errors(A, M, C, np.ones(A.n_cols), dev, torch)
    del M, C, ws
    return {"workload": f"convdiff2d_{N}^2_upwind_Pe10", "n_rows": A.n_rows, "nnz": A.nnz,
            "seed": seed, "restart": p.restart, "gse": res["gse"], "fp64": res["fp64"],
            "median_ms": {k: round(v, 3) for k, v in med.items()},
            "speedup": round(med["fp64"] / med["gse"], 3) if med["gse"] else None,
            "spmv_error": errs,
            "lowprec_gmres": leg_lowprec_solve(torch, G, A, b, x_true, G.GMRES, res["gse"],
                                               res["fp64"])}


def run_gmres(args, torch, G):
    t0 = time.perf_counter()
    leg = leg_gmres(torch, G, args.seed, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    out = base_record(args, "GMRES(30) time-to-1e-10, stepped GSE vs FP64 CSR",
                      round(leg["median_ms"]["gse"], 3), "ms", wall, higher=False)
    out["config"] = {k: leg[k] for k in ("workload", "n_rows", "nnz", "seed", "restart")}
    out["gmres"] = leg
    return out


# ------------------------------------------------------------ power law ---
def leg_powerlaw(torch, G, seed, steps, warmup, reps, n_rows, extras=True):
    """Power-law SPD matrix (Zipf(2) row lengths up to 10^4, values over six
    decades): SpMV per segment count after the autotuner picked the tile
    shape (the planes, 0.4-0.8 GB, exceed the Infinity Cache, so every launch
    is cold without rotated copies), their errors, then stepped GSE CG vs
    FP64 CG to 1e-10."""
    from workloads import powerlaw, rhs_from_solution

    dev = torch.device("cuda:0")
    A = powerlaw(n_rows, seed)
    x_true, b = rhs_from_solution(A, seed)
    progress(f"powerlaw: {A.n_rows} rows, {A.nnz} non-zeros generated")
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    C = G.CsrMatrix(rp, ci, va, A.n_cols)
    del ci, va
    xs = torch.ones(A.n_cols, dtype=torch.float64, device=dev)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=dev)
    M.autotune(1, xs, y)
    C.autotune(xs, y)
    stream = torch.cuda.current_stream()
    progress(f"powerlaw: autotuned tile_nnz {M.A.tile_nnz} rv_lanes {M.A.rv_lanes}")
    kinds = [("s1", 6), ("s2", 8), ("s3", 12), ("fp64", 12)]
    times = {k: [] for k, _ in kinds}

    def run(kname):
        if kname == "fp64":
            C.spmv(xs, y)
        else:
            M.spmv(int(kname[1]), xs, y)

    # CG runs on the symmetrically diagonal-scaled system D^-1/2 A D^-1/2 z =
    # D^-1/2 b, x = D^-1/2 z (unit diagonal; Jacobi-preconditioned CG in exact
    # arithmetic): the rows' scales span six decades, and plain CG on A itself
    # stalls near 4e-6 at the 5000-iteration cap.  Its Gershgorin bound gives
    # kappa <= 21.
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    diag = np.zeros(A.n_rows)
    on = rows == A.indices
    diag[rows[on]] = A.data[on]
    dinv = 1.0 / np.sqrt(diag)
    sval = A.data * dinv[rows] * dinv[A.indices]
    del rows, on
    sv = torch.from_numpy(sval).to(dev)
    sc = torch.from_numpy(A.indices).to(dev)
    MS = G.GseMatrix(rp, sc, sv, A.n_cols)
    CS = G.CsrMatrix(rp, sc, sv, A.n_cols)
    MS.autotune(1, xs, y)
    CS.autotune(xs, y)
    del sv, sc, sval
    bd = torch.from_numpy(b * dinv).to(dev)
    z_true = x_true / dinv
    p = G.gse_default_params(G.CG)
    ws = torch.empty(G.gse_solver_workspace(G.CG, A.n_rows, A.nnz, 30, p.max_iter),
                     dtype=torch.uint8, device=dev)
    z = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
    cg_runs = {"gse": [], "fp64": []}

    def step(record):
        for kname, _ in kinds:
            for _ in range(reps):
                if record:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                run(kname)
                if record:
                    e1.record(stream)
                    times[kname].append((e0, e1))
        z.zero_()
        torch.cuda.synchronize()  # the SpMV launches above are not part of the solve
        rg = solve_record(G.gse_cg(MS.A, bd, z, p, ws), z, z_true)
        z.zero_()
        torch.cuda.synchronize()
        r64 = solve_record(G.gse_csr_cg(CS.M, bd, z, p, ws), z, z_true)
        if record:
            cg_runs["gse"].append(rg)
            cg_runs["fp64"].append(r64)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    spmv = {}
    for kname, pb in kinds:
        ms = np.array([a.elapsed_time(c) for a, c in times[kname]])
        nbytes = spmv_bytes(A.n_rows, A.n_cols, A.nnz, pb)
        mean = float(ms.mean())
        spmv[kname] = {"mean_us": round(mean * 1e3, 2),
                       "median_us": round(float(np.median(ms)) * 1e3, 2),
                       "bytes": int(nbytes), "GBps": round(nbytes / (mean * 1e-3) / 1e9, 1),
                       "frac_peak": round(nbytes / (mean * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    med = {k: float(np.median([r["time_ms"] for r in v])) for k, v in cg_runs.items()}
    errs = spmv_errors(A, M, C, np.ones(A.n_cols), dev, torch)
    kname = kernel_name(M.A)
    tile, rv = M.A.tile_nnz, M.A.rv_lanes
    eta_scaled = [float(e) for e in MS.eta]
    del M, C, MS, CS, ws
    lowprec = ksweep = None
    if extras:
        progress("powerlaw: FP16 / BF16 SpMV and the k sweep")
        lowprec = leg_lowprec_spmv(torch, G, A, 1)
        ksweep = leg_k_sweep(torch, G, A, 1)
    return {"workload": f"powerlaw_{A.n_rows}_zipf2_spd", "n_rows": A.n_rows, "nnz": A.nnz,
            "max_row": int(np.diff(A.indptr).max()), "seed": seed, "x": "ones",
            "tile_nnz": tile, "rv_lanes": rv, "kernel": kname,
            "spmv": spmv, "spmv_error": errs, "lowprec_spmv": lowprec, "k_sweep": ksweep,
            "cg": {"system": "D^-1/2 A D^-1/2 z = D^-1/2 b (unit diagonal); x_err on z",
                   "gse": cg_runs["gse"][-1], "fp64": cg_runs["fp64"][-1],
                   "median_ms": {k: round(v, 3) for k, v in med.items()},
                   "speedup": round(med["fp64"] / med["gse"], 3) if med["gse"] else None,
                   "eta_scaled": eta_scaled},
            "wall_s": wall}


def run_powerlaw(args, torch, G):
    t0 = time.perf_counter()
    leg = leg_powerlaw(torch, G, args.seed, args.steps, args.warmup, args.reps, args.pl_rows,
                       extras=args.legs)
    wall = time.perf_counter() - t0
    spmv = leg["spmv"]
    out = base_record(args, "GSE-SpMV HBM GB/s (s=1), power-law SPD; CG time-to-1e-10 vs FP64 CSR",
                      spmv["s1"]["GBps"], "GB/s", leg["wall_s"])
    out["config"] = {k: leg[k] for k in ("workload", "n_rows", "nnz", "max_row", "seed", "x",
                                         "tile_nnz", "rv_lanes")}
    out["spmv"] = spmv
    out["spmv_error"] = leg["spmv_error"]
    out["roofline"] = {"bound": "hbm", "achieved": spmv["s1"]["GBps"], "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": spmv["s1"]["frac_peak"], "traffic": None,
                       "kernel": leg["kernel"], "bytes_per_launch": spmv["s1"]["bytes"],
                       "mean_launch_us": spmv["s1"]["mean_us"]}
    out["cg"] = leg["cg"]
    out["total_wall_s"] = round(wall, 2)
    return out


# -------------------------------------------------------------- Poisson ---
def leg_poisson(torch, G, seed, steps, warmup):
    """2-D Poisson 64 x 64 (exact stencil values, eta_1 = 0): stepped GSE CG
    and FP64 CG to 1e-10; the system is L2-resident, so this measures the
    launch-bound regime (median over the runs)."""
    from workloads import poisson2d, rhs_from_solution

    dev = torch.device("cuda:0")
    A = poisson2d(64)
    x_true, b = rhs_from_solution(A, seed)
    rp = torch.from_numpy(A.indptr).to(dev)
    ci = torch.from_numpy(A.indices).to(dev)
    va = torch.from_numpy(A.data).to(dev)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    C = G.CsrMatrix(rp, ci, va, A.n_cols)
    bd = torch.from_numpy(b).to(dev)
    p = G.gse_default_params(G.CG)
    ws = torch.empty(G.gse_solver_workspace(G.CG, A.n_rows, A.nnz, 30, p.max_iter),
                     dtype=torch.uint8, device=dev)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
    runs = {"gse": [], "fp64": []}

    def step():
        x.zero_()
        torch.cuda.synchronize()
        rg = solve_record(G.gse_cg(M.A, bd, x, p, ws), x, x_true)
        x.zero_()
        torch.cuda.synchronize()
        return rg, solve_record(G.gse_csr_cg(C.M, bd, x, p, ws), x, x_true)

    for _ in range(warmup):
        step()
    for _ in range(steps):
        rg, r64 = step()
        runs["gse"].append(rg)
        runs["fp64"].append(r64)
    med = {k: float(np.median([r["time_ms"] for r in v])) for k, v in runs.items()}
    return {"workload": "poisson2d_64^2_5pt", "n_rows": A.n_rows, "nnz": A.nnz, "seed": seed,
            "gse": runs["gse"][-1], "fp64": runs["fp64"][-1],
            "median_ms": {k: round(v, 3) for k, v in med.items()},
            "speedup": round(med["fp64"] / med["gse"], 3) if med["gse"] else None,
            "spmv_error": spmv_errors(A, M, C, np.ones(A.n_cols), dev, torch)}


def run_poisson(args, torch, G):
    t0 = time.perf_counter()
    leg = leg_poisson(torch, G, args.seed, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    out = base_record(args, "CG time-to-1e-10, stepped GSE vs FP64 CSR (2-D Poisson 64x64)",
                      round(leg["median_ms"]["gse"], 3), "ms", wall, higher=False)
    out["config"] = {k: leg[k] for k in ("workload", "n_rows", "nnz", "seed")}
    out["cg"] = leg
    return out


# ---------------------------------------------------------------- batch ---
def run_batch(args, torch, G):
    """One batch of K 3-D diffusion systems (grid^3 each, own coefficients
    and right-hand side per system, below the size that takes the row-tile
    ring's product), solved together by the batched CG at a fixed segment
    count, then the same systems as FP64 CSR.  Reports solve time, the
    iterations and the algorithmic bytes of one batched product at each
    segment count (every system's planes, row pointers, p and q once), the
    figure the batched product's kernel time is divided by.  A fixed count
    below 3 floors the true residual near its eta (about 5e-10 at s = 2 on
    these systems), so such runs end NOT_CONVERGED: they measure the product,
    the stepped default the time to 1e-10."""
    from workloads import diffusion3d, rhs_from_solution

    dev = torch.device("cuda:0")
    K, s = args.batch_systems, args.batch_segments
    mats, rhs = [], []
    for i in range(K):
        A = diffusion3d(args.batch_grid, args.seed + i)
        _, b = rhs_from_solution(A, args.seed + i)
        mats.append(A)
        rhs.append(torch.from_numpy(b).to(dev))
    progress(f"batch: {K} systems of {mats[0].n_rows} rows generated")
    res = {}
    t0 = time.perf_counter()
    kinds = [k for k in args.batch_kinds.split(",") if k]
    if not kinds or any(k not in ("gse", "fp64") for k in kinds):
        raise SystemExit(f"--batch-kinds: gse and/or fp64, not {args.batch_kinds!r}")
    for kind in kinds:
        holders, triples = [], []
        for A, b in zip(mats, rhs):
            rp = torch.from_numpy(A.indptr).to(dev)
            ci = torch.from_numpy(A.indices).to(dev)
            va = torch.from_numpy(A.data).to(dev)
            H = G.GseMatrix(rp, ci, va, A.n_cols) if kind == "gse" else G.CsrMatrix(rp, ci, va, A.n_cols)
            x = torch.zeros(A.n_rows, dtype=torch.float64, device=dev)
            holders.append((H, rp, ci, va))
            triples.append((H.A if kind == "gse" else H.M, b, x))
        p = G.gse_default_params(G.CG)
        p.max_iter = 20000
        p.fixed_segments = s if kind == "gse" else 0
        ws = torch.empty(G.gse_batch_workspace(triples, p), dtype=torch.uint8, device=dev)
        times = []
        for rep in range(args.warmup + args.steps):
            for _, _, x in triples:
                x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            reps = G.gse_batch_cg(triples, p, ws)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                times.append((time.perf_counter() - t) * 1e3)
        segs = (1, 2, 3) if kind == "gse" else (0,)
        nbytes = {f"s{k}" if k else "fp64":
                  int(sum(spmv_bytes(A.n_rows, A.n_cols, A.nnz, {0: 12, 1: 6, 2: 8, 3: 12}[k])
                          for A in mats)) for k in segs}
        res[kind] = {"solve_ms": round(float(np.median(times)), 3),
                     "iters": [int(r.iters) for r in reps],
                     "iters_per_seg_total": [int(sum(r.iters_per_seg[k] for r in reps))
                                             for k in range(3)],
                     "status": [int(r.status) for r in reps],
                     "relres_true_max": float(max(r.relres_true for r in reps)),
                     "product_bytes": nbytes}
        progress(f"batch: {kind} {res[kind]['solve_ms']} ms, iterations "
                 f"{min(res[kind]['iters'])}-{max(res[kind]['iters'])}")
        del holders, triples, ws
    wall = time.perf_counter() - t0
    label = "stepped GSE" if s == 0 else f"GSE s={s}"
    first = res[kinds[0]]
    out = base_record(args, f"batched CG time-to-1e-10, {K} systems, {label} vs FP64 CSR",
                      first["solve_ms"], "ms", wall, higher=False)
    if "gse" in res and "fp64" in res:
        out["speedup"] = round(res["fp64"]["solve_ms"] / res["gse"]["solve_ms"], 3)
    out["config"] = {"workload": f"{K}x diffusion3d_{args.batch_grid}^3_7pt_varcoef_4decades",
                     "n_rows_each": mats[0].n_rows, "nnz_each": mats[0].nnz,
                     "fixed_segments": s, "seed": args.seed}
    out["batch"] = res
    return out


# -------------------------------------------------------------- serving ---
def run_serving(args, torch, G):
    from workloads import rhs_from_solution, serving_request_matrix, serving_stream

    dev = torch.device("cuda:0")
    stream_def = serving_stream(args.seed, count=args.requests, n_lo=1e3, n_hi=args.n_hi)
    systems = []
    for r in stream_def:
        A = serving_request_matrix(r)
        _, b = rhs_from_solution(A, r["seed"])
        systems.append((A, b))
        if len(systems) % 250 == 0:
            progress(f"serving: {len(systems)} of {len(stream_def)} requests generated")
    p = G.gse_default_params(G.CG)
    p.max_iter = 20000
    arena = torch.empty(int(args.arena_gb * (1 << 30)), dtype=torch.uint8, device=dev)

    def run(fmt, slots, gaps):
        """Submit every request after its gap (open loop); latencies in ms."""
        server = G.gse_solver_create(arena, slots)
        try:
            reqs = [G.Request(A, b, fmt, params=p) for A, b in systems]
            tickets, done = [], {}
            t0 = time.perf_counter()
            due = t0
            for rq, gap in zip(reqs, gaps):
                due += gap
                while time.perf_counter() < due:
                    for t in tickets:
                        if t not in done:
                            r = G.gse_solver_poll(server, t)
                            if r is not None:
                                done[t] = (r, time.perf_counter())
                    time.sleep(0.0005)
                tickets.append(G.gse_solver_submit(server, rq.rq))
                if len(tickets) % 250 == 0:
                    progress(f"serving: {len(tickets)} submitted, {len(done)} done")
            reported = len(done) // 250
            while len(done) < len(tickets):
                for t in tickets:
                    if t not in done:
                        r = G.gse_solver_poll(server, t)
                        if r is not None:
                            done[t] = (r, time.perf_counter())
                if len(done) // 250 > reported:
                    reported = len(done) // 250
                    progress(f"serving: {len(done)} of {len(tickets)} done")
                time.sleep(0.0005)
            t_end = max(v[1] for v in done.values())
            stats = G.gse_solver_stats(server).as_dict()
        finally:
            G.gse_solver_destroy(server)
        reps = [done[t][0] for t in tickets]
        lat = np.array([r.time_ms for r in reps])
        ok = sum(1 for r in reps if r.status == G.OK)
        return {"solves_per_s": round(len(reps) / (t_end - t0), 2),
                "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "converged": ok, "requests": len(reps), "peak_arena_GB":
                    round(stats["arena_peak"] / 2**30, 3)}, [rq.x.copy() for rq in reqs]

    t0 = time.perf_counter()
    zero = [0.0] * len(systems)
    progress(f"serving: {len(systems)} requests generated; FP64 one at a time")
    base, _ = run(G.FMT_CSR64, 1, zero)  # closed loop: the one-at-a-time throughput
    lam = base["solves_per_s"]
    progress(f"serving: FP64 one at a time {base}")
    rng = np.random.default_rng(args.seed + 1)
    levels = {}
    xs_mix = None
    for f in (0.5, 1.0, 2.0):
        gaps = list(rng.exponential(1.0 / (f * lam), size=len(systems)))
        levels[f"{f}x"], xs = run(G.FMT_GSE, args.slots, gaps)
        progress(f"serving: GSE batched at {f}x: {levels[f'{f}x']}")
        if f == 2.0:
            xs_mix = xs
    # the same requests one at a time through the same server: same bits
    _, xs_alone = run(G.FMT_GSE, 1, zero)
    bitwise = all(np.array_equal(a, b) for a, b in zip(xs_mix, xs_alone))
    wall = time.perf_counter() - t0
    out = base_record(args, "serving solves/s at 1x the one-at-a-time FP64 rate (stepped GSE, batched)",
                      levels["1.0x"]["solves_per_s"], "solves/s", wall)
    out["steps"] = 1
    out["warmup"] = 0
    ns = [A.n_rows for A, _ in systems]
    out["config"] = {"workload": f"serving_poisson_arrivals_{len(systems)}req_n1e3..{args.n_hi:.0e}_2d3d_diffusion",
                     "mean_n": int(np.mean(ns)), "max_n": int(max(ns)), "slots": args.slots,
                     "arena_GB": args.arena_gb, "tol": 1e-10}
    out["serving"] = {"fp64_one_at_a_time": base, "gse_batched": levels,
                      "alone_vs_mix_bitwise": bool(bitwise)}
    return out


def json_safe(v):
    """Non-finite floats as strings ("inf", "-inf", "nan"): the line stays strict JSON."""
    if isinstance(v, float) and not np.isfinite(v):
        return "nan" if np.isnan(v) else ("inf" if v > 0 else "-inf")
    if isinstance(v, dict):
        return {k: json_safe(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [json_safe(x) for x in v]
    return v


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    import torch

    from paper_2411_04686_amd import gse as G
    G.lib()
    if args.workload == "gmres":
        out = run_gmres(args, torch, G)
    elif args.workload == "serving":
        out = run_serving(args, torch, G)
    elif args.workload == "powerlaw":
        out = run_powerlaw(args, torch, G)
    elif args.workload == "poisson":
        out = run_poisson(args, torch, G)
    elif args.workload == "batch":
        out = run_batch(args, torch, G)
    elif args.workload == "blocks":
        t0 = time.perf_counter()
        leg = leg_blocks(torch, G, args.seed, args.copies)
        out = base_record(args, "GSE-SpMV with per-row-block tables, s=1 GB/s",
                          leg["blocks_sampled"]["s1"]["GBps"], "GB/s", time.perf_counter() - t0)
        out["config"] = {"workload": leg["workload"], "n_rows": leg["n_rows"], "nnz": leg["nnz"],
                         "block_rows": leg["block_rows"]}
        out["blocks"] = leg
    else:
        out = run_spmv_cg(args, torch, G)
    print(json.dumps(json_safe(out), allow_nan=False))


if __name__ == "__main__":
    main()
