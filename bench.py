#!/usr/bin/env python3
"""Benchmark: generalized canonical purification on one MI355X.

Workload: dense H = Q diag(lam) Q^T, M = 8192, N = 3000, eigenvalues uniform in
[-1, -0.025] U [0.025, 1] (gap 0.05), Q from the QR of a seeded Gaussian
matrix, bounds [-1, 1].  One step = one whole solve on the GPU: the initial
guess from H (already resident in HBM) plus the purification to convergence
(|Tr(D Dbar)| <= 1e-6) with D written to a caller buffer.

Reported: throughput of the mixed-precision path in algorithmic TFLOP/s
(M^2 (M+1) per symmetric product, every product launched counted once),
its time to solution, the FP64 GPU path's time to solution on the same input,
both errors ||D - D_ref||_F / sqrt(M) against the closed-form projector, the
roofline of the dominant kernel (the product kernel) and the CPU oracle timed
on a bounded sample of the same workload.  The adjoint of the mixed solve
(gcp_backward in FP32, loss u^T D u) and the FP64 acceptance checks of its
result (gcp_verify: trace, idempotency, energy against the sum of the N lowest
eigenvalues, commutator with H) are reported alongside as extra information,
as is a scheduled solve (the mixed encoding, then FP64 once |Tr(D Dbar)| <= 1e-2,
stopping at 1e-9; near convergence Tr(D Dbar) falls by orders of magnitude per
update, so the switch must come before the mixed encoding reaches its floor).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("GCP TFLOP/s & time-to-solution at M=8192, mixed vs FP64, at "
          "‖D−D_ref‖≤1e-6")
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def product_kernel_hash() -> str:
    """sha256 of the source the 16-bit product kernel is built from: its text
    in gcp_kernels.hip and the headers it includes from the package."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1512_07236_amd", "csrc")
    k = open(os.path.join(csrc, "gcp_kernels.hip")).read()
    a = k.index("// ------------------------------------------------ 16-bit product kernel")
    b = k.index("int pair_count(int nt)")
    h = hashlib.sha256(k[a:b].encode())
    for f in ("gcp_encode.h", "gcp_mma.h", "gcp_kernels.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def pmc_traffic(kernel_tag: str):
    """HBM bytes per launch of the product kernel from the committed rocprofv3
    counter summary (profiles/<kernel_tag>_pmc.json), or None when absent or
    taken from a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        if d.get("kernel_source_sha256") != product_kernel_hash():
            return None
        return float(d["hbm_bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(w, iters_per_solve: int, launches_per_solve: int, budget_s: float):
    """Time the oracle's plain-C FP64 product on a bounded row sample of D0 D0
    at the full size, scaled to TFLOP/s and to an extrapolated solve time."""
    import oracle
    oracle.build(force=False)
    D0, _, _ = oracle.initial_guess(w.H, w.N, w.emin, w.emax)
    M = w.M
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    r = max(threads, 16)
    t0 = time.perf_counter()
    oracle.matmul_rows(D0, D0, 0, r)
    t_probe = time.perf_counter() - t0
    rows = int(min(M, max(r, r * (budget_s / max(t_probe, 1e-3)))))
    rows = max(r, rows // r * r)
    t0 = time.perf_counter()
    oracle.matmul_rows(D0, D0, r, r + rows) if r + rows <= M else oracle.matmul_rows(D0, D0, 0, rows)
    t = time.perf_counter() - t0
    flops = 2.0 * rows * M * M
    tflops = flops / t / 1e12
    product_s = t * (M / rows)
    return {
        "value": tflops, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
        "sample": f"rows {rows} of the {M}x{M} FP64 product D0*D0 (plain C i-k-j loop, OpenMP), "
                  f"{t:.1f} s",
        "extrapolated_time_to_solution_s": product_s * launches_per_solve,
    }


COPY_BYTES = 1 << 30


def copy_calibration() -> None:
    """A plain device-to-device copy of exactly COPY_BYTES (read COPY_BYTES,
    write COPY_BYTES): the yardstick for the memory-traffic counters."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def _counter_rows(d: str):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    return rows


def summarize_pmc(precision: str, scale: int, fetch_dir: str, write_dir: str) -> int:
    """profiles/<kernel>_pmc.json from FETCH_SIZE / WRITE_SIZE runs (KiB per
    dispatch), each scaled by what the same counter reads for the 1 GiB copy."""
    import hashlib
    import paper_1512_07236_amd as gcp
    prec = gcp.Precision.parse(precision)
    M = 8192 // scale
    kname = "k_gemm16" if gcp.PRODUCTS[prec] > 1 or prec in (gcp.Precision.BF16, gcp.Precision.FP16) else "k_gemm"
    tag = f"gemm_{prec.name.lower()}_M{M}"
    out = {"kernel": f"{kname}<{int(prec)}>", "workload": f"M={M}", "precision": prec.name.lower()}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == name]
        kern = [float(r["Counter_Value"]) for r in rows if f"{kname}<{int(prec)}>" in r["Kernel_Name"]]
        # the calibration copy: FETCH_SIZE reads about half of its true bytes
        # (WRITE_SIZE all of them), so accept copy kernels above a quarter
        copy = [float(r["Counter_Value"]) for r in rows
                if ("copy" in r["Kernel_Name"].lower() or "elementwise" in r["Kernel_Name"].lower())
                and float(r["Counter_Value"]) * 1024 > 0.25 * COPY_BYTES]
        if not kern or not copy:
            print(f"no {name} rows for the kernel or the copy in {d}", file=sys.stderr)
            return 1
        factor = (max(copy) * 1024) / COPY_BYTES   # counter bytes per true byte
        out[name] = {"kib_per_launch_raw": sum(kern) / len(kern), "launches": len(kern),
                     "copy_kib_raw": max(copy), "copy_factor": factor,
                     "bytes_per_launch": sum(kern) / len(kern) * 1024 / factor}
    out["hbm_bytes_per_launch"] = out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"]
    out["kernel_source_sha256"] = product_kernel_hash()
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    path = os.path.join(ROOT, "profiles", f"{tag}_pmc.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16x3")
    ap.add_argument("--fold-every", type=int, default=0)
    ap.add_argument("--tol", type=float, default=None,
                    help="|Tr(D Dbar)| stop; default 1e-5 for the split 16-bit encodings "
                         "(their rounding floor at M=8192 is ~1e-6) and 1e-6 otherwise")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--bwd-steps", type=int, default=1,
                    help="timed adjoints (gcp_backward, FP32) of the mixed solve for L = u^T D u")
    ap.add_argument("--scale", type=int, default=1, help="divide M by this (quick runs only)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (the reference kernel that scales "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE to bytes)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "'bench.py --copy-calibration' into profiles/<kernel>_pmc.json and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        return summarize_pmc(args.precision, args.scale, *args.pmc_summary)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the purification path here runs on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_1512_07236_amd as gcp
    import workloads
    import oracle

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)

    log("[bench] generating workload (seeded)")
    w = workloads.config(3, scale=args.scale)
    M, N = w.M, w.N
    H = torch.from_numpy(w.H).cuda()
    log("[bench] reference projector (closed form)")
    D_ref = oracle.projector_from_spectrum(w.Q, w.lam, N)

    prec = gcp.Precision.parse(args.precision)
    mfma_dtype = gcp.MFMA_DTYPE[prec]

    def tol_for(p):
        if args.tol is not None:
            return args.tol
        return 1e-5 if gcp.PRODUCTS[gcp.Precision.parse(p)] > 1 else 1e-6

    def run(precision, steps, warmup, fold=0):
        ctx = gcp.Context(M, precision=precision, tol_ddbar=tol_for(precision), max_iter=100,
                          fold_every=fold, profile=True)
        D = torch.empty((M, M), dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            ctx.init(H, N, w.emin, w.emax)
            ctx.purify(out=D)
        torch.cuda.synchronize()
        results = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.init(H, N, w.emin, w.emax)
            _, res = ctx.purify(out=D)
            results.append(res)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        Dh = D.cpu().numpy()
        ctx.close()
        err = float(np.linalg.norm(Dh - D_ref) / math.sqrt(M))
        return dt / steps, results, err, abs(float(np.trace(Dh)) - N)

    log(f"[bench] {prec.name}: {args.warmup} warmup + {args.steps} timed solves")
    t_mixed, res_m, err_m, tr_m = run(prec, args.steps, args.warmup, args.fold_every)
    r0 = res_m[-1]
    log(f"[bench] {prec.name}: {t_mixed*1e3:.1f} ms/solve, iters={r0.iters}, err={err_m:.3e}")
    launches = r0.gemm_launches
    flops_solve = r0.gemm_flops
    value = flops_solve / t_mixed / 1e12
    gemm_ms_avg = sum(r.gemm_ms for r in res_m) / sum(r.gemm_launches for r in res_m)
    flops_launch = flops_solve / launches
    achieved = flops_launch / (gemm_ms_avg * 1e-3) / 1e12
    mfma_achieved = (r0.mfma_flops / launches) / (gemm_ms_avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[mfma_dtype]
    kernel_tag = f"gemm_{prec.name.lower()}_M{M}"
    traffic = pmc_traffic(kernel_tag)

    fp64 = None
    if args.fp64_steps > 0 and prec != gcp.Precision.FP64:
        log(f"[bench] FP64 reference path: {args.fp64_steps} solve(s)")
        t64, res64, err64, tr64 = run(gcp.Precision.FP64, args.fp64_steps, 0)
        g64 = sum(r.gemm_ms for r in res64) / sum(r.gemm_launches for r in res64)
        fp64 = {"time_to_solution_ms": t64 * 1e3, "iters": res64[-1].iters, "err": err64,
                "trace_err": tr64,
                "tflops": res64[-1].gemm_flops / t64 / 1e12,
                "gemm_ms_per_launch": g64,
                "gemm_frac_of_fp64_peak": (res64[-1].gemm_flops / res64[-1].gemm_launches)
                / (g64 * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"]}
        log(f"[bench] FP64: {t64*1e3:.1f} ms/solve, iters={res64[-1].iters}, err={err64:.3e}")

    sched = None
    if prec != gcp.Precision.FP64:
        log(f"[bench] schedule {prec.name} -> FP64 below |Tr(D Dbar)| = 1e-2, stop at 1e-9")
        with gcp.Context(M, precision=prec, late_precision="fp64", switch_ddbar=1e-2,
                         tol_ddbar=1e-9, max_iter=100, fold_every=args.fold_every) as sctx:
            Ds = torch.empty((M, M), dtype=torch.float64, device="cuda")
            for rep in range(2):   # warm-up + timed
                sctx.init(H, N, w.emin, w.emax)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, rs = sctx.purify(out=Ds)
                torch.cuda.synchronize()
                ts = time.perf_counter() - t0
        Dsh = Ds.cpu().numpy()
        sched = {"late_precision": "fp64", "switch_ddbar": 1e-2, "tol_ddbar": 1e-9,
                 "time_to_solution_ms": ts * 1e3, "iters": rs.iters, "status": rs.status,
                 "err": float(np.linalg.norm(Dsh - D_ref) / math.sqrt(M)), "idem": rs.idem,
                 "trace_err": abs(float(np.trace(Dsh)) - N)}
        del Ds, Dsh

    log("[bench] FP64 acceptance checks of the mixed result (gcp_verify)")
    with gcp.Context(M, precision=prec, tol_ddbar=tol_for(prec), max_iter=100,
                     fold_every=args.fold_every) as vctx:
        vctx.init(H, N, w.emin, w.emax)
        Dv, _ = vctx.purify()
        vctx.verify(Dv, H)   # warm-up (allocates the workspace)
        q = vctx.verify(Dv, H)
    e0 = float(np.sort(w.lam)[:N].sum())
    verify = {"ms": q["ms"], "trace_err": abs(q["trace"] - N), "fro2_minus_N": q["fro2"] - N,
              "idem": q["idem"], "energy_err": q["energy"] - e0, "comm": q["comm"]}

    bwd = None
    if args.bwd_steps > 0:
        log(f"[bench] adjoint of the {prec.name} solve (FP32): {args.bwd_steps} timed")
        ctx = gcp.Context(M, precision=prec, tol_ddbar=tol_for(prec), max_iter=100,
                          fold_every=args.fold_every, profile=True, keep_iterates=True,
                          bwd_precision="fp32")
        ctx.init(H, N, w.emin, w.emax)
        ctx.purify()
        u = torch.from_numpy(np.random.default_rng(33).standard_normal(M)).cuda()
        G = torch.outer(u, u)
        ctx.backward(G)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.bwd_steps):
            _, rb = ctx.backward(G)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / args.bwd_steps
        ctx.close()
        bwd = {"precision": "fp32", "updates": rb.iters, "ms": tb * 1e3,
               "tflops": rb.gemm_flops / tb / 1e12,
               "gemm_ms_per_launch": rb.gemm_ms / max(rb.gemm_launches, 1),
               "gemm_frac_of_fp32_peak": rb.gemm_flops / (rb.gemm_ms * 1e-3) / 1e12
               / PEAK_TFLOPS["fp32"]}
        log(f"[bench] adjoint: {tb*1e3:.1f} ms, {bwd['tflops']:.1f} TFLOP/s")

    if args.copy_calibration:
        copy_calibration()

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample")
        cpu = cpu_baseline(w, r0.iters, launches, args.cpu_budget)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": mfma_dtype,
        "data": "synthetic",
        "config": {"workload": f"spectral H=Q diag(lam) Q^T, M={M}, N={N}, gap 0.05, "
                               f"bounds [-1,1], stop |Tr(D Dbar)|<={tol_for(prec):g}",
                   "M": M, "N": N, "precision": prec.name.lower(),
                   "fold_every": args.fold_every},
        "time_to_solution_ms": t_mixed * 1e3,
        "iters": r0.iters,
        "iterations_per_s": r0.iters / t_mixed,
        "err": err_m,
        "trace_err": tr_m,
        "meets_1e-6": bool(err_m <= 1e-6 and tr_m <= 1e-10),
        "fp64": fp64,
        "speedup_vs_fp64": (fp64["time_to_solution_ms"] / (t_mixed * 1e3)) if fp64 else None,
        "backward": bwd,
        "verify": verify,
        "schedule": sched,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": (f"k_gemm16<{prec.name}>" if gcp.MFMA_DTYPE[prec] in ("fp16", "bf16")
                                else f"k_gemm<{prec.name}>"),
                     "launches_per_solve": launches,
                     "ms_per_launch": gemm_ms_avg,
                     "mfma_issued_tflops": mfma_achieved,
                     "mfma_issued_frac": mfma_achieved / peak},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
