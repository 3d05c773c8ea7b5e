#!/usr/bin/env python3
"""Benchmark: generalized canonical purification on one MI355X.

Workload: dense H = Q diag(lam) Q^T, M = 8192, N = 3000, eigenvalues uniform in
[-1, -0.025] U [0.025, 1] (gap 0.05), Q from the QR of a seeded Gaussian
matrix, bounds [-1, 1].  One step = one whole solve on the GPU: the initial
guess from H (already resident in HBM) plus the purification to convergence
(|Tr(D Dbar)| <= 1e-6) with D written to a caller buffer.

Reported: throughput of the mixed-precision path in algorithmic TFLOP/s
(2 M^2 (M+1) per update: the two symmetric products of each of the p updates;
the final D^2 that proves convergence is reported separately), its time to
solution, the FP64 GPU path's time to solution on the same input,
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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_oracle_solves():
    """The oracle's whole FP64 solve (plain C, OpenMP), timed: the 1D chain
    (M = 256, N = 100, stop at ||D^2 - D||_F < 1e-10) and the 16 x 16 x 8
    lattice (M = 2048, N = 682, stop at Tr(D Dbar) <= 1e-8)."""
    import oracle
    import workloads
    out = {}
    for k, kw in ((1, dict(tol_ddbar=0.0, tol_idem=1e-10)), (4, dict(tol_ddbar=1e-8, max_iter=200))):
        w = workloads.config(k)
        t0 = time.perf_counter()
        r = oracle.purify(w.H, w.N, w.emin, w.emax, **kw)
        t = time.perf_counter() - t0
        out[f"config{k}"] = {"workload": w.name, "M": w.M, "time_to_solution_s": t,
                             "iters": r.iters, "status": r.status}
        log(f"[bench] oracle solve {w.name}: {t:.2f} s, {r.iters} updates")
    return out


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
        "cpu_model": cpu_model(), "nproc": os.cpu_count(),
        "extrapolated_time_to_solution_s": product_s * launches_per_solve,
        "extrapolated_time_to_solution_note": "the M=8192 solve is not run on the CPU: "
                                              "sampled product time x products per solve",
    }


COPY_BYTES = 1 << 30


def copy_calibration() -> None:
    """The yardsticks for the memory-traffic counters: a plain device copy of
    exactly COPY_BYTES (reads and writes COPY_BYTES; the reference for
    WRITE_SIZE, whose stores are ordinary global stores), and the library's
    gcp_stream_lds over COPY_BYTES (reads them with the product kernel's own
    global-to-LDS loads and writes nothing; the reference for FETCH_SIZE)."""
    import ctypes
    import torch
    import paper_1512_07236_amd as gcp
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    L = gcp.load_library()
    st = L.gcp_stream_lds(ctypes.c_void_p(src.data_ptr()), COPY_BYTES,
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == gcp.OK, st
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
    kname = "k_gemm16" if gcp.MFMA_DTYPE[prec] in ("fp16", "bf16") else "k_gemm"
    tag = f"gemm_{prec.name.lower()}_M{M}"
    out = {"kernel": f"{kname}<{int(prec)}>", "workload": f"M={M}", "precision": prec.name.lower()}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == name]
        # launches that did work (a solve's launches past its stop do nothing)
        kern = [float(r["Counter_Value"]) for r in rows
                if f"{kname}<{int(prec)}>" in r["Kernel_Name"] and float(r["Counter_Value"]) > 1024]
        # yardsticks of known size: the global-to-LDS stream for FETCH_SIZE
        # (the product kernel's load type), the plain copy for WRITE_SIZE
        if name == "FETCH_SIZE":
            ref = [float(r["Counter_Value"]) for r in rows if "k_stream_lds" in r["Kernel_Name"]]
            ref_name = "gcp_stream_lds (global_load_lds, 128-byte rows)"
        else:
            ref = [float(r["Counter_Value"]) for r in rows
                   if ("copy" in r["Kernel_Name"].lower() or "elementwise" in r["Kernel_Name"].lower())
                   and float(r["Counter_Value"]) * 1024 > 0.25 * COPY_BYTES]
            ref_name = "device copy"
        if not kern or not ref:
            print(f"no {name} rows for the kernel or the yardstick in {d}", file=sys.stderr)
            return 1
        factor = (max(ref) * 1024) / COPY_BYTES   # counter bytes per true byte
        out[name] = {"kib_per_launch_raw": sum(kern) / len(kern), "launches": len(kern),
                     "yardstick": ref_name, "yardstick_kib_raw": max(ref),
                     "factor": factor,
                     "bytes_per_launch": sum(kern) / len(kern) * 1024 / factor}
    out["hbm_bytes_per_launch"] = out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"]
    out["kernel_source_sha256"] = product_kernel_hash()
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    path = os.path.join(ROOT, "profiles", f"{tag}_pmc.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path)
    return 0


def time_solve(gcp, H, w, steps, warmup, **opts):
    """Average wall time of init + purify (H resident) over `steps` solves
    after `warmup`; returns (seconds, last Result, D on the host)."""
    import torch
    ctx = gcp.Context(w.M, **opts)
    D = torch.empty((w.M, w.M), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ctx.init(H, w.N, w.emin, w.emax)
        ctx.purify(out=D)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.init(H, w.N, w.emin, w.emax)
        _, res = ctx.purify(out=D)
        results.append(res)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    Dh = D.cpu().numpy()
    ctx.close()
    return dt, results, Dh


def time_adjoint(gcp, H, w, prec, tol, args):
    """The FP32 adjoint (gcp_backward) of the solve for L = u^T D u: one
    warm-up and args.bwd_steps timed calls on the same kept iterates."""
    import torch
    M, N = w.M, w.N
    log(f"[bench] adjoint of the {prec.name} solve (FP32): {args.bwd_steps} timed")
    ctx = gcp.Context(M, precision=prec, tol_ddbar=tol, max_iter=100,
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
    del G
    bwd = {"precision": "fp32", "updates": rb.iters, "ms": tb * 1e3,
           "tflops": rb.gemm_flops / tb / 1e12,
           "gemm_ms_per_launch": rb.gemm_ms / max(rb.gemm_launches, 1),
           "gemm_frac_of_fp32_peak": rb.gemm_flops / (rb.gemm_ms * 1e-3) / 1e12
           / PEAK_TFLOPS["fp32"]}
    log(f"[bench] adjoint: {tb*1e3:.1f} ms, {bwd['tflops']:.1f} TFLOP/s")
    return bwd


def extra_configs(gcp, args):
    """The other standard workloads, each timed once after a warm-up: the 1D
    chain (FP64, with the host checking after every update and every 4), the
    dense M = 4096 case in FP64 and FP32, the 16 x 16 x 8 lattice's FP64
    solve and adjoint, and (--config5) M = 16384 in BF16X6 with the
    checkpointed FP32 adjoint."""
    import torch
    import oracle
    import workloads
    out = {}
    # config 1: launch- and sync-bound at M = 256
    w = workloads.config(1)
    H = torch.from_numpy(w.H).cuda()
    c1 = {}
    for k in (1, 4):
        t, rs, Dh = time_solve(gcp, H, w, 5, 2, precision="fp64", tol_ddbar=0.0, tol_idem=1e-10,
                               sync_every=k)
        c1[f"sync_every_{k}"] = {"time_to_solution_ms": t * 1e3, "iters": rs[-1].iters,
                                 "host_syncs": rs[-1].host_syncs}
    P, _ = oracle.ground_state_jacobi(w.H, w.N)
    c1["err"] = float(np.linalg.norm(Dh - P) / math.sqrt(w.M))
    out["config1_chain_M256_fp64"] = c1
    log(f"[bench] config 1: {c1}")
    # config 2: FP64 vs FP32 at M = 4096
    w = workloads.config(2)
    H = torch.from_numpy(w.H).cuda()
    ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
    c2 = {}
    for prec, tol in (("fp64", 1e-9), ("fp32", 1e-6)):
        t, rs, Dh = time_solve(gcp, H, w, 2, 1, precision=prec, tol_ddbar=tol)
        c2[prec] = {"time_to_solution_ms": t * 1e3, "iters": rs[-1].iters, "status": rs[-1].status,
                    "tol_ddbar": tol, "err": float(np.linalg.norm(Dh - ref) / math.sqrt(w.M)),
                    "trace_err": abs(float(np.trace(Dh)) - w.N)}
    out["config2_spectral_M4096"] = c2
    log(f"[bench] config 2: {c2}")
    del H, ref
    # config 4: FP64 solve and adjoint of L = Tr(D P) on the lattice
    w = workloads.config(4)
    H = torch.from_numpy(w.H).cuda()
    Pm = torch.from_numpy(workloads.sym_gaussian(w.M, 40)).cuda()
    with gcp.Context(w.M, precision="fp64", tol_ddbar=1e-8, max_iter=200, keep_iterates=True) as ctx:
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.init(H, w.N, w.emin, w.emax)
            _, r = ctx.purify()
            torch.cuda.synchronize()
            tf = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, rb = ctx.backward(Pm)
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
    out["config4_cubic_16x16x8_fp64"] = {"forward_ms": tf * 1e3, "backward_ms": tb * 1e3,
                                         "iters": r.iters, "status": r.status}
    log(f"[bench] config 4: {out['config4_cubic_16x16x8_fp64']}")
    del H, Pm
    if args.config5:
        w = workloads.config(5)
        H = torch.from_numpy(w.H).cuda()
        u = torch.from_numpy(np.random.default_rng(55).standard_normal(w.M)).cuda()
        with gcp.Context(w.M, precision="bf16x6", tol_ddbar=1e-5, keep_iterates=True,
                         checkpoint_every=8, bwd_precision="fp32") as ctx:
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.init(H, w.N, w.emin, w.emax)
                D, r = ctx.purify()
                torch.cuda.synchronize()
                tf = time.perf_counter() - t0
                t0 = time.perf_counter()
                _, rb = ctx.backward(torch.outer(u, u))
                torch.cuda.synchronize()
                tb = time.perf_counter() - t0
            Dh = D.cpu().numpy()
        ref = oracle.projector_from_spectrum(w.Q, w.lam, w.N)
        out["config5_spectral_M16384_bf16x6"] = {
            "forward_ms": tf * 1e3, "backward_checkpointed_fp32_ms": tb * 1e3, "iters": r.iters,
            "status": r.status, "err": float(np.linalg.norm(Dh - ref) / math.sqrt(w.M)),
            "forward_algorithmic_tflops": 2.0 * r.iters * w.M ** 2 * (w.M + 1) / tf / 1e12}
        log(f"[bench] config 5: {out['config5_spectral_M16384_bf16x6']}")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16x3")
    ap.add_argument("--fold-every", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-6,
                    help="|Tr(D Dbar)| stop (the paper's 1e-6)")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--bwd-steps", type=int, default=1,
                    help="timed adjoints (gcp_backward, FP32) of the mixed solve for L = u^T D u")
    ap.add_argument("--scale", type=int, default=1, help="divide M by this (quick runs only)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--config5", action="store_true",
                    help="also run M = 16384 (BF16X6 forward and checkpointed FP32 adjoint)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the warm-up and timed solves of the headline workload (for a "
                         "kernel trace that covers exactly those launches)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the timed FP32 adjoints (--bwd-steps) of the headline solve (for "
                         "a kernel trace of the adjoint)")
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
    if args.copy_calibration:
        copy_calibration()

    log("[bench] generating workload (seeded)")
    w = workloads.config(3, scale=args.scale)
    M, N = w.M, w.N
    H = torch.from_numpy(w.H).cuda()
    prec = gcp.Precision.parse(args.precision)
    mfma_dtype = gcp.MFMA_DTYPE[prec]
    tol = args.tol

    if args.adjoint_only:
        print(json.dumps(time_adjoint(gcp, H, w, prec, args.tol, args)), flush=True)
        return 0
    log(f"[bench] {prec.name}: {args.warmup} warmup + {args.steps} timed solves")
    t_mixed, res_m, Dh = time_solve(gcp, H, w, args.steps, args.warmup, precision=prec,
                                    tol_ddbar=tol, max_iter=100, fold_every=args.fold_every,
                                    profile=True)
    r0 = res_m[-1]
    if args.headline_only:
        print(json.dumps({"ms_per_step": t_mixed * 1e3, "iters": r0.iters,
                          "launches": r0.gemm_launches,
                          "gemm_ms_per_launch": sum(r.gemm_ms for r in res_m)
                          / sum(r.gemm_launches for r in res_m)}), flush=True)
        return 0
    log("[bench] reference projector (closed form)")
    D_ref = oracle.projector_from_spectrum(w.Q, w.lam, N)
    err_m = float(np.linalg.norm(Dh - D_ref) / math.sqrt(M))
    tr_m = abs(float(np.trace(Dh)) - N)
    del Dh
    log(f"[bench] {prec.name}: {t_mixed*1e3:.1f} ms/solve, iters={r0.iters}, status={r0.status}, "
        f"err={err_m:.3e}")
    p = r0.iters
    launches = r0.gemm_launches            # 2p (2p + 1 if the stop needed the last square)
    flops_product = float(M) * M * (M + 1)  # one symmetric product, upper triangle
    value = 2.0 * p * flops_product / t_mixed / 1e12
    gemm_ms_avg = sum(r.gemm_ms for r in res_m) / sum(r.gemm_launches for r in res_m)
    achieved = flops_product / (gemm_ms_avg * 1e-3) / 1e12
    mfma_achieved = (r0.mfma_flops / launches) / (gemm_ms_avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[mfma_dtype]
    ceiling = 1.0 / gcp.PRODUCTS[prec]
    kernel_tag = f"gemm_{prec.name.lower()}_M{M}"
    traffic = pmc_traffic(kernel_tag)

    fp64 = None
    if args.fp64_steps > 0 and prec != gcp.Precision.FP64:
        log(f"[bench] FP64 reference path: {args.fp64_steps} solve(s)")
        t64, res64, D64 = time_solve(gcp, H, w, args.fp64_steps, 0, precision="fp64",
                                     tol_ddbar=tol, max_iter=100, profile=True)
        g64 = sum(r.gemm_ms for r in res64) / sum(r.gemm_launches for r in res64)
        r64 = res64[-1]
        fp64 = {"time_to_solution_ms": t64 * 1e3, "iters": r64.iters, "status": r64.status,
                "err": float(np.linalg.norm(D64 - D_ref) / math.sqrt(M)),
                "trace_err": abs(float(np.trace(D64)) - N),
                "tflops": 2.0 * r64.iters * flops_product / t64 / 1e12,
                "gemm_ms_per_launch": g64,
                "gemm_frac_of_fp64_peak": flops_product / (g64 * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"]}
        del D64
        log(f"[bench] FP64: {t64*1e3:.1f} ms/solve, iters={r64.iters}, err={fp64['err']:.3e}")

    sched = None
    if prec != gcp.Precision.FP64:
        log(f"[bench] schedule {prec.name} -> FP64 below |Tr(D Dbar)| = 1e-2, stop at 1e-9")
        ts, rss, Ds = time_solve(gcp, H, w, 1, 1, precision=prec, late_precision="fp64",
                                 switch_ddbar=1e-2, tol_ddbar=1e-9, max_iter=100,
                                 fold_every=args.fold_every)
        rs = rss[-1]
        # ||D^2 - D||_F of the scheduled result in FP64 (gcp_verify)
        with gcp.Context(M, precision=prec, late_precision="fp64", switch_ddbar=1e-2,
                         tol_ddbar=1e-9, max_iter=100, fold_every=args.fold_every) as sctx:
            sctx.init(H, N, w.emin, w.emax)
            Dsv, _ = sctx.purify()
            sidem = sctx.verify(Dsv, H)["idem"]
            del Dsv
        sched = {"late_precision": "fp64", "switch_ddbar": 1e-2, "tol_ddbar": 1e-9,
                 "time_to_solution_ms": ts * 1e3, "iters": rs.iters, "status": rs.status,
                 "err": float(np.linalg.norm(Ds - D_ref) / math.sqrt(M)), "idem": sidem,
                 "trace_err": abs(float(np.trace(Ds)) - N)}
        del Ds

    log("[bench] FP64 acceptance checks of the mixed result (gcp_verify)")
    with gcp.Context(M, precision=prec, tol_ddbar=tol, max_iter=100,
                     fold_every=args.fold_every) as vctx:
        vctx.init(H, N, w.emin, w.emax)
        Dv, _ = vctx.purify()
        vctx.verify(Dv, H)   # warm-up (allocates the workspace)
        q = vctx.verify(Dv, H)
        del Dv
    e0 = float(np.sort(w.lam)[:N].sum())
    verify = {"ms": q["ms"], "trace_err": abs(q["trace"] - N), "fro2_minus_N": q["fro2"] - N,
              "idem": q["idem"], "energy_err": q["energy"] - e0, "comm": q["comm"]}

    bwd = time_adjoint(gcp, H, w, prec, tol, args) if args.bwd_steps > 0 else None
    del H, D_ref

    extra = None if args.no_extra or args.scale != 1 else extra_configs(gcp, args)


    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample")
        cpu = cpu_baseline(w, p, launches, args.cpu_budget)
        cpu["timed_solves"] = timed_oracle_solves()

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
                               f"bounds [-1,1], stop |Tr(D Dbar)|<={tol:g}",
                   "M": M, "N": N, "precision": prec.name.lower(),
                   "fold_every": args.fold_every},
        "value_definition": "2 p M^2 (M+1) / time to solution: the two symmetric products of "
                            "each of the p updates (upper-triangle flops)",
        "time_to_solution_ms": t_mixed * 1e3,
        "iters": p,
        "status": r0.status,
        "host_syncs": r0.host_syncs,
        "iterations_per_s": p / t_mixed,
        "termination_product": {"launches": launches - 2 * p,
                                "note": ("the stop on Tr(D Dbar) was decided from the last "
                                         "update's traces; no product was launched for it")
                                if launches == 2 * p else
                                ("the last update's Tr(D Dbar) was above the tolerance, so "
                                 "one more D^2 was formed to decide the stop (at the "
                                 "encoding's rounding floor: status STOPPED_AT_FLOOR)")
                                if r0.status == gcp.STOPPED_AT_FLOOR else
                                "one more D^2 was formed to decide the stop",
                                "tflops_incl": launches * flops_product / t_mixed / 1e12},
        "err": err_m,
        "trace_err": tr_m,
        "meets_1e-6": bool(err_m <= 1e-6 and tr_m <= 1e-10),
        "fp64": fp64,
        "speedup_vs_fp64": (fp64["time_to_solution_ms"] / (t_mixed * 1e3)) if fp64 else None,
        "backward": bwd,
        "verify": verify,
        "schedule": sched,
        "other_workloads": extra,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": (("k_gemm16" if gcp.MFMA_DTYPE[prec] in ("fp16", "bf16") else "k_gemm")
                                + f"<{prec.name}>"),
                     "algorithmic_flops_per_launch": flops_product,
                     "launches_per_solve": launches,
                     "ms_per_launch": gemm_ms_avg,
                     "ceiling": ceiling,
                     "ceiling_note": "a split encoding issues 1/ceiling MFMA products per "
                                     "algorithmic product, so frac cannot exceed the ceiling",
                     "frac_of_ceiling": achieved / peak / ceiling,
                     "mfma_issued_tflops": mfma_achieved,
                     "mfma_issued_frac": mfma_achieved / peak},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
