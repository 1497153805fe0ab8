#!/usr/bin/env python3
"""Benchmark of the all-port solve at 32x32 thin-wire dipoles on one MI355X.

One step is the whole hot path for one frequency: block fill, block spectra,
preconditioner, preconditioned right-hand sides, batched GMRES for all 1024
port excitations, port impedance Z_p = Y_p^{-1}, S and the center-element
active impedance / ARC at 64 scan angles -- with nothing reused across steps
(the operator cache is bypassed).  The headline path runs the lattice FFTs
and per-bin block products in FP32 on the matrix cores (FP64 Arnoldi
accumulation, FP64 iterative refinement); the plain FP64 path is timed beside
it at matched Z_p accuracy.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
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

METRIC = "port-excitation solves/s at 32x32 dipoles, FP32-MFMA vs FP64; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_CODES = {"arnoldi_dots": 1, "arnoldi_update_dots": 2, "arnoldi_update_norm": 3, "fft_fwd_pad": 4,
                "fft_inv_crop": 5, "bin_product": 6, "precond_apply": 7}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def zp_errors(out, ref):
    Zp = out["Zp"]
    c = int(ref["center"])
    row = np.linalg.norm(Zp[c, :] - ref["Zp_center_row"]) / np.linalg.norm(ref["Zp_center_row"])
    samp = np.max(np.abs(Zp[ref["Zp_rows"], ref["Zp_cols"]] - ref["Zp_samples"])) / float(ref["Zp_max"])
    diag = np.max(np.abs(np.diag(Zp) - ref["Zp_diag"]) / np.abs(ref["Zp_diag"]))
    gam = np.max(np.abs(out["Gamma"] - ref["Gamma"]))
    return {"zp_center_row_rel": float(row), "zp_sample_max_rel": float(samp), "zp_diag_max_rel": float(diag),
            "gamma_max_abs": float(gam)}


def run_steps(mbt, ctx, arr, w, opts, steps, warmup, kernel=None):
    for _ in range(warmup):
        mbt.mbt_solve(ctx, arr, 1.0, opts, w.theta, w.phi, w.z0)
    import torch
    torch.cuda.synchronize()
    if kernel:
        mbt.mbt_prof_start(KERNEL_CODES[kernel])
    times, out = [], None
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        out = mbt.mbt_solve(ctx, arr, 1.0, opts, w.theta, w.phi, w.z0)
        times.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    prof = mbt.mbt_prof_read() if kernel else None
    if kernel:
        mbt.mbt_prof_start(0)
    return total, times, out, prof


def cpu_baseline(w):
    """The CPU oracle (dense fill from absolute positions, LAPACK LU, extraction)
    timed on a bounded sample: the same element, frequency and spacing on a
    14x14 lattice (N = 6076), each phase scaled to the 32x32 size by its
    complexity (fill ~ N^2, LU ~ N^3, solve ~ N^2 * ports); the extraction
    (P x P inverse, S, scans) is timed at the real P = 1024."""
    from oracle import mom
    from paper_2608_17844_amd import workloads as W
    lat_s = W.Lattice(14, 14, w.lattice.dx, w.lattice.dy)
    r = mom.solve_array(lat_s, w.dipole, 1.0, w.theta, w.phi, z0=w.z0)
    n1 = lat_s.nx * lat_s.ny * w.dipole.nbases
    p1 = lat_s.nx * lat_s.ny
    n2 = w.lattice.nx * w.lattice.ny * w.dipole.nbases
    p2 = w.lattice.nx * w.lattice.ny
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((p2, p2)) + 1j * rng.standard_normal((p2, p2)) + 30 * np.eye(p2)
    t0 = time.perf_counter()
    Zp = mom.port_impedance(Y)
    S = mom.s_matrix(Zp, w.z0)
    mom.active_impedance(Zp, w.lattice, 1.0, w.theta, w.phi)
    mom.wave_arc(S, w.lattice, 1.0, w.theta, w.phi)
    t_ext = time.perf_counter() - t0
    t_fill = r.times["fill"] * (n2 / n1) ** 2
    t_lu = r.times["lu"] * (n2 / n1) ** 3
    t_solve = r.times["solve"] * (n2 / n1) ** 2 * (p2 / p1)
    total = t_fill + t_lu + t_solve + t_ext
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    sample_s = sum(r.times.values()) + t_ext
    return {"value": p2 / total, "unit": "solves/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": "14x14 lattice of the same dipole (N=6076, 196 ports), dense fill + LAPACK LU + solve "
                      "+ extraction, %.1f s of CPU work, phases scaled to 32x32 (fill N^2, LU N^3, solve N^2*P); "
                      "extraction timed at P=1024" % sample_s,
            "phases_s": {"fill": t_fill, "lu": t_lu, "solve": t_solve, "extract": t_ext}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--pc", choices=["element_block", "normal_eq"], default="element_block")
    ap.add_argument("--kernel", choices=sorted(KERNEL_CODES), default="arnoldi_update_dots")
    ap.add_argument("--refine-tol", type=float, default=1e-7)
    ap.add_argument("--fp64-tol", type=float, default=1e-7, help="FP64 GMRES tolerance at matched Z_p accuracy")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver's workload fits one MI355X and no multi-GPU path "
              "is built (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    import torch

    w = W.gpu_size_32x32()
    ref = np.load(os.path.join(ROOT, "tests", "golden", "dipole_32x32_m31_reference.npz"))
    pc = mbt.MBT_PC_ELEMENT_BLOCK if args.pc == "element_block" else mbt.MBT_PC_NORMAL_EQ
    ctx = mbt.mbt_ctx_create(0)
    arr = mbt.mbt_array_create_dipole(ctx, w.dipole, w.lattice)
    P = w.lattice.nx * w.lattice.ny
    result = {}
    try:
        o32 = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=pc, restart=w.restart, refine_tol=args.refine_tol,
                                   flags=mbt.MBT_FLAG_NO_CACHE)
        log("fp32-mfma path: warmup %d, steps %d" % (args.warmup, args.steps))
        total, times, out, prof = run_steps(mbt, ctx, arr, w, o32, args.steps, args.warmup, args.kernel)
        err32 = zp_errors(out, ref)
        st32 = out["stats"]
        value = P * args.steps / total
        log("fp32: %.3f s/step  %.1f solves/s  err %s" % (total / args.steps, value, err32))
        fp64 = None
        if not args.no_fp64:
            o64 = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=pc, restart=w.restart, tol=args.fp64_tol,
                                       flags=mbt.MBT_FLAG_NO_CACHE)
            log("fp64 path (tol %g): warmup %d, steps %d" % (args.fp64_tol, args.warmup, args.steps))
            t64, times64, out64, _ = run_steps(mbt, ctx, arr, w, o64, args.steps, args.warmup)
            err64 = zp_errors(out64, ref)
            fp64 = {"value": P * args.steps / t64, "ms_per_step": 1e3 * t64 / args.steps, "tol": args.fp64_tol,
                    "errors": err64, "iters_max": out64["stats"]["iters_max"],
                    "matvecs": out64["stats"]["matvecs"]}
            log("fp64: %.3f s/step  %.1f solves/s  err %s" % (t64 / args.steps, fp64["value"], err64))
        achieved = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof and prof["ms"] > 0 else None
        roofline = {"kernel": args.kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": None,
                    "launches": prof["launches"] if prof else 0,
                    "avg_launch_ms": (prof["ms"] / prof["launches"]) if prof and prof["launches"] else None,
                    "alg_bytes_per_launch": (prof["bytes"] / prof["launches"]) if prof and prof["launches"] else None}
        lat = np.array(times) * 1e3
        result = {
            "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": w.name, "nx": w.lattice.nx, "ny": w.lattice.ny, "nbases": w.dipole.nbases,
                       "unknowns": P * w.dipole.nbases, "ports": P, "nscan": int(len(w.theta)),
                       "preconditioner": args.pc, "restart": w.restart,
                       "precision": "FP32 lattice FFT + FP32 MFMA block products, FP32-stored Krylov basis with "
                                    "FP64 dot products/Givens, FP64 refinement residual and extraction",
                       "refine_tol": args.refine_tol},
            "accuracy": err32, "iters_max": st32["iters_max"], "outer_steps": st32["outer_steps"],
            "matvecs_per_step": st32["matvecs"],
            "matvecs_per_s": st32["matvecs"] * args.steps / total,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "what": "per 1024-port request, whole hot path"},
            "fp64": fp64,
            "speedup_vs_fp64": (value / fp64["value"]) if fp64 else None,
            "roofline": roofline,
        }
        torch.cuda.synchronize()
    finally:
        mbt.mbt_array_destroy(arr)
        mbt.mbt_ctx_destroy(ctx)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, bounded sample)")
        result["cpu_baseline"] = cpu_baseline(w)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
