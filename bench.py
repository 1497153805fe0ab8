#!/usr/bin/env python3
"""Benchmark of the all-port solve at 32x32 thin-wire dipoles on one MI355X.

One step is the whole hot path for one frequency: block fill, block spectra,
preconditioner, preconditioned right-hand sides, batched GMRES for all 1024
port excitations, port impedance Z_p = Y_p^{-1}, S and the center-element
active impedance / ARC at 64 scan angles -- with nothing reused across steps
(the operator cache is bypassed).  The headline path runs the lattice FFTs
and per-bin block products in FP32 on the matrix cores (FP64 Arnoldi
accumulation, FP64 iterative refinement); the plain FP64 path is timed beside
it at the same accuracy target (Z_p entries and the center ARC within 1e-6
relative of the FP64 oracle), and so is FP64 COCG with the element-block
preconditioner, the fastest FP64 configuration.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]     headline 32x32 workload
  python bench.py --solver pcg | cocg                      the same workload with PCG or COCG on both paths
  python bench.py --serve 40 [--load 0.8] [--slots 4]     Poisson serving stream
  python bench.py --sweep                                  21-frequency precision sweep
  python bench.py --blocks 5                               64x64 elements of 96 bases (synthetic blocks)
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
    """Errors against the stored oracle results: Z_p center row (norm-wise),
    4096 sampled entries (each relative to itself and to max |Z_p|), the
    diagonal, and the ARC at the 64 scan angles (absolute and relative)."""
    Zp = out["Zp"]
    c = int(ref["center"])
    row = np.linalg.norm(Zp[c, :] - ref["Zp_center_row"]) / np.linalg.norm(ref["Zp_center_row"])
    d = np.abs(Zp[ref["Zp_rows"], ref["Zp_cols"]] - ref["Zp_samples"])
    samp = np.max(d) / float(ref["Zp_max"])
    elem = np.max(d / np.abs(ref["Zp_samples"]))
    diag = np.max(np.abs(np.diag(Zp) - ref["Zp_diag"]) / np.abs(ref["Zp_diag"]))
    dg = np.abs(out["Gamma"] - ref["Gamma"])
    return {"zp_center_row_rel": float(row), "zp_sample_max_rel": float(samp), "zp_sample_elementwise_rel": float(elem),
            "zp_diag_max_rel": float(diag), "gamma_max_abs": float(np.max(dg)),
            "gamma_max_rel": float(np.max(dg / np.abs(ref["Gamma"])))}


def run_steps(mbt, ctx, arr, w, opts, steps, warmup, kernel=None, allow_noconv=False):
    for _ in range(warmup):
        mbt.mbt_solve(ctx, arr, 1.0, opts, w.theta, w.phi, w.z0, allow_noconv=allow_noconv)
    import torch
    torch.cuda.synchronize()
    if kernel:
        mbt.mbt_prof_start(KERNEL_CODES[kernel])
    times, out = [], None
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        out = mbt.mbt_solve(ctx, arr, 1.0, opts, w.theta, w.phi, w.z0, allow_noconv=allow_noconv)
        times.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    prof = mbt.mbt_prof_read() if kernel else None
    if kernel:
        mbt.mbt_prof_start(0)
    return total, times, out, prof


def cpu_baseline(w, side=20):
    """The CPU oracle (dense fill from absolute positions, LAPACK LU, extraction)
    timed on a bounded sample: the same element, frequency and spacing on a
    20x20 lattice (N = 12,400), each phase scaled to the 32x32 size by its
    complexity (fill ~ N^2, LU ~ N^3, solve ~ N^2 * ports); the extraction
    (P x P inverse, S, scans) is timed at the real P = 1024."""
    from oracle import mom
    from paper_2608_17844_amd import workloads as W
    lat_s = W.Lattice(side, side, w.lattice.dx, w.lattice.dy)
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
            "sample": "%dx%d lattice of the same dipole (N=%d, %d ports), dense fill + LAPACK LU + solve "
                      "+ extraction, %.1f s of CPU work, phases scaled to 32x32 (fill N^2, LU N^3, solve N^2*P); "
                      "extraction timed at P=1024" % (side, side, n1, p1, sample_s),
            "phases_s": {"fill": t_fill, "lu": t_lu, "solve": t_solve, "extract": t_ext}}


CPU_FULL_PROFILE = os.path.join(ROOT, "profiles", "cpu_oracle_dipole_32x32_m31.txt")


def cpu_full(args):
    """The CPU oracle on the whole 32x32 workload (N = 31,744, all 1024 ports):
    dense fill, zgetrf, zgetrs of the 1024 port columns and the extraction, each
    timed, beside the bounded-sample extrapolation of two sample sizes on the
    same host (20x20 and 24x24 lattices scaled by fill N^2, LU N^3, solve N^2 P)."""
    import platform
    from oracle import mom
    from paper_2608_17844_amd import workloads as W
    w = W.gpu_size_32x32()
    samples = {str(side): cpu_baseline(w, side) for side in (20, 24)}
    log("cpu oracle, full 32x32 workload")
    r = mom.solve_array(w.lattice, w.dipole, 1.0, w.theta, w.phi, z0=w.z0)
    total = sum(r.times.values())
    P = w.lattice.nx * w.lattice.ny
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"metric": "CPU oracle solves/s, 32x32 dipoles (dense fill + LAPACK LU)", "value": P / total,
            "unit": "solves/s", "phases_s": r.times, "total_s": total,
            "host": platform.processor() or platform.machine(), "cores": cores,
            "threads": int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", cores))),
            "samples": {k: {"value": v["value"], "phases_s": v["phases_s"],
                            "error_vs_measured": v["value"] / (P / total) - 1.0} for k, v in samples.items()}}


def measured_full_cpu():
    """The full-size oracle run recorded in profiles/ (host, threads, phases)."""
    if not os.path.exists(CPU_FULL_PROFILE):
        return None
    for line in open(CPU_FULL_PROFILE):
        if line.startswith("{"):
            return json.loads(line)
    return None


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_dcgs2_update_dipole_32x32_m31_fp32.txt")


def measured_traffic(kernel, restart):
    """HBM bytes per launch of the dominant kernel class from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None when
    the summary does not cover this kernel and configuration or the kernel
    source changed since."""
    import hashlib
    if kernel != "arnoldi_update_dots" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    vals = {}
    for line in open(TRAFFIC_PROFILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2608_17844_amd", "csrc", "gmres.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if not vals.get("kernel_source", "").endswith(sha) or vals.get("restart") != str(restart):
        return None
    return float(vals["traffic_bytes_per_launch"].split()[0])


def kernel_rooflines(mbt, ctx, arr, w, opts, classes):
    """One extra (untimed) step per kernel class with HIP-event timing of that
    class: algorithmic bytes / measured time, against the HBM peak."""
    out = {}
    for name in classes:
        mbt.mbt_prof_start(KERNEL_CODES[name])
        mbt.mbt_solve(ctx, arr, 1.0, opts, w.theta, w.phi, w.z0, allow_noconv=True)
        p = mbt.mbt_prof_read()
        mbt.mbt_prof_start(0)
        if p["launches"] and p["ms"] > 0:
            gbs = p["bytes"] / (p["ms"] * 1e-3) / 1e9
            out[name] = {"achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS, "launches": p["launches"],
                         "avg_launch_ms": p["ms"] / p["launches"], "alg_bytes_per_launch": p["bytes"] / p["launches"],
                         "ms_total": p["ms"]}
    return out


def headline(args):
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    import torch

    w = W.gpu_size_32x32()
    ref = np.load(os.path.join(ROOT, "tests", "golden", "dipole_32x32_m31_reference.npz"))
    pc = mbt.MBT_PC_ELEMENT_BLOCK if args.pc == "element_block" else mbt.MBT_PC_NORMAL_EQ
    sflags = 0
    if args.solver == "pcg":
        # the paper's PCG solves the normal equations with P_A
        pc, sflags = mbt.MBT_PC_NORMAL_EQ, mbt.MBT_FLAG_PCG
        args.pc = "normal_eq"
        if args.kernel == "arnoldi_update_dots":
            args.kernel = "fft_inv_crop"
    elif args.solver == "cocg":
        # COCG on the complex symmetric Z with the symmetric P_K
        pc, sflags = mbt.MBT_PC_ELEMENT_BLOCK, mbt.MBT_FLAG_COCG
        args.pc = "element_block"
        if args.kernel == "arnoldi_update_dots":
            args.kernel = "fft_inv_crop"
    ctx = mbt.mbt_ctx_create(0)
    arr = mbt.mbt_array_create_dipole(ctx, w.dipole, w.lattice)
    P = w.lattice.nx * w.lattice.ny
    result = {}
    try:
        bflags = mbt.MBT_FLAG_FP32_BASIS if args.fp32_basis else 0
        # the FP32 COCG inner solves run away on a few RHS (the FP32 short recurrence): cap them at
        # 20 x 32 = 640 steps per refinement step instead of the default 400 x 32
        cyc = {"max_cycles": 20} if args.solver == "cocg" else {}
        o32 = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=pc, restart=args.restart, refine_tol=args.refine_tol,
                                   inner_tol=args.inner_tol, flags=mbt.MBT_FLAG_NO_CACHE | sflags | bflags, **cyc)
        log("fp32-mfma path: warmup %d, steps %d" % (args.warmup, args.steps))
        # the mixed COCG comparator is reported with the RHS it leaves short of the tolerance
        # (status and count in the line); every other configuration must converge
        total, times, out, prof = run_steps(mbt, ctx, arr, w, o32, args.steps, args.warmup, args.kernel,
                                            allow_noconv=args.solver == "cocg")
        err32 = zp_errors(out, ref)
        st32 = out["stats"]
        value = P * args.steps / total
        log("fp32: %.3f s/step  %.1f solves/s  err %s" % (total / args.steps, value, err32))
        fp64 = None
        if not args.no_fp64:
            o64 = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=pc, restart=args.fp64_restart, tol=args.fp64_tol,
                                       flags=mbt.MBT_FLAG_NO_CACHE | sflags)
            log("fp64 path (tol %g): warmup %d, steps %d" % (args.fp64_tol, args.warmup, args.steps))
            t64, times64, out64, _ = run_steps(mbt, ctx, arr, w, o64, args.steps, args.warmup)
            err64 = zp_errors(out64, ref)
            fp64 = {"value": P * args.steps / t64, "ms_per_step": 1e3 * t64 / args.steps, "tol": args.fp64_tol,
                    "restart": args.fp64_restart,
                    "errors": err64, "iters_max": out64["stats"]["iters_max"],
                    "matvecs": out64["stats"]["matvecs"]}
            log("fp64: %.3f s/step  %.1f solves/s  err %s" % (t64 / args.steps, fp64["value"], err64))
        fp64_cocg = None
        if not args.no_fp64 and args.solver == "gmres":
            # the fastest FP64 configuration measured here: COCG with P_K, ||r|| <= tol ||V||
            oc = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK, tol=args.fp64_tol,
                                      flags=mbt.MBT_FLAG_NO_CACHE | mbt.MBT_FLAG_COCG)
            log("fp64 COCG path (tol %g): warmup %d, steps %d" % (args.fp64_tol, args.warmup, args.steps))
            tc, _, outc, _ = run_steps(mbt, ctx, arr, w, oc, args.steps, args.warmup)
            fp64_cocg = {"value": P * args.steps / tc, "ms_per_step": 1e3 * tc / args.steps, "tol": args.fp64_tol,
                         "solver": "cocg", "errors": zp_errors(outc, ref), "iters_max": outc["stats"]["iters_max"],
                         "matvecs": outc["stats"]["matvecs"]}
            log("fp64 cocg: %.3f s/step  %.1f solves/s  err %s" % (tc / args.steps, fp64_cocg["value"],
                                                                      fp64_cocg["errors"]))
        kernels = {}
        if not args.no_kernel_table:
            log("per-kernel rooflines (one untimed step per kernel class)")
            classes = ["fft_fwd_pad", "fft_inv_crop", "bin_product", "precond_apply"]
            kernels = kernel_rooflines(mbt, ctx, arr, w, o32, (["arnoldi_dots"] if args.solver == "gmres" else []) + classes)
        achieved = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof and prof["ms"] > 0 else None
        # the committed counters cover the packed-basis sweep only
        traffic = None if args.fp32_basis else measured_traffic(args.kernel, args.restart)
        roofline = {"kernel": args.kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
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
                       "solver": args.solver, "preconditioner": args.pc, "restart": args.restart,
                       "fp64_restart": args.fp64_restart,
                       "precision": "FP32 lattice FFT + FP32 MFMA block products, Krylov basis "
                                    + ("in FP32" if args.fp32_basis else "packed to 24 bits per component")
                                    + " with FP32 work vectors and FP64 dot products/Givens, FP64 "
                                    "refinement residual and extraction",
                       "refine_tol": args.refine_tol, "inner_tol": args.inner_tol,
                       "accuracy_target": "Z_p entries and center ARC within 1e-6 relative of the FP64 oracle"},
            "accuracy": err32, "iters_max": st32["iters_max"], "outer_steps": st32["outer_steps"],
            "status": out["status"], "nconverged": st32["nconverged"],
            "matvecs_per_step": st32["matvecs"],
            "matvecs_per_s": st32["matvecs"] * args.steps / total,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "what": "per 1024-port request, whole hot path"},
            "fp64": fp64,
            "speedup_vs_fp64": (value / fp64["value"]) if fp64 else None,
            "fp64_cocg": fp64_cocg,
            "speedup_vs_fp64_cocg": (value / fp64_cocg["value"]) if fp64_cocg else None,
            "roofline": roofline,
            "kernels": kernels,
        }
        torch.cuda.synchronize()
    finally:
        mbt.mbt_array_destroy(arr)
        mbt.mbt_ctx_destroy(ctx)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, bounded sample)")
        result["cpu_baseline"] = cpu_baseline(w)
        full = measured_full_cpu()
        if full:
            # the whole workload measured on another host (the oracle takes minutes there)
            result["cpu_baseline"]["measured_full"] = {
                "value": full["value"], "unit": "solves/s", "host": full["host"], "threads": full["threads"],
                "phases_s": full["phases_s"], "source": os.path.relpath(CPU_FULL_PROFILE, ROOT),
                "sample_extrapolation_error_on_that_host": {k: v["error_vs_measured"]
                                                            for k, v in full["samples"].items()}}
    else:
        result["cpu_baseline"] = None
    return result


def serve(args):
    """Serving form: a seeded Poisson stream of heterogeneous requests (Nx, Ny
    in 8..48, 15 or 31 bases, 1-8 frequencies in 0.5-1.5 f0, 1-64 scans)
    through the continuous-batching server.  First the saturation throughput
    (all requests submitted at once), then the stream at a fraction of that
    request rate; latency is submit -> result on the server clock."""
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W

    ctx = mbt.mbt_ctx_create(0)
    srv = mbt.mbt_server_create(ctx, args.slots)
    opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=args.restart,
                                refine_tol=args.refine_tol, inner_tol=args.inner_tol, max_cycles=args.serve_max_cycles)

    def submit(r):
        return mbt.mbt_server_submit(srv, (r.dipole.length, r.dipole.radius, r.dipole.nbases),
                                     (r.lattice.nx, r.lattice.ny, r.lattice.dx, r.lattice.dy),
                                     r.freqs, r.theta, r.phi, opts, r.z0)

    def solves(r):
        return r.lattice.nx * r.lattice.ny * len(r.freqs)

    def collect(tickets, reqs, t0, keep=()):
        """Results in submission order; each is logged as it completes.  Only
        the requests in `keep` retain their Z_p (the rest drop it on arrival)."""
        out = [None] * len(tickets)
        pending = list(range(len(tickets)))
        while pending:
            still = []
            for i in pending:
                x = mbt.mbt_server_wait(srv, tickets[i], 0)
                if x is None:
                    still.append(i)
                    continue
                if i not in keep:
                    x["Zp"] = None
                out[i] = x
                r = reqs[i]
                log("  request %d (%dx%d, M=%d, %d freq, %d scans) status %d, latency %.2f s, iters %s, at %.1f s" % (
                    i, r.lattice.nx, r.lattice.ny, r.dipole.nbases, len(r.freqs), len(r.theta), x["status"],
                    x["t_done"] - x["t_submit"], list(int(v) for v in x["iters_max"]), x["t_done"] - t0))
            pending = still
            if pending:
                time.sleep(0.02)
        return out

    try:
        warm = W.serving_stream(args.serve_warmup, 0.0, seed=1)
        log("serving: warm-up with %d requests" % len(warm))
        collect([submit(r) for r in warm], warm, mbt.mbt_server_clock(srv))
        sat_n = args.serve_saturation if args.serve_saturation > 0 else args.serve
        if args.serve_rate > 0:
            sat_rate, sat_solves, bad = args.serve_rate, None, None
            log("serving: saturation rate given: %.3f requests/s" % sat_rate)
        else:
            reqs = W.serving_stream(sat_n, 1.0, seed=0)
            log("serving: saturation run, %d requests submitted at once" % len(reqs))
            t0 = mbt.mbt_server_clock(srv)
            tickets = [submit(r) for r in reqs]
            res = collect(tickets, reqs, t0)
            t_sat = max(x["t_done"] for x in res) - t0
            okm = [x["status"] == mbt.MBT_OK for x in res]
            sat_rate = len(reqs) / t_sat
            sat_solves = sum(solves(r) for r, g in zip(reqs, okm) if g) / t_sat
            bad = int(len(res) - sum(okm))
            log("serving: saturation %.3f requests/s, %.1f solves/s of converged requests (%d not converged)" % (
                sat_rate, sat_solves, bad))
        loads = [float(v) for v in str(args.load).split(",")]

        def summary(res, reqs, t0):
            """Throughput and latency count only requests that met the accuracy
            target (status MBT_OK); unconverged ones are reported beside them."""
            ok = [x["status"] == mbt.MBT_OK for x in res]
            lat = np.array([x["t_done"] - x["t_submit"] for x, g in zip(res, ok) if g]) * 1e3
            wait = np.array([x["t_start"] - x["t_submit"] for x, g in zip(res, ok) if g]) * 1e3
            lat_all = np.array([x["t_done"] - x["t_submit"] for x in res]) * 1e3
            span = max(x["t_done"] for x in res) - t0
            return {"solves_per_s": sum(solves(r) for r, g in zip(reqs, ok) if g) / span, "span_s": span,
                    "solves_per_s_incl_unconverged": sum(solves(r) for r in reqs) / span,
                    "requests_ok": int(sum(ok)), "requests": len(res),
                    "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                   "mean": float(lat.mean()), "queue_wait_p50": float(np.percentile(wait, 50)),
                                   "p99_incl_unconverged": float(np.percentile(lat_all, 99))},
                    "not_converged": int(len(res) - sum(ok)),
                    "not_converged_requests": [i for i, g in enumerate(ok) if not g]}

        runs = []
        checks = {}
        if not any(load > 0 for load in loads):
            # the latencies reported are those of the saturation run
            runs.append(dict(summary(res, reqs, t0), load_vs_saturation=0.0, rate_rps=None))
        for load in loads:
            if load <= 0:
                continue
            rate = load * sat_rate
            reqs = W.serving_stream(args.serve, rate, seed=0)
            # a seeded sample of requests small enough for the dense CPU oracle, and one of them
            # re-served alone afterwards for the alone-versus-in-the-mix comparison
            small = [i for i, r in enumerate(reqs) if r.lattice.nx * r.lattice.ny * r.dipole.nbases <= 6000]
            rng = np.random.default_rng(5)
            keep = set(int(i) for i in rng.choice(small, size=min(args.serve_verify, len(small)), replace=False)) \
                if args.serve_verify > 0 and small else set()
            log("serving: Poisson stream at %.3f requests/s (%.0f%% of saturation), %d requests" % (
                rate, 100 * load, len(reqs)))
            t0 = mbt.mbt_server_clock(srv)
            tickets = []
            for i, r in enumerate(reqs):
                dt = t0 + r.arrival - mbt.mbt_server_clock(srv)
                if dt > 0:
                    time.sleep(dt)
                tickets.append(submit(r))
                log("  submitted request %d (%dx%d, M=%d, %d freq) at %.1f s" % (
                    i, r.lattice.nx, r.lattice.ny, r.dipole.nbases, len(r.freqs), mbt.mbt_server_clock(srv) - t0))
            res = collect(tickets, reqs, t0, keep)
            runs.append(dict(summary(res, reqs, t0), load_vs_saturation=load, rate_rps=rate))
            log("serving: load %.2f: %.1f solves/s (converged requests), %d of %d converged, p50 %.1f s, "
                "p99 %.1f s" % (load, runs[-1]["solves_per_s"], runs[-1]["requests_ok"], len(reqs),
                                runs[-1]["latency_ms"]["p50"] / 1e3, runs[-1]["latency_ms"]["p99"] / 1e3))
            if keep and not checks:
                checks = verify_served(mbt, srv, submit, collect, reqs, res, sorted(keep))
                log("serving: verification %s" % checks)
    finally:
        mbt.mbt_server_destroy(srv)
        mbt.mbt_ctx_destroy(ctx)
    head = runs[0]
    return {"metric": "served port-excitation solves/s and p50/p99 request latency, Poisson stream",
            "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "dipole_serving_stream", "requests": len(reqs), "warmup_requests": len(warm),
                       "slots": args.slots, "rate_rps": head["rate_rps"],
                       "load_vs_saturation": head["load_vs_saturation"],
                       "nx_ny": [8, 48], "nbases": [15, 31], "nfreq": [1, 8], "nscan": [1, 64],
                       "restart": args.restart, "refine_tol": args.refine_tol, "inner_tol": args.inner_tol,
                       "max_cycles": args.serve_max_cycles},
            "latency_ms": head["latency_ms"],
            "saturation": {"requests_per_s": sat_rate, "solves_per_s": sat_solves, "not_converged": bad,
                           "requests": sat_n if args.serve_rate <= 0 else None},
            "not_converged": head["not_converged"], "span_s": head["span_s"], "loads": runs,
            "verification": checks}


def verify_served(mbt, srv, submit, collect, reqs, res, ids):
    """Served results of a seeded sample of the stream against the dense CPU
    oracle (every frequency: Z_p norm-wise and entry-wise, the ARC), and the
    first sampled request served again alone, compared bit for bit with its
    result from inside the stream."""
    from oracle import mom
    out = {"requests": [], "target": 1e-6}
    worst = 0.0
    for i in ids:
        r, x = reqs[i], res[i]
        if x["status"] != mbt.MBT_OK:
            out["requests"].append({"id": i, "status": int(x["status"])})
            continue
        ez, ee, eg = [], [], []
        for fi, s in enumerate(r.freqs):
            o = mom.solve_array(r.lattice, r.dipole, s, r.theta, r.phi, z0=r.z0)
            log("  verify: request %d (%dx%d, M=%d) frequency %.4f checked against the oracle"
                % (i, r.lattice.nx, r.lattice.ny, r.dipole.nbases, s))
            d = x["Zp"][fi] - o.Zp
            ez.append(float(np.linalg.norm(d) / np.linalg.norm(o.Zp)))
            ee.append(float(np.max(np.abs(d)) / np.max(np.abs(o.Zp))))
            eg.append(float(np.max(np.abs(x["Gamma"][fi] - o.Gamma) / np.maximum(1.0, np.abs(o.Gamma)))))
        worst = max(worst, max(ez), max(ee))
        out["requests"].append({"id": i, "nx": r.lattice.nx, "ny": r.lattice.ny, "nbases": r.dipole.nbases,
                                "freqs": list(r.freqs), "zp_rel": max(ez), "zp_max_entry_rel": max(ee),
                                "gamma_rel": max(eg)})
    out["zp_worst"] = worst
    out["meets_target"] = bool(worst <= 1e-6)
    j = ids[0]
    alone = collect([submit(reqs[j])], [reqs[j]], mbt.mbt_server_clock(srv), keep={0})[0]
    same = all(np.array_equal(alone[k], res[j][k]) for k in ("Zp", "Za", "Gamma", "Gamma_wave"))
    out["alone_vs_mix"] = {"id": j, "bit_identical": bool(same)}
    return out


def blocks_shape(args):
    """Largest single-GPU shape: 64 x 64 elements of 96 bases (N = 393,216, FFT
    grid 128 x 128) with seeded synthetic blocks (a solver-only variant of the
    bowtie workload, --bowtie), 32 port excitations per operator, 5 operators; FP32 products
    with FP64 refinement.  Reports operator applications per second and the
    rooflines of the per-bin product (large-block MFMA kernel) and the FFTs."""
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    nx, ny, M, seeds, ports = W.blocks_64x64_m96_shape()
    ctx = mbt.mbt_ctx_create(0)
    per = []
    kern = {}
    try:
        for seed in seeds[:args.blocks]:
            log("blocks: operator %d (64x64x96), generating" % seed)
            T = W.synthetic_blocks(nx, ny, M, seed=seed)
            arr = mbt.mbt_array_create_blocks(ctx, T)
            del T
            try:
                opts = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=32,
                                            refine_tol=1e-10)
                Y, it, st0 = mbt.mbt_port_admittance(ctx, arr, 1.0, ports, opts)   # builds and caches the operator
                classes = [0, 6, 4, 5] if seed == seeds[0] else [0]
                for kc in classes:
                    if kc:
                        mbt.mbt_prof_start(kc)
                    t0 = time.perf_counter()
                    Y, it, st = mbt.mbt_port_admittance(ctx, arr, 1.0, ports, opts)
                    dt = time.perf_counter() - t0
                    if kc:
                        p = mbt.mbt_prof_read()
                        mbt.mbt_prof_start(0)
                        kern[{6: "bin_product", 4: "fft_fwd_pad", 5: "fft_inv_crop"}[kc]] = p
                    else:
                        per.append({"seed": seed, "seconds": dt, "matvecs": st["matvecs"], "iters_max": st["iters_max"],
                                    "outer_steps": st["outer_steps"], "true_relres_max": st["true_relres_max"],
                                    "setup_s": st0["t_setup"]})
                        log("  solve %.3f s, %d matvecs, iters %d, outer %d, relres %.1e (setup %.1f s)" % (
                            dt, st["matvecs"], st["iters_max"], st["outer_steps"], st["true_relres_max"],
                            st0["t_setup"]))
            finally:
                mbt.mbt_array_destroy(arr)
    finally:
        mbt.mbt_ctx_destroy(ctx)
    tot_t = sum(x["seconds"] for x in per)
    tot_mv = sum(x["matvecs"] for x in per)
    out = {"metric": "operator applications per second, 64x64 elements of 96 bases (synthetic blocks)",
           "value": tot_mv / tot_t, "unit": "matvecs/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "blocks_64x64_m96", "nx": nx, "ny": ny, "nbases": M, "unknowns": nx * ny * M,
                      "grid": [128, 128], "rhs": len(ports), "operators": len(per), "restart": 32,
                      "refine_tol": 1e-10},
           "solves_per_s": len(ports) * len(per) / tot_t, "per_operator": per, "kernels": {}}
    for name, p in kern.items():
        if p["launches"] and p["ms"] > 0:
            gbs = p["bytes"] / (p["ms"] * 1e-3) / 1e9
            tfs = p["flops"] / (p["ms"] * 1e-3) / 1e12
            out["kernels"][name] = {"achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "achieved_TFs": tfs,
                                    "fp32_mfma_frac": tfs / 157.3, "avg_launch_ms": p["ms"] / p["launches"],
                                    "launches": p["launches"]}
    return out


# inner tolerance of the bowtie workload's mixed path: the best of 1e-4, 1e-3 and 3e-3 with GMRES(24..50)
# inner solves at s = 1.0 and 1.3 (four outer steps to 1e-9 either way)
BOWTIE_INNER_TOL = 3e-3


def bowtie(args):
    """Largest single-GPU instance: 64 x 64 planar bowties (96 RWG functions
    each, N = 393,216, FFT grid 128 x 128), 32 phased-voltage excitations
    (broadside first, then seeded scan directions) at 5 frequencies in 0.5-1.5
    f0, with the center element's active impedance and ARC.  Each frequency runs
    the whole path with nothing cached: RWG fill, block spectra, preconditioner,
    solve, extraction.  The mixed path (FP32 products, FP64 refinement) is timed
    against the FP64 path and their Za / Gamma are compared."""
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    mesh, lat, freqs, theta, phi = W.bowtie_64x64_workload()
    ctx = mbt.mbt_ctx_create(0)
    arr = mbt.mbt_array_create_rwg(ctx, mesh, lat)
    paths = {
        "mixed": mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=args.restart,
                                      refine_tol=1e-9, refine_max=6, inner_tol=BOWTIE_INNER_TOL,
                                      flags=mbt.MBT_FLAG_NO_CACHE),
        "fp64": mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=50, tol=1e-10,
                                     flags=mbt.MBT_FLAG_NO_CACHE),
    }
    res = {name: [] for name in paths}
    kern = {}
    try:
        log("bowtie: 64x64 x 96 RWG, %d frequencies x %d scans; warm-up" % (len(freqs), len(theta)))
        mbt.mbt_scan_solve(ctx, arr, float(freqs[2]), paths["mixed"], theta[:2], phi[:2], want_ip=False,
                           allow_noconv=True)
        for name, opts in paths.items():
            for s in freqs:
                t0 = time.perf_counter()
                r = mbt.mbt_scan_solve(ctx, arr, float(s), opts, theta, phi, want_ip=False, allow_noconv=True)
                dt = time.perf_counter() - t0
                st = r["stats"]
                res[name].append({"freq_ratio": float(s), "seconds": dt, "setup_s": st["t_setup"],
                                  "solve_s": st["t_solve"], "iters_min": st["iters_min"], "iters_max": st["iters_max"],
                                  "outer_steps": st["outer_steps"], "matvecs": st["matvecs"],
                                  "true_relres_max": st["true_relres_max"], "status": int(r["status"]),
                                  "Za": r["Za"], "Gamma": r["Gamma"]})
                log("  %s s=%.2f: %.3f s (setup %.3f, solve %.3f), iters %d..%d, outer %d, relres %.1e, status %d, "
                    "Za[0] %.4f%+.4fj" % (name, s, dt, st["t_setup"], st["t_solve"], st["iters_min"],
                                          st["iters_max"], st["outer_steps"], st["true_relres_max"], r["status"],
                                          r["Za"][0].real, r["Za"][0].imag))
        # kernel classes of the mixed path's solve (operator cached for these runs)
        cached = mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=args.restart,
                                      refine_tol=1e-9, refine_max=6, inner_tol=BOWTIE_INNER_TOL)
        mbt.mbt_scan_solve(ctx, arr, 1.0, cached, theta, phi, want_ip=False, allow_noconv=True)
        for kc, kname in ((6, "bin_product"), (4, "fft_fwd_pad"), (5, "fft_inv_crop"), (2, "arnoldi_update_dots")):
            mbt.mbt_prof_start(kc)
            mbt.mbt_scan_solve(ctx, arr, 1.0, cached, theta, phi, want_ip=False, allow_noconv=True)
            kern[kname] = mbt.mbt_prof_read()
            mbt.mbt_prof_start(0)
    finally:
        mbt.mbt_array_destroy(arr)
        mbt.mbt_ctx_destroy(ctx)
    nsolve = len(theta) * len(freqs)
    t_mixed = sum(x["seconds"] for x in res["mixed"])
    t_fp64 = sum(x["seconds"] for x in res["fp64"])
    za_err = max(float(np.max(np.abs(a["Za"] - b["Za"]) / np.abs(b["Za"]))) for a, b in zip(res["mixed"], res["fp64"]))
    g_err = max(float(np.max(np.abs(a["Gamma"] - b["Gamma"]) / np.maximum(1.0, np.abs(b["Gamma"]))))
                for a, b in zip(res["mixed"], res["fp64"]))
    for v in res.values():
        for x in v:
            x["Za_first"] = [float(x["Za"][0].real), float(x["Za"][0].imag)]
            del x["Za"], x["Gamma"]
    out = {"metric": "scan-excitation solves/s, 64x64 planar bowties (96 RWG bases), whole path per frequency",
           "value": nsolve / t_mixed, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "bowtie_64x64_m96", "nx": 64, "ny": 64, "nbases": 96, "unknowns": 64 * 64 * 96,
                      "grid": [128, 128], "scans": len(theta), "freq_ratio": [float(f) for f in freqs],
                      "mixed": {"restart": args.restart, "inner_tol": BOWTIE_INNER_TOL, "refine_tol": 1e-9,
                                "refine_max": 6},
                      "fp64": {"restart": 50, "tol": 1e-10}, "preconditioner": "element_block"},
           "fp64_solves_per_s": nsolve / t_fp64, "speedup_vs_fp64": t_fp64 / t_mixed,
           "mixed_vs_fp64": {"za_max_rel": za_err, "gamma_max_rel": g_err},
           "per_frequency": res, "kernels": {}}
    for name, p in kern.items():
        if p["launches"] and p["ms"] > 0:
            gbs = p["bytes"] / (p["ms"] * 1e-3) / 1e9
            out["kernels"][name] = {"achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                                    "avg_launch_ms": p["ms"] / p["launches"], "launches": p["launches"]}
    return out


def small(args):
    """The 5x5 array of 15-basis dipoles (25 ports, broadside + 10 scans): the
    whole path per request, operator rebuilt each time; latency-bound.  (Its
    accuracy against the oracle is checked by the GPU tests.)"""
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    w = W.cpu_size_5x5()
    ctx = mbt.mbt_ctx_create(0)
    arr = mbt.mbt_array_create_dipole(ctx, w.dipole, w.lattice)
    out = {}
    try:
        for name, opts in (("mixed", mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK,
                                                          flags=mbt.MBT_FLAG_NO_CACHE)),
                           ("fp64", mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK,
                                                         flags=mbt.MBT_FLAG_NO_CACHE))):
            mbt.mbt_solve(ctx, arr, 1.0, opts, w.theta, w.phi, w.z0)
            ts = []
            for _ in range(max(args.steps, 5)):
                t0 = time.perf_counter()
                r = mbt.mbt_solve(ctx, arr, 1.0, opts, w.theta, w.phi, w.z0)
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            out[name] = {"solves_per_s": 25 / t, "ms_per_request": 1e3 * t, "iters_max": r["stats"]["iters_max"],
                         "outer_steps": r["stats"]["outer_steps"]}
            log("small %s: %.2f ms per request, %.0f solves/s" % (name, 1e3 * t, 25 / t))
    finally:
        mbt.mbt_array_destroy(arr)
        mbt.mbt_ctx_destroy(ctx)
    return {"metric": "port-excitation solves/s, 5x5 dipoles (latency-bound, whole path per request)",
            "value": out["mixed"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic", "config": {"workload": w.name, "ports": 25, "nscan": len(w.theta)},
            "paths": out}


def shard(args):
    """One GPU's share of the all-port workload under a split of the ports over
    GPUs: the admittance columns of R ports of the 32x32 array (ports 0..R-1),
    mixed and FP64 paths with the headline settings; no extraction (Z_p needs
    every column, gathered across GPUs)."""
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    w = W.gpu_size_32x32()
    ctx = mbt.mbt_ctx_create(0)
    arr = mbt.mbt_array_create_dipole(ctx, w.dipole, w.lattice)
    ports = list(range(args.shard))
    out = {}
    try:
        for name, opts in (
                ("mixed", mbt.mbt_default_opts(prec=mbt.MBT_FP32, pc=mbt.MBT_PC_ELEMENT_BLOCK, restart=args.restart,
                                               refine_tol=args.refine_tol, inner_tol=args.inner_tol)),
                ("fp64", mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK,
                                              restart=args.fp64_restart, tol=args.fp64_tol))):
            mbt.mbt_port_admittance(ctx, arr, 1.0, ports, opts)   # builds the operator, warms up
            ts = []
            for _ in range(args.steps):
                t0 = time.perf_counter()
                Y, it, st = mbt.mbt_port_admittance(ctx, arr, 1.0, ports, opts)
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            out[name] = {"solves_per_s": len(ports) / t, "seconds": t, "iters_max": int(it.max()),
                         "outer_steps": st["outer_steps"]}
            log("shard %s: R=%d, %.3f s, %.1f solves/s, iters %d" % (name, len(ports), t, len(ports) / t, it.max()))
    finally:
        mbt.mbt_array_destroy(arr)
        mbt.mbt_ctx_destroy(ctx)
    return {"metric": "port-excitation solves/s of one GPU's port share (admittance columns only)",
            "value": out["mixed"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "dipole_32x32_m31_port_share", "rhs": len(ports), "steps": args.steps,
                       "operator_cached": True},
            "paths": out}


def sweep(args):
    """Precision form: the 5x5 array at 21 frequencies (one request, served
    concurrently) in FP64, FP32, FP16 and BF16 products with at most three FP64
    refinement steps; per-frequency Z_p and ARC errors against the stored
    oracle results."""
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    ref = np.load(os.path.join(ROOT, "tests", "golden", "dipole_5x5_m15_21f_reference.npz"))
    w = W.sweep_5x5_21f()
    ctx = mbt.mbt_ctx_create(0)
    srv = mbt.mbt_server_create(ctx, 4)
    out = {}
    try:
        for name, prec in (("fp64", 0), ("fp32", 1), ("fp16", 3), ("bf16", 2)):
            opts = mbt.mbt_default_opts(prec=prec, pc=mbt.MBT_PC_ELEMENT_BLOCK, refine_max=3, refine_tol=1e-9)
            t = mbt.mbt_server_submit(srv, (w.dipole.length, w.dipole.radius, w.dipole.nbases),
                                      (w.lattice.nx, w.lattice.ny, w.lattice.dx, w.lattice.dy),
                                      w.freqs, w.theta, w.phi, opts)
            r = mbt.mbt_server_wait(srv, t)
            ez = [float(np.linalg.norm(r["Zp"][i] - ref["Zp"][i]) / np.linalg.norm(ref["Zp"][i])) for i in range(21)]
            eg = [float(np.max(np.abs(r["Gamma"][i] - ref["Gamma"][i]) / np.abs(ref["Gamma"][i]))) for i in range(21)]
            out[name] = {"status": int(r["status"]), "seconds": r["t_done"] - r["t_submit"],
                         "zp_rel": ez, "gamma_rel": eg, "zp_rel_max": max(ez), "gamma_rel_max": max(eg)}
            log("%s: %.3f s, max |dZp|/|Zp| %.2e, max |dGamma|/|Gamma| %.2e" % (
                name, out[name]["seconds"], max(ez), max(eg)))
    finally:
        mbt.mbt_server_destroy(srv)
        mbt.mbt_ctx_destroy(ctx)
    return {"metric": "per-frequency Z_p and ARC error vs the FP64 oracle, 21-frequency sweep",
            "config": {"workload": w.name, "freqs": list(w.freqs), "refine_max": 3}, "data": "synthetic",
            "n_gpus": 1, "results": out}


def predict(args):
    """Array-size sweep of the coupling predictors (Sec. II-E) on N x N dipole
    arrays (odd N, so the center element is unique): the center element's
    active impedance at broadside and with the beam 30 degrees off broadside in
    the E-plane, its deviation xi(N) from the mean over the three largest
    arrays, xi_Z(N) of each array's own Z_p, xi_S(N) from the largest array's
    S_cc and S_1 (decay -2 and -2.4), and the decay of |C_n| of the largest
    array.  FP64 solves; all predictors computed on the GPU."""
    from paper_2608_17844_amd import mbt
    from paper_2608_17844_amd import workloads as W
    s = args.predict_freq
    dip = W.Dipole(0.5, 0.005, 15)
    sizes = list(range(3, args.predict + 1, 2))
    th = np.array([0.0, np.deg2rad(30.0)])
    ph = np.array([0.0, 0.0])
    ctx = mbt.mbt_ctx_create(0)
    rows = []
    t0 = time.perf_counter()
    try:
        opts = mbt.mbt_default_opts(prec=mbt.MBT_FP64, pc=mbt.MBT_PC_ELEMENT_BLOCK, tol=1e-10)
        for n in sizes:
            lat = W.Lattice(n, n, 0.5, 0.5)
            arr = mbt.mbt_array_create_dipole(ctx, dip, lat)
            try:
                out = mbt.mbt_solve(ctx, arr, s, opts, th, ph, 50.0)
            finally:
                mbt.mbt_array_destroy(arr)
            pr = mbt.mbt_predict(ctx, lat, out["Zp"], z0=50.0, nq=2 * n)
            c = pr["center"]
            rows.append({"n": n, "electrical_size": n * 0.5 * s, "za_broadside": out["Za"][0], "za_30": out["Za"][1],
                         "zp_cc": out["Zp"][c, c], "xi_z": pr["xi_z"], "xi_z_max": pr["xi_z_max"],
                         "border_sum": pr["border_sum"], "pred": pr, "Zp_row": out["Zp"][c, :]})
            log("predict: %dx%d  Za(0) %s  Za(30) %s  xi_Z %.3e" % (n, n, out["Za"][0], out["Za"][1], pr["xi_z"]))
        big = rows[-1]
        ref0 = np.mean([r["za_broadside"] for r in rows[-3:]])
        ref30 = np.mean([r["za_30"] for r in rows[-3:]])
        for r in rows:
            lat = W.Lattice(r["n"], r["n"], 0.5, 0.5)
            r["xi_broadside"] = abs(r["za_broadside"] / ref0 - 1)
            r["xi_30"] = abs(r["za_30"] / ref30 - 1)
            r["xi_s_2"] = mbt.mbt_predict_xi_s(ctx, lat, s, big["pred"]["s_cc"], big["pred"]["s_1"], abs(r["zp_cc"]),
                                               50.0, -2.0)
            r["xi_s_24"] = mbt.mbt_predict_xi_s(ctx, lat, s, big["pred"]["s_cc"], big["pred"]["s_1"],
                                                abs(r["zp_cc"]), 50.0, -2.4)
    finally:
        mbt.mbt_ctx_destroy(ctx)
    pr = big["pred"]
    n = pr["n"]
    pos = n > 0
    Cn = np.abs(pr["Cn"][pos])
    nmax = big["n"]
    fit = lambda k, v: float(np.polyfit(np.log(k), np.log(v), 1)[0])
    kk = n[pos]
    sel = kk >= 3
    out = {"metric": "coupling predictors over an array-size sweep (Sec. II-E)", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "dipole_NxN_m15_sweep", "sizes": sizes, "freq_ratio": s, "spacing_wavelengths":
                      0.5 * s, "scan": ["broadside", "30 deg E-plane"], "z0": 50.0},
           "seconds": time.perf_counter() - t0,
           "rows": [{k: (v if not isinstance(v, complex) else [v.real, v.imag]) for k, v in r.items()
                     if k not in ("pred", "Zp_row")} for r in rows],
           "largest": {"n": nmax, "C_n_abs": Cn.tolist(), "n_values": kk.tolist(),
                       "C_n_slope_n_ge_3": fit(kk[sel], Cn[sel]) if sel.sum() >= 2 else None,
                       "s_cc": [pr["s_cc"].real, pr["s_cc"].imag], "s_1": [pr["s_1"].real, pr["s_1"].imag]}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--pc", choices=["element_block", "normal_eq"], default="element_block")
    ap.add_argument("--solver", choices=["gmres", "pcg", "cocg"], default="gmres",
                    help="pcg: the paper's PCG on the normal equations with P_A (both paths); "
                         "cocg: COCG on Z with P_K (both paths)")
    ap.add_argument("--kernel", choices=sorted(KERNEL_CODES), default="arnoldi_update_dots")
    ap.add_argument("--restart", type=int, default=32, help="restart length of the mixed path's inner GMRES")
    ap.add_argument("--fp64-restart", type=int, default=50, help="restart length of the FP64 path (the workload's)")
    ap.add_argument("--refine-tol", type=float, default=1e-7, help="FP64 refinement stop of the mixed path")
    ap.add_argument("--inner-tol", type=float, default=1e-3, help="inner FP32 GMRES tolerance of the mixed path")
    ap.add_argument("--fp64-tol", type=float, default=1e-9,
                    help="FP64 GMRES tolerance giving the same accuracy target (1e-6 on Z_p entries and ARC)")
    ap.add_argument("--fp32-basis", action="store_true",
                    help="keep the mixed path's Krylov basis in FP32 instead of the packed 24-bit format")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-kernel-table", action="store_true")
    ap.add_argument("--serve", type=int, default=0, help="run the serving stream with this many requests instead")
    ap.add_argument("--serve-warmup", type=int, default=20)
    ap.add_argument("--serve-saturation", type=int, default=0,
                    help="requests of the saturation run (default: as many as the stream)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="use this saturation rate (requests/s) instead of measuring it")
    ap.add_argument("--serve-verify", type=int, default=3,
                    help="served requests checked against the dense CPU oracle (and one re-served alone)")
    ap.add_argument("--serve-max-cycles", type=int, default=8,
                    help="restart cycles per inner solve in the serving run (slow-converging requests report ENOCONV)")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--load", default="0.8",
                    help="stream rates as fractions of saturation, comma-separated (the first is the headline "
                         "of the JSON line; 0: report the saturation run only)")
    ap.add_argument("--sweep", action="store_true", help="run the 21-frequency precision sweep instead")
    ap.add_argument("--small", action="store_true", help="time the 5x5 array's whole path instead")
    ap.add_argument("--shard", type=int, default=0,
                    help="time one GPU's share of the ports (this many RHS, admittance only) instead")
    ap.add_argument("--blocks", type=int, default=0,
                    help="run the 64x64x96 synthetic-block shape with this many operators (1..5) instead")
    ap.add_argument("--bowtie", action="store_true",
                    help="run the 64x64 planar-bowtie scan workload (RWG fill, 5 frequencies x 32 scans) instead")
    ap.add_argument("--predict", type=int, default=0,
                    help="run the coupling-predictor sweep over N x N arrays up to this N (odd) instead")
    ap.add_argument("--predict-freq", type=float, default=1.1,
                    help="frequency ratio of the predictor sweep (1.1: spacing 0.55 wavelengths)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the CPU oracle on the whole 32x32 workload (minutes; no GPU) instead")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy kernel three times (a known-size reference "
                         "for hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver's workload fits one MI355X and no multi-GPU path "
              "is built (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of %d bytes" % (src.numel() * 4))
        del src, dst
    if args.serve > 0:
        result = serve(args)
    elif args.sweep:
        result = sweep(args)
    elif args.shard > 0:
        result = shard(args)
    elif args.small:
        result = small(args)
    elif args.blocks > 0:
        result = blocks_shape(args)
    elif args.bowtie:
        result = bowtie(args)
    elif args.predict > 0:
        result = predict(args)
    elif args.cpu_full:
        result = cpu_full(args)
    else:
        result = headline(args)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
