#!/usr/bin/env python3
"""Helmholtz solves/s of the additive overlapping DDM on one MI355X.

Headline workload (one "step" = one batch solve): the 2D layered medium on
the unit square, 2048^2 interior cells (8 flat layers with velocities
1.5-4.5 plus a 10% smoothed perturbation, 8 points per wavelength at the
slowest velocity), 5-point PML operator with a 20-cell PML (sigma0 for 1e-6
reflection), 16x16 subdomains of 128^2 cells with 8-cell overlap, 16 seeded
unit-mass Gaussian sources (std 2h) solved together.  `value`: the mixed
path as the workload states it -- block inverses and local solves in
complex64, FGMRES(30) right-preconditioned by K = N1 + N2 DDM steps with the
Krylov vectors, residual and assembly in FP64 -- to FP64 relative residual
1e-6, counting only the right-hand sides that reached it.  The same solve in
plain FP64 (complex128 everywhere) is timed beside it (`fp64`), with each
result's difference to it, and both as stationary iterations.  The
factorisation runs once before the timed region (reported separately), as in
the paper's timings.  The 1024^2 constant-medium workload (8x8 subdomains,
4 RHS) is measured briefly as a sub-record (`const_1024`).

`roofline` is for the dominant kernel of `value`, the complex64 block
substitution, from a live pass with HIP events around every substitution
launch on the library's stream: algorithmic bytes (every stored block
inverse read once per sweep, plus the block vectors) / summed launch time;
`traffic` is the HBM traffic per launch from the committed rocprofv3 counter
record of the same kernel source.  `cpu_baseline` runs the CPU oracle
(unchanged, FP64) on a 4x4-subdomain cut of the same medium and scales its
per-step time to the 256 subdomains and to the local-solve steps of the
measured solve.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Helmholtz solves/sec at rel.resid 1e-6 (mixed vs FP64 DDM); p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def workloads():
    """name -> (builder, stationary tolerance, description).  2d-1024 is the
    default (the headline configuration); the others are measured with
    --workload and are not the bench line's `value`."""
    import ddm_inputs as di
    return {
        "2d-1024": (lambda: di.const_2d_1024(nrhs=4), 1e-6,
                 "2D constant medium, 1024^2 interior (h=1/1024, omega=2*pi*102.4, 10 ppw), 5-point FD, PML 16 "
                 "(R=1e-6), 8x8 subdomains of 128^2 with overlap 8, 4 seeded Gaussian sources (std 2h)"),
        "2d-80": (di.const_2d_80, 1e-8,
                 "2D constant medium, 80^2 interior (omega=2*pi*8, 10 ppw), 5-point FD, PML 10 (R=1e-6), 2x2 "
                 "subdomains, overlap 4, one Gaussian source (std 2h) at the centre"),
        "2d-2048-layered": (lambda: di.layered_2d_2048(nrhs=16), 1e-6,
                 "2D layered medium, 2048^2 interior (8 layers 1.5-4.5 plus 10% smoothed perturbation, 8 ppw at "
                 "c=1.5), 5-point FD, PML 20 (R=1e-6), 16x16 subdomains, overlap 8, 16 seeded Gaussian sources"),
        "3d-96": (di.const_3d_96, 1e-6,
                 "3D constant medium, 96^3 interior (omega=2*pi*9.6, 10 ppw), 7-point FD, PML 6 (R=1e-6), 3x3x3 "
                 "subdomains, overlap 2, plane blocks of up to 46^2, one Gaussian source (std 2h) at the centre"),
    }


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(v, p):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=float), p)) if len(v) else None


SUBST_KERNELS = {"chain": "k_solve_chain", "chain2": "k_solve_chain2", "perline": "k_solve_line",
                 "mma": "k_solve_mma"}


# kernel sources whose hash a counter record of the variant is valid for
SUBST_SOURCES = {"mma": ["ddm_solve_mma.hip", "ddm_mma.h", "ddm_sync.h"]}


def kernel_sha(kernel_variant):
    import hashlib
    hsh = hashlib.sha256()
    for f in SUBST_SOURCES.get(kernel_variant, ["ddm_solve.hip", "ddm_sync.h"]):
        with open(os.path.join(ROOT, "paper_1807_04180_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def recorded_traffic(kernel_variant, tag, profiles_dir=None):
    """HBM traffic per launch of the substitution kernel from the committed
    rocprofv3 counter record profiles/<kernel>_<tag>_traffic.json, only if the
    kernel source is unchanged since the counters were taken."""
    name = SUBST_KERNELS.get(kernel_variant)
    if name is None:
        return None
    path = os.path.join(profiles_dir or os.path.join(ROOT, "profiles"), "%s_%s_traffic.json" % (name, tag))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_sha(kernel_variant):
        return None
    return rec["traffic_bytes_per_launch"]


def run_cpu_baseline(nrhs_full, nsub_full, steps_full, tol):
    """Oracle on a 4x4 cut of the workload; per-step time scaled by subdomain
    count (the oracle's work per step is linear in it) and by the full
    solve's step count."""
    import numpy as np
    import ddm_inputs as di
    from oracle import Oracle

    w = di.const_2d_1024_cut(4, nrhs=nrhs_full)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    t0 = time.perf_counter()
    o.factor()
    t_fac = time.perf_counter() - t0
    nsteps = 12
    t0 = time.perf_counter()
    u, rr = o.ddm_run(w.f, nsteps)
    t_run = time.perf_counter() - t0
    t_step = t_run / nsteps
    conv = [int(np.argmax(rr[:, q] <= tol)) + 1 if np.any(rr[:, q] <= tol) else None for q in range(w.nrhs)]
    scale = nsub_full / o.nsub
    t_step_full = t_step * scale
    value = nrhs_full / (t_step_full * steps_full)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": value, "unit": "solves/s", "cores": threads, "kind": "oracle",
        "sample": ("oracle (FP64 banded-LU local solves, OpenMP) on a 4x4-subdomain cut of the workload "
                   "(M=512, same h, omega, PML, overlap and 128^2 cores, %d seeded Gaussians): factor %.2f s, "
                   "%d DDM steps in %.2f s (%.3f s/step, steps to 1e-6 on the cut %s); per-step time scaled "
                   "x%.0f to the %d subdomains of the full workload and x%d steps of its FP64 GPU solve"
                   % (w.nrhs, t_fac, nsteps, t_run, t_step, conv, scale, nsub_full, steps_full)),
        "factor_s_sample": t_fac, "step_s_sample": t_step,
    }


def run_cpu_baseline_layered(nrhs_full, nsub_full, local_steps_full):
    """Oracle on the 4x4-subdomain cut of the layered 2048^2 medium (same h,
    omega, PML, overlap and 128^2 cores, 16 RHS): per-step time (one local
    solve of every subdomain for every RHS, plus transfers and assembly)
    scaled by the subdomain count and by the local-solve steps of the full
    solve."""
    import ddm_inputs as di
    from oracle import Oracle

    w = di.layered_2d_2048_cut(4, nrhs=nrhs_full)
    o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
    t0 = time.perf_counter()
    o.factor()
    t_fac = time.perf_counter() - t0
    nsteps = 3
    t0 = time.perf_counter()
    o.ddm_run(w.f, nsteps)
    t_run = time.perf_counter() - t0
    t_step = t_run / nsteps
    scale = nsub_full / o.nsub
    value = nrhs_full / (t_step * scale * local_steps_full)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": value, "unit": "solves/s", "cores": threads, "kind": "oracle",
        "sample": ("oracle (FP64 banded-LU local solves, OpenMP) on the 4x4-subdomain cut of the layered 2048^2 "
                   "medium around its centre (M=512, same h, omega, PML 20, overlap 8, 128^2 cores, %d seeded "
                   "Gaussians): factor %.2f s, %d DDM steps in %.2f s (%.3f s/step); per-step time scaled x%.0f to "
                   "the %d subdomains and x%d local-solve steps of the measured solve"
                   % (w.nrhs, t_fac, nsteps, t_run, t_step, scale, nsub_full, local_steps_full)),
        "factor_s_sample": t_fac, "step_s_sample": t_step,
    }


def _rel(a, b):
    import torch
    return (torch.linalg.vector_norm(a - b, dim=1) / torch.linalg.vector_norm(b, dim=1)).tolist()


def _timed_solves(s, f, reps, warmup, **kw):
    """warmup + reps batch solves; per-rep wall time, per-RHS info of the
    last, the solution (u of the last)."""
    import torch
    u = torch.empty_like(f)
    for _ in range(warmup):
        s.solve(f, u=u, **kw)
    torch.cuda.synchronize()
    times, lat, info, st = [], [], None, 0
    conv = 0
    for _ in range(reps):
        t0 = time.perf_counter()
        _, info, st = s.solve(f, u=u, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        lat += [x["seconds"] * 1e3 for x in info]
        conv += sum(1 for x in info if x["status"] == "OK")
    return u, info, st, times, lat, conv


def _roofline(s, f, **kw):
    """live event-profiled solve: the substitution kernel's achieved bytes/s"""
    import torch
    s.profile_enable(True)
    s.solve(f, u=torch.empty_like(f), **kw)
    prof = s.profile_read()
    s.profile_enable(False)
    sub = prof["substitution"]
    achieved = sub["bytes"] / (sub["ms"] * 1e-3) / 1e9 if sub["ms"] > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": SUBST_KERNELS[s.solve_variant()], "avg_launch_us": sub["ms"] / max(sub["launches"], 1) * 1e3,
            "launches": sub["launches"], "bytes_per_launch": sub["bytes"] / max(sub["launches"], 1)}, prof


def tune_handle(s, nrhs, args):
    """autotuned substitution plan (layout, variant, chain tile) of a handle,
    from the plan cache when it holds one for this shape"""
    if args.no_autotune:
        return None
    from paper_1807_04180_amd import tuning
    t0 = time.perf_counter()
    plan = tuning.tune(s, nrhs, reps=2, cache=tuning.PlanCache())
    plan["seconds"] = time.perf_counter() - t0
    log("bench: autotune %s: %s%s, tile %d, %.2f ms per local solve (%s)"
        % ("cached" if plan["cached"] else "timed", "twisted " if plan["twisted"] else "one-directional ",
           plan["variant"], plan["chain_tile"], plan["ms"], ", ".join("%s/%s/%d %.2f" % (
               "tw" if r["twisted"] else "od", r["variant"], r["chain_tile"], r["ms"]) for r in plan.get("table", []))))
    return plan


def run_headline(args):
    """The layered 2048^2, 16-RHS workload: mixed FGMRES (value) beside
    plain FP64, stationary legs, the 1024^2 sub-record and the oracle."""
    import numpy as np
    import torch

    import ddm_inputs as di
    import paper_1807_04180_amd as ddm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = di.layered_2d_2048(nrhs=16)
    nrhs = w.nrhs
    tol = args.tol if args.tol is not None else 1e-6
    K = int(sum(w.N))
    log("bench: workload %s nglob=%d nrhs=%d on %s" % (w.name, int(np.prod(w.grid_shape)), nrhs,
                                                        torch.cuda.get_device_name(0)))
    k2 = torch.from_numpy(w.k2.reshape(-1)).to(dev)
    f = torch.from_numpy(w.f.reshape(nrhs, -1)).to(dev)
    fg = dict(method="fgmres", tol=tol, maxiter=200, restart=30, K=K)
    stat = dict(method="stationary", tol=tol, maxiter=600)
    side_reps = max(1, min(args.steps, 3))

    # ---- mixed: complex64 inverses / local solves, FP64 Krylov ----------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smx = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=True), k2, nrhs, factor=False)
    try:
        smx.factor()
        torch.cuda.synchronize()
        t_fac_mx = time.perf_counter() - t0
        log("bench: mixed setup+factor %.3f s (%.2f GB of complex64 block inverses), substitution %s"
            % (t_fac_mx, smx.factor_bytes / 1e9, smx.solve_variant()))
        if args.probe == "traffic":
            g = torch.zeros((nrhs, smx.etot), dtype=torch.complex128, device=dev)
            g[:, ::7] = 1.0
            for _ in range(3):
                smx.local_solve(g)
            src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            log("bench: traffic probe done (3 complex64 local solves, 1 GiB copy)")
            return
        plan_mx = tune_handle(smx, nrhs, args)
        umx, info_mx, st_mx, t_mx, lat_mx, conv_mx = _timed_solves(smx, f, args.steps, args.warmup, **fg)
        roof_mx, prof_mx = _roofline(smx, f, **fg)
        roof_mx["traffic"] = recorded_traffic(smx.solve_variant(), "layered2048_c64")
        us_mx, info_smx, st_smx, t_smx, lat_smx, conv_smx = _timed_solves(smx, f, side_reps, 1, **stat)
    finally:
        smx.close()
    torch.cuda.empty_cache()
    t_timed = sum(t_mx)
    value = conv_mx / t_timed
    log("bench: mixed FGMRES(30)+DDM(K=%d): %.2f solves/s (%d of %d RHS converged), %.1f ms/batch, iters %s"
        % (K, value, conv_mx, nrhs * args.steps, 1e3 * t_timed / args.steps, sorted({x["iters"] for x in info_mx})))

    # ---- plain FP64 -------------------------------------------------------
    t0 = time.perf_counter()
    s64 = ddm.HelmholtzDDM(ddm.Problem.from_workload(w), k2, nrhs, factor=False)
    try:
        s64.factor()
        torch.cuda.synchronize()
        t_fac_64 = time.perf_counter() - t0
        plan_64 = tune_handle(s64, nrhs, args)
        u64, info_64, st_64, t_64, lat_64, conv_64 = _timed_solves(s64, f, side_reps, 1, **fg)
        roof_64, prof_64 = _roofline(s64, f, **fg)
        us_64, info_s64, st_s64, t_s64, lat_s64, conv_s64 = _timed_solves(s64, f, side_reps, 1, **stat)
    finally:
        s64.close()
    torch.cuda.empty_cache()
    v64 = conv_64 / sum(t_64)
    log("bench: FP64 FGMRES: %.2f solves/s; mixed x%.2f; substitution mixed %.0f GB/s, FP64 %.0f GB/s"
        % (v64, value / v64, roof_mx["achieved"], roof_64["achieved"]))

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_timed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": ("2D layered medium, 2048^2 interior (8 layers 1.5-4.5 plus 10%% smoothed "
                                "perturbation, 8 ppw at c=1.5), 5-point FD, PML 20 (R=1e-6), 16x16 subdomains of "
                                "128^2, overlap 8, 16 seeded Gaussian sources (std 2h) in one batch; complex64 block "
                                "inverses and local solves, FP64 FGMRES(30) + DDM(K=%d) to relres %.0e" % (K, tol)),
                   "global_batch": nrhs, "grid": list(w.M), "subdomains": list(w.N), "method": "fgmres",
                   "precision": "mixed"},
        "latency_ms": {"p50": pct(lat_mx, 50), "p99": pct(lat_mx, 99)},
        "converged": conv_mx, "solved": nrhs * args.steps,
        "relres": [x["relres"] for x in info_mx], "gmres_iters": [x["iters"] for x in info_mx],
        "local_solves": [x["local_solves"] for x in info_mx], "status": st_mx,
        "rel_diff_vs_fp64": _rel(umx, u64), "factor_s": t_fac_mx,
        "roofline": roof_mx,
        "kernel_time_ms_per_solve_batch": {k: v["ms"] for k, v in prof_mx.items()},
        "kernel_achieved_GBs": {k: (v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None)
                                for k, v in prof_mx.items()},
        "fp64": {"solves_per_s": v64, "ms_per_batch": sum(t_64) / side_reps * 1e3, "converged": conv_64,
                 "gmres_iters": [x["iters"] for x in info_64], "relres": [x["relres"] for x in info_64],
                 "status": st_64, "factor_s": t_fac_64, "mixed_speedup": value / v64, "roofline": roof_64},
        "autotune": {"mixed": plan_mx, "fp64": plan_64},
        # single-shot use: one batch solved once, its factorisation included
        "single_shot_solves_per_s": {
            "mixed": conv_mx / args.steps / (t_fac_mx + t_timed / args.steps),
            "fp64": conv_64 / side_reps / (t_fac_64 + sum(t_64) / side_reps)},
        "stationary": {
            "mixed": {"solves_per_s": conv_smx / sum(t_smx), "steps": [x["iters"] for x in info_smx],
                      "relres": [x["relres"] for x in info_smx], "status": st_smx,
                      "rel_diff_vs_fp64": _rel(us_mx, u64)},
            "fp64": {"solves_per_s": conv_s64 / sum(t_s64), "steps": [x["iters"] for x in info_s64],
                     "relres": [x["relres"] for x in info_s64], "status": st_s64,
                     "rel_diff_vs_fp64_fgmres": _rel(us_64, u64)},
        },
    }
    log("bench: stationary: mixed %.2f, FP64 %.2f solves/s" % (out["stationary"]["mixed"]["solves_per_s"],
                                                              out["stationary"]["fp64"]["solves_per_s"]))
    if not args.no_extras:
        out["const_1024"] = run_const_1024_brief(side_reps)
    if not args.no_cpu_baseline:
        log("bench: CPU baseline (oracle) ...")
        local_steps = max(x["local_solves"] for x in info_mx)
        out["cpu_baseline"] = run_cpu_baseline_layered(nrhs, int(np.prod(w.N)), local_steps)
        log("bench: CPU baseline %.5f solves/s" % out["cpu_baseline"]["value"])
    print(json.dumps(out), flush=True)


def run_const_1024_brief(reps):
    """the 1024^2 constant-medium workload (8x8, 4 RHS), stationary DDM to
    1e-6: FP64 (split substitution) and mixed, a few batches each"""
    import torch

    import ddm_inputs as di
    import paper_1807_04180_amd as ddm

    dev = torch.device("cuda:0")
    w = di.const_2d_1024(nrhs=4)
    k2 = torch.from_numpy(w.k2.reshape(-1)).to(dev)
    f = torch.from_numpy(w.f.reshape(w.nrhs, -1)).to(dev)
    rec = {"workload": "2D constant medium, 1024^2, 8x8 subdomains of 128^2, overlap 8, PML 16, 4 Gaussians; "
                       "stationary DDM to relres 1e-6"}
    u64 = None
    for mixed in (False, True):
        s = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), k2, w.nrhs)
        try:
            u, info, st, times, lat, conv = _timed_solves(s, f, reps, 1, method="stationary", tol=1e-6, maxiter=400)
            roof, _ = _roofline(s, f, method="stationary", tol=1e-6, maxiter=400)
        finally:
            s.close()
        key = "mixed" if mixed else "fp64"
        rec[key] = {"solves_per_s": conv / sum(times), "steps": [x["iters"] for x in info], "status": st,
                    "substitution": {"kernel": roof["kernel"], "avg_launch_us": roof["avg_launch_us"],
                                     "achieved_GBs": roof["achieved"], "frac": roof["frac"]}}
        if mixed:
            rec[key]["rel_diff_vs_fp64"] = _rel(u, u64)
        else:
            u64 = u
        log("bench: 1024^2 %s: %.1f solves/s, substitution %.0f GB/s" % (key, rec[key]["solves_per_s"], roof["achieved"]))
    torch.cuda.empty_cache()
    return rec


def make_traffic_record(fetch_dir, write_dir, tag, variant="mma", profiles_dir=None):
    """profiles/<kernel>_<tag>_traffic.json from two rocprofv3 --pmc runs of
    `bench.py --probe traffic` (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch): each counter is scaled by what it reads for the probe's 1 GiB
    device copy (the largest copy dispatch of the run)."""
    import csv
    import glob

    kname = SUBST_KERNELS[variant]

    def read(d, counter):
        rows = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    if r.get("Counter_Name") == counter:
                        rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        per = {}
        for did, name, v in rows:
            per.setdefault(did, [name, 0.0])[1] += v
        disp = sorted((did, nv[0], nv[1]) for did, nv in per.items())
        sub = [v for _, n, v in disp if kname in n]
        copies = [v for _, n, v in disp if "copy" in n.lower() and kname not in n]
        if not sub or not copies:
            raise SystemExit("no %s or copy dispatches with %s under %s" % (kname, counter, d))
        return sub, max(copies)

    fsub, fcopy = read(fetch_dir, "FETCH_SIZE")
    wsub, wcopy = read(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    fscale, wscale = gib_kib / fcopy, gib_kib / wcopy
    fb = sum(fsub) / len(fsub) * 1024.0 * fscale
    wb = sum(wsub) / len(wsub) * 1024.0 * wscale
    rec = {"kernel": kname, "workload": tag, "source_sha256": kernel_sha(variant),
           "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "traffic_bytes_per_launch": fb + wb,
           "fetch_scale": fscale, "write_scale": wscale, "fetch_kib_raw": fsub, "write_kib_raw": wsub,
           "copy_fetch_kib": fcopy, "copy_write_kib": wcopy}
    path = os.path.join(profiles_dir or os.path.join(ROOT, "profiles"), "%s_%s_traffic.json" % (kname, tag))
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote %s: reads %.3f GB + writes %.3f GB = %.3f GB per launch (scales %.4f / %.4f, %d launches)"
          % (path, fb / 1e9, wb / 1e9, (fb + wb) / 1e9, fscale, wscale, len(fsub)))


def overlap_report(trace_csv):
    """Concurrency of kernels from different HIP streams in a rocprofv3
    kernel trace (CSV with Stream_Id, Kernel_Name, Start/End_Timestamp):
    GPU busy time, time with kernels of two or more streams in flight, and
    the share of each kernel class's time that overlaps another stream's
    kernel."""
    import csv

    ev = []
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), int(r["Stream_Id"]), r["Kernel_Name"]))
    # sweep over start / end points: streams in flight at every instant
    pts = sorted([(a, 1, s) for a, b, s, _ in ev] + [(b, -1, s) for a, b, s, _ in ev])
    active = {}
    busy = multi = 0
    last = None
    multi_iv = []
    for t, d, st in pts:
        if last is not None and t > last:
            n = sum(1 for v in active.values() if v > 0)
            if n >= 1:
                busy += t - last
            if n >= 2:
                multi += t - last
                multi_iv.append((last, t))
        active[st] = active.get(st, 0) + d
        last = t

    def cls(name):
        for k, c in (("k_solve", "substitution"), ("k_transfer", "transfer"), ("k_assemble", "assembly"),
                     ("k_stencil", "residual"), ("k_factor", "factorisation")):
            if k in name:
                return c
        return "other"
    # share of each class's kernel time inside a multi-stream interval
    import bisect
    starts = [a for a, _ in multi_iv]
    by = {}
    for a, b, st, name in ev:
        c = cls(name)
        tot, ov = by.get(c, (0, 0))
        i = max(bisect.bisect_right(starts, a) - 1, 0)
        o = 0
        while i < len(multi_iv) and multi_iv[i][0] < b:
            lo, hi = max(a, multi_iv[i][0]), min(b, multi_iv[i][1])
            if hi > lo:
                o += hi - lo
            i += 1
        by[c] = (tot + (b - a), ov + o)
    streams = sorted({s for _, _, s, _ in ev})
    return {"kernels": len(ev), "streams": len(streams), "busy_ms": busy / 1e6, "multi_stream_ms": multi / 1e6,
            "multi_stream_share_of_busy": multi / busy if busy else 0.0,
            "overlapped_share_by_class": {c: (ov / tot if tot else 0.0) for c, (tot, ov) in sorted(by.items())},
            "ms_by_class": {c: tot / 1e6 for c, (tot, _) in sorted(by.items())}}


def run_serving(args):
    """Continuous-batching serving stream (Poisson arrivals of 2D solves on
    256^2 / 512^2 / 1024^2 grids, four media per grid, 1-32 sources per
    request), mixed precision, factorisations cached per problem under an HBM
    budget.  The capacity is measured first (a burst of requests all
    arriving at once), then streams of args.requests requests arrive at 0.5,
    0.8 and 1.0 x that rate; a sample of requests is solved again alone (same
    slot count) and by the oracle's global solve."""
    import numpy as np
    import torch

    import ddm_inputs as di
    import paper_1807_04180_amd as ddm
    from paper_1807_04180_amd import tuning
    from paper_1807_04180_amd.serving import Request, Server

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # warm-up: load the mixed-precision kernels on a small problem
    ws = di.small_2d(M=64, N=(2, 2), n_pml=6, n_ov=4, nrhs=2)
    sw = ddm.HelmholtzDDM(ddm.Problem.from_workload(ws, mixed=True), torch.from_numpy(ws.k2.reshape(-1)).to(dev), 2)
    sw.slot_admit(0, torch.from_numpy(ws.f[0].reshape(-1)).to(dev))
    sw.slots_step(2)
    sw.slots_poll()
    sw.close()
    # tuned plans for the stream's shapes (one per grid), outside the timed runs
    plans = None
    tuned = {}
    serve_layouts = {"any": (True, False), "onedir": (False,)}[args.serve_layouts]
    if not args.no_autotune:
        plans = tuning.PlanCache()
        for r in di.serving_stream(n_requests=40, rate=1.0):
            M = r.key[0]
            if M in tuned:
                continue
            h = ddm.HelmholtzDDM(ddm.Problem.from_workload(r.base, mixed=True),
                                 torch.from_numpy(r.base.k2.reshape(-1)).to(dev), args.slots)
            try:
                p = tuning.tune(h, args.slots, reps=2, cache=plans, layouts=serve_layouts)
            finally:
                h.close()
            tuned[M] = {k: p[k] for k in ("twisted", "variant", "chain_tile", "ms", "cached")}
            log("bench: serve plan for %d^2: %s" % (M, tuned[M]))
    torch.cuda.synchronize()

    def make_requests(stream, keep_ids=()):
        def maker(w):
            return lambda: (ddm.Problem.from_workload(w, mixed=True), torch.from_numpy(w.k2.reshape(-1)).to(dev))

        def sources(sr):
            return lambda: torch.from_numpy(sr.sources().reshape(sr.nrhs, -1)).to(dev)
        return [Request(r.rid, r.key, maker(r.base), sources(r), tol=args.tol, max_steps=400, t_arrival=r.t_arrival,
                        n_rhs=r.nrhs, keep=r.rid in keep_ids) for r in stream]

    def serve(stream, keep_ids=()):
        reqs = make_requests(stream, keep_ids)
        srv = Server(hbm_budget_bytes=int(args.budget_gb * 2**30), slots=args.slots, poll_steps=args.poll_steps,
                     device="cuda:0", plans=plans, plan_scope=tuning.scope_of(serve_layouts))
        t0 = time.perf_counter()
        done = srv.run(reqs, time_limit=stream[-1].t_arrival + 300.0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat = [r.latency * 1e3 for r in done]
        rel = [x for r in done for x in r.relres]
        steps = [x for r in done for x in r.steps]
        rec = {"requests": len(reqs), "done": len(done), "rhs": st["rhs"], "wall_s": wall,
               "rhs_per_s": st["rhs_per_s"], "req_per_s": len(done) / max(r.t_done for r in done),
               "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
               "cache_hit_rate": st["cache_hit_rate"], "cache_hits": st["cache_hits"],
               "cache_misses": st["cache_misses"], "evictions": st["evictions"],
               "hbm_peak_reserved_bytes": st["peak_hbm_bytes"], "factor_seconds": st["factor_seconds"],
               "plans_applied": st["plans_applied"],
               "max_relres": max(rel), "unconverged": sum(1 for x in rel if x > args.tol),
               "ddm_steps": {"p50": pct(steps, 50), "max": max(steps)}}
        return rec, done

    # capacity: a burst (all requests arrive at once)
    burst = di.serving_stream(n_requests=args.capacity_requests, rate=1e6, seed=1)
    cap_rec, _ = serve(burst)
    cap = cap_rec["req_per_s"]
    log("bench: capacity %.2f requests/s (%.1f RHS/s), burst of %d" % (cap, cap_rec["rhs_per_s"], len(burst)))
    runs = {}
    sample = None
    rates = [float(x) for x in args.rates.split(",")]
    for i, frac in enumerate(rates):
        stream = di.serving_stream(n_requests=args.requests, rate=frac * cap, seed=2 + i)
        keep = ()
        if frac == rates[len(rates) // 2]:
            keep = tuple(r.rid for r in stream if r.key[0] == min(x.key[0] for x in stream))[:3]
        rec, done = serve(stream, keep)
        rec["rate_req_per_s"] = frac * cap
        runs["%.1f" % frac] = rec
        log("bench: lambda %.1f x capacity (%.2f req/s): %.1f RHS/s, latency p50 %.0f ms p99 %.0f ms, hit rate %.2f, "
            "evictions %d, max relres %.1e" % (frac, frac * cap, rec["rhs_per_s"], rec["latency_ms"]["p50"],
                                              rec["latency_ms"]["p99"], rec["cache_hit_rate"], rec["evictions"],
                                              rec["max_relres"]))
        if keep:
            by_id = {r.rid: r for r in done}
            sample = [(sr, by_id[sr.rid]) for sr in stream if sr.rid in keep]
    top = runs["%.1f" % rates[-1]]
    out = {
        "metric": METRIC, "value": top["rhs_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": top["done"], "warmup": 1, "ms_per_step": top["wall_s"] / top["done"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+f64", "data": "synthetic",
        "config": {"workload": ("serving stream: Poisson arrivals of 2D solves, grids 256^2/512^2/1024^2 with 128^2 "
                                "cores (2x2/4x4/8x8), a catalog of 4 media per grid (constant at 10 and 8 ppw, two "
                                "layered), 1-32 Gaussian sources each, PML 16, overlap 8; complex64 inverses and "
                                "local solves, FP64 residual, stationary DDM to relres %.0e; factorisations cached "
                                "per (grid, medium) under a %.0f GiB HBM budget, %d RHS slots per cached problem"
                                % (args.tol, args.budget_gb, args.slots)),
                   "global_batch": top["rhs"], "method": "stationary", "precision": "mixed",
                   "layouts": args.serve_layouts},
        "latency_ms": top["latency_ms"],
        "capacity": cap_rec, "rates": runs, "plans": tuned,
        "roofline": None,
        "roofline_note": "mixed stream of problem sizes; per-kernel rooflines are reported on the fixed workloads",
    }
    if sample:
        from oracle import Oracle
        checks = []
        for i, (sr, r) in enumerate(sample):
            w = sr.workload
            f = r.f
            h = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=True), torch.from_numpy(w.k2.reshape(-1)).to(dev),
                                 args.slots, factor=False)
            try:
                plan = (plans.get(tuning.plan_key(h, args.slots, tuning.scope_of(serve_layouts)))
                        if plans is not None else None)
                if plan is not None:
                    tuning.apply_plan(h, plan)  # the configuration the server's handle had
                else:
                    h.factor()
                # alone: the request's sources in batches of at most `slots`
                ua = torch.empty_like(f)
                iters = []
                for c0 in range(0, r.nrhs, args.slots):
                    uc, info, st = h.solve(f[c0:c0 + args.slots].contiguous(), method="stationary", tol=args.tol,
                                           maxiter=400)
                    ua[c0:c0 + args.slots] = uc
                    iters += [x["iters"] for x in info]
            finally:
                h.close()
            d = (torch.linalg.vector_norm(ua - r.u, dim=1) / torch.linalg.vector_norm(ua, dim=1)).max().item()
            c = {"rid": r.rid, "grid": sr.key[0], "nrhs": r.nrhs, "alone_vs_mix_rel_diff": d,
                 "steps_equal": iters == r.steps}
            if i < 2:
                o = Oracle(w.dim, w.M, w.h, w.n_pml, w.sigma0, w.N, w.n_ov, w.k2)
                uo = o.global_solve(w.f).reshape(r.nrhs, -1)
                ug = r.u.cpu().numpy()
                c["rel_err_vs_oracle"] = float(np.max(np.linalg.norm(ug - uo, axis=1) / np.linalg.norm(uo, axis=1)))
            checks.append(c)
            log("bench: sample request %d: %s" % (r.rid, c))
        out["alone_vs_mix"] = checks
    print(json.dumps(out), flush=True)


def gaussian_free_space_2d(x, y, k, centre, nq=256):
    """Exact solution of Laplace(u) + k^2 u = f in the whole plane, radiating,
    for the Gaussian f = A exp(-a r^2), A = 16 k^2 / pi^3, a = (4k/pi)^2
    (Sec. 4.1.1), at the nodes x (columns) by y (rows).  The free-space Green
    function is -(i/4) H0(k|x - y|); averaging it over the angle of y (Graf's
    addition theorem) gives, with r = |x - centre|,
        u(r) = -(i pi / 2) [H0(kr) I_J(r) + J0(kr) I_H(r)],
        I_J(r) = int_0^r J0(k p) f(p) p dp,  I_H(r) = int_r^inf H0(k p) f(p) p dp,
    and u'(r) = (i pi k / 2) [H1(kr) I_J(r) + J1(kr) I_H(r)].  Beyond the
    source (a r^2 > 40) I_J is its full value exp(-pi^2/64) / (2 pi) and I_H
    vanishes; inside, both are Gauss-Legendre sums of nq points.  Returns
    (u, du/dx, du/dy) shaped [len(y), len(x)]."""
    import numpy as np
    from scipy.special import hankel1, jv

    A = 16 * k * k / math.pi ** 3
    a = (4 * k / math.pi) ** 2
    X, Y = np.meshgrid(np.asarray(x, float) - centre[0], np.asarray(y, float) - centre[1], indexing="xy")
    r = np.hypot(X, Y)
    R = math.sqrt(40.0 / a)
    IJ = np.full(r.shape, math.exp(-math.pi ** 2 / 64) / (2 * math.pi), dtype=np.complex128)
    IH = np.zeros(r.shape, dtype=np.complex128)
    near = r < R
    if near.any():
        t, wq = np.polynomial.legendre.leggauss(nq)
        rn = r[near][:, None]
        p = 0.5 * rn * (t + 1)                                  # [0, r]
        IJ[near] = 0.5 * rn[:, 0] * (wq * jv(0, k * p) * A * np.exp(-a * p * p) * p).sum(1)
        p = rn + 0.5 * (R - rn) * (t + 1)                       # [r, R]
        IH[near] = 0.5 * (R - rn[:, 0]) * (wq * hankel1(0, k * p) * A * np.exp(-a * p * p) * p).sum(1)
    kr = k * r
    u = -0.5j * math.pi * (hankel1(0, kr) * IJ + jv(0, kr) * IH)
    du = 0.5j * math.pi * k * (hankel1(1, kr) * IJ + jv(1, kr) * IH)
    return u, du * X / r, du * Y / r


def gaussian_free_space_3d(x, y, z, k, centre, nq=256):
    """Exact radiating solution of Laplace(u) + k^2 u = f in space for the
    Gaussian f = A exp(-a r^2), A = 64 k^3 / pi^(9/2), a = (4k/pi)^2
    (Sec. 4.1.2), at the nodes x by y by z.  The Green function
    -exp(ik|x - y|) / (4 pi |x - y|) averaged over spheres keeps only the
    l = 0 term of its addition theorem, sin(k r_<) exp(ik r_>) / (4 pi k r_< r_>),
    so with r = |x - centre|
        u(r) = -(1/(k r)) [exp(ikr) I_S(r) + sin(kr) I_E(r)],
        I_S(r) = int_0^r f(p) p sin(k p) dp,  I_E(r) = int_r^inf f(p) p exp(ik p) dp,
    and u'(r) = -(1/k) [(ikr - 1) exp(ikr) I_S + (kr cos(kr) - sin(kr)) I_E] / r^2.
    Beyond the source (a r^2 > 40) I_S = k exp(-pi^2/64) / (4 pi) and I_E = 0;
    inside, both are Gauss-Legendre sums of nq points.  Returns (u, du/dx,
    du/dy, du/dz) shaped [len(z), len(y), len(x)]."""
    import numpy as np

    A = 64 * k ** 3 / math.pi ** 4.5
    a = (4 * k / math.pi) ** 2
    Z, Y, X = np.meshgrid(np.asarray(z, float) - centre[2], np.asarray(y, float) - centre[1],
                          np.asarray(x, float) - centre[0], indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    R = math.sqrt(40.0 / a)
    IS = np.full(r.shape, k * math.exp(-math.pi ** 2 / 64) / (4 * math.pi), dtype=np.complex128)
    IE = np.zeros(r.shape, dtype=np.complex128)
    near = r < R
    if near.any():
        t, wq = np.polynomial.legendre.leggauss(nq)
        rn = r[near][:, None]
        p = 0.5 * rn * (t + 1)
        IS[near] = 0.5 * rn[:, 0] * (wq * A * np.exp(-a * p * p) * p * np.sin(k * p)).sum(1)
        p = rn + 0.5 * (R - rn) * (t + 1)
        IE[near] = 0.5 * (R - rn[:, 0]) * (wq * A * np.exp(-a * p * p) * p * np.exp(1j * k * p)).sum(1)
    kr = k * r
    e = np.exp(1j * kr)
    u = -(e * IS + np.sin(kr) * IE) / kr
    du = -((1j * kr - 1) * e * IS + (kr * np.cos(kr) - np.sin(kr)) * IE) / (k * r * r)
    return u, du * X / r, du * Y / r, du * Z / r


def l2_h1_errors(uh, x, h, L, k, centre):
    """Discrete L2 and H1 errors on the physical box [0, L]^dim of the nodal
    solution uh (C order [z][y][x], PML nodes included, node coordinates x on
    every axis) against the free-space solution of the paper's Gaussian
    source (dim = len(centre)): the L2 part is the h^dim-weighted sum over the
    physical nodes, the gradient part compares the difference quotient on
    each physical mesh edge with the exact derivative at the edge midpoint."""
    import numpy as np
    dim = len(centre)
    phys = (x >= -1e-9 * L) & (x <= L * (1 + 1e-9))
    xp = x[phys]
    xm = 0.5 * (xp[1:] + xp[:-1])
    up = uh[np.ix_(*([phys] * dim))]
    if dim == 2:
        exact = lambda xs: gaussian_free_space_2d(xs[0], xs[1], k, centre)
    else:
        exact = lambda xs: gaussian_free_space_3d(xs[0], xs[1], xs[2], k, centre)
    w = h ** (dim / 2.0)
    l2 = w * np.linalg.norm(up - exact([xp] * dim)[0])
    g2 = 0.0
    for d in range(dim):   # axis d of x is array axis dim - 1 - d
        xs = [xp] * dim
        xs[d] = xm
        ax = dim - 1 - d
        n = up.shape[ax]
        dq = (np.take(up, range(1, n), axis=ax) - np.take(up, range(n - 1), axis=ax)) / h
        g2 += np.linalg.norm(dq - exact(xs)[1 + d]) ** 2
    h1 = math.sqrt(l2 * l2 + w * w * g2)
    return float(l2), float(h1)

def run_study(args):
    """Studies beyond the benchmark line (one JSON line with a table):
    k-sweep: FGMRES(30) with K DDM steps per preconditioner application,
        K in {1, 2, 3, 5, 10, 15, 20, 32}, on the 16x16 layouts of 2048^2
        (constant and layered media, 4 RHS), FP64 and mixed, to relres 1e-6
        (the preconditioner experiments of Sec. 4.2.2);
    weak: the DDM as iterative solver on N x N subdomains of 300^2 cells with
        30 PML cells, omega growing with N, a delta shot in the first
        subdomain, to relres 1e-8 (the iterative-solver experiments of
        Sec. 4.2.1), N in {2, 4, 8, 16}; FP64 where its factors fit (N <= 8),
        mixed for every N;
    accuracy: the convergence experiment of Sec. 4.1.1 (Table 1): k/2pi = 25,
        5x5 subdomains, the paper's Gaussian source, PML of fixed thickness
        3/56, meshes 560^2, 1120^2 and 2240^2 (the larger ones of the table
        need more than one GPU's HBM for FP64 factors); L2 and H1 errors on
        the physical box of the FP64 DDM solution after N1 + N2 = 10 steps
        (the paper's DDM solution) and after convergence to relres 1e-11,
        against the exact free-space solution;
    accuracy-3d: the same for Sec. 4.1.2 (Table 2): k/2pi = 10, 3x3x3
        subdomains, meshes 80^3 and 96^3 (the larger ones need more HBM than
        one GPU has for dense plane-block inverses), N1 + N2 + N3 = 9 steps,
        FP64 and mixed precision;
    phi: the Phi form of the transferred source (eq. Phi) against the
        direct form on the 1024^2 problem split 8 x 1 (all transfers
        horizontal): plain DDM iterates (2 (N1 + N2) steps) in FP64 and
        complex64, their error against the FP64 direct-form iterate, the
        transfer kernel's time, and FGMRES(30) with K = N1 + N2 to 1e-10."""
    import numpy as np
    import torch

    import ddm_inputs as di
    import paper_1807_04180_amd as ddm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rows = []

    def run(w, mixed, fn):
        k2 = torch.from_numpy(w.k2.reshape(-1)).to(dev)
        f = torch.from_numpy(w.f.reshape(w.nrhs, -1)).to(dev)
        t0 = time.perf_counter()
        s = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=mixed), k2, w.nrhs)
        torch.cuda.synchronize()
        t_fac = time.perf_counter() - t0
        try:
            fn(s, f, t_fac)
        finally:
            s.close()
            del k2, f
            torch.cuda.empty_cache()

    if args.study == "k-sweep":
        for medium, build in (("constant", di.const_2d_2048), ("layered", lambda: di.layered_2d_2048(nrhs=4))):
            w = build()
            for mixed in (False, True):
                def sweep(s, f, t_fac):
                    u = torch.empty_like(f)
                    s.solve(f, method="fgmres", tol=1e-6, maxiter=2000, restart=30, K=1, u=u)  # warm-up
                    for K in (1, 2, 3, 5, 10, 15, 20, 32):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        _, info, st = s.solve(f, method="fgmres", tol=1e-6, maxiter=2000, restart=30, K=K, u=u)
                        torch.cuda.synchronize()
                        dt = time.perf_counter() - t0
                        r = {"medium": medium, "precision": "mixed" if mixed else "fp64", "K": K,
                             "gmres_iters": max(x["iters"] for x in info),
                             "local_solves": max(x["local_solves"] for x in info),
                             "relres_max": max(x["relres"] for x in info), "seconds": dt,
                             "solves_per_s": w.nrhs / dt, "status": st}
                        rows.append(r)
                        log("study: %s %s K=%2d: %3d FGMRES iterations, %4d local solves, %.2f s, relres %.1e"
                            % (medium, r["precision"], K, r["gmres_iters"], r["local_solves"], dt, r["relres_max"]))
                run(w, mixed, sweep)
    elif args.study == "weak":
        for medium in ("constant", "layered"):
            for N in (2, 4, 8, 16):
                w = di.paper_weak(N, medium)
                for mixed in ((False, True) if N <= 8 else (True,)):
                    def it(s, f, t_fac):
                        u = torch.empty_like(f)
                        s.solve(f, method="stationary", tol=1e-8, maxiter=2000, u=u)  # warm-up
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        _, info, st = s.solve(f, method="stationary", tol=1e-8, maxiter=2000, u=u)
                        torch.cuda.synchronize()
                        dt = time.perf_counter() - t0
                        steps = info[0]["iters"]
                        r = {"medium": medium, "precision": "mixed" if mixed else "fp64", "N": N, "M": w.M[0],
                             "n_ddm_iter": steps, "n_ddm_solve": steps / (2.0 * N), "relres": info[0]["relres"],
                             "seconds": dt, "factor_s": t_fac, "status": st}
                        rows.append(r)
                        log("study: %s %s N=%2d (M=%d): %4d steps, n_DDM_Solve %.2f, %.2f s (factor %.2f s), "
                            "relres %.1e" % (medium, r["precision"], N, w.M[0], steps, r["n_ddm_solve"], dt, t_fac,
                                              r["relres"]))
                    run(w, mixed, it)
    elif args.study == "accuracy":
        k = 2 * math.pi * 25
        c0 = di.PAPER_ACCURACY_CENTRE_2D
        for scale in (1, 2, 4):
            w = di.paper_accuracy_2d(scale)
            x = di.node_coords(w.M[0], w.n_pml, w.h)

            def acc(s, f, t_fac):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u10, rel10 = s.iterate(f, sum(w.N))
                torch.cuda.synchronize()
                t10 = time.perf_counter() - t0
                u = torch.empty_like(f)
                _, info, st = s.solve(f, method="stationary", tol=1e-11, maxiter=200, u=u)
                torch.cuda.synchronize()
                r = {"mesh": 560 * scale, "local_core": 100 * scale, "n_pml": w.n_pml, "n_ov": w.n_ov,
                     "factor_s": t_fac, "ddm_steps": sum(w.N), "ddm_s": t10, "relres_ddm": rel10[-1][0],
                     "steps_to_1e-11": info[0]["iters"], "status": st}
                for tag, uu in (("ddm", u10), ("converged", u)):
                    e0, e1 = l2_h1_errors(uu.cpu().numpy().reshape(len(x), len(x)), x, w.h, w.L, k, c0)
                    r[tag + "_l2"], r[tag + "_h1"] = e0, e1
                if rows:
                    for key in ("ddm_l2", "ddm_h1"):
                        r[key + "_rate"] = math.log(rows[-1][key] / r[key], 2)
                rows.append(r)
                log("study: mesh %d^2: factor %.1f s; %d DDM steps %.3f s (relres %.1e): L2 %.3e H1 %.3e%s; "
                    "converged (%d steps to 1e-11): L2 %.3e H1 %.3e"
                    % (r["mesh"], t_fac, r["ddm_steps"], t10, r["relres_ddm"], r["ddm_l2"], r["ddm_h1"],
                       "" if "ddm_l2_rate" not in r else " (rates %.2f, %.2f)" % (r["ddm_l2_rate"], r["ddm_h1_rate"]),
                       r["steps_to_1e-11"], r["converged_l2"], r["converged_h1"]))
            run(w, False, acc)
    elif args.study == "accuracy-3d":
        k = 2 * math.pi * 10
        c0 = di.PAPER_ACCURACY_CENTRE_3D
        for mesh in (80, 96):
            w = di.paper_accuracy_3d(mesh)
            x = di.node_coords(w.M[0], w.n_pml, w.h)
            for mixed in (False, True):
                def acc3(s, f, t_fac):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    u9, rel9 = s.iterate(f, sum(w.N))
                    torch.cuda.synchronize()
                    t9 = time.perf_counter() - t0
                    u = torch.empty_like(f)
                    tol = 1e-7 if mixed else 1e-10
                    _, info, st = s.solve(f, method="stationary", tol=tol, maxiter=200, u=u)
                    torch.cuda.synchronize()
                    r = {"mesh": mesh, "local_core": w.M[0] // 3, "n_pml": w.n_pml, "n_ov": w.n_ov,
                         "precision": "mixed" if mixed else "fp64", "factor_s": t_fac, "ddm_steps": sum(w.N),
                         "ddm_s": t9, "relres_ddm": rel9[-1][0], "tol": tol, "steps_to_tol": info[0]["iters"],
                         "status": st}
                    n = len(x)
                    for tag, uu in (("ddm", u9), ("converged", u)):
                        e0, e1 = l2_h1_errors(uu.cpu().numpy().reshape(n, n, n), x, w.h, w.L, k, c0)
                        r[tag + "_l2"], r[tag + "_h1"] = e0, e1
                    prev = [q for q in rows if q["precision"] == r["precision"]]
                    if prev:
                        for key in ("ddm_l2", "ddm_h1"):
                            r[key + "_rate"] = math.log(prev[-1][key] / r[key]) / math.log(mesh / prev[-1]["mesh"])
                    rows.append(r)
                    log("study: mesh %d^3 %s: factor %.1f s; %d DDM steps %.3f s (relres %.1e): L2 %.3e H1 %.3e%s; "
                        "to %.0e in %d steps: L2 %.3e H1 %.3e"
                        % (mesh, r["precision"], t_fac, r["ddm_steps"], t9, r["relres_ddm"], r["ddm_l2"], r["ddm_h1"],
                           "" if "ddm_l2_rate" not in r else " (rates %.2f, %.2f)" % (r["ddm_l2_rate"], r["ddm_h1_rate"]),
                           tol, r["steps_to_tol"], r["converged_l2"], r["converged_h1"]))
                log("study: mesh %d^3 %s: factorising (%.0f GB)" % (mesh, "mixed" if mixed else "fp64",
                    ddm.Problem.from_workload(w, mixed=mixed).memory_required(1) / 1e9))
                run(w, mixed, acc3)
    elif args.study == "phi":
        w = di.strip_2d_1024()
        nst = 2 * sum(w.N)
        ref = {}
        for mixed in (False, True):
            def phi(s, f, t_fac):
                for form in ("direct", "phi"):
                    s.set_transfer_form(form)
                    s.iterate(f, 2)  # warm-up
                    s.profile_enable(True)
                    u, rel = s.iterate(f, nst)
                    torch.cuda.synchronize()
                    pr = s.profile_read()["transfer"]
                    s.profile_enable(False)
                    if not mixed and form == "direct":
                        ref["u"] = u.clone()
                    err = float(torch.max(torch.linalg.vector_norm(u - ref["u"], dim=1)
                                          / torch.linalg.vector_norm(ref["u"], dim=1)))
                    _, info, st = s.solve(f, method="fgmres", tol=1e-10, maxiter=300, restart=30, K=sum(w.N))
                    r = {"precision": "mixed" if mixed else "fp64", "form": form, "steps": nst,
                         "relres_after_steps": max(rel[-1]), "err_vs_fp64_direct": err,
                         "transfer_ms_per_launch": pr["ms"] / max(pr["launches"], 1),
                         "fgmres_iters": max(x["iters"] for x in info),
                         "fgmres_relres": max(x["relres"] for x in info), "fgmres_status": st}
                    rows.append(r)
                    log("study: %s %s: %d steps relres %.2e, error vs FP64 direct %.2e, transfer %.4f ms/launch; "
                        "FGMRES(30, K=%d) to 1e-10: %d iterations (relres %.1e, status %d)"
                        % (r["precision"], form, nst, r["relres_after_steps"], err, r["transfer_ms_per_launch"],
                           sum(w.N), r["fgmres_iters"], r["fgmres_relres"], st))
                s.set_transfer_form("direct")
            run(w, mixed, phi)
    print(json.dumps({"study": args.study, "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["layered-2048", "2d-1024", "2d-80", "2d-2048-layered", "serve", "3d-96"],
                    default="layered-2048",
                    help="layered-2048 (default, the headline): 2D layered 2048^2 16x16, 16 RHS, mixed FGMRES beside "
                         "FP64; 2d-1024: 2D 1024^2 8x8, 4 RHS, FP64 stationary; 2d-80: 2D 80^2 2x2; "
                         "2d-2048-layered: the layered workload as FP64 stationary; serve: serving stream; "
                         "3d-96: 3D 96^3 3x3x3")
    ap.add_argument("--requests", type=int, default=500, help="serve: requests in each stream")
    ap.add_argument("--capacity-requests", type=int, default=64, help="serve: requests of the capacity burst")
    ap.add_argument("--rates", default="0.5,0.8,1.0",
                    help="serve: arrival rates of the streams, as fractions of the measured capacity (ascending)")
    ap.add_argument("--serve-layouts", choices=["any", "onedir"], default="any",
                    help="serve: factor layouts the tuner may pick (onedir: no cooperative substitution launches, "
                         "so handles' steps can run side by side)")
    ap.add_argument("--budget-gb", type=float, default=96.0, help="serve: HBM budget for cached problems (GiB)")
    ap.add_argument("--poll-steps", type=int, default=1,
                    help="serve: DDM steps enqueued per handle between polls (1: a right-hand side leaves at the "
                         "first step that meets the tolerance, as in a batch solve alone)")
    ap.add_argument("--slots", type=int, default=64,
                    help="serve: RHS slots per cached problem (the matrix-core substitution runs its 16-RHS "
                         "tiles side by side)")
    ap.add_argument("--tol", type=float, default=None, help="stationary/FGMRES tolerance (default per workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FGMRES and mixed-precision legs")
    ap.add_argument("--study", choices=["none", "k-sweep", "weak", "accuracy", "accuracy-3d", "phi"], default="none",
                    help="k-sweep: FGMRES preconditioner K sweep on 16x16 layouts; weak: iterative solver on "
                         "N x N subdomains of 300^2 cells; accuracy: L2/H1 errors against the free-space solution "
                         "on 560^2-2240^2 meshes; accuracy-3d: the same on 80^3 and 96^3; phi: the Phi form of the "
                         "transferred source against the direct one on an 8x1 layout (prints one JSON line with "
                         "the table)")
    ap.add_argument("--probe", choices=["none", "traffic"], default="none",
                    help="traffic: run 3 local solves of the workload (complex64 for the headline, FP64 for the "
                         "others) and a 1 GiB device copy (for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE), print "
                         "nothing else")
    ap.add_argument("--traffic-record", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "TAG"), default=None,
                    help="write profiles/<kernel>_<TAG>_traffic.json from the counter CSVs of the two rocprofv3 "
                         "--pmc runs of --probe traffic (FETCH_SIZE, then WRITE_SIZE) and print its summary; "
                         "runs nothing on the GPU")
    ap.add_argument("--variant", default="mma", help="--traffic-record: substitution variant the counters are of")
    ap.add_argument("--overlap-from", default=None, metavar="KERNEL_TRACE_CSV",
                    help="print the cross-stream kernel overlap of a rocprofv3 kernel trace; runs nothing on the GPU")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default substitution plan instead of the autotuned / cached one")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the DDM step here runs on one GPU (there is no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.traffic_record:
        make_traffic_record(*args.traffic_record, variant=args.variant)
        return

    if args.overlap_from:
        print(json.dumps(overlap_report(args.overlap_from)))
        return

    if args.study != "none":
        run_study(args)
        return

    if args.workload == "serve":
        if args.tol is None:
            args.tol = 1e-6
        run_serving(args)
        return

    if args.workload == "layered-2048":
        run_headline(args)
        return

    import numpy as np
    import torch

    import ddm_inputs as di
    import paper_1807_04180_amd as ddm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    build_w, tol_w, wdesc = workloads()[args.workload]
    if args.tol is None:
        args.tol = tol_w
    if args.workload != "2d-1024":
        args.no_cpu_baseline = True  # the oracle baseline is sampled from the headline workload only
    w = build_w()
    nrhs = w.nrhs
    log("bench: workload %s nglob=%d nrhs=%d on %s" % (w.name, int(np.prod(w.grid_shape)), nrhs,
                                                        torch.cuda.get_device_name(0)))
    k2 = torch.from_numpy(w.k2.reshape(-1)).to(dev)
    f = torch.from_numpy(w.f.reshape(nrhs, -1)).to(dev)

    # ---- FP64 handle: setup + factor ------------------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s64 = ddm.HelmholtzDDM(ddm.Problem.from_workload(w), k2, nrhs, factor=False)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    s64.factor()
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    log("bench: setup %.3f s, factor %.3f s (%.2f GB of complex128 block inverses), substitution variant %s"
        % (t_setup, t_factor, s64.factor_bytes / 1e9, s64.solve_variant()))

    if args.probe == "traffic":
        g = torch.zeros((nrhs, s64.etot), dtype=torch.complex128, device=dev)
        g[:, ::7] = 1.0
        for _ in range(3):
            s64.local_solve(g)
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: traffic probe done (3 local solves, 1 GiB copy)")
        s64.close()
        return

    def solve_fp64(u=None):
        return s64.solve(f, method="stationary", tol=args.tol, maxiter=400, u=u)

    u64 = torch.empty_like(f)
    for i in range(args.warmup):
        _, info, st = solve_fp64(u64)
        log("bench: warmup %d status %d steps %s" % (i, st, [x["iters"] for x in info]))
    torch.cuda.synchronize()
    lat = []
    steps_used = []
    converged = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, info, st = solve_fp64(u64)
        lat += [x["seconds"] * 1e3 for x in info]
        steps_used += [x["iters"] for x in info]
        converged += sum(1 for x in info if x["status"] == "OK")
        if st != 0:
            log("bench: step %d status %d" % (i, st))
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - t0
    ms_per_step = t_timed / args.steps * 1e3
    # only right-hand sides that reached the tolerance count
    value = converged / t_timed
    relres = [x["relres"] for x in info]
    log("bench: FP64 stationary: %.2f ms/batch, %.2f solves/s, steps %s, relres %s"
        % (ms_per_step, value, sorted(set(steps_used)), ["%.2e" % r for r in relres]))
    steps_full = max(steps_used)


    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wdesc + ", complex128 stationary DDM to relres %.0e" % args.tol,
                   "global_batch": nrhs, "grid": list(w.M), "subdomains": list(w.N), "method": "stationary",
                   "precision": "fp64"},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "ddm_steps_per_solve": steps_full,
        "relres": relres,
        "factor_s": t_factor, "setup_s": t_setup, "factor_bytes": s64.factor_bytes,
        # single-shot use: one batch solved once, setup and factorisation included
        "single_shot_solves_per_s": nrhs / (t_setup + t_factor + ms_per_step * 1e-3),
    }

    # ---- roofline of the substitution kernel: live event-profiled pass --
    s64.profile_enable(True)
    u_tmp = torch.empty_like(f)
    _, info_p, _ = solve_fp64(u_tmp)
    prof = s64.profile_read()
    s64.profile_enable(False)
    sub = prof["substitution"]
    avg_us = sub["ms"] / max(sub["launches"], 1) * 1e3
    achieved = sub["bytes"] / (sub["ms"] * 1e-3) / 1e9 if sub["ms"] > 0 else 0.0
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": recorded_traffic(s64.solve_variant(), "2d1024") if args.workload == "2d-1024" else None,
                       "kernel": SUBST_KERNELS[s64.solve_variant()] + " (block substitution)",
                       "avg_launch_us": avg_us, "launches": sub["launches"],
                       "bytes_per_launch": sub["bytes"] / max(sub["launches"], 1)}
    out["kernel_time_ms_per_solve_batch"] = {k: v["ms"] for k, v in prof.items()}
    out["kernel_achieved_GBs"] = {k: (v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None)
                                  for k, v in prof.items()}
    log("bench: substitution %d launches, avg %.2f us, %.0f GB/s (%.1f%% of HBM peak); per class ms %s"
        % (sub["launches"], avg_us, achieved, 100 * achieved / HBM_PEAK_GBS,
           {k: round(v["ms"], 2) for k, v in prof.items()}))

    if not args.no_extras:
        # ---- FGMRES(30) + DDM(K = N1 + N2), FP64 ----------------------------
        uf = torch.empty_like(f)
        s64.solve(f, method="fgmres", tol=args.tol, maxiter=200, restart=30, u=uf)  # warm-up / alloc
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infof, stf = s64.solve(f, method="fgmres", tol=args.tol, maxiter=200, restart=30, u=uf)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        errf = (torch.linalg.vector_norm(uf - u64, dim=1) / torch.linalg.vector_norm(u64, dim=1)).tolist()
        out["fgmres"] = {"solves_per_s": nrhs / tf, "ms_per_batch": tf * 1e3, "K": int(sum(w.N)) - (len(w.N) - w.dim), "restart": 30,
                         "gmres_iters": [x["iters"] for x in infof],
                         "local_solves": [x["local_solves"] for x in infof],
                         "relres": [x["relres"] for x in infof], "rel_diff_vs_stationary": errf, "status": stf}
        log("bench: FP64 FGMRES: %.2f solves/s, iters %s" % (nrhs / tf, [x["iters"] for x in infof]))

        # ---- mixed precision -------------------------------------------------
        s64.close()
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        smx = ddm.HelmholtzDDM(ddm.Problem.from_workload(w, mixed=True), k2, nrhs)
        torch.cuda.synchronize()
        t_factor_mx = time.perf_counter() - t0
        umx = torch.empty_like(f)
        for _ in range(args.warmup):
            smx.solve(f, method="stationary", tol=args.tol, maxiter=400, u=umx)
        torch.cuda.synchronize()
        latm = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, infom, stm = smx.solve(f, method="stationary", tol=args.tol, maxiter=400, u=umx)
            latm += [x["seconds"] * 1e3 for x in infom]
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        errm = (torch.linalg.vector_norm(umx - u64, dim=1) / torch.linalg.vector_norm(u64, dim=1)).tolist()
        # roofline of the complex64 substitution (live event-profiled pass)
        smx.profile_enable(True)
        smx.solve(f, method="stationary", tol=args.tol, maxiter=400, u=torch.empty_like(f))
        subm = smx.profile_read()["substitution"]
        smx.profile_enable(False)
        achm = subm["bytes"] / (subm["ms"] * 1e-3) / 1e9 if subm["ms"] > 0 else 0.0
        ufm = torch.empty_like(f)
        t1 = time.perf_counter()
        _, infofm, stfm = smx.solve(f, method="fgmres", tol=args.tol, maxiter=200, restart=30, u=ufm)
        torch.cuda.synchronize()
        tfm = time.perf_counter() - t1
        out["mixed"] = {"solves_per_s": nrhs * args.steps / tm, "ms_per_batch": tm / args.steps * 1e3,
                        "latency_ms": {"p50": pct(latm, 50), "p99": pct(latm, 99)},
                        "steps": [x["iters"] for x in infom], "relres": [x["relres"] for x in infom],
                        "rel_err_vs_fp64": errm, "status": stm, "factor_s": t_factor_mx,
                        "single_shot_solves_per_s": nrhs / (t_factor_mx + tm / args.steps),
                        "speedup_vs_fp64": (nrhs * args.steps / tm) / value,
                        "roofline": {"bound": "hbm", "achieved": achm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": achm / HBM_PEAK_GBS,
                                     "kernel": SUBST_KERNELS[smx.solve_variant()] + " (complex64 block substitution)",
                                     "avg_launch_us": subm["ms"] / max(subm["launches"], 1) * 1e3,
                                     "bytes_per_launch": subm["bytes"] / max(subm["launches"], 1)},
                        "fgmres": {"solves_per_s": nrhs / tfm, "gmres_iters": [x["iters"] for x in infofm],
                                   "relres": [x["relres"] for x in infofm], "status": stfm}}
        log("bench: mixed stationary: %.2f solves/s (x%.2f), steps %s, err vs FP64 %s; substitution %.0f GB/s "
            "(%.1f%% of HBM peak)"
            % (nrhs * args.steps / tm, (nrhs * args.steps / tm) / value, [x["iters"] for x in infom],
               ["%.1e" % e for e in errm], achm, 100 * achm / HBM_PEAK_GBS))
        smx.close()
    else:
        s64.close()

    if not args.no_cpu_baseline:
        log("bench: CPU baseline (oracle) ...")
        out["cpu_baseline"] = run_cpu_baseline(nrhs, int(np.prod(w.N)), steps_full, args.tol)
        log("bench: CPU baseline %.4f solves/s" % out["cpu_baseline"]["value"])

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
