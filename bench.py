"""Benchmark of the tensor-product multigrid hot path on one MI355X.

Workload (default): periodic 1024 x 1024 columns x 128 geometrically graded
layers (134M DOF), a_z/a_h = 1e4, c_f = 1 + 0.5 U[0,1), b ~ N(0,1), 7-level
V-cycle (2+2 line sweeps, omega 0.8, 2 sweeps on the 16 x 16 coarsest level).

One step = the whole path on that input: setup_hierarchy (coarse levels +
FP32 copies), the mixed-precision solve to 1e-8 (FP32 V-cycle inside FP64
CG), and the adjoint of J = 0.5 ||x||^2 (solve for lambda, then dJ/dc on
every face).  Inputs are resident in HBM before the timed region.

Beside the steps the plain FP64 solve is timed on the same input for the
FP32-MG vs FP64 comparison, the finest-level FP32 sweep kernel is timed with
HIP events for the roofline line, and the CPU oracle (built for the host,
OpenMP over columns) runs one step of the same workload on the host's cores.
`--cpu-baseline` times the oracle's solves on several workloads, single- and
multi-threaded.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Compulsory HBM bytes per finest-level DOF (words x 4 bytes for the FP32 V-cycle):
SWEEP_WORDS = 6            # reads u, b, c_E, c_N, c_U; writes u'
VCYCLE_WORDS = 28.5 * 4 / 3  # 28.5 words on the finest level, times sum 4^-l
KERNEL_SOURCES = ["paper_1605_00492_amd/csrc/tpmg_kernels.hip", "paper_1605_00492_amd/csrc/tpmg_device.h"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sweep_fp32_1024x1024x128_counters.json")
DG1_SOURCES = ["paper_1605_00492_amd/csrc/tpmg_dg1.hip", "paper_1605_00492_amd/csrc/tpmg_device.h"]
DG1_COUNTERS_FILE = os.path.join(ROOT, "profiles", "dg1_sweep_256x256x64_counters.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in sources:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(launch_dof: int, path=COUNTERS_FILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch of the roofline kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source;
    else None."""
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_hash(sources) or d.get("dof") != launch_dof:
        return None
    return d.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def native_oracle():
    """The oracle built for this host (gcc -O3 -march=native -ffp-contract=off
    -fopenmp) in a temporary directory, loaded in place of the portable build."""
    import tempfile

    import oracle
    d = tempfile.mkdtemp(prefix="tpmg_oracle_")
    path = oracle.build(path=os.path.join(d, "liboracle_native.so"), native=True)
    oracle.use_library(path)
    return oracle


def oracle_step(oracle, w, c, b):
    """One step of the path on the oracle: setup, mixed solve, adjoint.
    Returns (setup_s, solve_s, adjoint_s, forward iterations, adjoint iterations)."""
    t0 = time.perf_counter()
    P = oracle.problem_for(w, c)
    t1 = time.perf_counter()
    x, info = P.pcg(b, rtol=w.rtol, maxit=100, mixed=True, flexible=True)
    t2 = time.perf_counter()
    lam, info2 = P.pcg(x, rtol=w.rtol, maxit=100, mixed=True, flexible=True)
    P.face_gradient(lam, x)
    t3 = time.perf_counter()
    del P
    return t1 - t0, t2 - t1, t3 - t2, info["iterations"], info2["iterations"]


def cpu_baseline(w, syn):
    """The CPU oracle (plain C, OpenMP over columns, built for this host) on
    the whole workload: one step (setup + mixed solve + adjoint) on all the
    threads OpenMP is given (OMP_NUM_THREADS, else every core)."""
    oracle = native_oracle()
    threads = oracle.threads()
    c, b = w.coefficients(), w.rhs()
    t_setup, t_solve, t_adj, it, it2 = oracle_step(oracle, w, c, b)
    dt = t_setup + t_solve + t_adj
    return {"value": w.dof / dt, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole {w.n}x{w.n}x{w.nz} workload, one step: setup {t_setup:.1f} s, mixed solve "
                      f"({it} it) {t_solve:.1f} s, adjoint ({it2} it) {t_adj:.1f} s; gcc -O3 -march=native "
                      f"-fopenmp, {threads} threads on {os.cpu_count()} logical CPUs ({cpu_model()})",
            "ms_per_step": dt * 1e3}


def cpu_protocol(args):
    """The oracle's time per solve on the host (median of 3 after 1 warm-up,
    setup timed apart): the 32^2 x 16, 512^2 x 64 and 256^2 x 32 workloads
    single-threaded and on all threads, the 1024^2 x 128 workload on all
    threads; FP64 and mixed solves.  One JSON line."""
    import synthetic as syn
    oracle = native_oracle()
    all_threads = oracle.threads()
    out = {"cpu": cpu_model(), "logical_cpus": os.cpu_count(), "threads_all": all_threads,
           "build": "gcc -O3 -march=native -ffp-contract=off -fopenmp", "runs": []}
    plan = [("fp64_ref_32x32x16", (1, all_threads)), ("fp64_512x512x64", (1, all_threads)),
            ("adjoint_256x256x32", (1, all_threads)), ("large_1024x1024x128", (all_threads,))]
    for name, thread_counts in plan:
        if args.cpu_only and name not in args.cpu_only.split(","):
            continue
        w = syn.CONFIGS[name]
        c, b = w.coefficients(), w.rhs()
        for nt in thread_counts:
            oracle.threads(nt)
            t0 = time.perf_counter()
            P = oracle.problem_for(w, c)
            setup_s = time.perf_counter() - t0
            for mixed in (False, True):
                ts = []
                for rep in range(4):
                    t0 = time.perf_counter()
                    x, info = P.pcg(b, rtol=w.rtol, maxit=100, mixed=mixed, flexible=mixed)
                    if rep > 0:
                        ts.append(time.perf_counter() - t0)
                s = sorted(ts)[1]
                word = 4 if mixed else 8
                row = dict(workload=name, dof=w.dof, threads=nt, precision="mixed" if mixed else "fp64",
                           setup_s=setup_s, solve_s=s, iterations=info["iterations"],
                           dof_iterations_per_s=w.dof * info["iterations"] / s,
                           vcycle_model_bytes_per_dof=VCYCLE_WORDS * word)
                out["runs"].append(row)
                log(f"cpu {row}")
            del P
        oracle.threads(all_threads)
    print(json.dumps(out), flush=True)


def probe(tp, torch, w, c, b, kw, args):
    """Each finest-level kernel of the V-cycle (both precisions), the face
    gradient and a plain 1 GiB device copy, timed with HIP events: the
    workload for rocprofv3 counter passes and for kernel tuning.  Algorithmic
    bytes per DOF are words x word size: sweep0 5, sweep 6,
    prolongation+sweep 6.25, residual+restriction 5.25, apply 5, face
    gradient 5 (FP64)."""
    H = tp.Hierarchy(c, precision="mixed", **kw)
    nc = H.level_n(1)
    res = {}
    for dt, S in ((torch.float32, 4), (torch.float64, 8)):
        tag = "fp32" if S == 4 else "fp64"
        bb = b.to(dt)
        u = torch.empty_like(bb).normal_()
        e = torch.empty((w.nz, nc, nc), dtype=dt, device=c.device).normal_()
        kernels = {
            "sweep0": (lambda: H.smooth(bb), 5.0),
            "sweep": (lambda: H.smooth(bb, u), 6.0),
            "prolsweep": (lambda: H.prolong_smooth(u, e, bb), 6.25),
            "restrict": (lambda: H.residual_restrict(u, bb), 5.25),
            "apply": (lambda: H.apply(u), 5.0),
        }
        if S == 8:
            # adjoint face gradient: lambda, x in; three face arrays out
            lam = torch.empty_like(bb).normal_()
            g = torch.empty((3,) + tuple(bb.shape), dtype=dt, device=c.device)
            kernels["face_gradient"] = (lambda: H.face_gradient(lam, u, out=g), 5.0)
        for name, (fn, words) in kernels.items():
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            res[f"{tag}_{name}_ms"] = ms
            res[f"{tag}_{name}_GBps"] = words * S * w.dof / (ms * 1e-3) / 1e9
    # CG kernels and the V-cycle inside a profiled mixed solve (HIP events)
    from paper_1605_00492_amd.binding import K_PCG_APPLY, K_PCG_UPDATE, K_VCYCLE
    H.solve(b, rtol=w.rtol)
    H.profile_enable(True)
    H.solve(b, rtol=w.rtol)
    for name, cls in (("pcg_apply", K_PCG_APPLY), ("pcg_update", K_PCG_UPDATE), ("vcycle_fp32", K_VCYCLE)):
        ms, cnt = H.profile_read(cls)
        res[f"{name}_ms"] = ms / max(cnt, 1)
    H.profile_enable(False)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=c.device)
    dst = torch.empty_like(src)
    tp.bandwidth_probe(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        tp.bandwidth_probe(dst, src)
    e1.record()
    torch.cuda.synchronize()
    res["copy_ms"] = e0.elapsed_time(e1) / args.steps
    res["copy_GBps"] = 2 * nbytes / (res["copy_ms"] * 1e-3) / 1e9
    res["copy_bytes_each_way"] = nbytes
    res["dof"] = w.dof
    res["kernel_source_hash"] = kernel_hash()
    res["env"] = {k: v for k, v in os.environ.items() if k.startswith("TPMG_")}
    print(json.dumps(res), flush=True)
    H.close()


def robustness(tp, torch, w, dev, args):
    """Sec. 5.2 robustness study on the GPU (mixed precision, rtol 1e-8).

    PCG iterations and solve time against the Courant number, with the
    horizontal coupling a_h = (nu_CFL / 2)^2 on the workload's grid, and
    against the horizontal resolution at nu_CFL = 8, for: the single-level
    method (two line-Jacobi sweeps per iteration), multigrid with three fewer
    levels (coarsest grid n/2^(L-4)) and two or sixteen coarse sweeps,
    multigrid to a 16 x 16 coarsest grid with two (the default) or sixteen
    coarse sweeps, and multigrid down to a single column with an exact
    coarsest solve."""
    import numpy as np

    import synthetic as syn

    def variants(n):
        deep = int(round(np.log2(n))) + 1
        lv = int(round(np.log2(n // 16))) + 1
        sh = max(1, lv - 3)   # coarsest grid 8x finer than 16 x 16: a harder coarse problem
        return [("single_level", dict(levels=1, coarse="smooth", n_coarse=2)),
                ("mg_shallow_2sweeps", dict(levels=sh, coarse="smooth", n_coarse=2)),
                ("mg_shallow_16sweeps", dict(levels=sh, coarse="smooth", n_coarse=16)),
                ("mg_16x16_2sweeps", dict(levels=lv, coarse="smooth", n_coarse=2)),
                ("mg_16x16_16sweeps", dict(levels=lv, coarse="smooth", n_coarse=16)),
                ("mg_1x1_direct", dict(levels=deep, coarse="direct"))]

    def run(ww, a_h, names):
        c = torch.from_numpy(ww.coefficients()).to(dev)
        b = torch.from_numpy(ww.rhs()).to(dev)
        rows = []
        for name, kw in variants(ww.n):
            if name not in names:
                continue
            H = tp.Hierarchy(c, dz=ww.dz(), a_h=a_h, a_z=ww.a_z, nu=ww.nu, omega=ww.omega, precision="mixed",
                             **kw)
            H.solve(b, rtol=1e-8, maxit=1000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = H.solve(b, rtol=1e-8, maxit=1000)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            H.close()
            rows.append(dict(variant=name, n=ww.n, nz=ww.nz, levels=kw["levels"], a_h=a_h,
                             iterations=info["iterations"], converged=info["converged"],
                             true_rel_residual=info["true_rel_residual"], solve_ms=ms))
            log(f"robustness {rows[-1]}")
        del c, b
        return rows

    all_names = [v[0] for v in variants(w.n)]
    out = {"workload": w.name, "a_h_rule": "a_h = (nu_CFL/2)^2", "courant": [], "resolution": []}
    for nu in (2, 4, 8, 16, 32, 64):
        for r in run(w, (nu / 2.0) ** 2, all_names):
            out["courant"].append(dict(nu_cfl=nu, **r))
    for n in (128, 256, 512, 1024):
        if n > w.n:
            break
        ww = syn.scaled(w, n, levels=int(round(np.log2(n // 16))) + 1, name=f"{w.name}@{n}")
        for r in run(ww, 16.0, ["mg_16x16_2sweeps", "mg_1x1_direct"]):
            out["resolution"].append(dict(nu_cfl=8, **r))
    print(json.dumps(out), flush=True)


def mixed_system(tp, torch, w, dev, args):
    """The velocity-pressure system around the pressure solve (Sec. 4.2,
    Sec. 5.1): restarted flexible GMRES to rtol 1e-5 with the Schur-complement
    preconditioner, the pressure block approximated by one multigrid V-cycle
    (FP64 or FP32) or by the single-level method, at nu_CFL = 2 (a_h = 1, the
    workload) and nu_CFL = 8 (a_h = 16, the paper's runs).  GMRES(30) on
    512^2 x 64 and GMRES(20) on the full grid (memory: 2 m + 1 mixed vectors).
    --mixed-only N:A_H:NAME (each part may be *) keeps the matching runs."""
    import numpy as np

    import synthetic as syn
    out = {"rtol": 1e-5, "runs": []}
    only = (args.mixed_only or "*:*:*").split(":")

    def keep(i, v):
        return only[i] == "*" or only[i] == str(v)

    for n, nz, restart in ((512, 64, 30), (w.n, w.nz, 20)):
        if not keep(0, n):
            continue
        ww = syn.scaled(w, n, nz=nz, levels=int(round(np.log2(n // 16))) + 1, name=f"{w.name}@{n}x{n}x{nz}")
        c = torch.from_numpy(ww.coefficients()).to(dev)
        b = torch.from_numpy(ww.mixed_rhs()).to(dev)
        for a_h in (1.0, 16.0):
            for name, kw in (("mg_fp32", dict(levels=ww.levels, precision="mixed")),
                             ("mg_fp64", dict(levels=ww.levels, precision="fp64")),
                             ("single_level", dict(levels=1, precision="mixed"))):
                if not (keep(1, int(a_h)) and keep(2, name)):
                    continue
                H = tp.Hierarchy(c, dz=ww.dz(), a_h=a_h, a_z=ww.a_z, nu=ww.nu, omega=ww.omega, **kw)
                ws = torch.empty(H.mixed_workspace_bytes(restart), dtype=torch.uint8, device=dev)
                H.mixed_solve(b, rtol=1e-5, restart=restart, maxit=300, workspace=ws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = H.mixed_solve(b, rtol=1e-5, restart=restart, maxit=300, workspace=ws)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                H.close()
                del ws, x
                torch.cuda.empty_cache()
                row = dict(grid=[n, n, nz], unknowns=4 * ww.dof - n * n, a_h=a_h, nu_cfl=2.0 * a_h ** 0.5,
                           preconditioner=name, restart=restart, iterations=info["iterations"],
                           converged=info["converged"], true_rel_residual=info["true_rel_residual"], solve_ms=ms,
                           ms_per_iteration=ms / max(info["iterations"], 1))
                out["runs"].append(row)
                log(f"mixed system {row}")
        del c, b
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def nlo(tp, torch, dev, args):
    """The next-to-lowest-order (DG1) workload: band LU of every column block
    (setup), CG with the NLO V-cycle (DG1 line sweeps, p-coarsening to the
    lowest-order hierarchy in FP64 or FP32) to rtol 1e-8, and the DG1 general
    sweep (residual + forward / back substitution + update, one launch) timed
    with HIP events against its algorithmic bytes: band factors 11 words,
    u, b, out 3 words and the faces 0.5 word per unknown (116 B; 72 B in the
    mixed hierarchy, whose factors are stored in FP32).  The oracle
    (native build, all threads) solves the same system once for the CPU line
    and the error of the GPU solutions against it.  One JSON line."""
    import numpy as np

    import synthetic as syn
    from paper_1605_00492_amd.binding import K_DG1_PCG_APPLY, K_DG1_SWEEP, K_DG1_VCYCLE, K_VCYCLE
    w = syn.NLO_WORKLOADS[args.nlo_workload]
    nv = 6 * w.dof
    c = torch.from_numpy(w.coefficients()).to(dev)
    b = torch.from_numpy(w.dg1_rhs()).to(dev)
    kw = dict(dz=w.dz(), a_h=w.a_h, a_z=w.a_z, levels=w.levels, nu=w.nu, omega=w.omega, coarse=w.coarse,
              n_coarse=w.n_coarse)
    out = {"workload": w.name, "grid": [w.n, w.n, w.nz], "cells": w.dof, "unknowns": nv,
           "rows_per_column": 6 * w.nz, "band": [5, 5], "runs": []}
    sols = {}
    for prec in ("fp64", "mixed"):
        H = tp.Hierarchy(c, precision=prec, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D = tp.DG1Level(H)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            D.solve(b, rtol=w.rtol, maxit=200)
        ts = []
        for _ in range(max(args.steps, 1)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = D.solve(b, rtol=w.rtol, maxit=200)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = sorted(ts)[len(ts) // 2] * 1e3
        H.profile_enable(True)
        D.solve(b, rtol=w.rtol, maxit=200)
        prof = {name: H.profile_read(cls) for name, cls in (("sweep", K_DG1_SWEEP), ("pcg_apply", K_DG1_PCG_APPLY),
                                                             ("vcycle", K_DG1_VCYCLE), ("lo_vcycle", K_VCYCLE))}
        H.profile_enable(False)
        avg = {k: v[0] / max(v[1], 1) for k, v in prof.items()}
        sweep_bytes = (116 if prec == "fp64" else 72) * nv
        row = dict(precision=prec, factor_bytes=8 if prec == "fp64" else 4, sweep_bytes_per_unknown=sweep_bytes // nv,
                   setup_ms=setup_ms, solve_ms=ms, iterations=info["iterations"],
                   true_rel_residual=info["true_rel_residual"],
                   unknown_iterations_per_s=nv * info["iterations"] / (ms * 1e-3),
                   sweep_ms=avg["sweep"], sweep_GBps=sweep_bytes / (avg["sweep"] * 1e-3) / 1e9,
                   pcg_apply_ms=avg["pcg_apply"], vcycle_ms=avg["vcycle"], lowest_order_vcycle_ms=avg["lo_vcycle"],
                   workspace_GiB=D.ws_bytes / 2 ** 30)
        row["sweep_frac_hbm_peak"] = row["sweep_GBps"] / HBM_PEAK_GBS
        out["runs"].append(row)
        log(f"nlo {row}")
        sols[prec] = x.cpu().numpy()
        D.close()
        H.close()
    out["roofline"] = {"kernel": "k_dg1_sweep (general): residual + band forward/back substitution + update",
                       "bound": "hbm", "achieved": out["runs"][0]["sweep_GBps"], "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": out["runs"][0]["sweep_frac_hbm_peak"],
                       "traffic": measured_traffic(nv, DG1_COUNTERS_FILE, DG1_SOURCES),
                       "kernel_source_hash": kernel_hash(DG1_SOURCES),
                       "algorithmic_bytes_per_launch": 116 * nv, "launch_ms": out["runs"][0]["sweep_ms"]}
    m = out["runs"][1]
    out["roofline_fp32_factors"] = {"kernel": "k_dg1_sweep (general) with FP32 band factors (mixed hierarchy)",
                                    "bound": "hbm", "achieved": m["sweep_GBps"], "peak": HBM_PEAK_GBS,
                                    "unit": "GB/s", "frac": m["sweep_frac_hbm_peak"],
                                    "algorithmic_bytes_per_launch": 72 * nv, "launch_ms": m["sweep_ms"]}
    if not args.no_cpu_baseline:
        oracle = native_oracle()
        cn, bn = w.coefficients(), w.dg1_rhs()
        t0 = time.perf_counter()
        P = oracle.problem_for(w, cn)
        G = oracle.DG1(P)
        t1 = time.perf_counter()
        x_or, info_or = G.pcg(bn, rtol=w.rtol, maxit=200)
        t2 = time.perf_counter()
        out["cpu_baseline"] = {"value": nv / (t2 - t1), "unit": "unknowns/s (FP64 solve)", "cores": oracle.threads(),
                               "kind": "oracle", "sample": f"the whole workload: setup {t1 - t0:.1f} s, FP64 solve "
                               f"({info_or['iterations']} it) {t2 - t1:.1f} s; gcc -O3 -march=native -fopenmp, "
                               f"{oracle.threads()} threads ({cpu_model()})"}
        nrm = np.linalg.norm(x_or)
        out["error_vs_oracle"] = {p: float(np.linalg.norm(sols[p] - x_or) / nrm) for p in sols}
        out["oracle_iterations"] = info_or["iterations"]
    print(json.dumps(out), flush=True)


def all_configs(tp, torch, dev, args):
    """Time per solve (to each workload's rtol) for every workload, FP64 and
    mixed: setup, solve (median of 5 after 2 warm-ups), iterations, DOF
    iterations/s and the V-cycle time against its byte model.  On the smaller
    grids the level data fits the 256 MB last-level cache, so the model
    bandwidth there is an effective figure, not HBM."""
    from paper_1605_00492_amd.binding import K_VCYCLE

    import synthetic as syn
    out = []
    for name, w in syn.CONFIGS.items():
        c = torch.from_numpy(w.coefficients()).to(dev)
        b = torch.from_numpy(w.rhs()).to(dev)
        kw = dict(dz=w.dz(), a_h=w.a_h, a_z=w.a_z, levels=w.levels, nu=w.nu, omega=w.omega, coarse=w.coarse,
                  n_coarse=w.n_coarse)
        for prec in ("fp64", "mixed"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = tp.Hierarchy(c, precision=prec, **kw)
            torch.cuda.synchronize()
            setup_ms = (time.perf_counter() - t0) * 1e3
            for _ in range(2):
                H.solve(b, rtol=w.rtol)
            ts = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = H.solve(b, rtol=w.rtol)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            ms = sorted(ts)[2] * 1e3
            H.profile_enable(True)
            H.solve(b, rtol=w.rtol)
            vc_ms, vc_n = H.profile_read(K_VCYCLE)
            H.profile_enable(False)
            H.close()
            vc = vc_ms / max(vc_n, 1)
            word = 4 if prec == "mixed" else 8
            row = dict(workload=name, grid=[w.n, w.n, w.nz], dof=w.dof, precision=prec, setup_ms=setup_ms,
                       solve_ms=ms, iterations=info["iterations"], true_rel_residual=info["true_rel_residual"],
                       dof_iterations_per_s=w.dof * info["iterations"] / (ms * 1e-3), vcycle_ms=vc,
                       vcycle_model_GBps=VCYCLE_WORDS * word * w.dof / (vc * 1e-3) / 1e9)
            out.append(row)
            log(f"config {row}")
        del c, b
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="large_1024x1024x128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--configs", action="store_true",
                    help="time per solve for every workload, FP64 and mixed")
    ap.add_argument("--mixed-system", action="store_true",
                    help="velocity-pressure system: GMRES with multigrid vs single-level preconditioners")
    ap.add_argument("--mixed-only", default=None, metavar="N:A_H:NAME",
                    help="with --mixed-system: only the runs on grid width N, a_h and preconditioner NAME "
                         "(mg_fp32, mg_fp64, single_level; * matches all)")
    ap.add_argument("--robustness", action="store_true",
                    help="Courant-number and resolution study (single level vs multigrid variants)")
    ap.add_argument("--nlo", action="store_true",
                    help="the next-to-lowest-order (DG1) workload: banded LU line smoother, NLO V-cycle, CG")
    ap.add_argument("--nlo-workload", default="nlo_dg1_256x256x64")
    ap.add_argument("--probe", action="store_true",
                    help="only run the finest-level FP32 sweep and a 1 GiB copy (for counter runs)")
    ap.add_argument("--cpu-baseline", action="store_true",
                    help="the oracle's time per solve on this host, single-threaded and on all threads")
    ap.add_argument("--cpu-only", default=None, help="with --cpu-baseline: comma-separated workload names")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              f"documented but not built", file=sys.stderr)
        sys.exit(2)

    if args.cpu_baseline:
        cpu_protocol(args)
        return

    import numpy as np
    import torch

    import paper_1605_00492_amd as tp
    import synthetic as syn
    from paper_1605_00492_amd.binding import K_PCG_APPLY, K_SWEEP, K_VCYCLE

    w = syn.CONFIGS[args.config]
    dev = torch.device("cuda:0")
    if args.robustness:
        robustness(tp, torch, w, dev, args)
        return
    if args.mixed_system:
        mixed_system(tp, torch, w, dev, args)
        return
    if args.configs:
        all_configs(tp, torch, dev, args)
        return
    if args.nlo:
        nlo(tp, torch, dev, args)
        return
    log(f"generating {w.name} ({w.dof} DOF)")
    c = torch.from_numpy(w.coefficients()).to(dev)
    b = torch.from_numpy(w.rhs()).to(dev)
    kw = dict(dz=w.dz(), a_h=w.a_h, a_z=w.a_z, levels=w.levels, nu=w.nu, omega=w.omega,
              coarse=w.coarse, n_coarse=w.n_coarse)
    torch.cuda.synchronize()
    if args.probe:
        probe(tp, torch, w, c, b, kw, args)
        return

    def step(record=None):
        H = tp.Hierarchy(c, precision="mixed", **kw)
        if record is not None:
            H.profile_enable(True)
        x, info = H.solve(b, rtol=w.rtol, maxit=100)
        lam, info_adj = H.solve(x, rtol=w.rtol, maxit=100)   # dJ/dx = x for J = 0.5 ||x||^2
        g = H.face_gradient(lam, x)
        if record is not None:
            record.append(dict(info=info, info_adj=info_adj, sweep=H.profile_read(K_SWEEP),
                               vcycle=H.profile_read(K_VCYCLE), cg_apply=H.profile_read(K_PCG_APPLY)))
            # per-level breakdown from separate V-cycles (events around every launch)
            b32 = b.float()
            H.vcycle(b32)
            H.profile_enable(True, levels=True)
            for _ in range(5):
                H.vcycle(b32)
            record[-1]["levels"] = [H.profile_read_level(l) for l in range(w.levels)]
            record[-1]["levels_vcycle"] = H.profile_read(K_VCYCLE)
            del b32
        H.close()
        return x, g

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, g = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps

    # Instrumented step: kernel timings from HIP events on the launch stream.
    rec = []
    step(rec)
    torch.cuda.synchronize()
    r = rec[0]
    sweep_ms, sweep_n = r["sweep"]
    vc_ms, vc_n = r["vcycle"]
    sweep_avg_s = sweep_ms / max(sweep_n, 1) * 1e-3
    sweep_bytes = SWEEP_WORDS * 4 * w.dof
    achieved = sweep_bytes / sweep_avg_s / 1e9
    vc_avg_s = vc_ms / max(vc_n, 1) * 1e-3
    vc_gbs = VCYCLE_WORDS * 4 * w.dof / vc_avg_s / 1e9
    # The CG direction update + operator apply, the single launch with the
    # largest share of the step: 52 B/DOF (z32, p_old, 3 faces in FP64; p, q
    # out), 8 B less on the first iteration of each solve (no p_old).
    cg_ms, cg_n = r["cg_apply"]
    cg_avg_s = cg_ms / max(cg_n, 1) * 1e-3
    cg_bytes = (52 * cg_n - 8 * 2) * w.dof / max(cg_n, 1)   # two solves in the step
    cg_achieved = cg_bytes / cg_avg_s / 1e9

    # Mixed vs plain FP64 solve (solve only, hierarchies already set up).
    Hm = tp.Hierarchy(c, precision="mixed", **kw)
    H64 = tp.Hierarchy(c, precision="fp64", **kw)
    for H in (Hm, H64):
        H.solve(b, rtol=w.rtol)
    times = {}
    sols = {}
    for name, H in (("mixed", Hm), ("fp64", H64)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            xs, inf = H.solve(b, rtol=w.rtol)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t1) / args.steps
        sols[name] = (xs, inf)
    xm, im = sols["mixed"]
    x64, i64 = sols["fp64"]
    diff = float(torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64))
    Hm.close()
    H64.close()

    # Achievable HBM rate on this GPU: a plain 1 GiB device copy (library kernel).
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    tp.bandwidth_probe(dst, src)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        tp.bandwidth_probe(dst, src)
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes / ((time.perf_counter() - t1) / 20) / 1e9
    del src, dst

    traffic = measured_traffic(w.dof)
    out = {
        "metric": "time per solve to 1e-8 rel. residual (DOF/s, % HBM peak), FP32-MG vs FP64",
        "value": w.dof / dt,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle / f64 CG",
        "data": "synthetic (seeded SplitMix64 inputs of the stated distributions)",
        "config": {"workload": w.name, "grid": [w.n, w.n, w.nz], "dof": w.dof, "levels": w.levels,
                   "a_h": w.a_h, "a_z": w.a_z, "graded": w.graded, "rtol": w.rtol,
                   "step": "setup + mixed solve + adjoint (lambda solve + dJ/dc)"},
        "solve": {
            "mixed_ms": times["mixed"] * 1e3, "fp64_ms": times["fp64"] * 1e3,
            "speedup_mixed_vs_fp64": times["fp64"] / times["mixed"],
            "mixed_iterations": im["iterations"], "fp64_iterations": i64["iterations"],
            "mixed_true_rel_residual": im["true_rel_residual"],
            "fp64_true_rel_residual": i64["true_rel_residual"],
            "mixed_vs_fp64_rel_diff": diff,
            "mixed_dof_iterations_per_s": w.dof * im["iterations"] / times["mixed"],
            "fp64_dof_iterations_per_s": w.dof * i64["iterations"] / times["fp64"],
            "forward_iterations": r["info"]["iterations"], "adjoint_iterations": r["info_adj"]["iterations"],
        },
        "vcycle_fp32": {"ms": vc_avg_s * 1e3, "model_bytes_per_dof": VCYCLE_WORDS * 4,
                        "model_GBps": vc_gbs, "frac_hbm_peak": vc_gbs / HBM_PEAK_GBS,
                        "frac_of_copy": vc_gbs / copy_gbs,
                        # per V-cycle, the kernels on each level (finest first), from 5 separate
                        # V-cycles timed with events around every launch, and those V-cycles' time
                        "levels_ms": [lv[0] / max(r["levels_vcycle"][1], 1) for lv in r["levels"]],
                        "levels_vcycle_ms": r["levels_vcycle"][0] / max(r["levels_vcycle"][1], 1)},
        "stream": {"copy_GBps": copy_gbs, "copy_frac_hbm_peak": copy_gbs / HBM_PEAK_GBS,
                   "sweep_frac_of_copy": achieved / copy_gbs},
        "roofline": {"kernel": "k_sweep<float> finest level (general sweep)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "launch_ms": sweep_avg_s * 1e3, "launches": sweep_n,
                     "algorithmic_bytes_per_launch": sweep_bytes},
        "roofline_cg": {"kernel": "k_pcg_apply (FP64 CG: p = z + beta p, q = H p)", "bound": "hbm",
                        "achieved": cg_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": cg_achieved / HBM_PEAK_GBS, "launch_ms": cg_avg_s * 1e3, "launches": cg_n,
                        "algorithmic_bytes_per_launch": cg_bytes},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (the oracle on the whole workload, all threads)")
        del c, b, x, g, xm, x64, xs
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(w, syn)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
