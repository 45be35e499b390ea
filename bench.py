"""Benchmark of the Chebyshev-filtered FE Hamiltonian hot path on one MI355X.

Workload (default): the 24x24x48-bohr slab, 24x24x48 cubic cells of GLL
degree 4 (1,760,256 free DoFs, periodic x/y, Dirichlet z), Gaussian-well
potential on a 6-layer 4x4 lattice plus the field -E z (E = 0.005), N = 256
random vectors, filter degree m = 30, FP64 cell products.  One step is one
pass of the path over the block: the potential update (fe_set_potential)
and the degree-m filter (fe_cheb_filter), with spectrum bounds from a
10-step Lanczos run on the device beforehand.

Metric: GDoF.vec/s = m * n * N / t_step / 1e9.

Prints one JSON line.  Also reports the roofline of the dominant kernel (the
fused step kernel, timed live with HIP events on the stream it runs on) and
the CPU oracle timed on this host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H·X GDoF·vec/s in Chebyshev filter, FP64 vs FP32/BF16 at ≤1e-7 Ha Ritz err"
UNIT = "GDoF·vec/s"
PEAK = {"f64": (78.6, "mfma"), "f32": (157.3, "mfma"), "bf16": (2500.0, "mfma")}  # TFLOP/s, dense MFMA
# sustained rate of the instruction each default step kernel multiplies with,
# measured on an MI355X with a register-only loop (FP64: 4x4x4 blocks, FP32:
# 16x16x4); see paper_2504_00998_amd/microbench/mfma_rate.hip
MEASURED_PEAK = {"f64": 74.2, "f32": 155.0}
# HBM bytes per colour launch of the default step kernel on the p=4 slab
# (N=256), from FETCH_SIZE/WRITE_SIZE counters scaled by a plain copy of known
# size, averaged over the launches of a degree-30 filter (the first step reads
# no previous iterate: FP64 1.467e9 B, FP32 1.588e9 B, BF16 1.779e9 B; the 29
# others 1.950e9 / 2.065e9 / 2.235e9 B); valid for these kernel builds only
# (None: not counted)
COUNTED_TRAFFIC = {("slab-p4-24x24x48", 256, "f64"): (1.934e9, "step_tab_kernel<4,0,1,2,3,2>"),
                   ("slab-p4-24x24x48", 256, "f32"): (2.049e9, "step_tab_kernel<4,1,1,2,3,1,false,2>"),
                   ("slab-p4-24x24x48", 256, "bf16"): (2.220e9, "step_pipe_kernel<4,2,2,true>")}
# MI355X ceilings of the filter rate (GDoF.vec/s) of the large workloads:
# the dense-MFMA roofline of one H~X (2 n_c^2 flop per cell and vector; FP64
# 78.6, FP32 157.3 TFLOP/s) expressed per DoF and vector
CEILING = {("slab-p6-16x16x32", "f64"): 71.8, ("slab-p5-40x40x80-nonlocal", "f32"): 210.0}
GOLDEN_RITZ = os.path.join(ROOT, "tests", "golden", "cfg3_ritz_oracle.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_description():
    """CPU model, thread count and memory of this host (the oracle's machine)."""
    import subprocess
    model, mem_gib = None, None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    try:
        out = subprocess.run(["free", "-g"], capture_output=True, text=True, timeout=10).stdout
        mem_gib = int(out.splitlines()[1].split()[1])
    except (OSError, subprocess.SubprocessError, IndexError, ValueError):
        pass
    return {"lscpu_model": model, "nproc": os.cpu_count(), "free_g_total": mem_gib}


def cpu_baseline(wl, a, b, a0, ncols: int = 4):
    """The oracle (CSR SpMM recurrence) on `ncols` columns of the same workload."""
    import numpy as np
    import oracle as O
    from paper_2504_00998_amd import workloads as W

    t0 = time.time()
    om = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, om.quad_points())
    op = O.Operator(om, Vq, wl.E, wl.z0)
    X = wl.X(om.n, cols=range(ncols))
    log(f"[cpu_baseline] assembled H~ (nnz {op.A.nnz}) in {time.time() - t0:.1f} s")
    t = time.perf_counter()
    op.filter(X, wl.m, a, b, a0)
    dt = time.perf_counter() - t
    rec = {
        "value": wl.m * om.n * ncols / dt / 1e9,
        "unit": UNIT,
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": f"degree-{wl.m} filter on {ncols} of {wl.N} columns of the full mesh "
                  f"(CSR SpMM, nnz {op.A.nnz}); assembly excluded; {dt:.1f} s",
    }
    rec.update(host_description())
    return rec


def golden_ritz():
    """Bounds (a0, b, a) and per-iteration Ritz values of the oracle's
    5-iteration subspace iteration on the cfg-3 block (written by
    tests/golden/make_cfg3_ritz.py from the CPU oracle alone)."""
    import numpy as np
    bounds, hist = None, {}
    for line in open(GOLDEN_RITZ):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        if t[0] == "bounds":
            bounds = tuple(float(x) for x in t[1:4])
        else:
            hist.setdefault(int(t[0]), []).append((int(t[1]), float(t[2])))
    return bounds, [np.array([v for _, v in sorted(hist[k])]) for k in sorted(hist)]


def mixed_precision_report(gm, wl, X, Y, work, a, b, a0, steps, ms_f64, launches, flops_per_launch, variant):
    """FP32 / BF16 cell products: filter throughput on the benchmark block,
    speedup over FP64, the step kernel's launch time against the MFMA peak of
    the precision (and its counted HBM rate where the counters of the kernel
    are known).  Accuracy on the cfg-3 block (same mesh and potential, cfg-3
    seeds): the Ritz values after 5 subspace iterations (filter in the given
    precision; CholQR2 and Rayleigh-Ritz in FP64), every iteration from the
    oracle's Lanczos bounds and updating its own cut, against the oracle's
    own 5 iterations (tests/golden/cfg3_ritz_oracle.txt); FP64 on the device
    is reported the same way.  The bar is max |Ritz error| <= 1e-7 Ha over
    all N values; the lowest N/2 are reported beside it.  Also the
    per-vector relative error of one filter pass against the device's FP64
    filter of the same block."""
    import numpy as np
    import torch
    from paper_2504_00998_amd import solver
    from paper_2504_00998_amd import workloads as W

    stream = torch.cuda.current_stream()
    n, N, m = gm.n, wl.N, wl.m
    (ga0, gb, ga), ref = golden_ritz()
    wl3 = W.CFG3
    X3 = torch.from_numpy(wl3.X(n)).to(X.device)
    out = {"ritz_iterations": len(ref), "ritz_reference": "CPU oracle, 5-iteration subspace iteration on the cfg-3 "
           "block (tests/golden/cfg3_ritz_oracle.txt)", "ritz_bar_Ha": 1e-7,
           "y_reference": "device FP64 filter of the cfg-3 block, one pass"}
    Y64 = gm.cheb_filter(X3, m, ga, gb, ga0, prec="f64")
    for prec in ("f64", "f32", "bf16"):
        rec = {}
        if prec != "f64":
            gm.cheb_filter(X, m, a, b, a0, prec=prec, Y=Y, work=work)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                gm.cheb_filter(X, m, a, b, a0, prec=prec, Y=Y, work=work)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            launch_ms = ms / launches
            tf = flops_per_launch / (launch_ms * 1e-3) / 1e12
            traffic = COUNTED_TRAFFIC.get((wl.name, N, prec)) if variant == 0 else None
            rec = {"value": round(m * n * N / (ms * 1e-3) / 1e9, 4), "ms_per_filter": round(ms, 4),
                   "speedup_vs_f64": round(ms_f64 / ms, 3),
                   "avg_launch_ms": round(launch_ms, 5), "achieved_TFLOPs": round(tf, 3),
                   "frac_of_mfma_peak": round(tf / PEAK[prec][0], 4),
                   "hbm_GBps": round(traffic[0] / (launch_ms * 1e-3) / 1e9, 1) if traffic and traffic[0] else None,
                   "kernel": traffic[1] if traffic else None}
            Yp = gm.cheb_filter(X3, m, ga, gb, ga0, prec=prec, Y=Y, work=work)
            rec["y_rel_err_max"] = float(((Yp - Y64).norm(dim=0) / Y64.norm(dim=0)).max().item())
        hist, _ = solver.subspace_iteration(gm, X3, m, len(ref), ga, gb, ga0, prec=prec, work=work)
        d = np.abs(hist[-1] - ref[-1])
        rec.update({"ritz_err_max_Ha": float(d.max()), "ritz_err_lowest_half_Ha": float(d[: N // 2].max()),
                    "ritz_err_max_all_iterations_Ha": float(max(np.abs(h - r).max() for h, r in zip(hist, ref))),
                    "ritz_ok_1e-7": bool(d.max() <= 1e-7)})
        if prec == "bf16" and not rec["ritz_ok_1e-7"]:
            rec["note"] = ("BF16 cell products fail the 1e-7 Ha Ritz bar: their rate does not count toward the "
                           "metric")
        out[prec] = rec
    del X3, Y64
    torch.cuda.empty_cache()
    return out


def large_workloads(dev, steps):
    """The p = 6 slab (FP64 filter) and the p = 5 slab with nonlocal
    projectors (FP32 cell products) at full size, against their MFMA
    ceilings; X drawn on the device."""
    import numpy as np
    import torch

    import paper_2504_00998_amd as fe
    from paper_2504_00998_amd import workloads as W

    stream = torch.cuda.current_stream()
    out = {}
    for wl, prec in ((W.CFG4, "f64"), (W.CFG5, "f32")):
        t0 = time.time()
        gm = fe.Mesh.from_workload(wl)
        n, N, m = gm.n, wl.N, wl.m
        gm.set_potential(torch.from_numpy(W.workload_potential(wl, gm.quad_points())).to(dev), wl.E, wl.z0)
        if wl.nonlocal_sites:
            gm.set_nonlocal(wl.centres(), wl.nonlocal_coupling(), wl.r_cut, wl.r_g)
        v0 = torch.from_numpy(wl.lanczos_start(n)).to(dev)
        a0, b = gm.lanczos_bounds(v0, 10)
        a = a0 + (b - a0) * (N / n) ** (2.0 / 3.0)
        X = wl.X_device(n, N)
        Y = torch.empty_like(X)
        work = torch.empty(n * N, dtype=torch.float64, device=dev)
        setup_s = time.time() - t0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(2):
            gm.hx(X, Y=Y, prec=prec)
        torch.cuda.synchronize()
        reps = 3
        e0.record(stream)
        for _ in range(reps):
            gm.hx(X, Y=Y, prec=prec)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_hx = e0.elapsed_time(e1) / reps
        nf = 1 if wl.m * ms_hx > 2000 else min(steps, 3)  # the p = 5 filter takes seconds
        e0.record(stream)
        for _ in range(nf):
            gm.cheb_filter(X, m, a, b, a0, prec=prec, Y=Y, work=work)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_f = e0.elapsed_time(e1) / nf
        if not torch.isfinite(Y).all():
            raise RuntimeError(f"non-finite filter output on {wl.name}")
        nc = (wl.p + 1) ** 3
        flops_hx = 2.0 * nc * nc * wl.n_cells * N
        extra = {}
        if prec != "f64":
            # the same H~X with FP64 cell products (the row-owner kernel at p = 5)
            gm.hx(X, Y=Y, prec="f64")
            torch.cuda.synchronize()
            e0.record(stream)
            gm.hx(X, Y=Y, prec="f64")
            e1.record(stream)
            torch.cuda.synchronize()
            ms64 = e0.elapsed_time(e1)
            extra = {"ms_per_hx_f64": round(ms64, 3),
                     "hx_f64_TFLOPs": round(flops_hx / (ms64 * 1e-3) / 1e12, 3),
                     "hx_f64_frac_of_mfma_peak": round(flops_hx / (ms64 * 1e-3) / 1e12 / PEAK["f64"][0], 4)}
        value = m * n * N / (ms_f * 1e-3) / 1e9
        ceil = CEILING[(wl.name, prec)]
        out[wl.name] = {"prec": prec, "n_dof": n, "N": N, "m": m, "p": wl.p, "cells": list(wl.ncell),
                        "nonlocal_sites": int(wl.centres().shape[0]) if wl.nonlocal_sites else 0,
                        "value": round(value, 4), "unit": UNIT, "ceiling": ceil, "frac_of_ceiling": round(value / ceil, 4),
                        "ms_per_filter": round(ms_f, 3), "filters_timed": nf, "ms_per_hx": round(ms_hx, 4),
                        "hx_TFLOPs": round(flops_hx / (ms_hx * 1e-3) / 1e12, 3),
                        "hx_frac_of_mfma_peak": round(flops_hx / (ms_hx * 1e-3) / 1e12 / PEAK[prec][0], 4),
                        "setup_s": round(setup_s, 1), **extra}
        log(f"[bench] {wl.name} {prec}: {value:.2f} GDoF.vec/s ({value / ceil:.3f} of {ceil}), "
            f"H~X {ms_hx:.3f} ms")
        del X, Y, work, gm
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--cfg", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=64)
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32/BF16 report")
    ap.add_argument("--no-large", action="store_true", help="skip the p = 6 and p = 5 full-size workloads")
    ap.add_argument("--variant", type=int, default=0,
                    help="step-kernel variant (fe_mesh_set_kernel; 0 = the fastest measured)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the domain split across GPUs is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2504_00998_amd as fe
    from paper_2504_00998_amd import workloads as W

    wl = W.CONFIGS[args.cfg]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    gm = fe.Mesh.from_workload(wl)
    gm.set_kernel(args.variant)
    n, N, m = gm.n, wl.N, wl.m
    Vq = torch.from_numpy(W.workload_potential(wl, gm.quad_points())).to(dev)
    gm.set_potential(Vq, wl.E, wl.z0)
    X = torch.from_numpy(wl.X(n)).to(dev)
    Y = torch.empty_like(X)
    work = torch.empty(n * N, dtype=torch.float64, device=dev)
    v0 = torch.from_numpy(wl.lanczos_start(n)).to(dev)
    a0, b = gm.lanczos_bounds(v0, 10)
    a = a0 + (b - a0) * (N / n) ** (2.0 / 3.0)
    log(f"[bench] {wl.name}: n={n} N={N} m={m} prec={args.prec} bounds a0={a0:.4f} a={a:.4f} b={b:.4f} "
        f"(setup {time.time() - t0:.1f} s)")

    stream = torch.cuda.current_stream()

    def one_step():
        gm.set_potential(Vq, wl.E, wl.z0)
        gm.cheb_filter(X, m, a, b, a0, prec=args.prec, Y=Y, work=work)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    # potential update alone (to separate it from the step-kernel time)
    pe0, pe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pe0.record(stream)
    for _ in range(10):
        gm.set_potential(Vq, wl.E, wl.z0)
    pe1.record(stream)
    torch.cuda.synchronize()
    t_pot = pe0.elapsed_time(pe1) / 10.0

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        one_step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = m * n * N / (ms * 1e-3) / 1e9
    if not torch.isfinite(Y).all():
        raise RuntimeError("non-finite filter output")

    # dominant kernel: one colour pass of the fused step kernel (8 colours per step)
    ncol = 1
    for a_ in range(3):
        nce, bc = wl.ncell[a_], wl.bc[a_]
        ncol *= 3 if (bc == W.PERIODIC and nce % 2) else (2 if nce >= 2 else 1)
    launches = ncol * m
    nc = (wl.p + 1) ** 3
    cells = wl.n_cells
    flops_per_launch = 2.0 * nc * nc * (cells / ncol) * N
    launch_ms = (ms - t_pot) / launches
    achieved = flops_per_launch / (launch_ms * 1e-3) / 1e12
    peak, bound = PEAK[args.prec]
    # the counters belong to the default kernel
    traffic = COUNTED_TRAFFIC.get((wl.name, N, args.prec)) if args.variant == 0 else None
    # measured copy bandwidth of the same block (read + write), the practical
    # HBM ceiling the counted traffic is compared with
    W2 = work.view(n, N)
    W2.copy_(X)
    torch.cuda.synchronize()
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record(stream)
    for _ in range(3):
        W2.copy_(X)
    ce1.record(stream)
    torch.cuda.synchronize()
    copy_GBps = 2.0 * 8.0 * n * N / (ce0.elapsed_time(ce1) / 3 * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"{wl.name} (box {wl.L[0]:g}x{wl.L[1]:g}x{wl.L[2]:g} bohr, cells "
                               f"{wl.ncell[0]}x{wl.ncell[1]}x{wl.ncell[2]}, GLL p={wl.p}, n={n} free DoFs, "
                               f"N={N}, filter degree m={m}, cell products {args.prec})",
                   "n_dof": n, "N": N, "m": m, "p": wl.p, "cells": list(wl.ncell), "prec": args.prec,
                   "kernel_variant": args.variant},
        "roofline": {
            "bound": bound,
            "achieved": round(achieved, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": traffic[0] if traffic and traffic[0] else None,
            "traffic_unit": "B per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": 24.0 * n * N / ncol,
            "kernel": (traffic[1] if traffic else f"step kernel p={wl.p} {args.prec}") + " (one colour pass)",
            "measured_peak": MEASURED_PEAK.get(args.prec),
            "frac_of_measured_peak": round(achieved / MEASURED_PEAK[args.prec], 4) if args.prec in MEASURED_PEAK else None,
            "flops_per_launch": flops_per_launch,
            "avg_launch_ms": round(launch_ms, 5),
            "launches_per_step": launches,
            "hbm_GBps": round(traffic[0] / (launch_ms * 1e-3) / 1e9, 1) if traffic and traffic[0] else None,
            "hbm_frac_of_8TBps": round(traffic[0] / (launch_ms * 1e-3) / 8e12, 4) if traffic and traffic[0] else None,
            "copy_GBps_measured": round(copy_GBps, 1),
            "hbm_frac_of_measured_copy": round(traffic[0] / (launch_ms * 1e-3) / 1e9 / copy_GBps, 4) if traffic and traffic[0] else None,
        },
    }
    # density of the filtered block (Sec. 2.1) and its planar integral: HBM-bound
    # row reductions over the same (n, N) block
    f_occ = torch.ones(N, dtype=torch.float64, device=dev)
    rho = gm.density(Y, f_occ)
    gm.planar_average(rho)
    torch.cuda.synchronize()
    de0, de1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    de0.record(stream)
    for _ in range(5):
        gm.density(Y, f_occ, rho=rho)
    de1.record(stream)
    torch.cuda.synchronize()
    ms_rho = de0.elapsed_time(de1) / 5
    rho_bytes = 8.0 * n * N + 8.0 * N + 8.0 * n
    rec["density"] = {"ms": round(ms_rho, 4), "bytes": rho_bytes, "GB/s": round(rho_bytes / (ms_rho * 1e-3) / 1e9, 1),
                      "frac_of_hbm_peak": round(rho_bytes / (ms_rho * 1e-3) / 8e12, 4),
                      "kernel": "density_kernel (2 sum_n f_n X[I,n]^2 / M_I, 16 lanes per DoF, 16-byte column pairs)"}
    # electrostatics on the same space (Sec. 2.2): the constant-field boundary
    # conditions (periodic x, y, zero-Neumann z) on a mesh of the workload's
    # size, charge = the filtered block's density (zero at the wavefunction
    # mesh's Dirichlet z faces), neutralised by the solver
    em = fe.Mesh(wl.L, wl.ncell, wl.p, (fe.PERIODIC, fe.PERIODIC, fe.NEUMANN))
    charge = torch.zeros(em.nf[2], em.nf[1], em.nf[0], dtype=torch.float64, device=dev)
    nz_pad = (em.nf[2] - gm.nf[2]) // 2
    charge[nz_pad:nz_pad + gm.nf[2]] = rho.view(gm.nf[2], gm.nf[1], gm.nf[0])
    charge = charge.reshape(-1).contiguous()
    em.poisson(charge, tol=1e-10)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    _, p_it, p_rel = em.poisson(charge, tol=1e-10)
    torch.cuda.synchronize()
    p_s = time.perf_counter() - tp
    rec["poisson"] = {"n_dof": em.n, "bc": "periodic x,y / zero-Neumann z (zero-mean)", "tol": 1e-10,
                      "iterations": p_it, "relres": p_rel, "s": round(p_s, 4),
                      "ms_per_iteration": round(1e3 * p_s / max(p_it, 1), 4),
                      "solver": "Jacobi-preconditioned CG on the device; product = all cell products, then fixed-order nodal sums; batches of 8 iterations replayed from a HIP graph"}
    # Bloch form (Sec. 2.1): the same filter with complex H~^k at an in-plane
    # wave vector, on the same storage read as N/2 complex vectors
    # (interleaved re/im), FP64 only
    if args.prec == "f64" and wl.bc[0] == W.PERIODIC and wl.bc[1] == W.PERIODIC and N % 2 == 0:
        kb = (0.5 * math.pi / wl.L[0], 0.25 * math.pi / wl.L[1])
        gm.set_kpoint(*kb)
        kk = 0.5 * (kb[0] ** 2 + kb[1] ** 2)
        Xc, Yc = X.view(torch.complex128), Y.view(torch.complex128)
        gm.cheb_filter_k(Xc, m, a + kk, b + kk + 1.0, a0 + kk, Y=Yc, work=work)
        torch.cuda.synchronize()
        be0, be1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nb = max(1, min(args.steps, 3))
        be0.record(stream)
        for _ in range(nb):
            gm.cheb_filter_k(Xc, m, a + kk, b + kk + 1.0, a0 + kk, Y=Yc, work=work)
        be1.record(stream)
        torch.cuda.synchronize()
        ms_k = be0.elapsed_time(be1) / nb
        gm.set_kpoint(0.0, 0.0)
        if not torch.isfinite(Y).all():
            raise RuntimeError("non-finite Bloch filter output")
        Nc = N // 2
        # per colour launch: (1/2)K_c and k.G_c products on 2 Nc real columns
        fl_k = 2.0 * 2.0 * nc * nc * (cells / ncol) * (2 * Nc)
        lk_ms = ms_k / launches
        rec["bloch"] = {"k": list(kb), "complex_vectors": Nc, "ms_per_filter": round(ms_k, 4),
                        "GDoF_cvec_per_s": round(m * n * Nc / (ms_k * 1e-3) / 1e9, 3),
                        "avg_launch_ms": round(lk_ms, 5), "flops_per_launch": fl_k,
                        "achieved_TFLOPs": round(fl_k / (lk_ms * 1e-3) / 1e12, 3),
                        "frac_of_fp64_peak": round(fl_k / (lk_ms * 1e-3) / 1e12 / PEAK["f64"][0], 4),
                        "kernel": (f"step_tab_kernel<{wl.p},0,...,CPX> (complex H~^k, the table kernel with the k.G "
                                   "product, one colour pass)" if wl.p in (3, 4) else
                                   f"step_row_kernel<{wl.p},0,...,CPX> (complex H~^k, one colour pass)")}
    if not args.no_mixed and args.prec == "f64":
        t_pot_ms = t_pot
        rec["mixed_precision"] = mixed_precision_report(gm, wl, X, Y, work, a, b, a0, args.steps, ms - t_pot_ms,
                                                        launches, flops_per_launch, args.variant)
    if not args.no_large and args.cfg == 2:
        rec["large_workloads"] = large_workloads(dev, args.steps)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(wl, a, b, a0, args.cpu_cols)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
