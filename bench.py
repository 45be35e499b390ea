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
# size; valid for this kernel build only
COUNTED_TRAFFIC = {("slab-p4-24x24x48", 256, "f64"): (1.779e9, "step_pipe_kernel<4,0,2,true>"),
                   ("slab-p4-24x24x48", 256, "f32"): (1.779e9, "step_pipe_kernel<4,1,2,true>"),
                   ("slab-p4-24x24x48", 256, "bf16"): (1.779e9, "step_pipe_kernel<4,2,2,true>")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
    return {
        "value": wl.m * om.n * ncols / dt / 1e9,
        "unit": UNIT,
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": f"degree-{wl.m} filter on {ncols} of {wl.N} columns of the full mesh "
                  f"(CSR SpMM, nnz {op.A.nnz}); assembly excluded; {dt:.1f} s",
    }


def mixed_precision_report(gm, wl, X, Y, work, a, b, a0, steps, ms_f64, launches, flops_per_launch, variant):
    """FP32 / BF16 cell products on the same workload: filter throughput,
    speedup over FP64, the step kernel's launch time against the MFMA peak of
    the precision (and its counted HBM rate where the counters of the kernel
    are known), and the Ritz values after 5 subspace iterations (filter in the
    given precision; CholQR2 and Rayleigh-Ritz in FP64) against the same
    iteration with FP64 cell products."""
    import numpy as np
    import torch
    from paper_2504_00998_amd import solver

    stream = torch.cuda.current_stream()
    n, N, m = gm.n, wl.N, wl.m
    hist64, _ = solver.subspace_iteration(gm, X, m, 5, a, b, a0, prec="f64", work=work)
    out = {"ritz_iterations": 5, "ritz_reference": "same subspace iteration with FP64 cell products"}
    for prec in ("f32", "bf16"):
        gm.cheb_filter(X, m, a, b, a0, prec=prec, Y=Y, work=work)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            gm.cheb_filter(X, m, a, b, a0, prec=prec, Y=Y, work=work)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        hist, _ = solver.subspace_iteration(gm, X, m, 5, a, b, a0, prec=prec, work=work)
        d = np.abs(hist[-1] - hist64[-1])
        launch_ms = ms / launches
        tf = flops_per_launch / (launch_ms * 1e-3) / 1e12
        traffic = COUNTED_TRAFFIC.get((wl.name, N, prec)) if variant == 0 else None
        out[prec] = {"value": round(m * n * N / (ms * 1e-3) / 1e9, 4), "ms_per_filter": round(ms, 4),
                     "speedup_vs_f64": round(ms_f64 / ms, 3),
                     "avg_launch_ms": round(launch_ms, 5), "achieved_TFLOPs": round(tf, 3),
                     "frac_of_mfma_peak": round(tf / PEAK[prec][0], 4),
                     "hbm_GBps": round(traffic[0] / (launch_ms * 1e-3) / 1e9, 1) if traffic and traffic[0] else None,
                     "kernel": traffic[1] if traffic else None,
                     "ritz_err_max_Ha": float(d.max()), "ritz_err_lowest_half_Ha": float(d[: N // 2].max()),
                     "ritz_ok_1e-7": bool(d[: N // 2].max() <= 1e-7)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--cfg", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=24)
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32/BF16 report")
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
                      "kernel": "density_kernel (2 sum_n f_n X[I,n]^2 / M_I, 16 lanes per DoF)"}
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
                        "kernel": f"step_row_kernel<{wl.p},0,...,CPX> (complex H~^k, one colour pass)"}
    if not args.no_mixed and args.prec == "f64":
        t_pot_ms = t_pot
        rec["mixed_precision"] = mixed_precision_report(gm, wl, X, Y, work, a, b, a0, args.steps, ms - t_pot_ms,
                                                        launches, flops_per_launch, args.variant)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(wl, a, b, a0, args.cpu_cols)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
