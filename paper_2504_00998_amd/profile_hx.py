"""Profiling driver: one H~X per cell-product precision on a workload.

Run under ``rocprofv3`` to take per-kernel traces or counters of the step
kernels, e.g. (from any directory)::

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o run -- \\
        python3 REPO/paper_2504_00998_amd/profile_hx.py --cfg 2

Before the H~X launches it copies one (n x N) FP64 block with PyTorch, so the
same trace holds a plain copy kernel of known size (n*N*8 bytes read and
written) against which HBM byte counters can be calibrated.  With --filter M
it then runs a degree-M filter per precision as well, whose steps after the
first read the previous iterate (the launches the filter rate is made of).
With --nonlocal the workload's projector sites are set, so that each H~X
also runs the projection and expansion kernels.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cfg", type=int, default=2)
    ap.add_argument("--precs", default="f64,f32,bf16")
    ap.add_argument("--variant", type=int, default=0, help="step-kernel variant (fe_mesh_set_kernel)")
    ap.add_argument("--filter", type=int, default=0, help="also run a filter of this degree per precision")
    ap.add_argument("--nonlocal", dest="with_nonlocal", action="store_true", help="set the workload's nonlocal sites (cfg5)")
    args = ap.parse_args()

    import torch

    import paper_2504_00998_amd as fe
    from paper_2504_00998_amd import workloads as W

    wl = W.CONFIGS[args.cfg]
    gm = fe.Mesh.from_workload(wl)
    gm.set_kernel(args.variant)
    n, N = gm.n, wl.N
    Vq = torch.from_numpy(W.workload_potential(wl, gm.quad_points())).cuda()
    gm.set_potential(Vq, wl.E, wl.z0)
    if args.with_nonlocal and wl.nonlocal_sites:
        gm.set_nonlocal(wl.centres(), wl.nonlocal_coupling(), wl.r_cut, wl.r_g)
    X = torch.randn(n, N, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    torch.cuda.synchronize()
    Y.copy_(X)
    torch.cuda.synchronize()
    print(f"copy: {n * N * 8} bytes read and written", flush=True)
    for prec in args.precs.split(","):
        gm.hx(X, Y, prec=prec)
        torch.cuda.synchronize()
        print(f"hx {prec} done ({wl.name}, n={n}, N={N}, variant {args.variant})", flush=True)
        if args.filter > 0:
            # bounds of the slab workloads' spectra (the values only scale the recurrence)
            gm.cheb_filter(X, args.filter, 5.6, 314.0, 4.8, prec=prec, Y=Y)
            torch.cuda.synchronize()
            print(f"filter {prec} degree {args.filter} done", flush=True)


if __name__ == "__main__":
    main()
