"""Write cfg3_ritz_oracle.txt: the oracle's reference for the mixed-precision
Ritz errors.

Chebyshev-filtered subspace iteration on the p = 4 slab of 24x24x48 cells
(1,760,256 free DoFs; Gaussian-well lattice and field -E (z - z0) of the
slab recipe), N = 256 vectors drawn from the cfg-3 seeds, filter degree 30,
5 iterations: filter, two passes of Cholesky-QR, Rayleigh-Ritz, with the cut
a and the scaling point a0 taken from the current Ritz values after each
iteration.  The spectrum bounds come from the oracle's 10-step Lanczos run
(seeded start vector); the first cut is the Weyl-law guess.  Everything here
is the CPU oracle (FP64 CSR products, numpy/LAPACK dense steps); nothing
comes from the GPU library.

Usage (repository root):  python tests/golden/make_cfg3_ritz.py
Takes about 10-20 minutes on 8 cores and ~30 GB of host memory.
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2504_00998_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg3_ritz_oracle.txt")
ITERS = 5


def main():
    wl = W.CFG3
    t0 = time.time()
    om = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, om.quad_points())
    op = O.Operator(om, Vq, wl.E, wl.z0)
    n = op.n
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(n), 10)
    a = O.weyl_cut(a0, b, wl.N, n)
    print(f"assembled n={n} nnz={op.A.nnz}; bounds a0={a0!r} a={a!r} b={b!r} ({time.time() - t0:.0f} s)",
          flush=True)
    X = wl.X(n)
    hist = []
    aa, a00 = a, a0
    for it in range(ITERS):
        h, X = O.subspace_iteration(op, X, wl.m, 1, aa, b, a00)
        hist.append(h[0])
        aa, a00 = float(h[0][-1]), float(h[0][0])
        print(f"iteration {it + 1}: theta_1={h[0][0]!r} theta_N={h[0][-1]!r} ({time.time() - t0:.0f} s)",
              flush=True)
    with open(OUT, "w") as f:
        f.write("# Oracle reference of the mixed-precision Ritz errors (written by make_cfg3_ritz.py,\n")
        f.write("# which calls only the CPU oracle).  Workload: p=4 slab 24x24x48 cells, n=%d, N=%d,\n" % (n, wl.N))
        f.write("# filter degree %d, %d iterations of filter + CholQR2 + Rayleigh-Ritz, seeds of cfg %d.\n"
                % (wl.m, ITERS, wl.cfg))
        f.write("# Lanczos bounds (10 steps, seeded start) and the first cut:\n")
        f.write("bounds %r %r %r\n" % (a0, b, a))
        f.write("# iteration index ritz_value (Ha), ascending within each iteration\n")
        for it, th in enumerate(hist):
            for j, v in enumerate(th):
                f.write("%d %d %r\n" % (it + 1, j, float(v)))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
