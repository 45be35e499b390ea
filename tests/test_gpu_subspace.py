"""Subspace iteration on the device (filter + CholQR2 + Rayleigh-Ritz)
against the oracle's, and the mixed-precision Ritz error (cell products in
FP32/BF16, everything else FP64)."""
import numpy as np
import pytest

import oracle as O
from paper_2504_00998_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slab():
    import paper_2504_00998_amd as fe
    wl = W.small_slab((4, 4, 6), p=4, N=48, m=20)
    om = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, om.quad_points())
    op = O.Operator(om, Vq, wl.E, wl.z0)
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
    a = O.weyl_cut(a0, b, wl.N, op.n)
    hist_o, _ = O.subspace_iteration(op, wl.X(op.n), wl.m, 5, a, b, a0)
    gm = fe.Mesh.from_workload(wl)
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    return wl, op, gm, (a, b, a0), hist_o


def test_subspace_iteration_f64_matches_oracle(slab):
    from paper_2504_00998_amd import solver
    wl, op, gm, (a, b, a0), hist_o = slab
    X0 = torch.from_numpy(wl.X(op.n)).cuda()
    hist, _ = solver.subspace_iteration(gm, X0, wl.m, 5, a, b, a0, prec="f64")
    for t, (h, ho) in enumerate(zip(hist, hist_o)):
        assert np.abs(h - ho).max() < 1e-9, t


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_subspace_iteration_mixed_precision_ritz_error(slab, prec):
    from paper_2504_00998_amd import solver
    wl, op, gm, (a, b, a0), hist_o = slab
    X0 = torch.from_numpy(wl.X(op.n)).cuda()
    hist, _ = solver.subspace_iteration(gm, X0, wl.m, 5, a, b, a0, prec=prec)
    err_all = np.abs(hist[-1] - hist_o[-1]).max()
    err_low = np.abs(hist[-1][: wl.N // 2] - hist_o[-1][: wl.N // 2]).max()
    print(f"{prec}: max |Ritz - FP64 oracle| all {err_all:.3e} lowest half {err_low:.3e} Ha", flush=True)
    if prec == "f32":
        assert err_low < 1e-7


def test_rayleigh_ritz_refuses_aliased_blocks(slab):
    """fe_rayleigh_ritz writes X = Q W at the end: an X (or P) that shares
    memory with Q would be overwritten while still read, so the library
    refuses overlapping blocks."""
    import paper_2504_00998_amd as fe
    wl, op, gm, _, _ = slab
    Q = torch.from_numpy(wl.X(op.n)).cuda()
    gm.cholqr2(Q)
    P = torch.empty_like(Q)
    for X, Pp in ((Q, P), (P, P), (torch.empty_like(Q), Q)):
        with pytest.raises(RuntimeError, match="overlap"):
            gm.rayleigh_ritz(Q, X=X, P=Pp)
    theta, _ = gm.rayleigh_ritz(Q, X=torch.empty_like(Q), P=P)
    assert np.all(np.diff(theta) >= 0)
