"""The allocation-free form of H~X (fe_hx_apply_noalloc) against fe_hx_apply,
through the C ABI, on a mesh with a nonlocal term (the only part of H~X with
scratch: the projections diag(D) C~^T X, kept in a static device array)."""
import ctypes as C
import math

import numpy as np
import pytest

import oracle as O
from paper_2504_00998_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAX_DOUBLES = 4 * 1024 * 1024  # the static array, 32 MiB


def _mesh(wl):
    import paper_2504_00998_amd as fe
    gm = fe.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, gm.quad_points())
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    gm.set_nonlocal(wl.centres(), wl.nonlocal_coupling(), wl.r_cut, wl.r_g)
    return gm, Vq


def _call(gm, name, X, Y, prec=0):
    import paper_2504_00998_amd as fe
    L = fe.lib()
    N, ld = X.shape[1], X.stride(0)
    st = getattr(L, name)(gm._h, C.c_void_p(X.data_ptr()),
                          C.c_void_p(Y.data_ptr()), N, ld, prec, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, L.fe_last_error().decode()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_hx_equals_hx_apply_on_two_calls(prec):
    """Two calls in a row, the second with fewer vectors (the array keeps the
    first call's contents): both equal fe_hx_apply bit for bit, and the FP64
    result equals the oracle's nonlocal operator."""
    wl = W.small_slab((5, 5, 6), p=4, N=48, cfg=5)
    gm, Vq = _mesh(wl)
    om = O.Mesh.from_workload(wl)
    P = O.Projectors(om, wl.centres(), wl.r_cut, wl.r_g)
    op = O.Operator(om, Vq, wl.E, wl.z0, P, wl.nonlocal_coupling().reshape(-1))
    for N in (48, 17):
        print("case: noalloc hx", dict(prec=prec, N=N, sites=wl.centres().shape[0]), flush=True)
        Xh = wl.X(gm.n, cols=range(N))
        X = torch.from_numpy(Xh).cuda()
        Y0 = torch.full_like(X, math.nan)
        Y1 = torch.full_like(X, math.nan)
        st, msg = _call(gm, "fe_hx_apply", X, Y0, prec)
        assert st == 0, msg
        st, msg = _call(gm, "fe_hx_apply_noalloc", X, Y1, prec)
        assert st == 0, msg
        torch.cuda.synchronize()
        assert torch.equal(Y0, Y1)
        if prec == 0:
            R = op.apply(Xh)
            Yh = Y1.cpu().numpy()
            assert (np.linalg.norm(Yh - R, axis=0) / np.linalg.norm(R, axis=0)).max() < 1e-13


def test_noalloc_hx_at_and_beyond_the_maximum():
    """At the largest N the array holds (9 n_site N = 4,194,304 doubles for
    one site) the result equals fe_hx_apply; one more vector is refused with
    FE_ENOMEM before anything is enqueued (Y left untouched)."""
    import paper_2504_00998_amd as fe
    wl = W.small_slab((5, 5, 2), p=1, N=8, cfg=5, lattice=((2.5,), (2.5,), (1.0,)))
    gm, _ = _mesh(wl)
    assert wl.centres().shape[0] == 1
    Nmax = MAX_DOUBLES // 9
    g = torch.Generator(device="cuda")
    g.manual_seed(wl.seed(2))
    X = torch.randn(gm.n, Nmax, generator=g, dtype=torch.float64, device="cuda")
    print("case: noalloc hx at the maximum", dict(n=gm.n, N=Nmax), flush=True)
    Y0 = torch.full_like(X, math.nan)
    Y1 = torch.full_like(X, math.nan)
    st, msg = _call(gm, "fe_hx_apply", X, Y0)
    assert st == 0, msg
    st, msg = _call(gm, "fe_hx_apply_noalloc", X, Y1)
    assert st == 0, msg
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1)
    del Y0
    X2 = torch.randn(gm.n, Nmax + 1, generator=g, dtype=torch.float64, device="cuda")
    Y2 = torch.full_like(X2, math.nan)
    st, msg = _call(gm, "fe_hx_apply_noalloc", X2, Y2)
    assert st == fe.FE_ENOMEM and "static scratch" in msg, (st, msg)
    torch.cuda.synchronize()
    assert torch.isnan(Y2).all()
    # the binding raises the same refusal
    with pytest.raises(RuntimeError, match="static scratch"):
        gm.hx_noalloc(X2, Y2)
