"""GPU parity of the separable nonlocal term (Eq. V_nloc: nine Gaussian-radial
s, p, d projectors per site, couplings U(-1,1) Ha) against the oracle's
collocated projector matrix, for H~X, the filter and the adjoint."""
import numpy as np
import pytest

import oracle as O
from paper_2504_00998_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", params=[3, 4])
def nl_case(request):
    """p = 3 runs the row-owner step kernel, p = 4 the z-segment one (one
    segment of 6 cells per column here), each followed by the projector
    kernels."""
    import paper_2504_00998_amd as fe
    wl = W.small_slab((5, 5, 6), p=request.param, N=20, m=8, cfg=5)
    print("case: nonlocal p =", request.param, flush=True)
    om = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, om.quad_points())
    cen = wl.centres()
    D = wl.nonlocal_coupling()
    P = O.Projectors(om, cen, wl.r_cut, wl.r_g)
    op = O.Operator(om, Vq, wl.E, wl.z0, P, D.reshape(-1))
    gm = fe.Mesh.from_workload(wl)
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    gm.set_nonlocal(cen, D, wl.r_cut, wl.r_g)
    return wl, op, gm


def _err(Y, R):
    return (np.linalg.norm(Y - R, axis=0) / np.linalg.norm(R, axis=0)).max()


def test_hx_with_nonlocal(nl_case):
    wl, op, gm = nl_case
    X = wl.X(op.n)
    Y = gm.hx(torch.from_numpy(X).cuda()).cpu().numpy()
    assert _err(Y, op.apply(X)) < 1e-13


def test_hx_with_nonlocal_wide_block(nl_case):
    """150 columns: the projection and expansion kernels take their batched
    path on the full waves of 64 columns and the entry-by-entry path on the
    ragged last wave; two sites of this slab share nodes, so the expansion
    runs colour by colour.  Two calls give the same bits."""
    wl, op, gm = nl_case
    X = wl.X(op.n, cols=range(150))
    Xd = torch.from_numpy(X).cuda()
    Y = gm.hx(Xd).cpu().numpy()
    assert _err(Y, op.apply(X)) < 1e-13
    assert np.array_equal(gm.hx(Xd).cpu().numpy(), Y)


def test_filter_with_nonlocal(nl_case):
    wl, op, gm = nl_case
    X = wl.X(op.n)
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
    a0g, bg = gm.lanczos_bounds(torch.from_numpy(wl.lanczos_start(op.n)).cuda(), 10)
    assert abs(bg - b) < 1e-9 * abs(b) and abs(a0g - a0) < 1e-9 * abs(b)
    a = O.weyl_cut(a0, b, wl.N, op.n)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-4)):
        Y = gm.cheb_filter(torch.from_numpy(X).cuda(), wl.m, a, b, a0, prec=prec).cpu().numpy()
        assert _err(Y, op.filter(X, wl.m, a, b, a0)) < tol, prec


def test_vjp_with_nonlocal(nl_case):
    wl, op, gm = nl_case
    X = wl.X(op.n)
    G = np.random.default_rng(9).standard_normal(X.shape)
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
    a = O.weyl_cut(a0, b, wl.N, op.n)
    Xb_o, g_o = op.filter_vjp(X, G, wl.m, a, b, a0)
    Vb_o, Eb_o = op.potential_vjp(g_o)
    Xb, Vb, Eb = gm.cheb_filter_vjp(torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda(), wl.m, a, b, a0,
                                    ckpt_stride=3, col_chunk=8)
    assert _err(Xb.cpu().numpy(), Xb_o) < 1e-12
    assert np.abs(Vb.cpu().numpy() - Vb_o).max() < 1e-11 * np.abs(Vb_o).max()
    assert abs(Eb.item() - Eb_o) < 1e-11 * max(1.0, abs(Eb_o))


def test_nonlocal_clear_and_errors(nl_case):
    import paper_2504_00998_amd as fe
    wl, op, gm = nl_case
    om = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, om.quad_points())
    op_local = O.Operator(om, Vq, wl.E, wl.z0)
    gm2 = fe.Mesh.from_workload(wl)
    gm2.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    gm2.set_nonlocal(wl.centres(), wl.nonlocal_coupling(), wl.r_cut, wl.r_g)
    gm2.set_nonlocal(np.zeros((0, 3)), np.zeros((0, 9)), wl.r_cut, wl.r_g)  # clears the term
    X = wl.X(op.n)
    Y = gm2.hx(torch.from_numpy(X).cuda()).cpu().numpy()
    assert _err(Y, op_local.apply(X)) < 1e-13
    with pytest.raises(fe.FEError):
        gm2.set_nonlocal(wl.centres(), wl.nonlocal_coupling(), 3.0, wl.r_g)  # ball wraps on a 5-bohr period


@pytest.mark.parametrize("r_cut", [0.35, 0.9])
def test_hx_nonlocal_small_supports(r_cut):
    """Supports shorter than one batch of eight rows (r_cut = 0.35 bohr,
    including a site at the centre of the widest gap between GLL nodes with
    no node inside its ball) and supports of about a hundred rows over two
    expansion chunks (0.9 bohr), overlapping sites in several colours, 70
    columns: H~X against the oracle."""
    import paper_2504_00998_amd as fe
    wl = W.small_slab((5, 5, 6), p=3, N=70, cfg=5)
    print("case: small supports r_cut =", r_cut, flush=True)
    rng = np.random.default_rng(31)
    cen = np.concatenate([[[2.5, 2.5, 3.5]], rng.uniform((0.0, 0.0, 1.0), (5.0, 5.0, 5.0), size=(11, 3))])
    D = rng.uniform(-1.0, 1.0, size=(cen.shape[0], 9))
    om = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, om.quad_points())
    P = O.Projectors(om, cen, r_cut, 0.3)
    op = O.Operator(om, Vq, wl.E, wl.z0, P, D.reshape(-1))
    gm = fe.Mesh.from_workload(wl)
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    gm.set_nonlocal(cen, D, r_cut, 0.3)
    X = wl.X(op.n)
    Y = gm.hx(torch.from_numpy(X).cuda()).cpu().numpy()
    assert _err(Y, op.apply(X)) < 1e-13
