"""GPU parity of the C-ABI hot path against the CPU oracle.

Inputs are the seeded synthetic slabs of `paper_2504_00998_amd.workloads`,
with the potential sampled at the oracle's own GLL points and handed to both
sides.  The bar for FP64 is 1e-12 relative per vector for the filter (the
target tolerance) and 1e-13 for a single H~ application.  Mixed precision is
reported against the FP64 oracle with tolerances derived from the unit
roundoff of the cell-product format.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2504_00998_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fe():
    import paper_2504_00998_amd as fe
    return fe


def _setup(wl, rule=None):
    """Oracle operator and GPU mesh for a workload, same potential on both."""
    fe = _fe()
    om = O.Mesh.from_workload(wl, rule)
    Vq = W.workload_potential(wl, om.quad_points())
    op = O.Operator(om, Vq, wl.E, wl.z0)
    gm = fe.Mesh.from_workload(wl, rule)
    assert gm.n == om.n
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    return op, gm, Vq


def _relerr(Y, R):
    return (np.linalg.norm(Y - R, axis=0) / np.maximum(np.linalg.norm(R, axis=0), 1e-300)).max()


def _print_case(**kw):
    print("case:", kw, flush=True)


CASES = [
    # (label, workload) -- several tiles of every axis, ragged vector chunks
    ("cfg1", W.CFG1),
    ("slab-p4-3x3x4-N20", W.small_slab((3, 3, 4), p=4, N=20)),
    ("slab-p4-odd-periodic-N7", W.small_slab((3, 5, 3), p=4, N=7)),
    ("slab-p1-N33", W.small_slab((4, 4, 5), p=1, N=33)),
    ("slab-p2", W.small_slab((2, 3, 4), p=2, N=16)),
    ("slab-p3-gll", W.small_slab((3, 2, 3), p=3, N=17, rule=W.RULE_GLL)),
    ("slab-p5", W.small_slab((2, 2, 3), p=5, N=18)),
    ("slab-p6", W.small_slab((2, 2, 2), p=6, N=16)),
    ("slab-p7", W.small_slab((2, 2, 2), p=7, N=5)),
    ("neumann-box-p3", W.small_slab((2, 3, 2), p=3, N=9, bc=(W.NEUMANN, W.NEUMANN, W.NEUMANN))),
    ("mixed-bc-p4", W.small_slab((3, 2, 2), p=4, N=16, bc=(W.DIRICHLET, W.PERIODIC, W.NEUMANN))),
]


@pytest.mark.parametrize("label,wl", CASES, ids=[c[0] for c in CASES])
def test_hx_f64_matches_oracle(label, wl):
    _print_case(test="hx_f64", label=label, ncell=wl.ncell, p=wl.p, N=wl.N)
    op, gm, _ = _setup(wl)
    X = wl.X(op.n)
    Y = gm.hx(torch.from_numpy(X).cuda()).cpu().numpy()
    R = op.apply(X)
    assert _relerr(Y, R) < 1e-13


# filter cases: every H~X case, plus p = 5, 6, 7 at N >= 32, where the step
# kernel's recurrence path (the beta Y_{k-1} read, the first writer's old
# value, the rotation of the two blocks) runs in the one-cell row-owner kernel
FILTER_CASES = CASES + [
    ("slab-p5-N40", W.small_slab((2, 2, 3), p=5, N=40)),
    ("slab-p6-N33", W.small_slab((2, 2, 3), p=6, N=33)),
    ("slab-p7-N32", W.small_slab((2, 2, 2), p=7, N=32)),
    ("slab-p6-odd-periodic-N32", W.small_slab((3, 2, 2), p=6, N=32)),
]


@pytest.mark.parametrize("label,wl", FILTER_CASES, ids=[c[0] for c in FILTER_CASES])
@pytest.mark.parametrize("scaled", [True, False])
def test_filter_f64_matches_oracle(label, wl, scaled):
    _print_case(test="filter_f64", label=label, scaled=scaled)
    op, gm, _ = _setup(wl)
    X = wl.X(op.n)
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
    a = O.weyl_cut(a0, b, wl.N, op.n)
    a0s = a0 if scaled else math.nan
    m = wl.m if scaled else min(wl.m, 9)
    R = op.filter(X, m, a, b, a0s)
    Y = gm.cheb_filter(torch.from_numpy(X).cuda(), m, a, b, a0s).cpu().numpy()
    assert _relerr(Y, R) < 1e-12


@pytest.mark.parametrize("m", [1, 2, 3, 6])
def test_filter_degrees_and_leading_dimension(m):
    wl = W.small_slab((3, 3, 4), p=4, N=20)
    _print_case(test="filter_ld", m=m)
    op, gm, _ = _setup(wl)
    X = wl.X(op.n)
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
    a = O.weyl_cut(a0, b, wl.N, op.n)
    R = op.filter(X, m, a, b, a0)
    # X inside a wider buffer (ld = N + 5)
    Xb = torch.zeros((op.n, wl.N + 5), dtype=torch.float64, device="cuda")
    Xb[:, :wl.N] = torch.from_numpy(X).cuda()
    Yb = torch.full_like(Xb, float("nan"))
    gm.cheb_filter(Xb[:, :wl.N], m, a, b, a0, Y=Yb[:, :wl.N])
    Y = Yb[:, :wl.N].cpu().numpy()
    assert _relerr(Y, R) < 1e-12
    assert torch.isnan(Yb[:, wl.N:]).all()  # padding untouched


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("p", [2, 4, 5])
def test_kernel_variants_bitwise_equal(prec, p):
    """The multi-vector kernels and the one-cell-per-workgroup kernel perform
    the same operations in the same order.  The default at p = 4 is the
    table kernel (variant 10) for FP64 and FP32 products and the z-segment
    kernel (variant 9) for BF16, and at p = 5 the table kernel for FP32; both
    sum shared nodes in another order (the table kernel also multiplies with
    the folded cell matrix, BF16 takes the products transposed): equal to
    rounding, and bitwise equal to the variant they run.  Where the table
    kernel does not apply (p = 2; p = 5 in FP64 and BF16; BF16) variant 10
    runs the one-cell kernel.  The removed variants are refused."""
    wl = W.small_slab((3, 3, 4), p=p, N=40)
    op, gm, _ = _setup(wl)
    X = torch.from_numpy(wl.X(op.n)).cuda()
    for gone in (2, 5, 8, 11, -1):
        with pytest.raises(RuntimeError, match="kernel variant"):
            gm.set_kernel(gone)
    gm.set_kernel(1)
    Y1 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec)
    tab = (p == 4 and prec in ("f64", "f32")) or (p == 5 and prec == "f32")
    # above p = 4 variant 9 runs what variant 7 runs (one-cell kernels)
    for var in (0, 3, 4, 6, 7, 10) + ((9,) if p > 4 else ()):
        gm.set_kernel(var)
        Y0 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec)
        if (var == 0 and (p == 4 or tab)) or (var == 10 and tab):
            # two FP32 product orders, each within about 1e-6 of the exact
            # degree-5 filter (5e-7 at p = 4, up to 1.1e-6 apart at p = 5)
            rel = ((Y0 - Y1).norm(dim=0) / Y1.norm(dim=0)).max().item()
            assert 0 < rel < {"f64": 1e-13, "f32": 3e-6, "bf16": 1e-5}[prec], rel
        else:
            assert torch.equal(Y0, Y1), var
    if p == 4 or tab:
        gm.set_kernel(0)
        Y0 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec)
        gm.set_kernel(10 if tab else 9)
        assert torch.equal(gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec), Y0)
    gm.set_kernel(0)


def test_bitwise_reproducible():
    wl = W.small_slab((3, 3, 4), p=4, N=32)
    op, gm, _ = _setup(wl)
    X = torch.from_numpy(wl.X(op.n)).cuda()
    Y1 = gm.cheb_filter(X, 12, 2.0, 60.0, -0.5)
    Y2 = gm.cheb_filter(X, 12, 2.0, 60.0, -0.5)
    assert torch.equal(Y1, Y2)


@pytest.mark.parametrize("prec,tol", [("f32", 2e-5), ("bf16", 5e-2)])
def test_hx_mixed_precision_error(prec, tol):
    """Cell products in FP32 / BF16 with FP32 accumulation: the error of H~X
    against the FP64 oracle is bounded by a small multiple of the format's
    unit roundoff times ||D A D|| ||X|| / ||H~X|| (reported, loose bar)."""
    wl = W.small_slab((3, 3, 4), p=4, N=16)
    op, gm, _ = _setup(wl)
    X = wl.X(op.n)
    Y = gm.hx(torch.from_numpy(X).cuda(), prec=prec).cpu().numpy()
    R = op.apply(X)
    err = _relerr(Y, R)
    print(f"hx {prec} rel err {err:.3e}")
    assert err < tol


def test_potential_update_and_state_errors():
    fe = _fe()
    wl = W.small_slab((2, 2, 3), p=3, N=4)
    gm = fe.Mesh.from_workload(wl)
    X = torch.zeros((gm.n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FEError) as e:
        gm.hx(X)
    assert e.value.status == fe.FE_ESTATE
    gm.set_potential(None, wl.E, wl.z0)
    om = O.Mesh.from_workload(wl)
    op = O.Operator(om, None, wl.E, wl.z0)
    Xn = wl.X(gm.n)[:, :4]
    Y = gm.hx(torch.from_numpy(np.ascontiguousarray(Xn)).cuda()).cpu().numpy()
    assert _relerr(Y, op.apply(np.ascontiguousarray(Xn))) < 1e-13
    with pytest.raises(fe.FEError) as e:
        gm.cheb_filter(X, 3, 1.0, 0.5)
    assert e.value.status == fe.FE_EINVAL


def test_lanczos_cholqr_rayleigh_ritz_on_device():
    """Device Lanczos bound b >= lambda_max (dense eigh), CholQR2
    orthonormality and Rayleigh-Ritz values against the oracle's."""
    wl = W.CFG1
    op, gm, _ = _setup(wl)
    H = op.A.to_scipy().toarray()
    lam = np.linalg.eigvalsh(H)
    v0 = wl.lanczos_start(op.n)
    a0g, bg = gm.lanczos_bounds(torch.from_numpy(v0).cuda(), 10)
    a0o, bo, _ = O.lanczos_bounds(op.apply, v0, 10)
    assert bg >= lam[-1] and abs(bg - bo) < 1e-10 * abs(bo) and abs(a0g - a0o) < 1e-10 * abs(bo)
    Y = torch.from_numpy(wl.X(op.n)).cuda()
    Q = gm.cholqr2(Y.clone())
    Qh = Q.cpu().numpy()
    assert np.abs(Qh.T @ Qh - np.eye(wl.N)).max() < 1e-13
    Qo, _ = O.cholqr2(wl.X(op.n))
    # same span: projectors agree
    assert np.abs(Qh @ Qh.T - Qo @ Qo.T).max() < 1e-12
    theta, Xr = gm.rayleigh_ritz(Q)
    th_o, _ = O.rayleigh_ritz(op.apply, Qh)
    np.testing.assert_allclose(theta, th_o, atol=1e-12 * np.abs(lam).max())


@pytest.mark.parametrize("shape,p", [((3, 5, 4), 2), ((5, 4, 7), 3), ((6, 6, 9), 4), ((3, 3, 4), 5)])
def test_single_vector_cell_batched_kernel(shape, p):
    """N = 1 in FP64 runs the cell-batched kernel (16 cells in the MFMA vector
    columns): bitwise equal to the one-cell kernel, equal to the oracle, on
    colours whose cell counts are not multiples of 16; the recurrence form
    (beta != 0, Y_{k-1} read) through a short filter."""
    wl = W.small_slab(shape, p=p, N=1)
    print("case:", dict(shape=shape, p=p), flush=True)
    op, gm, _ = _setup(wl)
    X = torch.from_numpy(wl.X(op.n)).cuda()
    gm.set_kernel(1)
    Y1 = gm.hx(X)
    F1 = gm.cheb_filter(X, 6, 2.0, 400.0, -0.5)
    gm.set_kernel(0)
    Y0 = gm.hx(X)
    F0 = gm.cheb_filter(X, 6, 2.0, 400.0, -0.5)
    assert torch.equal(Y0, Y1) and torch.equal(F0, F1)
    assert _relerr(Y0.cpu().numpy(), op.apply(wl.X(op.n))) < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("p", [2, 3, 4])
def test_pipelined_variant_several_items_per_workgroup(p, prec):
    """The persistent pipelined kernel (variant 7, FP64 and FP32) walks several items per
    workgroup only when a colour pass has more items than resident
    workgroups: 24 x 24 x 16 cells and 64 vectors give 2304 items per pass
    (about 9 per workgroup at p = 4).  Bitwise equal to the one-cell kernel
    for one application and for the filter (previous-iterate path)."""
    wl = W.small_slab((24, 24, 16), p=p, N=64)
    fe = _fe()
    _print_case(test="pipelined_multi_item", p=p, prec=prec, ncell=wl.ncell, N=wl.N)
    gm = fe.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, gm.quad_points())
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    g = torch.Generator(device="cuda")
    g.manual_seed(wl.seed(2))
    X = torch.randn(gm.n, wl.N, generator=g, dtype=torch.float64, device="cuda")
    gm.set_kernel(1)
    Y1 = gm.hx(X, prec=prec)
    F1 = gm.cheb_filter(X, 6, 2.0, 400.0, -0.5, prec=prec)
    gm.set_kernel(7)
    assert torch.equal(gm.hx(X, prec=prec), Y1)
    assert torch.equal(gm.cheb_filter(X, 6, 2.0, 400.0, -0.5, prec=prec), F1)


def test_empty_blocks_and_the_one_dof_mesh():
    """N = 0 is a no-op for every apply / filter entry point (the output is
    left untouched); a single Dirichlet cell of degree 2 has one free DoF,
    and H~X and the filter on it match the oracle."""
    fe = _fe()
    wl = W.small_slab((3, 3, 4), p=2, N=4)
    _print_case(test="empty_and_one_dof")
    op, gm, _ = _setup(wl)
    L = fe.lib()
    Y = torch.full((op.n, 4), 7.0, dtype=torch.float64, device="cuda")
    X = torch.ones_like(Y)
    W0 = torch.empty(8 * op.n, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.fe_hx_apply(gm._h, X.data_ptr(), Y.data_ptr(), 0, 4, fe._PREC["f64"], s) == fe.FE_OK
    assert L.fe_cheb_filter(gm._h, X.data_ptr(), Y.data_ptr(), 0, 4, 5, 1.0, 9.0, float("nan"), fe._PREC["f64"],
                            W0.data_ptr(), W0.numel() * 8, s) == fe.FE_OK
    assert L.fe_hx_apply_k(gm._h, X.data_ptr(), Y.data_ptr(), 0, 2, s) == fe.FE_OK
    assert L.fe_cheb_filter_k(gm._h, X.data_ptr(), Y.data_ptr(), 0, 2, 5, 1.0, 9.0, float("nan"), W0.data_ptr(),
                              W0.numel() * 8, s) == fe.FE_OK
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
    # one free DoF: a single cube, Dirichlet on every face, p = 2
    one = W.small_slab((1, 1, 1), p=2, N=3, bc=(W.DIRICHLET, W.DIRICHLET, W.DIRICHLET))
    op1, gm1, _ = _setup(one)
    assert op1.n == 1 and gm1.n == 1
    X1 = one.X(1)
    assert _relerr(gm1.hx(torch.from_numpy(X1).cuda()).cpu().numpy(), op1.apply(X1)) < 1e-13
    lam = float(op1.apply(np.ones((1, 1)))[0, 0])
    Yf = gm1.cheb_filter(torch.from_numpy(X1).cuda(), 4, lam + 1.0, lam + 3.0, lam - 1.0).cpu().numpy()
    assert _relerr(Yf, op1.filter(X1, 4, lam + 1.0, lam + 3.0, lam - 1.0)) < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape,p,bc,zl", [
    ((3, 3, 12), 4, None, 6),                                 # Dirichlet z, 2 segments
    ((3, 3, 9), 3, (W.PERIODIC, W.PERIODIC, W.PERIODIC), 3),  # periodic z, 3 segments: 3 colours
    ((3, 2, 8), 4, (W.DIRICHLET, W.PERIODIC, W.PERIODIC), 4),  # periodic z, 2 segments
    ((2, 3, 10), 3, (W.NEUMANN, W.NEUMANN, W.NEUMANN), 5),    # Neumann z
    ((3, 3, 7), 2, None, 1),                                  # no divisor: plain cells
    ((2, 2, 18), 4, (W.PERIODIC, W.PERIODIC, W.PERIODIC), 6),  # p = 4, periodic z, 3 segment colours
    ((3, 2, 10), 4, (W.PERIODIC, W.DIRICHLET, W.NEUMANN), 5),  # p = 4, Neumann z
    ((3, 3, 12), 1, None, 6),                                 # p = 1: 4-node faces, 32-row padded tile
    ((4, 3, 8), 1, (W.PERIODIC, W.PERIODIC, W.PERIODIC), 4),  # p = 1, periodic z
])
def test_zsegment_variant_matches_oracle_and_is_reproducible(prec, shape, p, bc, zl):
    """Variant 9 walks z segments of zl cells (the largest length up to 6 that
    divides the z cell count, at least two segments on a periodic axis) and
    keeps the faces shared inside a segment in LDS.  Each node's
    contributions are summed in another fixed order, so the result equals the
    one-cell kernel to rounding and itself bit for bit; with zl = 1 it is the
    plain pipelined kernel, bitwise equal to the one-cell kernel (FP64, FP32;
    BF16 products are taken transposed there, equal to rounding)."""
    kw = {} if bc is None else dict(bc=bc)
    if bc is not None and bc[2] == W.PERIODIC:
        kw["E"] = 0.0  # a linear field has no periodic form along z
    wl = W.small_slab(shape, p=p, N=40, **kw)
    _print_case(test="zsegment", prec=prec, shape=shape, p=p, bc=bc)
    op, gm, _ = _setup(wl)
    X = torch.from_numpy(wl.X(op.n)).cuda()
    gm.set_kernel(1)
    Y1 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec)
    H1 = gm.hx(X, prec=prec)
    gm.set_kernel(9)
    Y9 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec)
    assert torch.equal(Y9, gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec))
    H9 = gm.hx(X, prec=prec)
    if zl == 1 and prec != "bf16":
        assert torch.equal(Y9, Y1) and torch.equal(H9, H1)
    elif prec == "f64":
        assert not torch.equal(Y9, Y1)  # equal bits would mean the cell path ran
    tol = {"f64": 1e-13, "f32": 1e-6, "bf16": 1e-5}[prec]
    for A, B in ((Y9, Y1), (H9, H1)):
        rel = ((A - B).norm(dim=0) / B.norm(dim=0)).max().item()
        assert rel < tol, rel
    if prec == "f64":
        Xn = wl.X(op.n)
        assert _relerr(H9.cpu().numpy(), op.apply(Xn)) < 1e-13
        a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
        a = O.weyl_cut(a0, b, wl.N, op.n)
        assert _relerr(gm.cheb_filter(X, wl.m, a, b, a0).cpu().numpy(), op.filter(Xn, wl.m, a, b, a0)) < 1e-12
    gm.set_kernel(0)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("p,N", [(2, 128), (4, 64)])
def test_zsegment_variant_several_items_per_workgroup(p, N, prec):
    """24 x 24 x 24 cells: segments of 6 cells, 2 per colour pass, so that a
    workgroup walks several segments and the two-deep prefetch crosses from
    one segment to the next.  Equal to the one-cell kernel to rounding,
    reproducible, for one application and for the filter."""
    wl = W.small_slab((24, 24, 24), p=p, N=N)
    fe = _fe()
    _print_case(test="zsegment_multi_item", p=p, prec=prec, ncell=wl.ncell, N=wl.N)
    gm = fe.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, gm.quad_points())
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    g = torch.Generator(device="cuda")
    g.manual_seed(wl.seed(2))
    X = torch.randn(gm.n, wl.N, generator=g, dtype=torch.float64, device="cuda")
    gm.set_kernel(1)
    Y1 = gm.hx(X, prec=prec)
    F1 = gm.cheb_filter(X, 6, 2.0, 400.0, -0.5, prec=prec)
    gm.set_kernel(9)
    Y9 = gm.hx(X, prec=prec)
    F9 = gm.cheb_filter(X, 6, 2.0, 400.0, -0.5, prec=prec)
    assert torch.equal(gm.hx(X, prec=prec), Y9)
    assert torch.equal(gm.cheb_filter(X, 6, 2.0, 400.0, -0.5, prec=prec), F9)
    tol = {"f64": 1e-13, "f32": 1e-6, "bf16": 1e-5}[prec]
    for A, B in ((Y9, Y1), (F9, F1)):
        rel = ((A - B).norm(dim=0) / B.norm(dim=0)).max().item()
        assert rel < tol, rel
    gm.set_kernel(0)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("N", [1, 17])
def test_zsegment_variant_ragged_blocks(prec, N):
    """Blocks of 1 and 17 vectors through the z-segment kernel (p = 4): the
    second 16-vector chunk of every item is wholly or partly outside N, so
    those lanes load clamped columns, and their outputs (and holds) must not
    leak into the block.  Equal to the one-cell kernel to rounding; columns
    past N of the wider buffers untouched.  X and Y share one leading
    dimension (N + 3 here); a Y of another layout is refused."""
    wl = W.small_slab((3, 3, 12), p=4, N=N)
    _print_case(test="zsegment_ragged", prec=prec, N=N)
    op, gm, _ = _setup(wl)
    Xb = torch.full((op.n, N + 3), float("nan"), dtype=torch.float64, device="cuda")
    Xb[:, :N] = torch.from_numpy(wl.X(op.n)).cuda()
    X = Xb[:, :N]
    gm.set_kernel(1)
    Y1 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec)
    gm.set_kernel(9)
    Yb = torch.full((op.n, N + 3), float("nan"), dtype=torch.float64, device="cuda")
    gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec, Y=Yb[:, :N])
    Y9 = Yb[:, :N]
    with pytest.raises(ValueError):
        gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, prec=prec, Y=torch.empty((op.n, N), dtype=torch.float64, device="cuda"))
    rel = ((Y9 - Y1).norm(dim=0) / Y1.norm(dim=0)).max().item()
    assert rel < {"f32": 1e-6, "bf16": 1e-5}[prec], rel
    assert torch.isnan(Yb[:, N:]).all()
    gm.set_kernel(0)


def test_binding_rejects_mismatched_buffers():
    """The binding refuses, before any library call, buffers whose layout the
    C entry points would misread: an output block of another leading
    dimension or width, a start vector or output vector of the wrong length
    or type, a scratch buffer that is not contiguous on the device."""
    wl = W.small_slab((3, 3, 4), p=2, N=4)
    _print_case(test="binding_checks")
    op, gm, _ = _setup(wl)
    n = op.n
    dev = "cuda"
    X = torch.from_numpy(wl.X(n)).cuda()
    f64 = dict(dtype=torch.float64, device=dev)
    bad_ld = torch.empty((n, 6), **f64)[:, :4]
    with pytest.raises(ValueError):
        gm.hx(X, bad_ld)
    with pytest.raises(ValueError):
        gm.cheb_filter(X, 3, 2.0, 40.0, Y=bad_ld)
    with pytest.raises(ValueError):
        gm.cheb_filter(X, 3, 2.0, 40.0, Y=torch.empty((n, 3), **f64))
    with pytest.raises(ValueError):
        gm.cheb_filter(X, 3, 2.0, 40.0, work=torch.empty(2 * n * 4, **f64)[::2])
    with pytest.raises(ValueError):
        gm.cheb_filter_vjp(X, bad_ld, 3, 2.0, 40.0)
    with pytest.raises(ValueError):
        gm.lanczos_bounds(torch.ones(n - 1, **f64))
    with pytest.raises(ValueError):
        gm.lanczos_bounds(torch.ones(n, dtype=torch.float32, device=dev))
    f = torch.ones(4, **f64)
    with pytest.raises(ValueError):
        gm.density(X, f, rho=torch.empty(n + 1, **f64))
    with pytest.raises(ValueError):
        gm.planar_average(torch.ones(n, **f64), out=torch.empty(1, **f64))
    with pytest.raises(ValueError):
        gm.rayleigh_ritz(X, X=bad_ld)
    # a float32 scratch buffer is sized by its own element size (half the
    # bytes of as many doubles): too small here, so the library refuses it
    with pytest.raises(RuntimeError):
        gm.cheb_filter(X, 3, 2.0, 40.0, work=torch.empty(n * 4, dtype=torch.float32, device=dev))
