"""The table kernel with direct-to-LDS prefetch (kernel variant 10):
parity with the oracle, reproducibility, the cases where it does not apply
(it falls back to the one-cell kernel), walks of several segments per
workgroup, and the split of N into whole 32-vector groups (table kernel)
and the rest (z-segment kernel).  It multiplies with the cell matrix
pre-scaled by the per-local-index M^-1/2 (meshes without a zero-Neumann
axis) and folds the epilogue into fused multiply-adds, so its rounding
differs from the other kernels'; it is compared with the oracle and with
them to rounding."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2504_00998_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _setup(wl):
    import paper_2504_00998_amd as fe
    om = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, om.quad_points())
    op = O.Operator(om, Vq, wl.E, wl.z0)
    gm = fe.Mesh.from_workload(wl)
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    return op, gm


def _relerr(Y, R):
    return (np.linalg.norm(Y - R, axis=0) / np.maximum(np.linalg.norm(R, axis=0), 1e-300)).max()


CASES = [
    # (label, workload): Dirichlet / periodic axes (the table's Dirichlet and
    # wrap masks), segment colours, odd periodic axes (three colours), no z
    # segments, N with and without a rest past the last 32-vector group, and
    # p = 1, 2 and N < 32 (the kernel does not apply: the one-cell kernel)
    ("p4-D-z12-N40", W.small_slab((3, 3, 12), p=4, N=40)),
    ("p4-odd-periodic-x-N64", W.small_slab((3, 2, 12), p=4, N=64)),
    ("p4-periodic-z-3seg-N34", W.small_slab((2, 2, 18), p=4, N=34, bc=(W.PERIODIC,) * 3, E=0.0)),
    ("p4-periodic-odd-all-N96", W.small_slab((3, 5, 9), p=4, N=96, bc=(W.PERIODIC,) * 3, E=0.0)),
    ("p4-no-segments-z7-N32", W.small_slab((2, 3, 7), p=4, N=32)),
    ("p4-DPP-N48", W.small_slab((3, 2, 8), p=4, N=48, bc=(W.DIRICHLET, W.PERIODIC, W.PERIODIC), E=0.0)),
    ("p3-periodic-z-N52", W.small_slab((3, 3, 9), p=3, N=52, bc=(W.PERIODIC,) * 3, E=0.0)),
    ("p3-dirichlet-all-N32", W.small_slab((3, 4, 8), p=3, N=32, bc=(W.DIRICHLET,) * 3)),
    # x bricks (3 or 2 cells per brick, inner x faces in LDS): periodic x
    # with two bricks, three bricks (three colours), Dirichlet x with one and
    # two bricks
    ("p4-bricks3-periodic-x6-N64", W.small_slab((6, 2, 12), p=4, N=64)),
    ("p4-bricks3-3colour-x9-N32", W.small_slab((9, 2, 6), p=4, N=32, bc=(W.PERIODIC,) * 3, E=0.0)),
    ("p4-bricks2-periodic-x4-N48", W.small_slab((4, 3, 8), p=4, N=48)),
    ("p4-bricks2-dirichlet-x2-N32", W.small_slab((2, 3, 8), p=4, N=32, bc=(W.DIRICHLET, W.PERIODIC, W.DIRICHLET))),
    ("p3-bricks3-dirichlet-x6-N40", W.small_slab((6, 2, 6), p=3, N=40, bc=(W.DIRICHLET, W.PERIODIC, W.DIRICHLET))),
    # y bricks (2 cells along y, inner y faces in LDS): periodic y with two
    # bricks, x and y bricks together, three y bricks (three colours),
    # Dirichlet y with one brick
    ("p4-ybricks-periodic-y4-N32", W.small_slab((3, 4, 6), p=4, N=32)),
    ("p4-xybricks-6x4-N64", W.small_slab((6, 4, 6), p=4, N=64)),
    ("p4-ybricks-3colour-y6-N48", W.small_slab((4, 6, 4), p=4, N=48, bc=(W.PERIODIC,) * 3, E=0.0)),
    ("p4-ybricks-dirichlet-y2-N40", W.small_slab((3, 2, 6), p=4, N=40, bc=(W.DIRICHLET,) * 3)),
    ("p3-xybricks-6x4-N32", W.small_slab((6, 4, 6), p=3, N=32)),
    ("p2-dirichlet-all-N64", W.small_slab((3, 4, 8), p=2, N=64, bc=(W.DIRICHLET,) * 3)),
    ("p1-N2", W.small_slab((4, 3, 12), p=1, N=2)),
    ("p4-N20", W.small_slab((3, 2, 8), p=4, N=20)),
]


@pytest.mark.parametrize("label,wl", CASES, ids=[c[0] for c in CASES])
def test_dma_kernel_matches_oracle_and_is_reproducible(label, wl):
    print("case: dma", label, wl.ncell, wl.p, wl.N, flush=True)
    op, gm = _setup(wl)
    Xh = wl.X(op.n)
    X = torch.from_numpy(Xh).cuda()
    gm.set_kernel(10)
    try:
        H = gm.hx(X)
        assert torch.equal(gm.hx(X), H)
        assert _relerr(H.cpu().numpy(), op.apply(Xh)) < 1e-13
        a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
        a = O.weyl_cut(a0, b, wl.N, op.n)
        for a0s, m in ((a0, wl.m), (math.nan, 6)):
            Y = gm.cheb_filter(X, m, a, b, a0s)
            assert torch.equal(gm.cheb_filter(X, m, a, b, a0s), Y)
            assert _relerr(Y.cpu().numpy(), op.filter(Xh, m, a, b, a0s)) < 1e-12
        # and the one-cell kernel to rounding (another summation order)
        gm.set_kernel(1)
        H1 = gm.hx(X)
        rel = ((H - H1).norm(dim=0) / H1.norm(dim=0)).max().item()
        assert rel < 1e-13, rel
    finally:
        gm.set_kernel(0)


def test_dma_kernel_leading_dimension_and_padding_untouched():
    """Blocks inside wider buffers (even leading dimension N + 6, N = 40: one
    whole group and a rest of 8): columns past N are neither read into the
    product nor written.  The filter's work block has leading dimension N, so
    the steps that mix the two run the one-cell kernel."""
    wl = W.small_slab((3, 3, 12), p=4, N=40)
    op, gm = _setup(wl)
    Xh = wl.X(op.n)
    Xb = torch.full((op.n, wl.N + 6), float("nan"), dtype=torch.float64, device="cuda")
    Xb[:, :wl.N] = torch.from_numpy(Xh).cuda()
    Yb = torch.full_like(Xb, float("nan"))
    gm.set_kernel(10)
    try:
        a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
        a = O.weyl_cut(a0, b, wl.N, op.n)
        gm.cheb_filter(Xb[:, :wl.N], wl.m, a, b, a0, Y=Yb[:, :wl.N])
        assert _relerr(Yb[:, :wl.N].cpu().numpy(), op.filter(Xh, wl.m, a, b, a0)) < 1e-12
        assert torch.isnan(Yb[:, wl.N:]).all()
    finally:
        gm.set_kernel(0)


@pytest.mark.parametrize("why,wl,ld_extra", [
    ("N-below-32", W.small_slab((3, 3, 12), p=4, N=17), 0),
    ("neumann-axis", W.small_slab((3, 2, 10), p=4, N=32, bc=(W.PERIODIC, W.DIRICHLET, W.NEUMANN)), 0),
    ("odd-leading-dimension", W.small_slab((3, 3, 12), p=4, N=32), 1),
    ("p5", W.small_slab((2, 2, 3), p=5, N=32), 0),
])
def test_dma_kernel_falls_back_where_it_does_not_apply(why, wl, ld_extra):
    """Fewer than 32 vectors (no whole group), a Neumann axis (no folded
    cell matrix), an odd leading dimension (unaligned rows) and p > 4:
    variant 10 runs the one-cell kernel, bit for bit."""
    print("case: dma fallback", why, flush=True)
    op, gm = _setup(wl)
    Xb = torch.zeros((op.n, wl.N + ld_extra), dtype=torch.float64, device="cuda")
    Xb[:, :wl.N] = torch.from_numpy(wl.X(op.n)).cuda()
    X = Xb[:, :wl.N]
    Yb = torch.zeros_like(Xb)
    gm.set_kernel(1)
    Y1 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, Y=Yb[:, :wl.N]).clone()
    gm.set_kernel(10)
    try:
        Y10 = gm.cheb_filter(X, 5, 2.0, 400.0, -0.5, Y=Yb[:, :wl.N])
        assert torch.equal(Y10, Y1)
    finally:
        gm.set_kernel(0)


@pytest.mark.parametrize("p,N", [(4, 64), (3, 96)])
def test_dma_kernel_several_segments_per_workgroup(p, N):
    """24 x 24 x 24 cells: a workgroup walks several segments per colour
    pass, so the three LDS buffers rotate through position counts that are
    and are not multiples of three, and the two-ahead requests cross from
    one segment into the next.  Against the z-segment kernel (variant 9) and
    the one-cell kernel to rounding; reproducible."""
    import paper_2504_00998_amd as fe
    wl = W.small_slab((24, 24, 24), p=p, N=N)
    print("case: dma multi-item", p, N, flush=True)
    gm = fe.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, gm.quad_points())
    gm.set_potential(torch.from_numpy(Vq).cuda(), wl.E, wl.z0)
    g = torch.Generator(device="cuda")
    g.manual_seed(wl.seed(2))
    X = torch.randn(gm.n, N, generator=g, dtype=torch.float64, device="cuda")
    try:
        gm.set_kernel(1)
        Y1, F1 = gm.hx(X), gm.cheb_filter(X, 6, 2.0, 400.0, -0.5)
        gm.set_kernel(10)
        Y10, F10 = gm.hx(X), gm.cheb_filter(X, 6, 2.0, 400.0, -0.5)
        assert torch.equal(gm.hx(X), Y10)
        assert torch.equal(gm.cheb_filter(X, 6, 2.0, 400.0, -0.5), F10)
        for A, B in ((Y10, Y1), (F10, F1)):
            rel = ((A - B).norm(dim=0) / B.norm(dim=0)).max().item()
            assert rel < 1e-13, rel
    finally:
        gm.set_kernel(0)


# p = 5 (FP32 products only): 14 waves, 16 vectors per item;
# three colours along x and one-cell bricks, bricks of 2 and 3 cells, all
# axes periodic with a rest of 8 columns
P5_CASES = [
    ("p5-3colour-x3-N48", W.small_slab((3, 2, 6), p=5, N=48)),
    ("p5-bricks2-periodic-x4-N32", W.small_slab((4, 2, 4), p=5, N=32)),
    ("p5-bricks3-dirichlet-x3-N64", W.small_slab((3, 2, 5), p=5, N=64, bc=(W.DIRICHLET, W.PERIODIC, W.DIRICHLET))),
    ("p5-periodic-all-N40", W.small_slab((2, 3, 4), p=5, N=40, bc=(W.PERIODIC,) * 3, E=0.0)),
    ("p5-xybricks-4x4-N32", W.small_slab((4, 4, 4), p=5, N=32)),
    ("p5-ybricks-3colour-y6-N48", W.small_slab((2, 6, 3), p=5, N=48, bc=(W.DIRICHLET, W.PERIODIC, W.DIRICHLET))),
]
TAB_CASES = [c for c in CASES if c[1].p in (3, 4) and c[1].N >= 32]
F32_CASES = TAB_CASES + P5_CASES


@pytest.mark.parametrize("label,wl", F32_CASES, ids=[c[0] for c in F32_CASES])
def test_dma_kernel_f32_products(label, wl):
    """FP32 cell products (the folded matrix rounded to FP32, X rounded to
    FP32 as it leaves LDS, FP32 accumulation; the epilogue in FP64) on every
    mesh form the table applies to (and p = 5): H~X and the filter against
    the FP64 oracle within the FP32 bound of the other FP32 kernels, the
    FP32 products of variant 9 (the z-segment kernel; at p = 5 the one-cell
    pipelined kernel) to the same order, and reproducible."""
    print("case: dma f32", label, wl.ncell, wl.p, wl.N, flush=True)
    op, gm = _setup(wl)
    Xh = wl.X(op.n)
    X = torch.from_numpy(Xh).cuda()
    gm.set_kernel(10)
    try:
        H = gm.hx(X, prec="f32")
        assert torch.equal(gm.hx(X, prec="f32"), H)
        eh = _relerr(H.cpu().numpy(), op.apply(Xh))
        a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
        a = O.weyl_cut(a0, b, wl.N, op.n)
        Y = gm.cheb_filter(X, wl.m, a, b, a0, prec="f32")
        assert torch.equal(gm.cheb_filter(X, wl.m, a, b, a0, prec="f32"), Y)
        ef = _relerr(Y.cpu().numpy(), op.filter(Xh, wl.m, a, b, a0))
        gm.set_kernel(9)
        H9 = gm.hx(X, prec="f32")
        e9 = _relerr(H9.cpu().numpy(), op.apply(Xh))
        print(f"f32 rel err: table {eh:.2e} (z-segment {e9:.2e}), filter {ef:.2e}", flush=True)
        assert 0 < eh < 1e-6 and ef < 5e-6
        assert ((H - H9).norm(dim=0) / H9.norm(dim=0)).max().item() < 1e-6
    finally:
        gm.set_kernel(0)
