"""Pins of the CPU oracle against what the finite-element theory and the
mathematics fix (no GPU).  Each part of the oracle is checked by a route that
does not reuse its own code: closed forms, numpy library routines, exact
polynomial integration, separable spectra, dense eigendecompositions and
brute force.  References are to the paper's sections and equations.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2504_00998_amd import workloads as W
from tests import _fe_numpy as F

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mesh(L, ncell, p, bc, rule=0):
    return O.Mesh(L, ncell, p, bc, rule)


# ------------------------------------------------------------ 1-D GLL (Sec. 2.3)

def test_gll_matches_closed_forms():
    rows = [l.split() for l in open(os.path.join(GOLD, "gll_closed_forms.txt")) if l.strip() and not l.startswith("#")]
    for p in range(1, 5):
        ref = np.array([[float(a), float(b)] for q, a, b in rows if int(q) == p])
        xi, w = O.gll(p)
        np.testing.assert_allclose(xi, ref[:, 0], atol=2e-16)
        np.testing.assert_allclose(w, ref[:, 1], rtol=2e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_nodes_are_legendre_derivative_roots(p):
    xi, w = O.gll(p)
    xr, wr = F.gll_numpy(p)
    np.testing.assert_allclose(xi, xr, atol=1e-14)
    np.testing.assert_allclose(w, wr, rtol=1e-12)
    assert abs(w.sum() - 2.0) < 1e-14
    # exact for x^k, k <= 2p-1; the closed-form integral over [-1,1] is 2/(k+1) for even k
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * xi ** k).sum() - exact) < 1e-13
    # and not exact at k = 2p (the defining property of the Lobatto rule)
    k = 2 * p
    assert abs((w * xi ** k).sum() - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("q", [1, 2, 5, 8, 10])
def test_gauss_matches_numpy_leggauss(q):
    x, w = O.gauss(q)
    xr, wr = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(x, xr, atol=1e-14)
    np.testing.assert_allclose(w, wr, rtol=1e-13)


@pytest.mark.parametrize("p", [1, 3, 4, 6])
def test_lagrange_interpolates_and_differentiates(p):
    xi, _ = O.gll(p)
    ls = F.lagrange_polys(F.gll_numpy(p)[0])
    for x in [-1.0, -0.37, 0.0, 0.81, 1.0]:
        l, dl = O.lagrange(p, x)
        np.testing.assert_allclose(l, [P(x) for P in ls], atol=1e-13)
        np.testing.assert_allclose(dl, [P.deriv()(x) for P in ls], atol=1e-11)
        # reproduces x^k and its derivative for k <= p
        for k in range(p + 1):
            assert abs((l * xi ** k).sum() - x ** k) < 1e-13
            assert abs((dl * xi ** k).sum() - (k * x ** (k - 1) if k else 0.0)) < 1e-11
    for j in range(p + 1):
        l, _ = O.lagrange(p, xi[j])
        np.testing.assert_allclose(l, np.eye(p + 1)[j], atol=1e-14)


# ------------------------------------------------------- cell stiffness (Sec. 2.3)

@pytest.mark.parametrize("p,rule", [(1, 0), (2, 0), (3, 0), (4, 0), (4, 1), (5, 0), (3, 1)])
def test_cell_stiffness_equals_kronecker_sum_of_exact_1d_integrals(p, rule):
    h = 0.7
    Kc = O.cell_stiffness(p, rule, h)
    ref = F.cell_stiffness_kron(p, rule, h)
    np.testing.assert_allclose(Kc, ref, atol=1e-13 * np.abs(ref).max())
    assert np.array_equal(Kc, Kc.T) or np.abs(Kc - Kc.T).max() < 1e-15 * np.abs(Kc).max()
    np.testing.assert_allclose(Kc.sum(axis=1), 0.0, atol=1e-12 * np.abs(Kc).max())


def test_cell_stiffness_energy_of_polynomial():
    """u^T Kc u = int_cell |grad u|^2 for u = x^2 y + z on [0,h]^3 (closed form)."""
    p, h = 3, 1.3
    xi, _ = O.gll(p)
    n1 = p + 1
    Kc = O.cell_stiffness(p, 0, h)
    xs = 0.5 * h * (xi + 1.0)
    u = np.array([xs[l % n1] ** 2 * xs[(l // n1) % n1] + xs[l // n1 ** 2] for l in range(n1 ** 3)])
    # |grad u|^2 = (2xy)^2 + (x^2)^2 + 1 integrated over the cube
    exact = 4 * (h ** 3 / 3) * (h ** 3 / 3) * h + (h ** 5 / 5) * h * h + h ** 3
    assert abs(u @ Kc @ u - exact) < 1e-12 * exact


# ------------------------------------------------------ mesh maps & mass (Sec. 2.3)

def test_free_dof_counts_match_configs():
    assert O.Mesh.from_workload(W.CFG1).n == 1331
    assert W.CFG2.n_free() == 1_760_256
    assert W.CFG4.n_free() == 1_760_256
    assert W.CFG5.n_free() == 15_960_000
    m = _mesh((2, 2, 2), (2, 2, 2), 3, (2, 2, 2))
    assert m.n == 7 ** 3


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (2, 2, 2), (1, 1, 2)])
def test_mass_sums_to_volume_and_is_separable(bc):
    L, nc, p = (3.0, 3.0, 4.0), (3, 3, 4), 3
    m = _mesh(L, nc, p, bc)
    M = m.mass()
    # sum over free nodes = volume minus the mass of Dirichlet nodes (1-D products)
    oneD = [F.global_1d(nc[a], p, L[a] / nc[a], bc[a], 0) for a in range(3)]
    Mref = np.kron(oneD[2][2], np.kron(oneD[1][2], oneD[0][2]))
    np.testing.assert_allclose(M, Mref, rtol=1e-14)
    if all(b != 0 for b in bc):
        assert abs(M.sum() - np.prod(L)) < 1e-12


def test_cell_dof_map_consistency():
    m = _mesh((3, 2, 4), (3, 2, 4), 2, (1, 1, 0))
    cd = m.cell_dofs()
    qp = m.quad_points()
    xyz = m.dof_coords()
    free = cd >= 0
    # every free DoF appears, and the coordinates of a cell's point and its DoF agree modulo the period
    assert set(cd[free].tolist()) == set(range(m.n))
    d = qp[free] - xyz[cd[free]]
    d[:, 0] -= 3.0 * np.round(d[:, 0] / 3.0)
    d[:, 1] -= 2.0 * np.round(d[:, 1] / 2.0)
    assert np.abs(d).max() < 1e-13
    # Dirichlet points lie on the z faces
    z = qp[~free][:, 2]
    assert np.all((np.abs(z) < 1e-14) | (np.abs(z - 4.0) < 1e-14))


# ----------------------------------------------------- assembled K (Sec. 2.3)

def _K(m):
    return O.stiffness(m)


@pytest.mark.parametrize("bc", [(2, 2, 2), (1, 1, 2)])
@pytest.mark.parametrize("rule", [0, 1])
def test_K_symmetric_with_constants_in_null_space(bc, rule):
    """Zero-Neumann (and periodic-xy + Neumann-z, the CEF electrostatics
    setting of Sec. 2.2.1, Eq. governing_equations CEF): K 1 = 0."""
    m = _mesh((3.0, 3.0, 6.0), (3, 3, 6), 3, bc, rule)
    K = _K(m)
    assert (K - K.T).count_nonzero() == 0 or abs(K - K.T).max() == 0.0
    r = K @ np.ones(m.n)
    assert np.abs(r).max() < 1e-12 * abs(K).max()


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("p", [2, 3, 4])
def test_K_reproduces_laplacian_of_degree_p_polynomials(rule, p):
    """(K u)_I = M_I (-lap u)(x_I) + face terms, exactly, for total degree <= p
    (all-Neumann box; GLL quadrature is exact for the integrands)."""
    L, nc = (2.0, 3.0, 2.0), (2, 3, 2)
    m = _mesh(L, nc, p, (2, 2, 2), rule)
    K = _K(m)
    M = m.mass()
    X = m.dof_coords()
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    rng = np.random.default_rng(7)
    # a random polynomial of total degree p
    terms = [(a, b, c) for a in range(p + 1) for b in range(p + 1) for c in range(p + 1) if a + b + c <= p]
    coef = rng.standard_normal(len(terms))
    u = sum(cf * x ** a * y ** b * z ** c for cf, (a, b, c) in zip(coef, terms))
    lap = sum(cf * (a * (a - 1) * x ** max(a - 2, 0) * y ** b * z ** c
                    + b * (b - 1) * x ** a * y ** max(b - 2, 0) * z ** c
                    + c * (c - 1) * x ** a * y ** b * z ** max(c - 2, 0)) for cf, (a, b, c) in zip(coef, terms))
    grad = [sum(cf * a * x ** max(a - 1, 0) * y ** b * z ** c for cf, (a, b, c) in zip(coef, terms)),
            sum(cf * b * x ** a * y ** max(b - 1, 0) * z ** c for cf, (a, b, c) in zip(coef, terms)),
            sum(cf * c * x ** a * y ** b * z ** max(c - 1, 0) for cf, (a, b, c) in zip(coef, terms))]
    # face weights: lumped mass of the face (product of the other two axes' 1-D lumped masses)
    oneD = [F.global_1d(nc[a], p, L[a] / nc[a], 2, rule) for a in range(3)]
    lm = [o[2] for o in oneD]
    cz = [o[3] for o in oneD]
    face = np.zeros(m.n)
    for a in range(3):
        others = [b for b in range(3) if b != a]
        # weight of node I on the face normal to axis a = product of the other axes' 1-D lumped masses
        w3 = [np.ones_like(lm[b]) if b == a else lm[b] for b in range(3)]
        wf = np.kron(w3[2], np.kron(w3[1], w3[0]))
        coord = X[:, a]
        lo = np.abs(coord - 0.0) < 1e-12
        hi = np.abs(coord - L[a]) < 1e-12
        face += np.where(hi, wf * grad[a], 0.0) - np.where(lo, wf * grad[a], 0.0)
    expected = -M * lap + face
    got = K @ u
    assert np.abs(got - expected).max() < 1e-10 * max(1.0, np.abs(expected).max())


def test_linear_bias_is_laplace_exact():
    """u = -E (z - z0): K u vanishes off the z faces and equals the outward
    flux -/+E times the face mass on them (the field of Sec. 2.2.1; also the
    FE solution of the CPD Laplace problem with linear Dirichlet data)."""
    L, nc, p, E, z0 = (3.0, 3.0, 6.0), (3, 3, 6), 4, 0.01, 3.0
    m = _mesh(L, nc, p, (1, 1, 2))
    K = _K(m)
    X = m.dof_coords()
    u = -E * (X[:, 2] - z0)
    r = K @ u
    lm = [F.global_1d(nc[a], p, L[a] / nc[a], (1, 1, 2)[a], 0)[2] for a in range(3)]
    wf = np.kron(np.ones_like(lm[2]), np.kron(lm[1], lm[0]))
    top = np.abs(X[:, 2] - L[2]) < 1e-12
    bot = np.abs(X[:, 2]) < 1e-12
    expected = np.where(top, -E * wf, 0.0) + np.where(bot, E * wf, 0.0)
    assert np.abs(r - expected).max() < 1e-14 * 1e3


# -------------------------------------------------- spectra (Sec. 2.1, Sec. 2.3)

def _Hdense(op):
    return op.A.to_scipy().toarray()


def test_separable_spectrum_gll_rule_with_field():
    """gll rule, V = V_ext(z) only: H~ is a Kronecker sum of 1-D operators, so
    its spectrum is {1/2 mu_x + 1/2 mu_y + (1/2 mu_z + field)} exactly."""
    L, nc, p, bc, E, z0 = (3.0, 3.0, 5.0), (3, 3, 5), 3, (1, 1, 0), 0.01, 2.5
    m = _mesh(L, nc, p, bc, rule=1)
    op = O.Operator(m, None, E, z0)
    H = _Hdense(op)
    assert np.abs(H - H.T).max() < 1e-14 * np.abs(H).max()
    lam = np.linalg.eigvalsh(H)
    fac = []
    for a in range(3):
        Kg, _, Lg, xc = F.global_1d(nc[a], p, L[a] / nc[a], bc[a], 1)
        D = 1.0 / np.sqrt(Lg)
        A = 0.5 * D[:, None] * Kg * D[None, :]
        if a == 2:
            A = A + np.diag(-E * (xc - z0))
        fac.append(np.linalg.eigvalsh(A))
    ref = np.sort((fac[0][:, None, None] + fac[1][None, :, None] + fac[2][None, None, :]).ravel())
    np.testing.assert_allclose(lam, ref, atol=1e-12 * np.abs(ref).max())


def test_particle_in_box_levels_and_convergence():
    """V = 0 Dirichlet cube: discrete levels approach pi^2/(2L^2)(n1^2+n2^2+n3^2)
    with error falling ~ h^(2p) under refinement.  (With the lumped GLL mass
    the discrete levels are not upper bounds, so only |error| is checked.)"""
    line = [l.split() for l in open(os.path.join(GOLD, "particle_in_box.txt")) if l.strip() and not l.startswith("#")][0]
    L = float(line[0]); sums = np.array([float(s) for s in line[1:]])
    exact = np.pi ** 2 / (2 * L * L) * sums
    errs = []
    for ncell in (2, 4):
        m = _mesh((L, L, L), (ncell,) * 3, 3, (0, 0, 0))
        lam = np.linalg.eigvalsh(_Hdense(O.Operator(m, None, 0.0, 0.0)))[:10]
        errs.append(np.abs(lam - exact))
    rate = np.log2(errs[0][0] / errs[1][0])
    assert rate > 5.0  # 2p = 6
    assert errs[1][:4].max() < 2e-4 and errs[1][0] < 5e-6


def test_cfg1_dense_symmetric_and_lanczos_bound():
    wl = W.CFG1
    m = O.Mesh.from_workload(wl)
    Vq = W.wells_potential(m.quad_points(), wl.centres(), wl.depth, wl.sigma, wl.L, [b == 1 for b in wl.bc])
    op = O.Operator(m, Vq, wl.E, wl.z0)
    H = _Hdense(op)
    assert np.abs(H - H.T).max() == 0.0
    lam = np.linalg.eigvalsh(H)
    a0, b, theta = O.lanczos_bounds(op.apply, wl.lanczos_start(m.n), 10)
    assert b >= lam[-1]
    assert a0 >= lam[0] - 1e-12
    # Lanczos Ritz values interlace the spectrum
    assert theta[0] >= lam[0] - 1e-12 and theta[-1] <= lam[-1] + 1e-12
    # a 1331-step run is exact
    a0e, be, th = O.lanczos_bounds(lambda v: H @ v, wl.lanczos_start(m.n), 60)
    assert abs(a0e - lam[0]) < 1e-8


def test_potential_diagonal_equals_nodal_value():
    """With GLL-collocated quadrature the potential part of H~ is diagonal and
    v_I is the mass-weighted mean of V over the cells sharing I; for a
    continuous V this is V(x_I) - E (z_I - z0)."""
    wl = W.small_slab((2, 2, 3), p=3)
    m = O.Mesh.from_workload(wl)
    qp = m.quad_points()
    Vq = W.wells_potential(qp, wl.centres(), wl.depth, wl.sigma, wl.L, [b == 1 for b in wl.bc])
    H1 = O.Operator(m, Vq, wl.E, wl.z0).A.to_scipy()
    H0 = O.Operator(m, None, 0.0, wl.z0).A.to_scipy()
    dv = (H1 - H0)
    off = dv - sp.diags(dv.diagonal())
    assert abs(off).max() < 1e-15
    X = m.dof_coords()
    v = W.wells_potential(X, wl.centres(), wl.depth, wl.sigma, wl.L, [b == 1 for b in wl.bc]) - wl.E * (X[:, 2] - wl.z0)
    np.testing.assert_allclose(dv.diagonal(), v, atol=1e-13)


# -------------------------------------------------------- filter (CheFSI)

@pytest.fixture(scope="module")
def cfg1_op():
    wl = W.CFG1
    m = O.Mesh.from_workload(wl)
    Vq = W.wells_potential(m.quad_points(), wl.centres(), wl.depth, wl.sigma, wl.L, [b == 1 for b in wl.bc])
    op = O.Operator(m, Vq, wl.E, wl.z0)
    H = _Hdense(op)
    lam, Q = np.linalg.eigh(H)
    return wl, m, op, H, lam, Q


@pytest.mark.parametrize("scaled", [True, False])
@pytest.mark.parametrize("mdeg", [1, 2, 7, 20])
def test_filter_equals_spectral_closed_form(cfg1_op, scaled, mdeg):
    """Y = Q diag(tau(lambda)) Q^T X, tau = T_m(t(lambda)) / T_m(t0) (scaled) or
    T_m(t(lambda)) (unscaled); T_m from its cos/cosh closed forms."""
    wl, m, op, H, lam, Q = cfg1_op
    X = wl.X(m.n)
    a0 = -0.6 if scaled else float("nan")
    a, b = 0.4, 21.0
    Y = op.filter(X, mdeg, a, b, a0)
    e, c = 0.5 * (b - a), 0.5 * (b + a)
    tau = O.chebyshev_T(mdeg, (lam - c) / e)
    if scaled:
        tau = tau / O.chebyshev_T(mdeg, np.array([(a0 - c) / e]))[0]
    ref = Q @ (tau[:, None] * (Q.T @ X))
    err = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() < 1e-11


def test_filter_degree_one_and_scaling_relation(cfg1_op):
    wl, m, op, H, lam, Q = cfg1_op
    X = wl.X(m.n)
    a, b, a0 = 0.4, 21.0, -0.6
    e, c = 0.5 * (b - a), 0.5 * (b + a)
    s1 = e / (a0 - c)
    Y1 = op.filter(X, 1, a, b, a0)
    np.testing.assert_allclose(Y1, (s1 / e) * (H @ X - c * X), rtol=1e-13, atol=1e-13 * np.abs(Y1).max())
    Ys = op.filter(X, 20, a, b, a0)
    Yu = op.filter(X, 20, a, b, float("nan"))
    t0 = (a0 - c) / e
    np.testing.assert_allclose(Yu / O.chebyshev_T(20, np.array([t0]))[0], Ys, rtol=1e-10, atol=1e-12 * np.abs(Ys).max())


def test_filter_on_eigenvectors_separable_large():
    """gll rule + field only: eigenvectors of the 1-D factors give exact
    eigenvectors of H~, and the filter multiplies each by tau(lambda)."""
    L, nc, p, bc, E, z0 = (4.0, 4.0, 6.0), (4, 4, 6), 4, (1, 1, 0), 0.005, 3.0
    m = _mesh(L, nc, p, bc, rule=1)
    op = O.Operator(m, None, E, z0)
    vecs, vals = [], []
    f = []
    for a in range(3):
        Kg, _, Lg, xc = F.global_1d(nc[a], p, L[a] / nc[a], bc[a], 1)
        D = 1.0 / np.sqrt(Lg)
        A = 0.5 * D[:, None] * Kg * D[None, :]
        if a == 2:
            A = A + np.diag(-E * (xc - z0))
        f.append(np.linalg.eigh(A))
    for (i, j, k) in [(0, 0, 0), (1, 0, 0), (2, 3, 1), (5, 1, 7)]:
        q = np.kron(f[2][1][:, k], np.kron(f[1][1][:, j], f[0][1][:, i]))
        vecs.append(q); vals.append(f[0][0][i] + f[1][0][j] + f[2][0][k])
    Xq = np.stack(vecs, axis=1)
    lam = np.array(vals)
    np.testing.assert_allclose(op.apply(Xq), Xq * lam, atol=1e-11)
    a, b, a0 = 1.0, 280.0, 0.1  # b above lambda_max = 274.6
    Y = op.filter(Xq, 9, a, b, a0)
    e, c = 0.5 * (b - a), 0.5 * (b + a)
    tau = O.chebyshev_T(9, (lam - c) / e) / O.chebyshev_T(9, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Y, Xq * tau, atol=1e-12 * np.abs(tau).max())


# ------------------------------------------------- CholQR2 and Rayleigh-Ritz

def test_cholqr2_and_rayleigh_ritz_on_invariant_subspace(cfg1_op):
    wl, m, op, H, lam, Q = cfg1_op
    rng = np.random.default_rng(3)
    # a basis of the lowest 8 eigenvectors mixed by a random well-conditioned matrix
    B = Q[:, :8] @ (np.eye(8) + 0.3 * rng.standard_normal((8, 8)))
    Qc, R = O.cholqr2(B)
    assert np.abs(Qc.T @ Qc - np.eye(8)).max() < 1e-13
    np.testing.assert_allclose(Qc @ R, B, atol=1e-13)
    theta, Xr = O.rayleigh_ritz(op.apply, Qc)
    np.testing.assert_allclose(theta, lam[:8], atol=1e-12)


def test_subspace_iteration_converges_to_lowest_levels(cfg1_op):
    wl, m, op, H, lam, Q = cfg1_op
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(m.n), 10)
    a = O.weyl_cut(a0, b, wl.N, m.n)
    hist, _ = O.subspace_iteration(op, wl.X(m.n), wl.m, 5, a, b, a0)
    err = np.abs(hist[-1][:11] - lam[:11])
    assert err.max() < 1e-7


# ----------------------------------------------------------- the adjoint

def _loss(op, X, w, m, a, b, a0):
    Y = op.filter(X, m, a, b, a0)
    return float(np.sum(w * np.sum(X * Y, axis=0))), Y


def test_vjp_closed_form_dX(cfg1_op):
    """L = sum_i w_i <x_i, T(H) x_i> is quadratic with a symmetric kernel, so
    dL/dX = 2 Y W."""
    wl, m, op, H, lam, Q = cfg1_op
    X = wl.X(m.n); w = wl.weights()
    a, b, a0 = 0.4, 21.0, -0.6
    L0, Y = _loss(op, X, w, 20, a, b, a0)
    Xb, g = op.filter_vjp(X, X * w, 20, a, b, a0)
    np.testing.assert_allclose(Xb + Y * w, 2 * Y * w, rtol=1e-10, atol=1e-12 * np.abs(Y).max())


def test_vjp_daleckii_krein_diagonal(cfg1_op):
    """g_I = [dL/dH~]_II with dL/dH~ = Q (Gamma o (Q^T G X^T Q)) Q^T (symmetrised),
    Gamma_ij = divided differences of tau (Daleckii-Krein)."""
    wl, m, op, H, lam, Q = cfg1_op
    X = wl.X(m.n)[:, :4]
    w = wl.weights()[:4]
    a, b, a0, mdeg = 0.4, 21.0, -0.6, 9
    e, c = 0.5 * (b - a), 0.5 * (b + a)
    T0 = O.chebyshev_T(mdeg, np.array([(a0 - c) / e]))[0]
    tau = O.chebyshev_T(mdeg, (lam - c) / e) / T0
    # tau' from T_m' = m U_{m-1}; use a centred difference of the closed form in extended precision instead
    hstep = 1e-6
    dtau = (O.chebyshev_T(mdeg, (lam + hstep - c) / e) - O.chebyshev_T(mdeg, (lam - hstep - c) / e)) / (2 * hstep) / T0
    Gm = X * w
    diff = lam[:, None] - lam[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        Gam = (tau[:, None] - tau[None, :]) / diff
    close = np.abs(diff) < 1e-9
    Gam[close] = 0.5 * (dtau[:, None] + dtau[None, :])[close]
    S = Q.T @ Gm @ X.T @ Q
    dH = Q @ (Gam * S) @ Q.T
    Xb, g = op.filter_vjp(X, Gm, mdeg, a, b, a0)
    np.testing.assert_allclose(g, np.diag(dH), atol=1e-7 * np.abs(np.diag(dH)).max())


def test_vjp_finite_differences_in_V_and_E(cfg1_op):
    """Central differences of L in V (at the quadrature points) and in E
    (Sec. 2.2.1: V_app enters V_eff linearly) against the chain rule."""
    wl, m, op, H, lam, Q = cfg1_op
    X = wl.X(m.n)[:, :6]; w = wl.weights()[:6]
    a, b, a0, mdeg = 0.4, 21.0, -0.6, 8
    Vq = W.wells_potential(m.quad_points(), wl.centres(), wl.depth, wl.sigma, wl.L, [False] * 3)
    Xb, g = op.filter_vjp(X, X * w, mdeg, a, b, a0)
    Vb, Eb = op.potential_vjp(g)
    rng = np.random.default_rng(11)
    for t in range(3):
        dV = rng.standard_normal(Vq.shape)
        dE = rng.standard_normal()
        hs = 1e-6
        Lp, _ = _loss(O.Operator(m, Vq + hs * dV, wl.E + hs * dE, wl.z0), X, w, mdeg, a, b, a0)
        Lm, _ = _loss(O.Operator(m, Vq - hs * dV, wl.E - hs * dE, wl.z0), X, w, mdeg, a, b, a0)
        fd = (Lp - Lm) / (2 * hs)
        an = float((Vb * dV).sum() + Eb * dE)
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an))
    # chain rule identity: Ebar = -sum Vbar (z_q - z0) over the quadrature points
    zq = m.quad_points()[..., 2]
    assert abs(Eb - (-(Vb * (zq - wl.z0)).sum())) < 1e-10 * max(1.0, abs(Eb))


def test_vjp_hellmann_feynman_on_eigenvectors():
    """x_i = q_i exact eigenvectors: g_I = sum_i w_i tau'(lambda_i) q_i,I^2, and
    dL/dE = -sum_i w_i tau'(lambda_i) <q_i, (z - z0) q_i>."""
    L, nc, p, bc, E, z0 = (3.0, 3.0, 5.0), (3, 3, 5), 3, (1, 1, 0), 0.01, 2.5
    m = _mesh(L, nc, p, bc, rule=1)
    op = O.Operator(m, None, E, z0)
    H = _Hdense(op)
    lam, Q = np.linalg.eigh(H)
    idx = [0, 3, 10]
    Xq = Q[:, idx]; w = np.array([0.3, 0.9, 0.5])
    a, b, a0, mdeg = 2.0, 60.0, 0.3, 7
    e, c = 0.5 * (b - a), 0.5 * (b + a)
    T0 = O.chebyshev_T(mdeg, np.array([(a0 - c) / e]))[0]
    l = lam[idx]
    hstep = 1e-5
    dtau = (O.chebyshev_T(mdeg, (l + hstep - c) / e) - O.chebyshev_T(mdeg, (l - hstep - c) / e)) / (2 * hstep) / T0
    Xb, g = op.filter_vjp(Xq, Xq * w, mdeg, a, b, a0)
    ref = (Xq ** 2 * (w * dtau)).sum(axis=1)
    np.testing.assert_allclose(g, ref, atol=1e-8 * np.abs(ref).max())
    _, Eb = op.potential_vjp(g)
    zz = m.dof_coords()[:, 2] - z0
    Eref = -sum(w[t] * dtau[t] * (Xq[:, t] ** 2 * zz).sum() for t in range(3))
    assert abs(Eb - Eref) < 1e-8 * abs(Eref)


# -------------------------------------------------------- nonlocal (Eq. V_nloc)

def test_nonlocal_term_symmetric_and_reduces():
    wl = W.small_slab((3, 3, 4), p=3, cfg=5)
    m = O.Mesh.from_workload(wl)
    cen = wl.centres()
    P = O.Projectors(m, cen, wl.r_cut, wl.r_g)
    Cm = P.to_scipy()
    M = m.mass()
    # unit discrete M-norm: sum_I M_I p(x_I)^2 = 1, and C~ = M^1/2 p
    np.testing.assert_allclose(np.asarray(Cm.multiply(Cm).sum(axis=0)).ravel(), 1.0, rtol=1e-13)
    D = np.random.default_rng(5).uniform(-1, 1, P.nproj)
    Vq = W.wells_potential(m.quad_points(), cen, wl.depth, wl.sigma, wl.L, [b == 1 for b in wl.bc])
    opl = O.Operator(m, Vq, wl.E, wl.z0)
    opn = O.Operator(m, Vq, wl.E, wl.z0, P, D)
    op0 = O.Operator(m, Vq, wl.E, wl.z0, P, np.zeros(P.nproj))
    X = wl.X(m.n, cols=range(5))
    np.testing.assert_allclose(op0.apply(X), opl.apply(X), rtol=0, atol=0)
    Hn = opn.apply(np.eye(m.n))
    assert np.abs(Hn - Hn.T).max() < 1e-13 * np.abs(Hn).max()
    ref = opl.apply(X) + Cm @ (D[:, None] * (Cm.T @ X))
    np.testing.assert_allclose(opn.apply(X), ref, atol=1e-13 * np.abs(ref).max())
    # s-projector values follow the Gaussian radial form at the DoFs
    xyz = m.dof_coords()
    col = Cm[:, 0].toarray().ravel()
    d = xyz - cen[0]
    for a in range(2):
        d[:, a] -= wl.L[a] * np.round(d[:, a] / wl.L[a])
    r2 = (d ** 2).sum(axis=1)
    raw = np.where(r2 < wl.r_cut ** 2, np.exp(-r2 / (2 * wl.r_g ** 2)), 0.0)
    raw = raw / np.sqrt((M * raw ** 2).sum()) * np.sqrt(M)
    np.testing.assert_allclose(col, raw, atol=1e-14)


def _real_solid_harmonic(l, mm, d):
    """r^l times the real spherical harmonic of degree l and order mm at the
    displacements d (k, 3), from scipy's complex Y_l^m (polar angle theta,
    azimuth phi): Y_l^0; sqrt(2) (-1)^m Re Y_l^m for m > 0; sqrt(2) (-1)^m
    Im Y_l^|m| for m < 0.  An independent route to the angular factors (no
    Cartesian polynomial is written out)."""
    from scipy.special import sph_harm_y
    r = np.sqrt((d ** 2).sum(axis=1))
    theta = np.arccos(np.clip(d[:, 2] / np.where(r > 0, r, 1.0), -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = sph_harm_y(l, abs(mm), theta, phi)
    if mm == 0:
        re = Y.real
    elif mm > 0:
        re = np.sqrt(2.0) * (-1) ** mm * Y.real
    else:
        re = np.sqrt(2.0) * (-1) ** mm * Y.imag
    return r ** l * re


# projector beta -> (l, m) of the real harmonic: s; p_x, p_y, p_z; d_xy, d_yz,
# d_zx, d_{x^2-y^2}, d_{3z^2-r^2} (the order the projector columns take)
_BETA_LM = [(0, 0), (1, 1), (1, -1), (1, 0), (2, -2), (2, -1), (2, 1), (2, 2), (2, 0)]


def test_projector_angular_factors_are_real_solid_harmonics():
    """Pin of all nine projector shapes (Sec. 2.1, Eq. V_nloc; s, p and d
    channels): column (s, beta) of C~ equals M^1/2 p with p = r^l Y_lm(x - R)
    exp(-r^2 / 2 r_g^2) [r < r_cut], the real harmonic taken from scipy,
    normalised to unit discrete M-norm -- up to the sign convention of the
    harmonic, which the normalisation leaves free.  The sites sit at generic
    points, one of them with a ball wrapping through the periodic x face, so
    no two channels coincide on the node set and a permuted or mistyped
    channel (yz for zx, z^2 - r^2 for 3z^2 - r^2) misses by O(1)."""
    m = _mesh((6.0, 5.0, 7.0), (6, 5, 7), 3, (1, 1, 0))
    cen = np.array([[2.37, 2.61, 3.43], [0.31, 4.12, 3.77]])
    P = O.Projectors(m, cen, 2.0, 0.5)
    Cm = P.to_scipy().toarray()
    M = m.mass()
    xyz = m.dof_coords()
    for s in range(cen.shape[0]):
        d = xyz - cen[s]
        for a in range(2):
            d[:, a] -= m.L[a] * np.round(d[:, a] / m.L[a])
        r2 = (d ** 2).sum(axis=1)
        inside = r2 < 4.0
        rad = np.exp(-r2 / (2 * 0.5 ** 2))
        for beta, (l, mm) in enumerate(_BETA_LM):
            ref = np.where(inside, _real_solid_harmonic(l, mm, d) * rad, 0.0)
            ref = ref / np.sqrt((M * ref ** 2).sum()) * np.sqrt(M)
            col = Cm[:, 9 * s + beta]
            sign = np.sign(col @ ref)
            assert sign != 0
            err = np.abs(col - sign * ref).max()
            assert err < 1e-12, (s, beta, err)
            # and it is far from every other channel's shape
            for b2, (l2, m2) in enumerate(_BETA_LM):
                if b2 == beta:
                    continue
                o = np.where(inside, _real_solid_harmonic(l2, m2, d) * rad, 0.0)
                o = o / np.sqrt((M * o ** 2).sum()) * np.sqrt(M)
                assert min(np.abs(col - o).max(), np.abs(col + o).max()) > 1e-2, (s, beta, b2)


def test_projector_gram_is_diagonal_at_a_cubic_site():
    """At a site on a mesh node whose neighbourhood has the full symmetry of
    the cube (interior cell corner, cubic cells, GLL nodes symmetric in each
    cell), the discrete Gram C~^T C~ = sum_I M_I p_a p_b of one site is the
    identity: the nine real harmonics lie in different rows of the cube
    group's representations (A1g; T1u; T2g; Eg), so every cross term sums to
    zero over the symmetric node set, and the diagonal is 1 by the
    normalisation.  A duplicated or mixed channel breaks the zeros."""
    m = _mesh((8.0, 8.0, 8.0), (4, 4, 4), 4, (0, 0, 0))
    cen = np.array([[4.0, 4.0, 4.0]])
    Cm = O.Projectors(m, cen, 2.0, 0.5).to_scipy().toarray()
    G = Cm.T @ Cm
    np.testing.assert_allclose(G, np.eye(9), atol=1e-13)


def test_separable_wells_equal_pointwise_sum():
    """The tensor-grid evaluation of the Gaussian wells equals the pointwise
    minimum-image sum (input recipe, both periodic and bounded axes)."""
    for wl in [W.CFG1, W.small_slab((3, 5, 3), p=4), W.small_slab((2, 3, 4), p=2, bc=(2, 1, 0))]:
        m = O.Mesh.from_workload(wl)
        qp = m.quad_points()
        V1 = W.wells_potential(qp, wl.centres(), wl.depth, wl.sigma, wl.L, [b == 1 for b in wl.bc])
        V2 = W.workload_potential(wl, qp)
        assert np.abs(V1 - V2).max() < 1e-13


def test_apply_rows_equals_assembled_operator():
    """Rows summed one by one from their cell contributions equal the same
    rows of the assembled CSR product (with and without the nonlocal term)."""
    wl = W.small_slab((5, 5, 6), p=3, N=6, cfg=5)
    m = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, m.quad_points())
    P = O.Projectors(m, wl.centres(), wl.r_cut, wl.r_g)
    D = wl.nonlocal_coupling().reshape(-1)
    X = wl.X(m.n)
    rows = np.random.default_rng(2).choice(m.n, size=40, replace=False)
    for proj in (None, P):
        op = O.Operator(m, Vq, wl.E, wl.z0, proj, D if proj is not None else None)
        full = op.apply(X)[rows]
        part = O.apply_rows(m, Vq, wl.E, wl.z0, rows, X, proj, D if proj is not None else None)
        np.testing.assert_allclose(part, full, rtol=1e-13, atol=1e-13 * np.abs(full).max())


# ------------------------------------------- density and planar averages (Sec. 2.1, Sec. 3.2)

def test_density_and_planar_integral_sum_rule():
    """int rho = sum_I M_I rho_I = 2 sum_n f_n |x_n|^2 for any block, and the
    planar integrals integrate along z to the same total."""
    m = _mesh((3.0, 3.0, 4.0), (3, 3, 4), 3, (1, 1, 0))
    rng = np.random.default_rng(7)
    X = rng.standard_normal((m.n, 9))
    f = rng.uniform(-0.5, 2.0, 9)
    rho = O.density(m, X, f)
    total = 2.0 * (f * (X * X).sum(axis=0)).sum()
    assert abs((m.mass() * rho).sum() - total) < 1e-12 * abs(total)
    zc, mz = O.axis_positions(m, 2)
    pl = O.planar_integral(m, rho)
    assert pl.shape == (11,)
    assert abs((mz * pl).sum() - total) < 1e-12 * abs(total)


@pytest.mark.parametrize("bcz", [0, 2])
def test_planar_integral_of_separable_orbital_closed_form(bcz):
    """psi = a(z) with periodic x, y: rho^0(z) = 2 f a(z)^2 L_x L_y exactly (the
    GLL weights of a periodic axis sum to its length)."""
    L = (2.5, 3.5, 5.0)
    m = _mesh(L, (2, 3, 4), 4, (1, 1, bcz))
    z = m.dof_coords()[:, 2]
    a = np.cos(0.7 * z) + 0.3 * z
    X = (np.sqrt(m.mass()) * a)[:, None]
    f = np.array([0.75])
    pl = O.planar_integral(m, O.density(m, X, f))
    zc, _ = O.axis_positions(m, 2)
    ref = 2.0 * 0.75 * (np.cos(0.7 * zc) + 0.3 * zc) ** 2 * L[0] * L[1]
    np.testing.assert_allclose(pl, ref, rtol=1e-13)


def test_planar_average_of_constant_and_linear_fields():
    """The average over a plane of a constant is the constant, of -E(z - z0)
    is -E(z_k - z0), on any x-y boundary conditions."""
    for bc in [(1, 1, 0), (0, 2, 2), (2, 0, 1)]:
        m = _mesh((2.0, 3.0, 4.0), (2, 3, 4), 3, bc)
        z = m.dof_coords()[:, 2]
        zc, _ = O.axis_positions(m, 2)
        np.testing.assert_allclose(O.planar_integral(m, np.full(m.n, 1.7), normalize=True), 1.7, rtol=1e-14)
        np.testing.assert_allclose(O.planar_integral(m, -0.01 * (z - 2.0), normalize=True), -0.01 * (zc - 2.0),
                                   rtol=1e-12, atol=1e-16)


def test_planar_integral_brute_force_p2():
    """p = 2 by hand: GLL weights (1/3, 4/3, 1/3) on [-1, 1], assembled masses
    on each axis written out, plane sums by explicit loops over node positions."""
    h = 1.5
    m = _mesh((3 * h, 2 * h, 2 * h), (3, 2, 2), 2, (1, 0, 2))
    w = np.array([1.0, 4.0, 1.0]) / 3.0

    def masses(nce, bc):
        mass = np.zeros(2 * nce + 1)
        for c in range(nce):
            for i in range(3):
                mass[2 * c + i] += 0.5 * h * w[i]
        if bc == 1:
            mass[0] += mass[-1]
            return mass[:-1]
        if bc == 0:
            return mass[1:-1]
        return mass

    mx, my, mz = masses(3, 1), masses(2, 0), masses(2, 2)
    rng = np.random.default_rng(3)
    F = rng.standard_normal(m.n)
    xyz = m.dof_coords()
    # node positions along each axis from the coordinates (h/2 spacing at p = 2)
    ix = np.rint(xyz[:, 0] / (0.5 * h)).astype(int)
    iy = np.rint(xyz[:, 1] / (0.5 * h)).astype(int) - 1  # Dirichlet: first free position is 1
    iz = np.rint(xyz[:, 2] / (0.5 * h)).astype(int)
    ref = np.zeros(len(mz))
    for I in range(m.n):
        ref[iz[I]] += mx[ix[I]] * my[iy[I]] * F[I]
    np.testing.assert_allclose(O.planar_integral(m, F), ref, rtol=1e-13, atol=1e-14)


def test_density_of_box_ground_state_matches_continuum():
    """Dirichlet cube, V = 0: the lowest orbital approaches (2/L)^{3/2} prod sin,
    so rho^0(z) -> (4/L) sin^2(pi z / L) for one doubly occupied orbital."""
    Lb = 4.0
    m = _mesh((Lb, Lb, Lb), (4, 4, 4), 4, (0, 0, 0))
    op = O.Operator(m, None, 0.0, 0.5 * Lb)
    import scipy.sparse.linalg as sla
    A = op.A.to_scipy() if hasattr(op.A, "to_scipy") else op.A
    vals, vecs = sla.eigsh(A, k=1, which="SA", tol=1e-12)
    x = vecs[:, :1]
    pl = O.planar_integral(m, O.density(m, x, np.array([1.0])))
    zc, _ = O.axis_positions(m, 2)
    ref = 4.0 / Lb * np.sin(np.pi * zc / Lb) ** 2
    assert np.abs(pl - ref).max() < 1e-5 * ref.max()  # discretisation error ~3e-6 at p = 4, h = 1


# ------------------------------------------------ electrostatics (Sec. 2.2)

def test_poisson_manufactured_periodic_neumann():
    """Periodic x, y and zero-Neumann z (the constant-field setup): phi =
    cos(2 pi z / L_z) (zero flux at both z faces, zero mean) from
    s = -lap(phi) / 4 pi; the FE solution matches at the nodes."""
    L = (3.0, 3.0, 8.0)
    m = _mesh(L, (3, 3, 8), 4, (1, 1, 2))
    z = m.dof_coords()[:, 2]
    k = 2 * np.pi / L[2]
    exact = np.cos(k * z)
    s = k * k * np.cos(k * z) / (4 * np.pi)
    phi = O.poisson(m, s)
    assert abs((m.mass() * phi).sum()) < 1e-10
    assert np.abs(phi - exact).max() < 2e-5


def test_poisson_manufactured_dirichlet_z_with_x_variation():
    L = (4.0, 2.0, 6.0)
    m = _mesh(L, (4, 2, 6), 4, (1, 1, 0))
    x, z = m.dof_coords()[:, 0], m.dof_coords()[:, 2]
    kx, kz = 2 * np.pi / L[0], np.pi / L[2]
    exact = np.sin(kz * z) * (1 + 0.3 * np.cos(kx * x))
    lap = -(kz ** 2) * exact - 0.3 * kx ** 2 * np.sin(kz * z) * np.cos(kx * x)
    phi = O.poisson(m, -lap / (4 * np.pi))
    assert np.abs(phi - exact).max() < 5e-5


def test_poisson_residual_mean_and_neutralisation():
    """The solve satisfies K phi = 4 pi M (s - mean) to rounding, phi has zero
    mean, and adding a constant to s changes nothing (neutral-slab reading)."""
    m = _mesh((3.0, 3.0, 4.0), (3, 3, 4), 3, (1, 1, 2))
    rng = np.random.default_rng(4)
    s = rng.standard_normal(m.n)
    phi = O.poisson(m, s)
    M = m.mass()
    s0 = s - (M @ s) / M.sum()
    K = O.stiffness(m)
    r = K @ phi - 4 * np.pi * M * s0
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(4 * np.pi * M * s0)
    assert abs(M @ phi) < 1e-10 * np.abs(phi).max()
    np.testing.assert_allclose(O.poisson(m, s + 2.5), phi, atol=1e-9 * np.abs(phi).max())


# --------------------------- constrained potential difference (Sec. 2.2.2)

def test_cpd_uniform_charge_gives_the_exact_quadratic():
    """Periodic x, y, conductors below z_lo and above z_hi on cell faces,
    uniform charge s0, w = 0: the continuum solution between them is
    phi = -2 pi s0 (z - z_lo)(z - z_hi) + dV (z - z_lo) / (z_hi - z_lo), a
    quadratic that the p = 2 and p = 4 spaces hold and that GLL quadrature
    of the uniform right-hand side integrates exactly, so the nodal values
    are exact; phi is 0 and dV inside the conductors (no field there)."""
    for p in (2, 4):
        L = (2.0, 3.0, 10.0)
        m = _mesh(L, (2, 3, 10), p, (1, 1, 2))
        z = m.dof_coords()[:, 2]
        z_lo, z_hi, s0, dV = 2.0, 7.0, 0.013, -0.4
        phi = O.poisson_cpd(m, np.full(m.n, s0), None, z_lo, z_hi, dV)
        exact = np.where(z <= z_lo, 0.0, np.where(z >= z_hi, dV,
                         -2 * np.pi * s0 * (z - z_lo) * (z - z_hi) + dV * (z - z_lo) / (z_hi - z_lo)))
        assert np.abs(phi - exact).max() < 1e-12, p
        reg = O.cpd_constrained(m, z_lo, z_hi)
        assert (phi[reg == 1] == 0.0).all() and (phi[reg == 2] == dV).all()


def test_cpd_conductor_data_enter_as_the_total_potential():
    """No charge, w = V_loc - V_sm varying in z and x inside the conductors:
    the constraint holds phi + w at 0 and dV there, and between the
    conductors phi is the linear interpolant of the two planes' values
    (w constant over each boundary plane)."""
    L = (3.0, 2.0, 9.0)
    m = _mesh(L, (3, 2, 9), 3, (1, 1, 2))
    xyz = m.dof_coords()
    x, z = xyz[:, 0], xyz[:, 2]
    z_lo, z_hi, dV = 3.0, 6.0, 0.25
    # w constant on the planes z = z_lo and z = z_hi, varying elsewhere
    w = 0.1 * np.cos(2 * np.pi * x / L[0]) * (z - z_lo) * (z - z_hi) + 0.05 + 0.02 * z
    phi = O.poisson_cpd(m, np.zeros(m.n), w, z_lo, z_hi, dV)
    reg = O.cpd_constrained(m, z_lo, z_hi)
    assert np.abs((phi + w)[reg == 1]).max() < 1e-15
    assert np.abs((phi + w)[reg == 2] - dV).max() < 1e-15
    glo, ghi = -(0.05 + 0.02 * z_lo), dV - (0.05 + 0.02 * z_hi)
    mid = reg == 0
    lin = glo + (ghi - glo) * (z[mid] - z_lo) / (z_hi - z_lo)
    assert np.abs(phi[mid] - lin).max() < 1e-12


def test_cpd_solution_satisfies_the_free_rows_and_reduces_to_dirichlet():
    """Random charge: K phi = 4 pi M s holds on every free row (rows of
    constrained nodes are not equations).  With z_lo, z_hi at the z faces of
    a zero-Neumann-z mesh the conductors hold only the face nodes, and with
    dV = 0, w = 0 the solution equals the homogeneous Dirichlet solve on the
    same cells (whose free nodes are the Neumann mesh's inner nodes, in the
    same order)."""
    rng = np.random.default_rng(12)
    L = (2.0, 2.0, 6.0)
    mN = _mesh(L, (2, 2, 6), 3, (1, 1, 2))
    s = rng.standard_normal(mN.n)
    z_lo, z_hi = 0.0, L[2]
    phi = O.poisson_cpd(mN, s, None, z_lo, z_hi, 0.0)
    reg = O.cpd_constrained(mN, z_lo, z_hi)
    K, M = O.stiffness(mN), mN.mass()
    r = (K @ phi - 4 * np.pi * M * s)[reg == 0]
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(4 * np.pi * M * s)
    mD = _mesh(L, (2, 2, 6), 3, (1, 1, 0))
    # the Dirichlet mesh's free nodes are the Neumann mesh's nodes strictly inside
    inner = reg == 0
    phiD = O.poisson(mD, s[inner])
    np.testing.assert_allclose(phi[inner], phiD, rtol=0, atol=1e-11 * np.abs(phiD).max())
    assert (phi[~inner] == 0.0).all()


def test_bare_potential_planar_average_of_plane_constant_fields():
    """Fields constant over each x-y plane average to their z profile at
    every free z position; the sawtooth of the constant-field setup comes
    back as -E (z - z0) exactly; the three terms add."""
    L = (3.0, 2.0, 6.0)
    m = _mesh(L, (3, 2, 6), 3, (1, 1, 2))
    z = m.dof_coords()[:, 2]
    zc, _ = O.axis_positions(m, 2)
    E, z0 = 0.02, 2.5
    phi, w, vapp = np.cos(z), 0.1 * z ** 2, -E * (z - z0)
    np.testing.assert_allclose(O.bare_potential_planar(m, np.zeros(m.n), None, vapp), -E * (zc - z0),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(O.bare_potential_planar(m, phi, w, vapp),
                               np.cos(zc) + 0.1 * zc ** 2 - E * (zc - z0), rtol=0, atol=1e-14)
    # a field varying in x averages over the plane: cos(2 pi x / L_x) has mean 0
    x = m.dof_coords()[:, 0]
    np.testing.assert_allclose(O.bare_potential_planar(m, np.cos(2 * np.pi * x / L[0]) + phi), np.cos(zc),
                               rtol=0, atol=1e-5)


# ------------------------------------------- dipole and polarisability (Sec. 3.1)

def test_dipole_of_polynomial_profile_is_exact():
    """psi = a(z) with a cubic: a^2 (z - z0) has degree 7, integrated exactly by
    the p = 4 GLL rule per cell; periodic x, y give the factor L_x L_y."""
    L = (2.0, 3.0, 6.0)
    m = _mesh(L, (2, 3, 6), 4, (1, 1, 2))
    z = m.dof_coords()[:, 2]
    a = np.polynomial.Polynomial([0.3, -0.2, 0.05, 0.01])
    X = (np.sqrt(m.mass()) * a(z))[:, None]
    rho = O.density(m, X, np.array([1.0]))
    z0 = 2.5
    integrand = a * a * np.polynomial.Polynomial([-z0, 1.0])
    exact = 2.0 * L[0] * L[1] * (integrand.integ()(L[2]) - integrand.integ()(0.0))
    assert abs(O.dipole(m, rho, z0) - exact) < 1e-12 * abs(exact)


@pytest.fixture(scope="module")
def biased_box():
    """A tiny Dirichlet box with two asymmetric wells; dense H~(E) and Z."""
    wl = W.CFG1
    m = O.Mesh.from_workload(wl)
    Vq = W.wells_potential(m.quad_points(), wl.centres(), wl.depth, wl.sigma, wl.L, [b == 1 for b in wl.bc])
    z = m.dof_coords()[:, 2] - wl.z0

    def H(E):
        return _Hdense(O.Operator(m, Vq, E, wl.z0))
    return m, wl, H, z


def test_hellmann_feynman_band_derivative_equals_minus_dipole(biased_box):
    """d(2 sum_{n<4} eps_n)/dE by central differences of dense eigenvalues
    equals -mu of the occupied eigenvectors (dH~/dE = -diag(z - z0))."""
    m, wl, H, z = biased_box
    E, h, nocc = 0.01, 1e-4, 4
    lam_p = np.linalg.eigvalsh(H(E + h))[:nocc]
    lam_m = np.linalg.eigvalsh(H(E - h))[:nocc]
    lam, Q = np.linalg.eigh(H(E))
    rho = O.density(m, Q[:, :nocc], np.ones(nocc))
    mu = O.dipole(m, rho, wl.z0)
    deb = 2.0 * (lam_p.sum() - lam_m.sum()) / (2 * h)
    assert abs(deb + mu) < 1e-7 * max(1.0, abs(mu))


def test_polarisability_sum_over_states_equals_dipole_derivative(biased_box):
    """Second-order perturbation theory, alpha = 4 sum_{n occ, k virt}
    |<x_k|Z|x_n>|^2 / (eps_k - eps_n), equals d mu / dE by central
    differences of the dipole of the occupied eigenvectors."""
    m, wl, H, z = biased_box
    E, h, nocc = 0.0, 1e-4, 3
    lam, Q = np.linalg.eigh(H(E))
    Zm = Q.T @ (z[:, None] * Q)
    occ, vir = slice(0, nocc), slice(nocc, None)
    alpha_sos = 4.0 * (Zm[vir, occ] ** 2 / (lam[vir][:, None] - lam[occ][None, :])).sum()

    def mu(e):
        _, Qe = np.linalg.eigh(H(e))
        return O.dipole(m, O.density(m, Qe[:, :nocc], np.ones(nocc)), wl.z0)
    alpha_fd = (mu(E + h) - mu(E - h)) / (2 * h)
    assert alpha_sos > 0
    assert abs(alpha_fd - alpha_sos) < 1e-5 * alpha_sos


def test_sawtooth_field_shape_and_collocation():
    """The sawtooth V_app (Sec. 2.2.1, extrema at 0.1 of the box from the z
    faces): zero at both faces, slope -E in the middle, extrema +-0.4 L E,
    return slope 4 E; supplied at the GLL points it is collocated exactly into
    the diagonal of H~."""
    Lz, E = 8.0, 0.02
    z = np.linspace(0.0, Lz, 801)
    v = W.sawtooth(z, Lz, E)
    assert abs(v[0]) < 1e-15 and abs(v[-1]) < 1e-15
    mid = (z > 0.1 * Lz + 1e-9) & (z < 0.9 * Lz - 1e-9)
    np.testing.assert_allclose(np.diff(v)[mid[:-1] & mid[1:]] / np.diff(z)[0], -E, rtol=1e-9)
    assert abs(v.max() - 0.4 * Lz * E) < 1e-12 and abs(z[v.argmax()] - 0.1 * Lz) < 1e-9
    assert abs(v.min() + 0.4 * Lz * E) < 1e-12 and abs(z[v.argmin()] - 0.9 * Lz) < 1e-9
    np.testing.assert_allclose((v[1:40] - v[:39]) / np.diff(z)[0], 4 * E, rtol=1e-9)
    m = _mesh((4.0, 4.0, Lz), (2, 2, 4), 3, (1, 1, 0))
    zq = m.quad_points()[:, :, 2]
    d = (O.Operator(m, W.sawtooth(zq, Lz, E), 0.0, 0.0).A.to_scipy()
         - O.Operator(m, np.zeros_like(zq), 0.0, 0.0).A.to_scipy())
    assert abs(d - sp.diags(d.diagonal())).max() < 1e-15
    np.testing.assert_allclose(d.diagonal(), W.sawtooth(m.dof_coords()[:, 2], Lz, E), atol=1e-15)


# ------------------------------------------------ Bloch-k operator (Sec. 2.3, k-point sampling)

@pytest.mark.parametrize("p,rule", [(2, 0), (3, 0), (3, 1)])
def test_cell_advection_is_a_kronecker_product(p, rule):
    """int N_l dN_l'/dx over the cell = (h/2)^2 Mhat (x) Mhat (x) Chat with the
    1-D Chat_ij = int l_i l_j' and the 1-D mass (consistent for the exact rule,
    GLL-lumped for rule 1), from exact numpy polynomial integration."""
    h = 1.7
    xi, w = F.gll_numpy(p)
    P = F.lagrange_polys(xi)
    Ch = np.array([[F.integ(P[i] * P[j].deriv()) for j in range(p + 1)] for i in range(p + 1)])
    Mh = np.diag(w) if rule == 1 else np.array([[F.integ(P[i] * P[j]) for j in range(p + 1)] for i in range(p + 1)])
    for axis in range(3):
        mats = [(h / 2) * Mh, (h / 2) * Mh, (h / 2) * Mh]
        mats[axis] = Ch
        ref = np.kron(mats[2], np.kron(mats[1], mats[0]))
        np.testing.assert_allclose(O.cell_advection(p, axis, rule, h), ref, atol=1e-13)


def test_bloch_operator_hermitian_and_reduces_at_gamma():
    wl = W.small_slab((3, 3, 4), p=3, N=6)
    m = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, m.quad_points())
    op = O.Operator(m, Vq, wl.E, wl.z0)
    B = O.BlochOperator(op, m, (0.3, -0.7))
    D = B.A - B.A.conj().T
    assert abs(D).max() < 1e-12 * abs(B.A).max()
    B0 = O.BlochOperator(op, m, (0.0, 0.0))
    assert abs(B0.A - op.A.to_scipy()).max() == 0.0
    X = wl.X(op.n)
    np.testing.assert_allclose(B0.filter(X, 7, 2.0, 300.0, -0.5).real, op.filter(X, 7, 2.0, 300.0, -0.5), rtol=0,
                               atol=1e-12 * np.abs(op.filter(X, 7, 2.0, 300.0, -0.5)).max())


def test_bloch_free_particle_levels():
    """V = 0, periodic x-y, Dirichlet z: the levels of H~^k approach
    (k_x + 2 pi a / L_x)^2 / 2 + (k_y + 2 pi b / L_y)^2 / 2 + (pi c / L_z)^2 / 2."""
    L = (4.0, 4.0, 6.0)
    m = _mesh(L, (4, 4, 6), 4, (1, 1, 0))
    op = O.Operator(m, None, 0.0, 0.0)
    k = (0.35, -0.2)
    B = O.BlochOperator(op, m, k)
    lam = np.linalg.eigvalsh(B.A.toarray())[:12]
    ref = sorted(0.5 * (k[0] + 2 * np.pi * a / L[0]) ** 2 + 0.5 * (k[1] + 2 * np.pi * b / L[1]) ** 2
                 + 0.5 * (np.pi * c / L[2]) ** 2
                 for a in range(-3, 4) for b in range(-3, 4) for c in range(1, 6))[:12]
    np.testing.assert_allclose(lam, ref, rtol=2e-6)


def test_bloch_sign_from_a_plane_wave():
    """psi = exp(i k.r) u with u = exp(i g x) sin(pi z / Lz): the Rayleigh
    quotient of H~^k at M^1/2 u is (k_x + g)^2/2 + k_y^2/2 + (pi/Lz)^2/2 up to
    the FE error; the opposite sign of the k.grad term would give (k_x - g)^2/2."""
    L = (4.0, 4.0, 6.0)
    m = _mesh(L, (4, 4, 6), 5, (1, 1, 0))
    op = O.Operator(m, None, 0.0, 0.0)
    k = (0.4, 0.25)
    g = 2 * np.pi / L[0]
    B = O.BlochOperator(op, m, k)
    xyz = m.dof_coords()
    u = np.exp(1j * g * xyz[:, 0]) * np.sin(np.pi * xyz[:, 2] / L[2])
    v = np.sqrt(m.mass()) * u
    rq = (v.conj() @ (B.A @ v)).real / (v.conj() @ v).real
    ref = 0.5 * (k[0] + g) ** 2 + 0.5 * k[1] ** 2 + 0.5 * (np.pi / L[2]) ** 2
    wrong = 0.5 * (k[0] - g) ** 2 + 0.5 * k[1] ** 2 + 0.5 * (np.pi / L[2]) ** 2
    assert abs(rq - ref) < 1e-6 < abs(wrong - ref) / 100


def test_bloch_band_folding_with_phase_twisted_projectors():
    """Bloch's theorem on a supercell: for a potential and sites of period L_x,
    the Gamma levels of the 2 L_x supercell are the union of the k_x = 0 and
    k_x = pi / L_x levels of the L_x cell, up to the FE error of the exp(i k x)
    factor (it shrinks from 2e-4 at p = 4 to 3e-7 at p = 6).  The site sits
    0.3 from the periodic face, so its cutoff ball wraps and the projector
    phase must use the minimum-image displacement; dropping the wrap, or
    conjugating the projector phase against the -i k.grad term, moves the
    folded levels by O(1)."""
    import scipy.sparse as sp
    p, Lx = 4, 3.0

    def build(nx, cen):
        m = _mesh((Lx * nx, 3.0, 4.0), (3 * nx, 3, 4), p, (1, 1, 0))
        q = m.quad_points()
        Vq = -1.5 * np.exp(-(q[..., 2] - 2.0) ** 2) * (1 + 0.5 * np.cos(2 * np.pi * q[..., 0] / Lx))
        P = O.Projectors(m, np.array(cen), 1.2, 0.45)
        D = np.tile([2.0, 0.7, 0.7, 0.7, 0.3, 0.3, 0.3, 0.3, 0.3], (len(cen), 1))
        return m, O.Operator(m, Vq, 0.0, 0.0, P, D)

    c0 = [0.3, 1.5, 2.0]
    m1, op1 = build(1, [c0])
    ms, ops = build(2, [c0, [c0[0] + Lx, c0[1], c0[2]]])
    nev = 12
    lam_sc = np.linalg.eigvalsh(O.BlochOperator(ops, ms, (0.0, 0.0)).A.toarray())[:nev]
    l0 = np.linalg.eigvalsh(O.BlochOperator(op1, m1, (0.0, 0.0)).A.toarray())
    k = np.pi / Lx
    B = O.BlochOperator(op1, m1, (k, 0.0))

    def folded(A):
        return np.sort(np.concatenate([l0, np.linalg.eigvalsh(A.toarray())]))[:nev]

    err = lambda lam: np.max(np.abs(lam - lam_sc) / np.abs(lam_sc))
    assert err(folded(B.A)) < 1e-3
    # the two plausible mistakes, planted in a copy of the operator
    Cm = op1.proj.to_scipy().tocoo()
    d = m1.dof_coords()[Cm.row] - op1.proj.centres[Cm.col // 9]
    dw = d[:, 0] - Lx * np.round(d[:, 0] / Lx)
    Dd = sp.diags(op1.Dnl.astype(complex))
    C_ok = sp.csr_matrix((Cm.data * np.exp(-1j * k * dw), (Cm.row, Cm.col)), shape=Cm.shape)
    base = B.A - C_ok @ Dd @ C_ok.conj().T
    for ph in (np.exp(-1j * k * d[:, 0]), np.exp(1j * k * dw)):
        Cb = sp.csr_matrix((Cm.data * ph, (Cm.row, Cm.col)), shape=Cm.shape)
        assert err(folded(base + Cb @ Dd @ Cb.conj().T)) > 0.1


def test_bloch_advection_rows_match_the_assembled_operator():
    """The cell-by-cell row route (used at full size) agrees with the
    assembled Bloch operator: rows of H~ X + |k|^2/2 X + S X_i - i S X_r."""
    wl = W.small_slab((3, 3, 4), p=3, N=5)
    m = O.Mesh.from_workload(wl)
    Vq = W.workload_potential(wl, m.quad_points())
    op = O.Operator(m, Vq, wl.E, wl.z0)
    k = (0.3, -0.55)
    X = wl.Xc(op.n)
    rows = np.array([0, 1, 17, op.n // 2, op.n - 1])
    kk = 0.5 * (k[0] ** 2 + k[1] ** 2)
    S = O.bloch_advection_rows(m, k, rows, X)
    R = (O.apply_rows(m, Vq, wl.E, wl.z0, rows, X.real.copy()) + 1j * O.apply_rows(m, Vq, wl.E, wl.z0, rows, X.imag.copy())
         + kk * X[rows] - 1j * S)
    ref = O.BlochOperator(op, m, k).apply(X)[rows]
    np.testing.assert_allclose(R, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_complex_cholqr2_and_rayleigh_ritz_on_a_known_hermitian_matrix():
    """Complex CholQR2 gives orthonormal columns spanning Y (Y = Q R, R upper
    triangular); Rayleigh-Ritz of a Hermitian matrix with known spectrum on an
    invariant subspace returns those eigenvalues and eigenvectors."""
    rng = np.random.default_rng(3)
    n, N = 60, 7
    Y = rng.standard_normal((n, N)) + 1j * rng.standard_normal((n, N))
    Q, R = O.cholqr2(Y)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(N), atol=1e-13)
    np.testing.assert_allclose(Q @ R, Y, atol=1e-12)
    assert np.allclose(np.tril(R, -1), 0.0)
    # H = U diag(lam) U^H with a random unitary U
    U, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(-3, 5, n))
    H = (U * lam) @ U.conj().T
    idx = [1, 4, 9, 20, 33, 41, 57]
    V = U[:, idx] @ np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))[0]
    theta, X = O.rayleigh_ritz(lambda Z: H @ Z, V)
    np.testing.assert_allclose(theta, lam[idx], atol=1e-12)
    np.testing.assert_allclose(H @ X, X * theta, atol=1e-11)


def test_bloch_subspace_iteration_converges_to_the_dense_levels():
    """Filtered subspace iteration with the Bloch operator (complex filter,
    complex CholQR2, Rayleigh-Ritz) converges to the lowest eigenvalues of the
    assembled complex matrix."""
    wl = W.small_slab((3, 3, 4), p=3, N=8)
    m = O.Mesh.from_workload(wl)
    op = O.Operator(m, W.workload_potential(wl, m.quad_points()), wl.E, wl.z0)
    k = (0.45, -0.3)
    B = O.BlochOperator(op, m, k)
    ev = np.linalg.eigvalsh(B.A.toarray())
    X0 = wl.Xc(op.n)
    a0, b = ev[0] - 0.1, ev[-1] + 0.1
    a = ev[12]
    hist, _ = O.subspace_iteration(B, X0, 12, 25, a, b, a0)
    np.testing.assert_allclose(hist[-1][:5], ev[:5], rtol=0, atol=1e-9)
