"""GPU electronic dipole (fe_dipole) and the field response built from the
device eigensolver (Sec. 3.1: mu_z, alpha_z = d mu / dE): parity of the
dipole with the oracle, the polarisability against second-order perturbation
theory on the oracle's dense operator, and the Hellmann-Feynman relation
d E_band / dE = -mu between band energies and dipoles from the device."""
import numpy as np
import pytest

import oracle as O
from paper_2504_00998_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("case", [((3.0, 3.0, 4.0), (3, 3, 4), 3, (1, 1, 0)),
                                  ((2.0, 3.0, 5.0), (2, 3, 5), 4, (0, 2, 2)),
                                  ((4.0, 2.0, 3.0), (4, 2, 3), 2, (2, 0, 1))])
def test_dipole_matches_oracle(case):
    import paper_2504_00998_amd as fe
    L, ncell, p, bc = case
    om, gm = O.Mesh(L, ncell, p, bc), fe.Mesh(L, ncell, p, bc)
    rho = np.random.default_rng(9).uniform(0.0, 1.0, om.n)
    for z0 in (0.0, 0.5 * L[2], 1.3):
        ref = O.dipole(om, rho, z0)
        got = gm.dipole(torch.from_numpy(rho).cuda(), z0)
        scale = (om.mass() * rho * np.abs(om.dof_coords()[:, 2] - z0)).sum()
        assert abs(got - ref) <= 1e-14 * scale, z0


@pytest.fixture(scope="module")
def response():
    import paper_2504_00998_amd as fe
    from paper_2504_00998_amd import solver
    wl = W.CFG1
    gm = fe.Mesh.from_workload(wl)
    om = O.Mesh.from_workload(wl)
    Vq_h = W.workload_potential(wl, om.quad_points())
    Vq = torch.from_numpy(Vq_h).cuda()
    X0 = torch.from_numpy(wl.X(gm.n)).cuda()
    v0 = torch.from_numpy(wl.lanczos_start(gm.n)).cuda()
    nocc = 4
    f = np.zeros(wl.N)
    f[:nocc] = 1.0
    dE = 1e-3
    res = solver.polarizability(gm, Vq, 0.0, dE, wl.z0, X0, v0, f, m=20, iters=25)
    return wl, om, Vq_h, nocc, dE, res


def test_polarisability_matches_dense_reference(response):
    """The same central difference on the oracle's dense eigenvectors (to the
    device eigensolver's convergence), and second-order perturbation theory
    (to the O(dE^2) truncation of the central difference)."""
    wl, om, Vq_h, nocc, dE, res = response

    def dense(E):
        return np.linalg.eigh(O.Operator(om, Vq_h, E, wl.z0).A.to_scipy().toarray())

    def mu(E):
        _, Q = dense(E)
        return O.dipole(om, O.density(om, Q[:, :nocc], np.ones(nocc)), wl.z0)
    alpha_fd = (mu(dE) - mu(-dE)) / (2 * dE)
    lam, Q = dense(0.0)
    z = om.dof_coords()[:, 2] - wl.z0
    Zm = Q.T @ (z[:, None] * Q)
    alpha_pt = 4.0 * (Zm[nocc:, :nocc] ** 2 / (lam[nocc:][:, None] - lam[:nocc][None, :])).sum()
    print("alpha device", res["alpha"], "dense FD", alpha_fd, "perturbation theory", alpha_pt, flush=True)
    assert abs(res["alpha"] - alpha_fd) < 1e-7 * alpha_fd
    assert abs(res["alpha"] - alpha_pt) < 2e-4 * alpha_pt


def test_hellmann_feynman_on_device_ground_states(response):
    """Band-energy difference and mean dipole from the device equal the same
    formulas on the dense eigenpairs; they satisfy d E_band / dE = -mu to the
    O(dE^2) truncation of the differences."""
    wl, om, Vq_h, nocc, dE, res = response
    eb, mus = [], []
    for E in (-dE, dE):
        lam, Q = np.linalg.eigh(O.Operator(om, Vq_h, E, wl.z0).A.to_scipy().toarray())
        eb.append(2.0 * lam[:nocc].sum())
        mus.append(O.dipole(om, O.density(om, Q[:, :nocc], np.ones(nocc)), wl.z0))
    deb = (eb[1] - eb[0]) / (2 * dE)
    mu_mid = 0.5 * (mus[0] + mus[1])
    assert abs(res["deband_dE"] - deb) < 1e-8 * abs(deb)
    assert abs(res["mu_mid"] - mu_mid) < 1e-10 * abs(mu_mid)
    assert abs(res["deband_dE"] + res["mu_mid"]) < 1e-4 * abs(res["mu_mid"])


def test_sawtooth_field_filter_and_polarisability():
    """The sawtooth V_app supplied at the GLL points: filter parity with the
    oracle, and the polarisability to it against the dense reference and
    second-order perturbation theory with the sawtooth as perturbation."""
    import paper_2504_00998_amd as fe
    from paper_2504_00998_amd import solver
    wl = W.CFG1
    gm = fe.Mesh.from_workload(wl)
    om = O.Mesh.from_workload(wl)
    Vq_h = W.workload_potential(wl, om.quad_points())
    shape_q = W.sawtooth(om.quad_points()[:, :, 2], wl.L[2], 1.0)
    E0 = 0.01
    gm.set_potential(torch.from_numpy(Vq_h + E0 * shape_q).cuda(), 0.0, wl.z0)
    op = O.Operator(om, Vq_h + E0 * shape_q, 0.0, wl.z0)
    X = wl.X(om.n)
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(om.n), 10)
    a = O.weyl_cut(a0, b, wl.N, om.n)
    Y = gm.cheb_filter(torch.from_numpy(X).cuda(), wl.m, a, b, a0).cpu().numpy()
    R = op.filter(X, wl.m, a, b, a0)
    assert (np.linalg.norm(Y - R, axis=0) / np.linalg.norm(R, axis=0)).max() < 1e-12

    nocc, dE = 4, 1e-3
    f = np.zeros(wl.N)
    f[:nocc] = 1.0
    res = solver.polarizability(gm, torch.from_numpy(Vq_h).cuda(), 0.0, dE, wl.z0,
                                torch.from_numpy(X).cuda(), torch.from_numpy(wl.lanczos_start(om.n)).cuda(), f,
                                m=20, iters=25, profile_q=torch.from_numpy(shape_q).cuda())

    def dense(e):
        return np.linalg.eigh(O.Operator(om, Vq_h + e * shape_q, 0.0, wl.z0).A.to_scipy().toarray())

    def mu(e):
        _, Q = dense(e)
        return O.dipole(om, O.density(om, Q[:, :nocc], np.ones(nocc)), wl.z0)
    alpha_fd = (mu(dE) - mu(-dE)) / (2 * dE)
    lam, Q = dense(0.0)
    z = om.dof_coords()[:, 2] - wl.z0
    s = W.sawtooth(om.dof_coords()[:, 2], wl.L[2], 1.0)
    Zm = Q.T @ (z[:, None] * Q)
    Sm = Q.T @ (s[:, None] * Q)
    alpha_pt = -4.0 * (Zm[nocc:, :nocc] * Sm[nocc:, :nocc] / (lam[nocc:][:, None] - lam[:nocc][None, :])).sum()
    print("sawtooth alpha device", res["alpha"], "dense FD", alpha_fd, "perturbation theory", alpha_pt, flush=True)
    assert abs(res["alpha"] - alpha_fd) < 1e-7 * abs(alpha_fd)
    assert abs(res["alpha"] - alpha_pt) < 2e-4 * abs(alpha_pt)
