"""GPU electrostatics of the constrained-potential-difference setup (Sec.
2.2.2): phi + w held at 0 in the conductor below z_lo and at dV in the one
above z_hi, K phi = 4 pi M s between, against the oracle's reduced direct
solve; the data inside the conductors exactly; the closed-form quadratic of
a uniform charge at a larger size; superposition of charge and bias; the
refusals."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [
    # (L, ncell, p, bc, z_lo, z_hi, dV): conductor planes inside cells and on
    # cell faces; Neumann-z, Dirichlet-z (faces absent) and Neumann-x meshes
    ((3.0, 3.0, 8.0), (3, 3, 8), 3, (1, 1, 2), 1.3, 6.1, 0.3),
    ((2.0, 2.0, 10.0), (2, 2, 10), 4, (1, 1, 2), 2.0, 8.0, -0.45),
    ((2.0, 3.0, 7.0), (2, 3, 7), 2, (1, 1, 0), 1.0, 5.5, 0.2),
    ((3.0, 2.0, 6.0), (3, 2, 6), 3, (2, 1, 2), 0.5, 4.9, 1.0),
]


def _g(om, w, z_lo, z_hi, dV):
    reg = O.cpd_constrained(om, z_lo, z_hi)
    return reg, np.where(reg == 2, dV, 0.0) - w


@pytest.mark.parametrize("case", CASES)
def test_cpd_matches_direct_solve_and_holds_the_conductors(case):
    import paper_2504_00998_amd as fe
    L, ncell, p, bc, z_lo, z_hi, dV = case
    print("case: cpd", case, flush=True)
    om, gm = O.Mesh(L, ncell, p, bc), fe.Mesh(L, ncell, p, bc)
    rng = np.random.default_rng(7)
    s = rng.standard_normal(om.n)
    xyz = om.dof_coords()
    w = 0.3 * np.exp(-((xyz[:, 0] - 0.4 * L[0]) ** 2 + (xyz[:, 2] - 0.5 * L[2]) ** 2)) + 0.05 * np.sin(xyz[:, 1])
    ref = O.poisson_cpd(om, s, w, z_lo, z_hi, dV)
    phi_t, it, rel = gm.poisson_cpd(torch.from_numpy(s).cuda(), z_lo, z_hi, dV, w=torch.from_numpy(w).cuda(),
                                    tol=1e-13)
    phi = phi_t.cpu().numpy()
    assert rel <= 1e-13 and it > 0
    assert np.abs(phi - ref).max() <= 1e-8 * np.abs(ref).max()
    reg, g = _g(om, w, z_lo, z_hi, dV)
    # the data themselves inside the conductors, so the total potential is flat there
    np.testing.assert_array_equal(phi[reg > 0], g[reg > 0])
    assert np.abs((phi + w)[reg == 1]).max() == 0.0
    assert np.abs((phi + w)[reg == 2] - dV).max() <= 4 * np.finfo(float).eps * (abs(dV) + np.abs(w).max())
    # reproducible bit for bit
    phi2, it2, _ = gm.poisson_cpd(torch.from_numpy(s).cuda(), z_lo, z_hi, dV, w=torch.from_numpy(w).cuda(),
                                  tol=1e-13)
    assert it2 == it and torch.equal(phi2, phi_t)


def test_cpd_uniform_charge_closed_form_at_size():
    """Uniform charge, w = 0, conductor planes on cell faces of a 8 x 8 x 40
    p = 4 slab (139,776 DoFs): the exact quadratic of the continuum problem,
    which the space holds, at every node."""
    import paper_2504_00998_amd as fe
    L, ncell = (8.0, 8.0, 40.0), (8, 8, 40)
    gm = fe.Mesh(L, ncell, 4, (1, 1, 2))
    om = O.Mesh(L, ncell, 4, (1, 1, 2))
    z = om.dof_coords()[:, 2]
    z_lo, z_hi, s0, dV = 10.0, 30.0, 0.004, 0.35
    phi, it, rel = gm.poisson_cpd(torch.full((gm.n,), s0, dtype=torch.float64, device="cuda"), z_lo, z_hi, dV,
                                  tol=1e-13)
    print(f"cpd closed form: n={gm.n} iterations {it} relres {rel:.2e}", flush=True)
    exact = np.where(z <= z_lo, 0.0, np.where(z >= z_hi, dV,
                     -2 * np.pi * s0 * (z - z_lo) * (z - z_hi) + dV * (z - z_lo) / (z_hi - z_lo)))
    assert np.abs(phi.cpu().numpy() - exact).max() <= 1e-9 * np.abs(exact).max()


def test_cpd_superposition_of_charge_and_bias():
    import paper_2504_00998_amd as fe
    L, ncell, p, bc, z_lo, z_hi, dV = CASES[0]
    gm = fe.Mesh(L, ncell, p, bc)
    rng = np.random.default_rng(8)
    s = torch.from_numpy(rng.standard_normal(gm.n)).cuda()
    w = torch.from_numpy(0.1 * rng.standard_normal(gm.n)).cuda()
    a, _, _ = gm.poisson_cpd(s, z_lo, z_hi, dV, w=w, tol=1e-13)
    b, _, _ = gm.poisson_cpd(s, z_lo, z_hi, 0.0, tol=1e-13)
    c, _, _ = gm.poisson_cpd(torch.zeros_like(s), z_lo, z_hi, dV, w=w, tol=1e-13)
    assert ((a - b - c).abs().max() / a.abs().max()).item() <= 1e-9


def test_cpd_rejects_bad_arguments():
    import paper_2504_00998_amd as fe
    gm = fe.Mesh((2.0, 2.0, 6.0), (2, 2, 6), 2, (1, 1, 2))
    s = torch.zeros(gm.n, dtype=torch.float64, device="cuda")
    for z_lo, z_hi, msg in ((3.0, 3.0, "z_lo < z_hi"), (4.0, 2.0, "z_lo < z_hi"), (-1.0, 7.0, "no node"),
                            (10.0, 20.0, "every node")):
        with pytest.raises(RuntimeError, match=msg):
            gm.poisson_cpd(s, z_lo, z_hi, 0.1)
    with pytest.raises(RuntimeError, match="overlaps"):
        gm.poisson_cpd(s, 1.0, 5.0, 0.1, phi=s)
    gp = fe.Mesh((2.0, 2.0, 6.0), (2, 2, 6), 2, (1, 1, 1))
    with pytest.raises(RuntimeError, match="periodic"):
        gp.poisson_cpd(torch.zeros(gp.n, dtype=torch.float64, device="cuda"), 1.0, 5.0, 0.1)


def test_bare_potential_planar_average_matches_oracle():
    """V0_bare(z) (Sec. 3.2): the planar average of phi + (V_loc - V_self) +
    V_app.  The constrained-potential setup (phi from the device solve,
    V_app = 0; V0_bare is 0 and dV inside the two conductors) and the
    constant-field setup (phi from the zero-mean solve, V_app the linear
    field), against the oracle's planar average of the same nodal sum."""
    import paper_2504_00998_amd as fe
    L, ncell, p, bc, z_lo, z_hi, dV = CASES[0]
    om, gm = O.Mesh(L, ncell, p, bc), fe.Mesh(L, ncell, p, bc)
    rng = np.random.default_rng(9)
    s = rng.standard_normal(om.n)
    xyz = om.dof_coords()
    w = 0.2 * np.cos(2 * np.pi * xyz[:, 0] / L[0]) * np.exp(-(xyz[:, 2] - 0.5 * L[2]) ** 2)
    st, wt = torch.from_numpy(s).cuda(), torch.from_numpy(w).cuda()
    phi, _, _ = gm.poisson_cpd(st, z_lo, z_hi, dV, w=wt, tol=1e-13)
    got = gm.bare_potential_planar(phi, w=wt).cpu().numpy()
    ref = O.bare_potential_planar(om, phi.cpu().numpy(), w)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    zc, _ = O.axis_positions(om, 2)
    assert np.abs(got[zc <= z_lo]).max() <= 1e-14 and np.abs(got[zc >= z_hi] - dV).max() <= 1e-14
    # constant-field setup
    E, z0 = 0.01, 0.5 * L[2]
    vapp = -E * (xyz[:, 2] - z0)
    phic, _, _ = gm.poisson(st, tol=1e-13)
    got = gm.bare_potential_planar(phic, w=wt, vapp=torch.from_numpy(vapp).cuda()).cpu().numpy()
    ref = O.bare_potential_planar(om, phic.cpu().numpy(), w, vapp)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
