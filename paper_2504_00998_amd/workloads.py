"""Seeded synthetic workloads for the biased-slab Hamiltonian filter.

This module only describes and draws inputs: mesh sizes, the Gaussian-well
stand-in for the local pseudopotential, the field strength, random wavefunction
blocks, loss weights and finite-difference directions.  It holds none of the
finite-element arithmetic (no basis, quadrature, assembly or filter); both the
CPU oracle and the GPU library receive the arrays drawn here.

The paper's slabs (LLZO, GaAs(111), Al(111) with vacuum, periodic in x and y,
bias along z; Sec. 3 and Fig. 2) need structures and pseudopotentials that are
not available, so a slab of attractive Gaussian wells in the middle third of
the box stands in for the atoms (V_loc of Sec. 2.1, Eq. for V_eff), with the
constant-field term of Sec. 2.2.1 added as a linear potential along z.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

# per-axis boundary conditions (shared integer codes of the C ABI)
DIRICHLET, PERIODIC, NEUMANN = 0, 1, 2
# stiffness integration rules
RULE_EXACT, RULE_GLL = 0, 1


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cfg: int                      # 1..5; seeds are 1000*cfg + k
    L: Tuple[float, float, float]  # box edge lengths (bohr)
    ncell: Tuple[int, int, int]
    p: int                        # GLL degree of the wavefunction basis
    bc: Tuple[int, int, int]
    N: int                        # number of wavefunction vectors
    m: int                        # Chebyshev filter degree
    E: float                      # field strength (Ha/bohr); V_ext = -E (z - z0)
    depth: float                  # well depth (Ha)
    sigma: float                  # well width (bohr)
    lattice: Optional[Tuple[Tuple[float, ...], Tuple[float, ...], Tuple[float, ...]]]
    n_random_wells: int = 0       # cfg1: wells at seeded uniform centres
    random_box: Tuple[float, float] = (1.0, 7.0)
    nonlocal_sites: bool = False  # cfg5: 9 projectors per well site
    r_cut: float = 2.0
    r_g: float = 0.5
    rule: int = RULE_EXACT

    @property
    def z0(self) -> float:
        """Field origin: the domain centre along z (the dipole is measured there)."""
        return 0.5 * self.L[2]

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple(self.L[a] / self.ncell[a] for a in range(3))

    def n_free(self) -> int:
        n = 1
        for a in range(3):
            k = self.ncell[a] * self.p
            n *= {DIRICHLET: k - 1, PERIODIC: k, NEUMANN: k + 1}[self.bc[a]]
        return n

    @property
    def n_cells(self) -> int:
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    # ---------------------------------------------------------------- seeds
    def seed(self, k: int) -> int:
        return 1000 * self.cfg + k

    def centres(self) -> np.ndarray:
        """Well centres, (n_site, 3)."""
        if self.lattice is not None:
            xs, ys, zs = self.lattice
            g = np.array([(x, y, z) for z in zs for y in ys for x in xs], dtype=np.float64)
            return g
        rng = np.random.default_rng(self.seed(1))
        lo, hi = self.random_box
        return rng.uniform(lo, hi, size=(self.n_random_wells, 3))

    def X(self, n: Optional[int] = None, cols=None) -> np.ndarray:
        """Random block, (n, len(cols)) row-major, i.i.d. N(0,1).

        Column j is drawn from its own PCG64 stream seeded (seed(2), j), so any
        subset of columns can be regenerated without drawing the others.
        """
        n = self.n_free() if n is None else n
        cols = range(self.N) if cols is None else cols
        cols = list(cols)
        out = np.empty((n, len(cols)), dtype=np.float64)
        for t, j in enumerate(cols):
            out[:, t] = np.random.default_rng([self.seed(2), int(j)]).standard_normal(n)
        return out

    def Xc(self, n: Optional[int] = None, cols=None) -> np.ndarray:
        """Complex random block for the Bloch-k operator: real part `X`, imaginary
        part i.i.d. N(0,1) from the streams (seed(7), j)."""
        n = self.n_free() if n is None else n
        cols = list(range(self.N) if cols is None else cols)
        im = np.empty((n, len(cols)), dtype=np.float64)
        for t, j in enumerate(cols):
            im[:, t] = np.random.default_rng([self.seed(7), int(j)]).standard_normal(n)
        return self.X(n, cols) + 1j * im

    def X_device(self, n: Optional[int] = None, N: Optional[int] = None, device="cuda"):
        """Random block (n, N), i.i.d. N(0,1), drawn on the device by torch's
        seeded generator (seed(2)).  Used where the host recipe `X` would be
        too slow (tens of GB); every consumer of a given test receives this
        same array."""
        import torch
        n = self.n_free() if n is None else n
        N = self.N if N is None else N
        g = torch.Generator(device=device)
        g.manual_seed(self.seed(2))
        return torch.randn((n, N), generator=g, dtype=torch.float64, device=device)

    def lanczos_start(self, n: Optional[int] = None) -> np.ndarray:
        n = self.n_free() if n is None else n
        return np.random.default_rng(self.seed(3)).standard_normal(n)

    def weights(self) -> np.ndarray:
        """Loss weights w_i ~ U(0,1)."""
        return np.random.default_rng(self.seed(4)).uniform(0.0, 1.0, size=self.N)

    def fd_directions(self, k: int, nX: int, nV: int):
        """k joint directions (dX, dV, dE) with per-entry N(0,1) entries."""
        rng = np.random.default_rng(self.seed(5))
        out = []
        for _ in range(k):
            out.append((rng.standard_normal(nX), rng.standard_normal(nV), float(rng.standard_normal())))
        return out

    def nonlocal_coupling(self) -> np.ndarray:
        """Per (site, projector) coupling D ~ U(-1, 1) Ha, (n_site, 9)."""
        n_site = self.centres().shape[0]
        return np.random.default_rng(self.seed(6)).uniform(-1.0, 1.0, size=(n_site, 9))


def wells_potential(points: np.ndarray, centres: np.ndarray, depth: float, sigma: float,
                    L, periodic) -> np.ndarray:
    """Sum of Gaussian wells  depth * exp(-|x - R_s|^2 / (2 sigma^2))  at `points`.

    Distances use the minimum image along periodic axes.  `points` is (..., 3);
    the result has the leading shape of `points`.
    """
    pts = np.asarray(points, dtype=np.float64)
    flat = pts.reshape(-1, 3)
    out = np.zeros(flat.shape[0], dtype=np.float64)
    inv = 1.0 / (2.0 * sigma * sigma)
    Lv = np.asarray(L, dtype=np.float64)
    for R in np.asarray(centres, dtype=np.float64):
        d = flat - R
        for a in range(3):
            if periodic[a]:
                d[:, a] -= Lv[a] * np.round(d[:, a] / Lv[a])
        out += depth * np.exp(-(d * d).sum(axis=1) * inv)
    return out.reshape(pts.shape[:-1])


def axis_points(quad_points: np.ndarray, ncell) -> list:
    """Per-axis coordinates (ncell_a, p+1) of a tensor-product set of cell
    GLL points given as (n_cells, (p+1)^3, 3), cells x fastest."""
    n1 = round(quad_points.shape[1] ** (1.0 / 3.0))
    nx, ny, _ = ncell
    q = quad_points.reshape(ncell[2], ny, nx, n1, n1, n1, 3)  # [cz, cy, cx, k, j, i, a]
    return [q[0, 0, :, 0, 0, :, 0], q[0, :, 0, 0, :, 0, 1], q[:, 0, 0, :, 0, 0, 2]]


def wells_potential_cells(axis_pts, centres: np.ndarray, depth: float, sigma: float, L, periodic) -> np.ndarray:
    """The Gaussian-well sum of `wells_potential` on a tensor-product set of
    cell points, using exp(-|d|^2/2s^2) = prod_a exp(-d_a^2/2s^2).

    axis_pts: three arrays (ncell_a, p+1) of coordinates.  Returns
    (n_cells, (p+1)^3) with cells x fastest and local index i + n1 (j + n1 k).
    """
    inv = 1.0 / (2.0 * sigma * sigma)
    G = []
    for a in range(3):
        x = np.asarray(axis_pts[a], dtype=np.float64).reshape(-1)          # (ncell_a * n1)
        d = x[None, :] - np.asarray(centres, dtype=np.float64)[:, a][:, None]  # (n_site, .)
        if periodic[a]:
            d -= L[a] * np.round(d / L[a])
        G.append(np.exp(-(d * d) * inv))
    gx, gy, gz = G
    ns = gx.shape[0]
    pxy = (gx[:, None, :] * gy[:, :, None]).reshape(ns, -1)    # (s, [cy j][cx i])
    V = depth * (gz.T @ pxy)                                   # ([cz k], [cy j][cx i])
    ncz, n1 = np.asarray(axis_pts[2]).shape
    ncy = np.asarray(axis_pts[1]).shape[0]
    ncx = np.asarray(axis_pts[0]).shape[0]
    V = V.reshape(ncz, n1, ncy, n1, ncx, n1)                   # cz k cy j cx i
    V = V.transpose(0, 2, 4, 1, 3, 5)                          # cz cy cx k j i
    return np.ascontiguousarray(V.reshape(ncz * ncy * ncx, n1 ** 3))


def sawtooth(z: np.ndarray, Lz: float, E: float, frac: float = 0.1) -> np.ndarray:
    """Sawtooth form of the constant-field potential along z (Sec. 2.2.1;
    extrema at `frac` of the box from either z face, Sec. 3.1): slope -E on
    [frac Lz, (1 - frac) Lz], centred on Lz / 2, and the return ramp through
    the z faces, so that V(0) = V(Lz) = 0."""
    z = np.asarray(z, dtype=np.float64)
    lo, hi = frac * Lz, (1.0 - frac) * Lz
    vmax = -E * (lo - 0.5 * Lz)
    ramp = (hi - lo) / (2.0 * lo)  # slope of the return ramp in units of E
    mid = -E * (z - 0.5 * Lz)
    below = vmax - ramp * E * (lo - z)
    above = -vmax + ramp * E * (z - hi)
    return np.where(z < lo, below, np.where(z > hi, above, mid))


def workload_potential(wl: "Workload", quad_points: np.ndarray) -> np.ndarray:
    """V_loc of the workload at the given cell GLL points, (n_cells, (p+1)^3)."""
    periodic = [b == PERIODIC for b in wl.bc]
    return wells_potential_cells(axis_points(quad_points, wl.ncell), wl.centres(), wl.depth, wl.sigma,
                                 wl.L, periodic)


def _lat(lo, n, s=3.0):
    return tuple(lo + s * i for i in range(n))


CFG1 = Workload("cube-p3-dirichlet", 1, (8.0, 8.0, 8.0), (4, 4, 4), 3,
                (DIRICHLET, DIRICHLET, DIRICHLET), N=16, m=20, E=0.01,
                depth=-2.0, sigma=0.7, lattice=None, n_random_wells=4)
CFG2 = Workload("slab-p4-24x24x48", 2, (24.0, 24.0, 48.0), (24, 24, 48), 4,
                (PERIODIC, PERIODIC, DIRICHLET), N=256, m=30, E=0.005,
                depth=-3.0, sigma=0.6, lattice=(_lat(7.5, 4), _lat(7.5, 4), _lat(16.5, 6)))
CFG3 = CFG2.with_(name="slab-p4-24x24x48-subspace", cfg=3)
CFG4 = Workload("slab-p6-16x16x32", 4, (16.0, 16.0, 32.0), (16, 16, 32), 6,
                (PERIODIC, PERIODIC, DIRICHLET), N=128, m=20, E=0.005,
                depth=-3.0, sigma=0.6, lattice=(_lat(3.5, 4), _lat(3.5, 4), _lat(11.5, 4)))
CFG5 = Workload("slab-p5-40x40x80-nonlocal", 5, (40.0, 40.0, 80.0), (40, 40, 80), 5,
                (PERIODIC, PERIODIC, DIRICHLET), N=384, m=40, E=0.01,
                depth=-3.0, sigma=0.6, lattice=(_lat(9.5, 8), _lat(9.5, 8), _lat(29.5, 8)),
                nonlocal_sites=True)

CONFIGS = {1: CFG1, 2: CFG2, 3: CFG3, 4: CFG4, 5: CFG5}


def small_slab(ncell=(3, 3, 4), p=4, N=24, m=7, cfg=2, **kw) -> Workload:
    """A small slab with the cfg-2 recipe scaled to a few cells (parity cases)."""
    L = tuple(float(c) for c in ncell)
    base = CONFIGS[cfg]
    cx = tuple(0.5 * L[0] + 3.0 * (i - 0.5) for i in range(2))
    cz = tuple(0.5 * L[2] + 3.0 * (i - 0.5) for i in range(2))
    d = dict(name=f"small-slab-p{p}-{ncell[0]}x{ncell[1]}x{ncell[2]}", L=L, ncell=tuple(ncell), p=p,
             N=N, m=m, lattice=(cx, cx, cz))
    d.update(kw)
    return base.with_(**d)
