"""FP64 CPU oracle for the Chebyshev-filtered FE Hamiltonian of a biased slab.

TEST INFRASTRUCTURE ONLY: the independent reference the GPU library is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark import it.  It shares no code with the GPU library.

The heavy parts (reference element, CSR assembly, sparse products, filter,
adjoint) are plain C in ``oracle.c``; the dense steps (Lanczos bounds,
Cholesky-QR, Rayleigh-Ritz) are numpy/LAPACK here.

Parity unpinned: nothing here is unpinned; every function has at least one pin
in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Mesh(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("ncell", C.c_int * 3), ("p", C.c_int),
                ("bc", C.c_int * 3), ("rule", C.c_int)]


class _CSR(C.Structure):
    _fields_ = [("n", C.c_int64), ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class _CSC(C.Structure):
    _fields_ = [("n", C.c_int64), ("nproj", C.c_int64), ("colptr", C.c_void_p),
                ("row", C.c_void_p), ("val", C.c_void_p)]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.or_gll.argtypes = [C.c_int, _dp, _dp]
        L.or_gauss.argtypes = [C.c_int, _dp, _dp]
        L.or_lagrange_eval.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.or_cell_stiffness.argtypes = [C.c_int, C.c_int, C.c_double, _dp]
        L.or_cell_advection.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, _dp]
        L.or_n_free.argtypes = [C.POINTER(_Mesh)]
        L.or_n_free.restype = C.c_int64
        L.or_cell_dofs.argtypes = [C.POINTER(_Mesh), _i64p]
        L.or_quad_points.argtypes = [C.POINTER(_Mesh), _dp]
        L.or_mass.argtypes = [C.POINTER(_Mesh), _dp]
        L.or_dof_coords.argtypes = [C.POINTER(_Mesh), _dp]
        L.or_assemble.argtypes = [C.POINTER(_Mesh), C.c_int, C.c_void_p, C.c_double, C.c_double]
        L.or_assemble.restype = C.POINTER(_CSR)
        L.or_csr_free.argtypes = [C.POINTER(_CSR)]
        L.or_csr_nnz.argtypes = [C.POINTER(_CSR)]
        L.or_csr_nnz.restype = C.c_int64
        L.or_csr_export.argtypes = [C.POINTER(_CSR), _i64p, _i32p, _dp]
        L.or_projectors.argtypes = [C.POINTER(_Mesh), C.c_int, _dp, C.c_double, C.c_double]
        L.or_projectors.restype = C.POINTER(_CSC)
        L.or_csc_free.argtypes = [C.POINTER(_CSC)]
        L.or_csc_nnz.argtypes = [C.POINTER(_CSC)]
        L.or_csc_nnz.restype = C.c_int64
        L.or_csc_export.argtypes = [C.POINTER(_CSC), _i64p, _i64p, _dp]
        L.or_apply.argtypes = [C.POINTER(_CSR), C.c_void_p, C.c_void_p, _dp, _dp, C.c_int64]
        L.or_cheb_coeffs.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp,
                                     C.POINTER(C.c_double)]
        L.or_cheb_filter.argtypes = [C.POINTER(_CSR), C.c_void_p, C.c_void_p, _dp, _dp, C.c_int64,
                                     C.c_int, C.c_double, C.c_double, C.c_double, C.c_void_p]
        L.or_cheb_filter.restype = C.c_int
        L.or_cheb_filter_vjp.argtypes = [C.POINTER(_CSR), C.c_void_p, C.c_void_p, _dp, _dp, C.c_int64,
                                         C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.or_cheb_filter_vjp.restype = C.c_int
        L.or_apply_rows.argtypes = [C.POINTER(_Mesh), C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                    _i64p, C.c_int64, _dp, C.c_int64, _dp]
        L.or_apply_rows.restype = C.c_int
        L.or_potential_vjp.argtypes = [C.POINTER(_Mesh), _dp, C.c_double, _dp, C.POINTER(C.c_double)]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


# ------------------------------------------------------------------ 1-D rules

def gll(p: int):
    """GLL nodes and weights of degree p on [-1, 1]."""
    xi = np.zeros(p + 1); w = np.zeros(p + 1)
    assert lib().or_gll(p, xi, w) == 0
    return xi, w


def gauss(q: int):
    x = np.zeros(q); w = np.zeros(q)
    assert lib().or_gauss(q, x, w) == 0
    return x, w


def lagrange(p: int, x: float):
    """Values and derivatives of the p+1 GLL Lagrange polynomials at x."""
    l = np.zeros(p + 1); dl = np.zeros(p + 1)
    lib().or_lagrange_eval(p, float(x), l, dl)
    return l, dl


def cell_stiffness(p: int, rule: int = 0, h: float = 1.0) -> np.ndarray:
    """Dense stiffness of one cubic cell, (p+1)^3 x (p+1)^3, local i fastest."""
    nc = (p + 1) ** 3
    K = np.zeros(nc * nc)
    assert lib().or_cell_stiffness(p, rule, h, K) == 0
    return K.reshape(nc, nc)


def cell_advection(p: int, axis: int, rule: int = 0, h: float = 1.0) -> np.ndarray:
    """int_c N_l dN_l'/dx_axis over one cubic cell, (p+1)^3 x (p+1)^3."""
    nc = (p + 1) ** 3
    G = np.zeros(nc * nc)
    assert lib().or_cell_advection(p, rule, h, axis, G) == 0
    return G.reshape(nc, nc)


# ------------------------------------------------------------------- the mesh

class Mesh:
    """Structured box of cubic cells with per-axis boundary conditions
    (0 Dirichlet, 1 periodic, 2 zero-Neumann) and GLL degree p."""

    def __init__(self, L, ncell, p, bc, rule=0):
        self.L = tuple(float(x) for x in L)
        self.ncell = tuple(int(x) for x in ncell)
        self.p = int(p)
        self.bc = tuple(int(x) for x in bc)
        self.rule = int(rule)
        self._m = _Mesh((C.c_double * 3)(*self.L), (C.c_int * 3)(*self.ncell), self.p,
                        (C.c_int * 3)(*self.bc), self.rule)

    @classmethod
    def from_workload(cls, wl, rule=None):
        return cls(wl.L, wl.ncell, wl.p, wl.bc, wl.rule if rule is None else rule)

    @property
    def nc(self) -> int:
        return (self.p + 1) ** 3

    @property
    def n_cells(self) -> int:
        return self.ncell[0] * self.ncell[1] * self.ncell[2]

    @property
    def n(self) -> int:
        return int(lib().or_n_free(C.byref(self._m)))

    def cell_dofs(self) -> np.ndarray:
        out = np.zeros(self.n_cells * self.nc, dtype=np.int64)
        lib().or_cell_dofs(C.byref(self._m), out)
        return out.reshape(self.n_cells, self.nc)

    def quad_points(self) -> np.ndarray:
        out = np.zeros(self.n_cells * self.nc * 3)
        lib().or_quad_points(C.byref(self._m), out)
        return out.reshape(self.n_cells, self.nc, 3)

    def mass(self) -> np.ndarray:
        out = np.zeros(self.n)
        lib().or_mass(C.byref(self._m), out)
        return out

    def dof_coords(self) -> np.ndarray:
        out = np.zeros(self.n * 3)
        lib().or_dof_coords(C.byref(self._m), out)
        return out.reshape(self.n, 3)


class CSR:
    """Owning wrapper of an assembled CSR matrix."""

    def __init__(self, ptr):
        if not ptr:
            raise MemoryError("oracle assembly failed")
        self._p = ptr
        self.n = ptr.contents.n

    def __del__(self):
        if getattr(self, "_p", None):
            lib().or_csr_free(self._p)
            self._p = None

    @property
    def nnz(self) -> int:
        return int(lib().or_csr_nnz(self._p))

    def to_scipy(self):
        import scipy.sparse as sp
        rp = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(self.nnz, dtype=np.int32)
        val = np.zeros(self.nnz)
        lib().or_csr_export(self._p, rp, col, val)
        return sp.csr_matrix((val, col, rp), shape=(self.n, self.n))


class Projectors:
    """Owning wrapper of the collocated projector matrix C~ (CSC, n x 9*n_site)."""

    def __init__(self, mesh: Mesh, centres, r_cut: float, r_g: float):
        centres = np.ascontiguousarray(centres, dtype=np.float64)
        self.centres = centres.copy()
        self.n_site = centres.shape[0]
        self._p = lib().or_projectors(C.byref(mesh._m), self.n_site, centres.reshape(-1),
                                      float(r_cut), float(r_g))
        if not self._p:
            raise MemoryError("projector construction failed")
        self.n = mesh.n
        self.nproj = 9 * self.n_site

    def __del__(self):
        if getattr(self, "_p", None):
            lib().or_csc_free(self._p)
            self._p = None

    def to_scipy(self):
        import scipy.sparse as sp
        nnz = int(lib().or_csc_nnz(self._p))
        cp = np.zeros(self.nproj + 1, dtype=np.int64)
        row = np.zeros(nnz, dtype=np.int64)
        val = np.zeros(nnz)
        lib().or_csc_export(self._p, cp, row, val)
        return sp.csc_matrix((val, row, cp), shape=(self.n, self.nproj))


class Operator:
    """H~ = M^-1/2 (1/2 K + V) M^-1/2 (+ C~ diag(D) C~^T), assembled on the CPU."""

    def __init__(self, mesh: Mesh, Vq: Optional[np.ndarray], E: float, z0: float,
                 projectors: Optional[Projectors] = None, Dnl: Optional[np.ndarray] = None):
        self.mesh = mesh
        self.E = float(E); self.z0 = float(z0)
        vq = None
        if Vq is not None:
            self._Vq = np.ascontiguousarray(Vq, dtype=np.float64).reshape(-1)
            assert self._Vq.size == mesh.n_cells * mesh.nc
            vq = self._Vq.ctypes.data
        self.A = CSR(lib().or_assemble(C.byref(mesh._m), 1, vq, self.E, self.z0))
        self.n = self.A.n
        self.proj = projectors
        self.Dnl = None
        if projectors is not None:
            self.Dnl = np.ascontiguousarray(Dnl, dtype=np.float64).reshape(-1)
            assert self.Dnl.size == projectors.nproj

    def _nl(self):
        if self.proj is None:
            return None, None
        return C.cast(self.proj._p, C.c_void_p), self.Dnl.ctypes.data

    def apply(self, X: np.ndarray) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64)
        one = X.ndim == 1
        X2 = X.reshape(self.n, -1)
        Y = np.zeros_like(X2)
        c, d = self._nl()
        lib().or_apply(self.A._p, c, d, X2, Y, X2.shape[1])
        return Y.reshape(X.shape) if one else Y

    def filter(self, X: np.ndarray, m: int, a: float, b: float, a0: float = float("nan"),
               store: bool = False):
        X = np.ascontiguousarray(X, dtype=np.float64)
        N = X.shape[1]
        Y = np.zeros_like(X)
        S = np.zeros((m + 1,) + X.shape) if store else None
        c, d = self._nl()
        rc = lib().or_cheb_filter(self.A._p, c, d, X, Y, N, m, a, b, a0,
                                  None if S is None else S.ctypes.data)
        if rc != 0:
            raise ValueError(f"oracle filter failed ({rc})")
        return (Y, S) if store else Y

    def filter_vjp(self, X: np.ndarray, G: np.ndarray, m: int, a: float, b: float,
                   a0: float = float("nan")):
        """(Xbar, g) with g_I = dL/dv_I for the diagonal potential term."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        G = np.ascontiguousarray(G, dtype=np.float64)
        Xb = np.zeros_like(X); g = np.zeros(self.n)
        c, d = self._nl()
        rc = lib().or_cheb_filter_vjp(self.A._p, c, d, X, G, X.shape[1], m, a, b, a0, Xb, g)
        if rc != 0:
            raise ValueError(f"oracle vjp failed ({rc})")
        return Xb, g

    def potential_vjp(self, g: np.ndarray):
        """(Vbar at quadrature points (n_cells, nc), Ebar) from g = dL/dv."""
        Vb = np.zeros(self.mesh.n_cells * self.mesh.nc)
        Eb = C.c_double(0.0)
        lib().or_potential_vjp(C.byref(self.mesh._m), np.ascontiguousarray(g), self.z0, Vb, C.byref(Eb))
        return Vb.reshape(self.mesh.n_cells, self.mesh.nc), Eb.value


def apply_rows(mesh: Mesh, Vq: Optional[np.ndarray], E: float, z0: float, rows, X: np.ndarray,
               projectors: Optional[Projectors] = None, Dnl: Optional[np.ndarray] = None) -> np.ndarray:
    """Rows `rows` of H~ X (nonlocal term included when given), summed row by
    row from the cell contributions; X is the full (n x N) block."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    N = X.shape[1]
    Yr = np.zeros((rows.size, N))
    vq = None
    if Vq is not None:
        Vq = np.ascontiguousarray(Vq, dtype=np.float64).reshape(-1)
        vq = Vq.ctypes.data
    cp, dp = None, None
    if projectors is not None:
        Dnl = np.ascontiguousarray(Dnl, dtype=np.float64).reshape(-1)
        cp, dp = C.cast(projectors._p, C.c_void_p), Dnl.ctypes.data
    rc = lib().or_apply_rows(C.byref(mesh._m), vq, float(E), float(z0), cp, dp, rows, rows.size, X, N, Yr)
    if rc != 0:
        raise MemoryError("or_apply_rows failed")
    return Yr


# ------------------------------------------------------------ Bloch-k operator

class BlochOperator:
    """Bloch form of H~ over the periodic x-y directions (paper Sec. 2.1,
    governing equations for u = exp(-i k.r) psi): the local part
    -1/2 lap - i k.grad + |k|^2/2 + V on the FE space is
        H~ + |k|^2 / 2 - i M^-1/2 (k_x G_x + k_y G_y) M^-1/2,
    G_a the assembled advection matrices int N_I dN_J/dx_a (real,
    antisymmetric on periodic axes), and the nonlocal part carries the phase
    exp(-i k.(x - R - L_r)) on the ket side and its conjugate on the bra side,
    i.e. C^k_I = exp(-i k.d_I) C~_I with d_I = x_I - R_s the displacement to
    the image of the site the entry belongs to (minimum image), and
    H~^k gains C^k diag(D) C^k^H.  Hermitian.  Complex sparse (scipy);
    vectors are complex (n, N)."""

    def __init__(self, op: "Operator", mesh: Mesh, k):
        import scipy.sparse as sp
        self.k = (float(k[0]), float(k[1]))
        for a in range(2):
            if self.k[a] != 0.0 and mesh.bc[a] != 1:
                raise ValueError("a Bloch wave number needs a periodic axis")
        n = op.n
        h = mesh.L[0] / mesh.ncell[0]
        dofs = mesh.cell_dofs()
        M = mesh.mass()
        rows, cols, vals = [], [], []
        Gk = self.k[0] * cell_advection(mesh.p, 0, mesh.rule, h) + self.k[1] * cell_advection(mesh.p, 1, mesh.rule, h)
        nc = mesh.nc
        li, lj = np.meshgrid(np.arange(nc), np.arange(nc), indexing="ij")
        for c in range(mesh.n_cells):
            I, J = dofs[c][li], dofs[c][lj]
            ok = (I >= 0) & (J >= 0)
            rows.append(I[ok]); cols.append(J[ok]); vals.append(Gk[ok])
        G = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        d = 1.0 / np.sqrt(M)
        S = sp.diags(d) @ G @ sp.diags(d)
        kk = 0.5 * (self.k[0] ** 2 + self.k[1] ** 2)
        self.A = (op.A.to_scipy().astype(np.complex128) + kk * sp.identity(n, dtype=np.complex128)
                  - 1j * S.astype(np.complex128)).tocsr()
        if op.proj is not None:
            Cm = op.proj.to_scipy().tocoo()
            xyz = mesh.dof_coords()
            site = Cm.col // 9
            d = xyz[Cm.row] - op.proj.centres[site]
            for a in range(3):
                if mesh.bc[a] == 1:
                    d[:, a] -= mesh.L[a] * np.round(d[:, a] / mesh.L[a])
            ph = np.exp(-1j * (self.k[0] * d[:, 0] + self.k[1] * d[:, 1]))
            Ck = sp.csr_matrix((Cm.data * ph, (Cm.row, Cm.col)), shape=Cm.shape)
            self.A = (self.A + Ck @ sp.diags(op.Dnl.astype(np.complex128)) @ Ck.conj().T).tocsr()
        self.n = n

    def apply(self, X: np.ndarray) -> np.ndarray:
        return self.A @ X

    def filter(self, X: np.ndarray, m: int, a: float, b: float, a0: float = float("nan")) -> np.ndarray:
        """The same scaled / unscaled three-term recurrence as Operator.filter
        (real coefficients), on complex vectors."""
        al, be, c = cheb_coeffs(m, a, b, a0)
        Ym1 = np.array(X, dtype=np.complex128)
        Y = al[0] * (self.A @ Ym1 - c * Ym1)
        for j in range(1, m):
            Yn = al[j] * (self.A @ Y - c * Y) - be[j] * Ym1
            Ym1, Y = Y, Yn
        return Y


def bloch_advection_rows(mesh: Mesh, k, rows, X: np.ndarray) -> np.ndarray:
    """Rows `rows` of M^-1/2 (k_x G_x + k_y G_y) M^-1/2 X, summed cell by cell
    from the cell advection matrices (the -i k.grad term of the Bloch form is
    -i times this); X is the full (n, N) block, real or complex.  No
    nonlocal term."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    h = mesh.L[0] / mesh.ncell[0]
    Gk = k[0] * cell_advection(mesh.p, 0, mesh.rule, h) + k[1] * cell_advection(mesh.p, 1, mesh.rule, h)
    dofs = mesh.cell_dofs()
    d = 1.0 / np.sqrt(mesh.mass())
    pos = {int(I): t for t, I in enumerate(rows)}
    out = np.zeros((rows.size, X.shape[1]), dtype=np.result_type(X.dtype, np.float64))
    for c, l in zip(*np.nonzero(np.isin(dofs, rows))):
        I = int(dofs[c, l])
        J = dofs[c]
        ok = J >= 0
        out[pos[I]] += d[I] * (Gk[l, ok] @ (d[J[ok], None] * X[J[ok]]))
    return out


# ------------------------------------------------------------ observables

def density(mesh: Mesh, X: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Electron density of Sec. 2.1, rho = 2 sum_n f_n |psi_n|^2, at the free
    GLL nodes, for orbitals psi_n = M^-1/2 x_n (x_n a column of X)."""
    M = mesh.mass()
    return 2.0 * ((X * X) @ np.asarray(f, dtype=np.float64)) / M


def axis_positions(mesh: Mesh, a: int):
    """Coordinates and assembled 1-D GLL lumped masses of the free node
    positions along axis a (Dirichlet ends dropped, periodic ends joined)."""
    xi, w = gll(mesh.p)
    p, nce = mesh.p, mesh.ncell[a]
    h = mesh.L[a] / nce
    K = nce * p
    mass = np.zeros(K + 1)
    coord = np.zeros(K + 1)
    for c in range(nce):
        for i in range(p + 1):
            mass[c * p + i] += 0.5 * h * w[i]
            coord[c * p + i] = c * h + 0.5 * h * (xi[i] + 1.0)
    if mesh.bc[a] == 1:  # periodic: position K is position 0
        mass[0] += mass[K]
        return coord[:K], mass[:K]
    if mesh.bc[a] == 0:  # Dirichlet
        return coord[1:K], mass[1:K]
    return coord, mass


def planar_integral(mesh: Mesh, field: np.ndarray, normalize: bool = False) -> np.ndarray:
    """Sec. 3.2 planar integral of a nodal field over the x-y plane S_z through
    each row of free z nodes (ascending z), by GLL quadrature in x and y:
    sum over the plane's nodes of m_x m_y F = M_I F_I / m_z.  With normalize,
    divided by the plane area sum m_x * sum m_y (the planar average)."""
    xyz = mesh.dof_coords()
    M = mesh.mass()
    zc, mz = axis_positions(mesh, 2)
    k = np.searchsorted(zc, xyz[:, 2] - 1e-9 * mesh.L[2])
    out = np.bincount(k, weights=M * np.asarray(field, dtype=np.float64), minlength=len(zc)) / mz
    if normalize:
        out = out / (axis_positions(mesh, 0)[1].sum() * axis_positions(mesh, 1)[1].sum())
    return out


def bare_potential_planar(mesh: Mesh, phi: np.ndarray, w: Optional[np.ndarray] = None,
                          vapp: Optional[np.ndarray] = None) -> np.ndarray:
    """Sec. 3.2 planar average of the bare potential V_bare = phi~ + V_app,
    phi~ = phi + (V_loc - V_self): the planar average of the nodal sum
    phi + w + vapp (w = V_loc - V_self and vapp at the nodes, None: 0)."""
    v = np.asarray(phi, dtype=np.float64).copy()
    if w is not None:
        v = v + np.asarray(w, dtype=np.float64)
    if vapp is not None:
        v = v + np.asarray(vapp, dtype=np.float64)
    return planar_integral(mesh, v, normalize=True)


def dipole(mesh: Mesh, rho: np.ndarray, z0: float) -> float:
    """Sec. 3.1 electronic dipole about z0, int rho (z - z0), by the GLL
    quadrature of the nodal density."""
    z = mesh.dof_coords()[:, 2]
    return float((mesh.mass() * np.asarray(rho, dtype=np.float64) * (z - z0)).sum())


def poisson(mesh: Mesh, s: np.ndarray) -> np.ndarray:
    """Sec. 2.2 electrostatics on the finite-element space: -lap(phi) / 4 pi = s
    in Galerkin form, K phi = 4 pi M s (GLL-collocated right-hand side), with
    phi = 0 on Dirichlet faces.  With no Dirichlet axis K is singular (the
    constants); then the charge's mean is removed and the zero-mean solution
    (sum M phi = 0) is taken, by a bordered sparse direct solve."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    K = stiffness(mesh).tocsc()
    M = mesh.mass()
    s = np.asarray(s, dtype=np.float64)
    if 0 in mesh.bc:
        return sla.spsolve(K, 4.0 * np.pi * M * s)
    s0 = s - (M @ s) / M.sum()
    A = sp.bmat([[K, sp.csc_matrix(M[:, None])], [sp.csc_matrix(M[None, :]), None]], format="csc")
    sol = sla.spsolve(A, np.concatenate([4.0 * np.pi * M * s0, [0.0]]))
    return sol[:-1]


def cpd_constrained(mesh: Mesh, z_lo: float, z_hi: float) -> np.ndarray:
    """Free nodes inside the conductor regions of the constrained-potential
    setup (Sec. 2.2.2): Omega_0 = {z <= z_lo}, Omega_1 = {z >= z_hi}.
    Returns 0 (not constrained), 1 (Omega_0) or 2 (Omega_1) per node."""
    z = mesh.dof_coords()[:, 2]
    return np.where(z <= z_lo, 1, np.where(z >= z_hi, 2, 0))


def poisson_cpd(mesh: Mesh, s: np.ndarray, w: Optional[np.ndarray], z_lo: float, z_hi: float,
                dV: float) -> np.ndarray:
    """Sec. 2.2.2 electrostatics with constrained potential difference:
    K phi = 4 pi M s at the nodes between the conductors, and phi prescribed
    inside them, phi = -w on Omega_0 = {z <= z_lo} and phi = dV - w on
    Omega_1 = {z >= z_hi}, where w = V_loc - V_sm at the nodes (None: 0), so
    that the total potential phi + w is 0 and dV in the two conductors.
    Rows of constrained nodes are replaced by the constraint, the rest is a
    sparse direct solve of the remaining block (data moved to the right-hand
    side)."""
    import scipy.sparse.linalg as sla
    n = mesh.n
    K = stiffness(mesh).tocsr()
    M = mesh.mass()
    s = np.asarray(s, dtype=np.float64)
    w = np.zeros(n) if w is None else np.asarray(w, dtype=np.float64)
    reg = cpd_constrained(mesh, z_lo, z_hi)
    C = reg > 0
    F = ~C
    if not C.any() or not F.any():
        raise ValueError("the conductor regions must hold some nodes and leave some free")
    g = np.where(reg == 2, dV, 0.0) - w
    phi = np.empty(n)
    phi[C] = g[C]
    KF = K[F]
    rhs = 4.0 * np.pi * M[F] * s[F] - KF[:, C] @ g[C]
    phi[F] = sla.spsolve(KF[:, F].tocsc(), rhs)
    return phi


def stiffness(mesh: Mesh):
    """Global stiffness K (no 1/2, unscaled) as scipy CSR."""
    return CSR(lib().or_assemble(C.byref(mesh._m), 0, None, 0.0, 0.0)).to_scipy()


def cheb_coeffs(m: int, a: float, b: float, a0: float = float("nan")):
    al = np.zeros(m); be = np.zeros(m); c = C.c_double(0.0)
    lib().or_cheb_coeffs(m, a, b, a0, al, be, C.byref(c))
    return al, be, c.value


# -------------------------------------------------------- dense steps (numpy)

def lanczos_bounds(op, v0: np.ndarray, k: int = 10):
    """k-step Lanczos with full reorthogonalisation from start vector v0.

    Returns (a0, b, theta): a0 = smallest Ritz value, b = largest Ritz value
    + |beta_k| (an upper bound of the spectrum, Zhou & Li 2011), theta all
    Ritz values.  `op(v)` applies the operator to a vector.
    """
    n = v0.size
    Q = np.zeros((n, k + 1))
    alpha = np.zeros(k); beta = np.zeros(k)
    Q[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(k):
        w = op(Q[:, j])
        alpha[j] = Q[:, j] @ w
        w = w - Q[:, : j + 1] @ (Q[:, : j + 1].T @ w)
        w = w - Q[:, : j + 1] @ (Q[:, : j + 1].T @ w)
        beta[j] = np.linalg.norm(w)
        if beta[j] == 0.0:
            k = j + 1
            break
        Q[:, j + 1] = w / beta[j]
    T = np.diag(alpha[:k]) + np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1)
    theta = np.linalg.eigvalsh(T)
    return float(theta[0]), float(theta[-1] + abs(beta[k - 1])), theta


def weyl_cut(a0: float, b: float, N: int, n: int) -> float:
    """First cut a = a0 + (b - a0) (N/n)^(2/3): a Weyl-law guess of lambda_N."""
    return a0 + (b - a0) * (N / n) ** (2.0 / 3.0)


def cholqr2(Y: np.ndarray):
    """Two passes of Cholesky-QR: Q = Y R^-1 with Q^H Q = I (real or complex
    blocks; for real ones the conjugations are the identity)."""
    Q = Y
    R = np.eye(Y.shape[1], dtype=Y.dtype)
    for _ in range(2):
        S = Q.conj().T @ Q
        Rk = np.linalg.cholesky(S).conj().T   # S = Rk^H Rk
        Q = np.linalg.solve(Rk.T, Q.T).T      # Q Rk^-1
        R = Rk @ R
    return Q, R


def rayleigh_ritz(apply, Q: np.ndarray):
    """Ritz values/vectors of the operator on span(Q) (Q orthonormal, real or
    complex): the Hermitian part of Q^H A Q."""
    P = apply(Q)
    Hs = Q.conj().T @ P
    Hs = 0.5 * (Hs + Hs.conj().T)
    theta, W = np.linalg.eigh(Hs)
    return theta, Q @ W


def subspace_iteration(op, X0: np.ndarray, m: int, iters: int, a: float, b: float, a0: float):
    """Chebyshev-filtered subspace iteration: filter, CholQR2, Rayleigh-Ritz;
    the cut a and the scaling point a0 follow the current Ritz values.  op is
    an Operator, or a BlochOperator with complex X0."""
    X = X0
    hist = []
    for _ in range(iters):
        Y = op.filter(X, m, a, b, a0)
        Q, _ = cholqr2(Y)
        theta, X = rayleigh_ritz(op.apply, Q)
        hist.append(theta)
        a, a0 = float(theta[-1]), float(theta[0])
    return hist, X


def chebyshev_T(m: int, t: np.ndarray) -> np.ndarray:
    """T_m(t) from the closed forms cos(m acos t) (|t|<=1) and
    sign(t)^m cosh(m acosh |t|) (|t|>1)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(m * np.arccos(t[inside]))
    ti = t[~inside]
    out[~inside] = np.sign(ti) ** m * np.cosh(m * np.arccosh(np.abs(ti)))
    return out
