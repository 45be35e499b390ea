"""MI355X (gfx950) finite-element Hamiltonian filter for biased slabs.

Thin ctypes binding of ``libfe.so`` (declared in ``include/fe.h``): argument
marshalling only.  Every step of the hot path runs in the library's HIP
kernels; PyTorch provides device memory and the current stream.  The library
must have been built (``python -m paper_2504_00998_amd.build``); importing
the binding without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfe.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EDEVICE, FE_ESTATE, FE_ENOTSUP = range(6)
DIRICHLET, PERIODIC, NEUMANN = 0, 1, 2
RULE_EXACT, RULE_GLL = 0, 1
F64, F32, BF16 = 0, 1, 2
_PREC = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}


class FEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fe status {status}: {msg}")
        self.status = status


class _Desc(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("ncell", C.c_int32 * 3), ("p", C.c_int32),
                ("bc", C.c_int32 * 3), ("k_rule", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libfe.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2504_00998_amd.build`")
    # torch ships its own HIP runtime under the same sonames; loading it first
    # makes libfe.so bind to that one copy, so streams and device pointers
    # are shared with PyTorch.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    sig = {
        "fe_last_error": ([], C.c_char_p),
        "fe_mesh_create": ([C.POINTER(_Desc), C.POINTER(vp)], C.c_int),
        "fe_mesh_destroy": ([vp], C.c_int),
        "fe_mesh_set_kernel": ([vp, i32], C.c_int),
        "fe_mesh_info": ([vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)], C.c_int),
        "fe_mesh_quad_points": ([vp, vp], C.c_int),
        "fe_mesh_dof_coords": ([vp, vp], C.c_int),
        "fe_reference_cell": ([i32, i32, dbl, vp, vp, vp], C.c_int),
        "fe_set_potential": ([vp, vp, dbl, dbl, vp], C.c_int),
        "fe_set_nonlocal": ([vp, i32, vp, vp, dbl, dbl, vp], C.c_int),
        "fe_hx_apply": ([vp, vp, vp, i64, i64, C.c_int, vp], C.c_int),
        "fe_hx_apply_noalloc": ([vp, vp, vp, i64, i64, C.c_int, vp], C.c_int),
        "fe_cheb_filter": ([vp, vp, vp, i64, i64, i32, dbl, dbl, dbl, C.c_int, vp, C.c_size_t, vp], C.c_int),
        "fe_cheb_filter_vjp_work_bytes": ([vp, i64, i32, i32, i32], C.c_size_t),
        "fe_cheb_filter_vjp": ([vp, vp, vp, i64, i64, i32, dbl, dbl, dbl, C.c_int, vp, vp, vp, i32, i32, vp,
                                C.c_size_t, vp], C.c_int),
        "fe_lanczos_bounds": ([vp, vp, i32, C.POINTER(dbl), C.POINTER(dbl), vp], C.c_int),
        "fe_cholqr2": ([vp, vp, i64, i64, vp], C.c_int),
        "fe_rayleigh_ritz": ([vp, vp, vp, vp, i64, i64, vp, vp], C.c_int),
        "fe_density": ([vp, vp, i64, i64, vp, vp, vp], C.c_int),
        "fe_planar_average": ([vp, vp, i32, vp, vp], C.c_int),
        "fe_dipole": ([vp, vp, dbl, C.POINTER(dbl), vp], C.c_int),
        "fe_poisson_work_bytes": ([vp], C.c_size_t),
        "fe_poisson_solve": ([vp, vp, vp, dbl, i32, vp, C.c_size_t, C.POINTER(i32), C.POINTER(dbl), vp], C.c_int),
        "fe_bare_potential_planar": ([vp, vp, vp, vp, vp, vp], C.c_int),
        "fe_poisson_solve_cpd": ([vp, vp, vp, dbl, dbl, dbl, vp, dbl, i32, vp, C.c_size_t, C.POINTER(i32),
                                  C.POINTER(dbl), vp], C.c_int),
        "fe_set_kpoint": ([vp, dbl, dbl], C.c_int),
        "fe_get_kpoint": ([vp, vp], C.c_int),
        "fe_hx_apply_k": ([vp, vp, vp, i64, i64, vp], C.c_int),
        "fe_cheb_filter_k": ([vp, vp, vp, i64, i64, i32, dbl, dbl, dbl, vp, C.c_size_t, vp], C.c_int),
        "fe_cholqr2_k": ([vp, vp, i64, i64, vp], C.c_int),
        "fe_rayleigh_ritz_k": ([vp, vp, vp, vp, i64, i64, vp, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int):
    if status != FE_OK:
        raise FEError(status, lib().fe_last_error().decode())


def reference_cell(p: int, rule: int = RULE_EXACT, h: float = 1.0):
    """(xi, w, A = 1/2 Kc) from the library's host reference element."""
    nc = (p + 1) ** 3
    xi = np.zeros(p + 1); w = np.zeros(p + 1); A = np.zeros(nc * nc)
    _check(lib().fe_reference_cell(p, rule, h, xi.ctypes.data, w.ctypes.data, A.ctypes.data))
    return xi, w, A.reshape(nc, nc)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _check_block(t, n: int, name: str):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 device tensor")
    if t.dim() != 2 or t.shape[0] != n or t.stride(1) != 1:
        raise ValueError(f"{name} must be (n={n}, N) with unit column stride")


def _check_vec(t, n: int, name: str):
    """A contiguous float64 device vector of exactly n values."""
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float64 device tensor of {n} values")


def _work_bytes(t) -> int:
    """Size in bytes of a caller's scratch buffer (any dtype, contiguous, on the device)."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("work must be a contiguous device tensor")
    return t.numel() * t.element_size()


def _check_cblock(t, n: int, name: str):
    import torch
    if t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 device tensor")
    if t.dim() != 2 or t.shape[0] != n or t.stride(1) != 1:
        raise ValueError(f"{name} must be (n={n}, N) with unit column stride")


class Mesh:
    """A structured slab mesh on the current device (fe_mesh_create)."""

    def __init__(self, L: Sequence[float], ncell: Sequence[int], p: int, bc: Sequence[int], rule: int = RULE_EXACT):
        d = _Desc((C.c_double * 3)(*[float(x) for x in L]), (C.c_int32 * 3)(*[int(x) for x in ncell]), int(p),
                  (C.c_int32 * 3)(*[int(x) for x in bc]), int(rule))
        h = C.c_void_p()
        _check(lib().fe_mesh_create(C.byref(d), C.byref(h)))
        self._h = h
        self.L, self.ncell, self.p, self.bc, self.rule = tuple(L), tuple(ncell), int(p), tuple(bc), int(rule)
        n, nce, nc = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().fe_mesh_info(h, C.byref(n), C.byref(nce), C.byref(nc)))
        self.n, self.n_cells, self.nc = n.value, nce.value, nc.value
        # free node positions per axis (Dirichlet faces removed, periodic ends identified)
        self.nf = tuple(int(ncell[a]) * self.p + (1 if bc[a] == NEUMANN else 0 if bc[a] == PERIODIC else -1)
                        for a in range(3))

    @classmethod
    def from_workload(cls, wl, rule: Optional[int] = None) -> "Mesh":
        return cls(wl.L, wl.ncell, wl.p, wl.bc, wl.rule if rule is None else rule)

    def close(self):
        if getattr(self, "_h", None):
            lib().fe_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_kernel(self, variant: int):
        """Step-kernel implementation (``fe_mesh_set_kernel``): 0 = fastest
        measured (default), 1 = one cell x 16 vectors per workgroup, 2-9 =
        the alternatives declared in ``include/fe.h``."""
        _check(lib().fe_mesh_set_kernel(self._h, int(variant)))

    # ------------------------------------------------------------- geometry
    def quad_points(self) -> np.ndarray:
        out = np.zeros(self.n_cells * self.nc * 3)
        _check(lib().fe_mesh_quad_points(self._h, out.ctypes.data))
        return out.reshape(self.n_cells, self.nc, 3)

    def dof_coords(self) -> np.ndarray:
        out = np.zeros(self.n * 3)
        _check(lib().fe_mesh_dof_coords(self._h, out.ctypes.data))
        return out.reshape(self.n, 3)

    # ------------------------------------------------------------ operators
    def set_potential(self, Vq, E: float, z0: float, stream=None):
        """Vq: float64 device tensor [n_cells, n_c] (or None for V_loc = 0)."""
        if Vq is not None:
            import torch
            if Vq.dtype != torch.float64 or not Vq.is_cuda or not Vq.is_contiguous() or Vq.numel() != self.n_cells * self.nc:
                raise ValueError("Vq must be a contiguous float64 device tensor of n_cells*n_c values")
        _check(lib().fe_set_potential(self._h, _ptr(Vq), float(E), float(z0), _stream(stream)))

    def set_nonlocal(self, centres: np.ndarray, D: np.ndarray, r_cut: float, r_g: float, stream=None):
        centres = np.ascontiguousarray(centres, dtype=np.float64)
        D = np.ascontiguousarray(D, dtype=np.float64)
        ns = centres.shape[0] if centres.size else 0
        if ns and D.shape != (ns, 9):
            raise ValueError("D must be (n_site, 9)")
        _check(lib().fe_set_nonlocal(self._h, ns, centres.ctypes.data if ns else None, D.ctypes.data if ns else None,
                                     float(r_cut), float(r_g), _stream(stream)))

    def hx(self, X, Y=None, prec="f64", stream=None):
        import torch
        _check_block(X, self.n, "X")
        N, ld = X.shape[1], X.stride(0)
        if Y is None:
            Y = torch.empty_strided(X.shape, X.stride(), dtype=torch.float64, device=X.device)
        _check_block(Y, self.n, "Y")
        if Y.shape[1] != N or Y.stride(0) != ld:
            raise ValueError("Y must have X's shape and leading dimension")
        _check(lib().fe_hx_apply(self._h, _ptr(X), _ptr(Y), N, ld, _PREC[prec], _stream(stream)))
        return Y

    def hx_noalloc(self, X, Y, prec="f64", stream=None):
        """Y = H~ X through fe_hx_apply_noalloc, which allocates nothing (its
        nonlocal scratch is a static device array): Y must be given."""
        _check_block(X, self.n, "X")
        N, ld = X.shape[1], X.stride(0)
        _check_block(Y, self.n, "Y")
        if Y.shape[1] != N or Y.stride(0) != ld:
            raise ValueError("Y must have X's shape and leading dimension")
        _check(lib().fe_hx_apply_noalloc(self._h, _ptr(X), _ptr(Y), N, ld, _PREC[prec], _stream(stream)))
        return Y

    def cheb_filter(self, X, m: int, a: float, b: float, a0: float = math.nan, prec="f64", Y=None, work=None,
                    stream=None):
        import torch
        _check_block(X, self.n, "X")
        N, ld = X.shape[1], X.stride(0)
        if Y is None:
            Y = torch.empty_strided(X.shape, X.stride(), dtype=torch.float64, device=X.device)
        _check_block(Y, self.n, "Y")
        if Y.shape[1] != N or Y.stride(0) != ld:
            raise ValueError("Y must have X's shape and leading dimension")
        if work is None:
            work = torch.empty(self.n * N, dtype=torch.float64, device=X.device)
        _check(lib().fe_cheb_filter(self._h, _ptr(X), _ptr(Y), N, ld, int(m), float(a), float(b), float(a0),
                                    _PREC[prec], _ptr(work), _work_bytes(work), _stream(stream)))
        return Y

    # --------------------------------------------------------------- Bloch-k
    def set_kpoint(self, kx: float, ky: float):
        """Bloch wave vector of the complex entry points (fe_set_kpoint)."""
        _check(lib().fe_set_kpoint(self._h, float(kx), float(ky)))

    def kpoint(self):
        k = np.zeros(2)
        _check(lib().fe_get_kpoint(self._h, k.ctypes.data))
        return float(k[0]), float(k[1])

    def hx_k(self, X, Y=None, stream=None):
        """Y = H~^k X for a complex128 (n, N) device block (fe_hx_apply_k)."""
        import torch
        _check_cblock(X, self.n, "X")
        N, ld = X.shape[1], X.stride(0)
        if Y is None:
            Y = torch.empty_strided(X.shape, X.stride(), dtype=torch.complex128, device=X.device)
        _check_cblock(Y, self.n, "Y")
        if Y.shape[1] != N or Y.stride(0) != ld:
            raise ValueError("Y must have X's shape and leading dimension")
        _check(lib().fe_hx_apply_k(self._h, _ptr(X), _ptr(Y), N, ld, _stream(stream)))
        return Y

    def cheb_filter_k(self, X, m: int, a: float, b: float, a0: float = math.nan, Y=None, work=None, stream=None):
        """Chebyshev filter with H~^k on a complex128 block (fe_cheb_filter_k)."""
        import torch
        _check_cblock(X, self.n, "X")
        N, ld = X.shape[1], X.stride(0)
        if Y is None:
            Y = torch.empty_strided(X.shape, X.stride(), dtype=torch.complex128, device=X.device)
        _check_cblock(Y, self.n, "Y")
        if Y.shape[1] != N or Y.stride(0) != ld:
            raise ValueError("Y must have X's shape and leading dimension")
        if work is None:
            work = torch.empty(2 * self.n * N, dtype=torch.float64, device=X.device)
        _check(lib().fe_cheb_filter_k(self._h, _ptr(X), _ptr(Y), N, ld, int(m), float(a), float(b), float(a0),
                                      _ptr(work), _work_bytes(work), _stream(stream)))
        return Y

    def cholqr2_k(self, Y, stream=None):
        """Complex CholQR2 in place (fe_cholqr2_k)."""
        _check_cblock(Y, self.n, "Y")
        _check(lib().fe_cholqr2_k(self._h, _ptr(Y), Y.shape[1], Y.stride(0), _stream(stream)))
        return Y

    def rayleigh_ritz_k(self, Q, X=None, P=None, stream=None):
        """(theta, X) of H~^k on span(Q) (fe_rayleigh_ritz_k)."""
        import torch
        _check_cblock(Q, self.n, "Q")
        N, ld = Q.shape[1], Q.stride(0)
        if X is None:
            X = torch.empty_strided(Q.shape, Q.stride(), dtype=torch.complex128, device=Q.device)
        if P is None:
            P = torch.empty_strided(Q.shape, Q.stride(), dtype=torch.complex128, device=Q.device)
        for t, name in ((X, "X"), (P, "P")):
            _check_cblock(t, self.n, name)
            if t.shape[1] != N or t.stride(0) != ld:
                raise ValueError(f"{name} must have Q's shape and leading dimension")
        theta = np.zeros(N)
        _check(lib().fe_rayleigh_ritz_k(self._h, _ptr(Q), _ptr(X), _ptr(P), N, ld, theta.ctypes.data,
                                        _stream(stream)))
        return theta, X

    def vjp_work_bytes(self, N: int, m: int, ckpt_stride: int = 1, col_chunk: int = 0) -> int:
        return int(lib().fe_cheb_filter_vjp_work_bytes(self._h, N, m, ckpt_stride, col_chunk))

    def cheb_filter_vjp(self, X, G, m: int, a: float, b: float, a0: float = math.nan, prec="f64",
                        ckpt_stride: int = 1, col_chunk: int = 0, work=None, stream=None):
        """(Xbar, Vbar_quad [n_cells, n_c], Ebar scalar tensor)."""
        import torch
        _check_block(X, self.n, "X")
        _check_block(G, self.n, "G")
        N, ld = X.shape[1], X.stride(0)
        if G.shape[1] != N or G.stride(0) != ld:
            raise ValueError("G must have X's shape and leading dimension")
        Xb = torch.empty_strided(X.shape, X.stride(), dtype=torch.float64, device=X.device)
        Vb = torch.empty((self.n_cells, self.nc), dtype=torch.float64, device=X.device)
        Eb = torch.empty((), dtype=torch.float64, device=X.device)
        nb = self.vjp_work_bytes(N, m, ckpt_stride, col_chunk)
        if work is None:
            work = torch.empty(max(1, (nb + 7) // 8), dtype=torch.float64, device=X.device)
        _check(lib().fe_cheb_filter_vjp(self._h, _ptr(X), _ptr(G), N, ld, int(m), float(a), float(b), float(a0),
                                        _PREC[prec], _ptr(Xb), _ptr(Vb), _ptr(Eb), int(ckpt_stride), int(col_chunk),
                                        _ptr(work), _work_bytes(work), _stream(stream)))
        return Xb, Vb, Eb

    # ------------------------------------------------------------ observables
    def density(self, X, f, rho=None, stream=None):
        """rho_I = 2 sum_n f_n X[I,n]^2 / M_I at the free nodes (fe_density).
        X: (n, N) float64 device block; f: N float64 device occupations."""
        import torch
        _check_block(X, self.n, "X")
        N, ld = X.shape[1], X.stride(0)
        if f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous() or f.numel() != N:
            raise ValueError("f must be a contiguous float64 device tensor of N values")
        if rho is None:
            rho = torch.empty(self.n, dtype=torch.float64, device=X.device)
        _check_vec(rho, self.n, "rho")
        _check(lib().fe_density(self._h, _ptr(X), N, ld, _ptr(f), _ptr(rho), _stream(stream)))
        return rho

    def density_k(self, X, f, rho=None, stream=None):
        """rho_I = 2 sum_n f_n |u_nk(x_I)|^2 / M_I for the complex Bloch vectors of
        one k-point (the k-point's term of the Brillouin-zone average): the same
        fe_density on the (n, 2N) real view of the interleaved block, each
        occupation applied to the real and the imaginary column."""
        import torch
        _check_cblock(X, self.n, "X")
        if f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous() or f.numel() != X.shape[1]:
            raise ValueError("f must be a contiguous float64 device tensor of N values")
        return self.density(X.view(torch.float64), f.repeat_interleave(2), rho, stream)

    def planar_average(self, field, normalize: bool = False, out=None, stream=None):
        """x-y planar integral (or average) of a nodal field, one value per
        free z node position, ascending z (fe_planar_average)."""
        import torch
        if field.dtype != torch.float64 or not field.is_cuda or not field.is_contiguous() or field.numel() != self.n:
            raise ValueError("field must be a contiguous float64 device tensor of n values")
        if out is None:
            out = torch.empty(self.nf[2], dtype=torch.float64, device=field.device)
        _check_vec(out, int(self.nf[2]), "out")
        _check(lib().fe_planar_average(self._h, _ptr(field), int(bool(normalize)), _ptr(out), _stream(stream)))
        return out

    def bare_potential_planar(self, phi, w=None, vapp=None, out=None, stream=None):
        """Planar average of V_bare = (phi + w) + vapp per free z position,
        ascending z (fe_bare_potential_planar); w = V_loc - V_self and vapp at
        the nodes, None for 0."""
        import torch
        _check_vec(phi, self.n, "phi")
        for t, nm in ((w, "w"), (vapp, "vapp")):
            if t is not None:
                _check_vec(t, self.n, nm)
        if out is None:
            out = torch.empty(self.nf[2], dtype=torch.float64, device=phi.device)
        _check_vec(out, int(self.nf[2]), "out")
        _check(lib().fe_bare_potential_planar(self._h, _ptr(phi), _ptr(w) if w is not None else None,
                                              _ptr(vapp) if vapp is not None else None, _ptr(out), _stream(stream)))
        return out

    def dipole(self, rho, z0: float, stream=None) -> float:
        """Electronic dipole sum_I M_I rho_I (z_I - z0) (fe_dipole)."""
        import torch
        if rho.dtype != torch.float64 or not rho.is_cuda or not rho.is_contiguous() or rho.numel() != self.n:
            raise ValueError("rho must be a contiguous float64 device tensor of n values")
        mu = C.c_double()
        _check(lib().fe_dipole(self._h, _ptr(rho), float(z0), C.byref(mu), _stream(stream)))
        return mu.value

    def poisson(self, charge, tol: float = 1e-12, maxit: int = 100000, phi=None, work=None, stream=None):
        """Electrostatic potential of a nodal charge density on this mesh's
        space and boundary conditions (fe_poisson_solve): K phi = 4 pi M s.
        Returns (phi, iterations, final relative residual)."""
        import torch
        if charge.dtype != torch.float64 or not charge.is_cuda or not charge.is_contiguous() or charge.numel() != self.n:
            raise ValueError("charge must be a contiguous float64 device tensor of n values")
        if phi is None:
            phi = torch.empty(self.n, dtype=torch.float64, device=charge.device)
        _check_vec(phi, self.n, "phi")
        need = int(lib().fe_poisson_work_bytes(self._h))
        if work is None:
            work = torch.empty((need + 7) // 8, dtype=torch.float64, device=charge.device)
        it, rel = C.c_int32(), C.c_double()
        _check(lib().fe_poisson_solve(self._h, _ptr(charge), _ptr(phi), float(tol), int(maxit), _ptr(work),
                                      _work_bytes(work), C.byref(it), C.byref(rel), _stream(stream)))
        return phi, it.value, rel.value

    def poisson_cpd(self, charge, z_lo: float, z_hi: float, dV: float, w=None, tol: float = 1e-12,
                    maxit: int = 100000, phi=None, work=None, stream=None):
        """Electrostatic potential of the constrained-potential-difference
        setup (fe_poisson_solve_cpd): phi + w = 0 for z <= z_lo and dV for
        z >= z_hi (w = V_loc - V_sm at the nodes, None: 0), K phi = 4 pi M s
        between.  Returns (phi, iterations, final relative residual)."""
        import torch
        if charge.dtype != torch.float64 or not charge.is_cuda or not charge.is_contiguous() or charge.numel() != self.n:
            raise ValueError("charge must be a contiguous float64 device tensor of n values")
        if w is not None:
            _check_vec(w, self.n, "w")
        if phi is None:
            phi = torch.empty(self.n, dtype=torch.float64, device=charge.device)
        _check_vec(phi, self.n, "phi")
        need = int(lib().fe_poisson_work_bytes(self._h))
        if work is None:
            work = torch.empty((need + 7) // 8, dtype=torch.float64, device=charge.device)
        it, rel = C.c_int32(), C.c_double()
        _check(lib().fe_poisson_solve_cpd(self._h, _ptr(charge), _ptr(w) if w is not None else None, float(z_lo),
                                          float(z_hi), float(dV), _ptr(phi), float(tol), int(maxit), _ptr(work),
                                          _work_bytes(work), C.byref(it), C.byref(rel), _stream(stream)))
        return phi, it.value, rel.value

    def lanczos_bounds(self, v0, k: int = 10, stream=None):
        """(a0, b): lowest Ritz value and upper spectral bound from k Lanczos
        steps started at the device vector v0 (fe_lanczos_bounds)."""
        _check_vec(v0, self.n, "v0")
        a0, b = C.c_double(), C.c_double()
        _check(lib().fe_lanczos_bounds(self._h, _ptr(v0), int(k), C.byref(a0), C.byref(b), _stream(stream)))
        return a0.value, b.value

    def cholqr2(self, Y, stream=None):
        _check_block(Y, self.n, "Y")
        _check(lib().fe_cholqr2(self._h, _ptr(Y), Y.shape[1], Y.stride(0), _stream(stream)))
        return Y

    def rayleigh_ritz(self, Q, X=None, P=None, stream=None):
        import torch
        _check_block(Q, self.n, "Q")
        N, ld = Q.shape[1], Q.stride(0)
        if X is None:
            X = torch.empty_strided(Q.shape, Q.stride(), dtype=torch.float64, device=Q.device)
        if P is None:
            P = torch.empty_strided(Q.shape, Q.stride(), dtype=torch.float64, device=Q.device)
        for t, name in ((X, "X"), (P, "P")):
            _check_block(t, self.n, name)
            if t.shape[1] != N or t.stride(0) != ld:
                raise ValueError(f"{name} must have Q's shape and leading dimension")
        theta = np.zeros(N)
        _check(lib().fe_rayleigh_ritz(self._h, _ptr(Q), _ptr(X), _ptr(P), N, ld, theta.ctypes.data,
                                      _stream(stream)))
        return theta, X


def _autograd_function():
    import torch

    class ChebFilter(torch.autograd.Function):
        """Y = T_m((H~ - c)/e) X / T_m((a0 - c)/e) with H~ built from (V_quad, E).

        Differentiable in X, V_quad ([n_cells, n_c] at the cell GLL points) and
        E (0-dim tensor); the bounds a, b, a0 are held fixed.  forward calls
        fe_set_potential + fe_cheb_filter, backward fe_cheb_filter_vjp.
        """

        @staticmethod
        def forward(ctx, X, Vq, E, mesh, m, a, b, a0=math.nan, prec="f64", z0=0.0, ckpt_stride=1, col_chunk=0):
            ctx.E_tensor = torch.is_tensor(E)
            Ev = float(E.item()) if ctx.E_tensor else float(E)
            mesh.set_potential(Vq.detach().contiguous(), Ev, z0)
            Y = mesh.cheb_filter(X.detach().contiguous(), m, a, b, a0, prec=prec)
            ctx.save_for_backward(X.detach(), Vq.detach())
            ctx.cfg = (mesh, m, a, b, a0, z0, prec, ckpt_stride, col_chunk, Ev)
            return Y

        @staticmethod
        def backward(ctx, G):
            X, Vq = ctx.saved_tensors
            mesh, m, a, b, a0, z0, prec, ckpt_stride, col_chunk, Ev = ctx.cfg
            mesh.set_potential(Vq.contiguous(), Ev, z0)
            Xb, Vb, Eb = mesh.cheb_filter_vjp(X.contiguous(), G.contiguous(), m, a, b, a0, prec=prec,
                                              ckpt_stride=ckpt_stride, col_chunk=col_chunk)
            # dL/dV in the caller's layout of V_quad; no gradient for a plain-number E
            Eb = Eb.reshape(()) if ctx.E_tensor else None
            return Xb, Vb.view_as(Vq), Eb, None, None, None, None, None, None, None, None, None

    return ChebFilter


_CHEB = None


def cheb_filter(X, Vq, E, mesh: "Mesh", m: int, a: float, b: float, a0: float = math.nan, z0: float = 0.0,
                prec="f64", ckpt_stride: int = 1, col_chunk: int = 0):
    """Differentiable Chebyshev filter (see ChebFilter)."""
    global _CHEB
    if _CHEB is None:
        _CHEB = _autograd_function()
    return _CHEB.apply(X, Vq, E, mesh, int(m), float(a), float(b), float(a0), prec, float(z0), int(ckpt_stride),
                       int(col_chunk))


def __getattr__(name):
    """`ChebFilter`, the torch.autograd.Function behind cheb_filter, created on
    first use (so that importing the package does not import torch):
    ChebFilter.apply(X, Vq, E, mesh, m, a, b[, a0, prec, z0, ckpt_stride,
    col_chunk])."""
    global _CHEB
    if name == "ChebFilter":
        if _CHEB is None:
            _CHEB = _autograd_function()
        return _CHEB
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
