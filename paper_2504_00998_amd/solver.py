"""Chebyshev-filtered subspace iteration on the device.

Each iteration: filter the block (fe_cheb_filter, cell products in the chosen
precision), orthonormalise it (fe_cholqr2, FP64), and take Rayleigh-Ritz
values and vectors (fe_rayleigh_ritz, FP64 products).  The cut a follows the
largest Ritz value of the block and the scaling point a0 the smallest; the
upper bound b comes from Lanczos once.  This is the eigensolver step of the
discrete problem H u = eps M u (paper Sec. 2.3), in the form of Zhou, Saad,
Tiago and Chelikowsky (2006); everything runs through the C ABI.
"""
from __future__ import annotations

import math
from typing import List, Optional, Tuple

import numpy as np


def spectrum_bounds(mesh, v0, k: int = 10) -> Tuple[float, float]:
    """(a0, b) from k-step Lanczos on the device."""
    return mesh.lanczos_bounds(v0, k)


def weyl_cut(a0: float, b: float, N: int, n: int) -> float:
    """First cut a = a0 + (b - a0)(N/n)^(2/3), a Weyl-law guess of lambda_N."""
    return a0 + (b - a0) * (N / n) ** (2.0 / 3.0)


def subspace_iteration(mesh, X0, m: int, iters: int, a: float, b: float, a0: float, prec: str = "f64",
                       work=None) -> Tuple[List[np.ndarray], "object"]:
    """Run `iters` filtered subspace iterations from X0 (device, n x N).

    Returns the Ritz values of every iteration (host arrays) and the final
    Ritz vectors (device).  X0 is not modified.
    """
    import torch
    X = X0.clone()
    Y = torch.empty_like(X)
    P = torch.empty_like(X)
    if work is None:
        work = torch.empty(X.numel(), dtype=torch.float64, device=X.device)
    hist = []
    for _ in range(iters):
        mesh.cheb_filter(X, m, a, b, a0, prec=prec, Y=Y, work=work)
        mesh.cholqr2(Y)
        theta, X = mesh.rayleigh_ritz(Y, X=X, P=P)
        hist.append(theta)
        a, a0 = float(theta[-1]), float(theta[0])
    return hist, X


def subspace_iteration_k(mesh, X0, m: int, iters: int, a: float, b: float, a0: float,
                         work=None) -> Tuple[List[np.ndarray], "object"]:
    """Filtered subspace iteration with the Bloch operator H~^k at the mesh's
    current wave vector (fe_set_kpoint): complex filter, complex CholQR2 and
    Rayleigh-Ritz, all on the device.  X0: complex128 (n, N) device block,
    not modified.  Returns the Ritz values of every iteration and the final
    Ritz vectors."""
    import torch
    X = X0.clone()
    Y = torch.empty_like(X)
    P = torch.empty_like(X)
    if work is None:
        work = torch.empty(2 * X.numel(), dtype=torch.float64, device=X.device)
    hist = []
    for _ in range(iters):
        mesh.cheb_filter_k(X, m, a, b, a0, Y=Y, work=work)
        mesh.cholqr2_k(Y)
        theta, X = mesh.rayleigh_ritz_k(Y, X=X, P=P)
        hist.append(theta)
        a, a0 = float(theta[-1]), float(theta[0])
    return hist, X


def ground_state(mesh, Vq, E: float, z0: float, X0, v0, m: int, iters: int, prec: str = "f64", work=None,
                 profile_q=None):
    """Set the potential (V_loc at the GLL points, field E about z0), bound the
    spectrum by Lanczos from v0, and run `iters` filtered subspace iterations
    from X0.  Returns (Ritz values of the last iteration, Ritz vectors).

    profile_q: optional field shape per unit E at the GLL points (e.g. the
    sawtooth of workloads.sawtooth divided by E); the field then enters as
    V_loc + E profile instead of the linear -E (z - z0)."""
    if profile_q is None:
        mesh.set_potential(Vq, E, z0)
    else:
        mesh.set_potential(Vq + E * profile_q, 0.0, z0)
    a0, b = spectrum_bounds(mesh, v0)
    a = weyl_cut(a0, b, X0.shape[1], mesh.n)
    hist, X = subspace_iteration(mesh, X0, m, iters, a, b, a0, prec=prec, work=work)
    return hist[-1], X


def polarizability(mesh, Vq, E: float, dE: float, z0: float, X0, v0, f, m: int, iters: int, prec: str = "f64",
                   profile_q=None):
    """Electronic response of the slab to the field (Sec. 3.1): ground states
    at E - dE and E + dE, densities (fe_density) with occupations f, dipoles
    about z0 (fe_dipole); alpha_z = (mu(E+dE) - mu(E-dE)) / (2 dE).  Also the
    band energy 2 sum f eps at both fields, whose central difference is the
    Hellmann-Feynman derivative -mu (for the linear field).  Returns a dict of
    host scalars.  profile_q: as in ground_state."""
    import torch
    f = torch.as_tensor(f, dtype=torch.float64, device=X0.device)
    out = {}
    for tag, e in (("minus", E - dE), ("plus", E + dE)):
        theta, X = ground_state(mesh, Vq, e, z0, X0, v0, m, iters, prec=prec, profile_q=profile_q)
        rho = mesh.density(X, f)
        out["mu_" + tag] = mesh.dipole(rho, z0)
        out["eband_" + tag] = 2.0 * float((f.cpu().numpy() * theta).sum())
    out["alpha"] = (out["mu_plus"] - out["mu_minus"]) / (2.0 * dE)
    out["deband_dE"] = (out["eband_plus"] - out["eband_minus"]) / (2.0 * dE)
    out["mu_mid"] = 0.5 * (out["mu_plus"] + out["mu_minus"])
    return out
