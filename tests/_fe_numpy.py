"""Independent numpy routes used to pin the oracle (test helpers only).

Everything here is computed a different way from the oracle: nodes from
numpy's Legendre-series routines, basis functions as exact numpy polynomials,
integrals by exact antiderivatives, and 3-D operators from Kronecker products
of 1-D global matrices assembled here.
"""
import numpy as np
from numpy.polynomial import Polynomial
from numpy.polynomial import legendre as npleg

DIRICHLET, PERIODIC, NEUMANN = 0, 1, 2


def gll_numpy(p):
    """GLL nodes: -1, +1 and the roots of d/dx P_p from numpy's Legendre
    series; weights 2/(p(p+1) P_p(x)^2)."""
    c = np.zeros(p + 1); c[p] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(c)))) if p > 1 else np.array([])
    x = np.concatenate([[-1.0], inner, [1.0]])
    Pp = npleg.legval(x, c)
    return x, 2.0 / (p * (p + 1) * Pp ** 2)


def lagrange_polys(x):
    out = []
    for i in range(len(x)):
        others = np.delete(x, i)
        P = Polynomial.fromroots(others)
        out.append(P / P(x[i]))
    return out


def integ(P, lo=-1.0, hi=1.0):
    Q = P.integ()
    return Q(hi) - Q(lo)


def ref_matrices(p):
    """Exact 1-D reference stiffness and consistent mass on [-1,1]."""
    x, w = gll_numpy(p)
    ls = lagrange_polys(x)
    K = np.array([[integ(a.deriv() * b.deriv()) for b in ls] for a in ls])
    Mc = np.array([[integ(a * b) for b in ls] for a in ls])
    return K, Mc, np.diag(w), x, w


def cell_stiffness_kron(p, rule, h):
    """(h/2)[Kx My Mz + Mx Ky Mz + Mx My Kz] with local index i + n1 (j + n1 k)."""
    K, Mc, Ml, _, _ = ref_matrices(p)
    M = Mc if rule == 0 else Ml
    kron3 = lambda a, b, c: np.kron(c, np.kron(b, a))  # a acts on x (fastest)
    return 0.5 * h * (kron3(K, M, M) + kron3(M, K, M) + kron3(M, M, K))


def global_1d(ncell, p, h, bc, rule):
    """Assembled 1-D stiffness (2/h) K^, mass (h/2) M^ and lumped mass on the
    free nodes of one axis; plus the free-node coordinates."""
    K, Mc, Ml, x, w = ref_matrices(p)
    nn = ncell * p + 1
    Kg = np.zeros((nn, nn)); Mg = np.zeros((nn, nn)); Lg = np.zeros(nn)
    for c in range(ncell):
        s = slice(c * p, c * p + p + 1)
        Kg[s, s] += (2.0 / h) * K
        Mg[s, s] += (0.5 * h) * (Mc if rule == 0 else Ml)
        Lg[s] += 0.5 * h * w
    coords = np.concatenate([c * h + 0.5 * h * (x[:-1] + 1.0) for c in range(ncell)] + [[ncell * h]])
    if bc == PERIODIC:
        Kg[0, :] += Kg[-1, :]; Kg[:, 0] += Kg[:, -1]
        Mg[0, :] += Mg[-1, :]; Mg[:, 0] += Mg[:, -1]
        Lg[0] += Lg[-1]
        keep = np.arange(nn - 1)
    elif bc == DIRICHLET:
        keep = np.arange(1, nn - 1)
    else:
        keep = np.arange(nn)
    return Kg[np.ix_(keep, keep)], Mg[np.ix_(keep, keep)], Lg[keep], coords[keep]
