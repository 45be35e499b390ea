/*
 * oracle.c -- plain FP64 CPU oracle for the Chebyshev-filtered finite-element
 * Kohn-Sham Hamiltonian of a biased slab.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  It shares no code, header, table or
 * constant generator with the library, and only tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.
 *
 * What it computes, in the paper's terms:
 *   - the C0 Lagrange basis on Gauss-Lobatto-Legendre nodes of degree p
 *     (Sec. 2.3, FE discretization);
 *   - the stiffness K_IJ = int grad N_I . grad N_J (Sec. 2.3), the GLL-lumped
 *     overlap M, and the local Hamiltonian H = 1/2 K + V with the effective
 *     potential V_eff + V_app sampled at the GLL points (Sec. 2.1, Eq. for
 *     H_loc and V_eff; Sec. 2.2.1, V_app with slope -E);
 *   - the symmetric standard form H~ = M^-1/2 H M^-1/2 of the generalised
 *     problem H u = eps M u (Sec. 2.3), assembled as a global CSR matrix;
 *   - the separable nonlocal term sum_a sum_beta p_beta D_beta <p_beta, .>
 *     (Sec. 2.1, Eq. V_nloc) as a rank-n_proj update with collocated
 *     projector coefficients;
 *   - the Chebyshev filter Y = T_m((H~ - c)/e) X by the three-term recurrence,
 *     scaled (Zhou, Saad, Tiago, Chelikowsky 2006) or unscaled, applied by
 *     sparse matrix products;
 *   - the reverse-mode derivative of that filter.
 *
 * Everything is written out from its definition, with no blocking, fusion or
 * reordering beyond what the definition states.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_DIRICHLET 0
#define OR_PERIODIC 1
#define OR_NEUMANN 2

/* ------------------------------------------------------------------ 1-D */

/* Legendre P_n(x) and P_n'(x) by Bonnet's recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; the derivative from
 * P_n' = sum over the same recurrence differentiated:
 * (k+1) P'_{k+1} = (2k+1) (P_k + x P'_k) - k P'_{k-1}. */
static void legendre(int n, double x, double *P, double *dP) {
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = ((2.0 * k + 1.0) * (p1 + x * d1) - k * d0) / (k + 1.0);
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *P = p1; *dP = d1;
}

/* Second derivative from Legendre's equation (1-x^2) P'' - 2x P' + n(n+1) P = 0
 * (valid for |x| < 1, where the interior GLL nodes lie). */
static double legendre_dd(int n, double x, double P, double dP) {
    return (2.0 * x * dP - n * (n + 1.0) * P) / (1.0 - x * x);
}

/* GLL rule of degree p: p+1 nodes, xi_0 = -1, xi_p = +1, interior nodes the
 * roots of P_p', weights w_i = 2 / (p (p+1) P_p(xi_i)^2). */
int or_gll(int p, double *xi, double *w) {
    if (p < 1) return -1;
    xi[0] = -1.0; xi[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double x = -cos(M_PI * i / p); /* Chebyshev-Gauss-Lobatto start */
        for (int it = 0; it < 100; ++it) {
            double P, dP; legendre(p, x, &P, &dP);
            double ddP = legendre_dd(p, x, P, dP);
            double dx = dP / ddP;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i <= p; ++i) {
        double P, dP; legendre(p, xi[i], &P, &dP);
        w[i] = 2.0 / (p * (p + 1.0) * P * P);
    }
    return 0;
}

/* Gauss-Legendre rule with q points: roots of P_q, w = 2 / ((1-x^2) P_q'(x)^2). */
int or_gauss(int q, double *x, double *w) {
    if (q < 1) return -1;
    for (int i = 0; i < q; ++i) {
        double t = -cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP; legendre(q, t, &P, &dP);
            double dt = P / dP;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        double P, dP; legendre(q, t, &P, &dP);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
    }
    return 0;
}

/* Lagrange basis l_i on the nodes xi[0..p] and its derivative at x, from the
 * product definitions l_i(x) = prod_{j!=i} (x - xi_j)/(xi_i - xi_j) and
 * l_i'(x) = sum_{k!=i} 1/(xi_i - xi_k) prod_{j!=i,k} (x - xi_j)/(xi_i - xi_j). */
static void lagrange(int p, const double *xi, double x, double *l, double *dl) {
    for (int i = 0; i <= p; ++i) {
        double v = 1.0, d = 0.0;
        for (int j = 0; j <= p; ++j) if (j != i) v *= (x - xi[j]) / (xi[i] - xi[j]);
        for (int k = 0; k <= p; ++k) {
            if (k == i) continue;
            double t = 1.0 / (xi[i] - xi[k]);
            for (int j = 0; j <= p; ++j) if (j != i && j != k) t *= (x - xi[j]) / (xi[i] - xi[j]);
            d += t;
        }
        l[i] = v; dl[i] = d;
    }
}

/* Export of the basis at arbitrary points (for pins). */
void or_lagrange_eval(int p, double x, double *l, double *dl) {
    double xi[16], w[16];
    or_gll(p, xi, w);
    lagrange(p, xi, x, l, dl);
}

/* ---------------------------------------------------------- cell matrix */

/* Stiffness of one cubic cell of edge h,
 *   Kc[l][l'] = int_cell grad N_l . grad N_l',
 * local index l = i + (p+1) (j + (p+1) k), i along x.
 * rule 0 ("exact"): tensor Gauss-Legendre quadrature with p+2 points per
 *                   axis, exact for the degree-2p integrand;
 * rule 1 ("gll")  : the (p+1)^3 GLL points collocated with the nodes.
 * The reference map x = x_c + (h/2)(xi+1) gives grad = (2/h) grad_xi and
 * dx = (h/2)^3 dxi. */
int or_cell_stiffness(int p, int rule, double h, double *Kc) {
    int n1 = p + 1, nc = n1 * n1 * n1;
    double xi[16], wg[16], qx[16], qw[16];
    int nq;
    or_gll(p, xi, wg);
    if (rule == 0) { nq = p + 2; or_gauss(nq, qx, qw); }
    else if (rule == 1) { nq = p + 1; memcpy(qx, xi, sizeof(double) * n1); memcpy(qw, wg, sizeof(double) * n1); }
    else return -1;
    double *L = malloc(sizeof(double) * nq * n1), *dL = malloc(sizeof(double) * nq * n1);
    for (int q = 0; q < nq; ++q) lagrange(p, xi, qx[q], L + q * n1, dL + q * n1);
    double s = 2.0 / h, jac = (h / 2.0) * (h / 2.0) * (h / 2.0);
    memset(Kc, 0, sizeof(double) * nc * nc);
    for (int qz = 0; qz < nq; ++qz)
    for (int qy = 0; qy < nq; ++qy)
    for (int qx_ = 0; qx_ < nq; ++qx_) {
        double wq = qw[qx_] * qw[qy] * qw[qz] * jac;
        for (int l = 0; l < nc; ++l) {
            int i = l % n1, j = (l / n1) % n1, k = l / (n1 * n1);
            double gx = s * dL[qx_ * n1 + i] * L[qy * n1 + j] * L[qz * n1 + k];
            double gy = s * L[qx_ * n1 + i] * dL[qy * n1 + j] * L[qz * n1 + k];
            double gz = s * L[qx_ * n1 + i] * L[qy * n1 + j] * dL[qz * n1 + k];
            for (int lp = 0; lp < nc; ++lp) {
                int ip = lp % n1, jp = (lp / n1) % n1, kp = lp / (n1 * n1);
                double hx = s * dL[qx_ * n1 + ip] * L[qy * n1 + jp] * L[qz * n1 + kp];
                double hy = s * L[qx_ * n1 + ip] * dL[qy * n1 + jp] * L[qz * n1 + kp];
                double hz = s * L[qx_ * n1 + ip] * L[qy * n1 + jp] * dL[qz * n1 + kp];
                Kc[(size_t)l * nc + lp] += wq * (gx * hx + gy * hy + gz * hz);
            }
        }
    }
    free(L); free(dL);
    return 0;
}

/* Cell advection matrix along axis a (0, 1, 2): G[l][l'] = int_c N_l dN_l'/dx_a
 * over a cube of edge h, by the same direct 3-D Gauss quadrature (exact rule,
 * p+2 points) or the GLL rule (rule 1).  The Bloch-k term of the Hamiltonian
 * (the -i k.grad part of (-i grad + k)^2 / 2) is assembled from these. */
int or_cell_advection(int p, int rule, double h, int axis, double *Gc) {
    int n1 = p + 1, nc = n1 * n1 * n1;
    double xi[16], wg[16], qx[16], qw[16];
    int nq;
    if (axis < 0 || axis > 2) return -1;
    or_gll(p, xi, wg);
    if (rule == 0) { nq = p + 2; or_gauss(nq, qx, qw); }
    else if (rule == 1) { nq = p + 1; memcpy(qx, xi, sizeof(double) * n1); memcpy(qw, wg, sizeof(double) * n1); }
    else return -1;
    double *L = malloc(sizeof(double) * nq * n1), *dL = malloc(sizeof(double) * nq * n1);
    for (int q = 0; q < nq; ++q) lagrange(p, xi, qx[q], L + q * n1, dL + q * n1);
    double s = 2.0 / h, jac = (h / 2.0) * (h / 2.0) * (h / 2.0);
    memset(Gc, 0, sizeof(double) * nc * nc);
    for (int qz = 0; qz < nq; ++qz)
    for (int qy = 0; qy < nq; ++qy)
    for (int qx_ = 0; qx_ < nq; ++qx_) {
        double wq = qw[qx_] * qw[qy] * qw[qz] * jac;
        int q3[3] = {qx_, qy, qz};
        for (int l = 0; l < nc; ++l) {
            int il[3] = {l % n1, (l / n1) % n1, l / (n1 * n1)};
            double v = L[q3[0] * n1 + il[0]] * L[q3[1] * n1 + il[1]] * L[q3[2] * n1 + il[2]];
            for (int lp = 0; lp < nc; ++lp) {
                int ip[3] = {lp % n1, (lp / n1) % n1, lp / (n1 * n1)};
                double g = s;
                for (int a = 0; a < 3; ++a)
                    g *= (a == axis) ? dL[q3[a] * n1 + ip[a]] : L[q3[a] * n1 + ip[a]];
                Gc[(size_t)l * nc + lp] += wq * v * g;
            }
        }
    }
    free(L); free(dL);
    return 0;
}

/* ----------------------------------------------------------------- mesh */

typedef struct {
    double L[3];
    int ncell[3];
    int p;
    int bc[3];
    int rule;
} or_mesh;

/* Number of distinct node positions along an axis and free-DoF count. */
static int64_t axis_free(const or_mesh *m, int a) {
    int64_t k = (int64_t)m->ncell[a] * m->p;
    if (m->bc[a] == OR_DIRICHLET) return k - 1;
    if (m->bc[a] == OR_PERIODIC) return k;
    return k + 1;
}

int64_t or_n_free(const or_mesh *m) {
    return axis_free(m, 0) * axis_free(m, 1) * axis_free(m, 2);
}

/* Free index of global node position g in [0, ncell*p] along axis a, or -1
 * for a Dirichlet node.  Periodic axes identify g = ncell*p with g = 0. */
static int64_t axis_index(const or_mesh *m, int a, int64_t g) {
    int64_t k = (int64_t)m->ncell[a] * m->p;
    if (m->bc[a] == OR_DIRICHLET) return (g == 0 || g == k) ? -1 : g - 1;
    if (m->bc[a] == OR_PERIODIC) return g % k;
    return g;
}

/* Global node position of free index t along axis a (inverse of axis_index). */
static int64_t axis_node(const or_mesh *m, int a, int64_t t) {
    return m->bc[a] == OR_DIRICHLET ? t + 1 : t;
}

/* Coordinate of the node with local GLL index i in cell c along axis a. */
static double node_coord(const or_mesh *m, int a, int c, int i, const double *xi) {
    double h = m->L[a] / m->ncell[a];
    return c * h + 0.5 * h * (xi[i] + 1.0);
}

/* Free-DoF index (x fastest, z slowest) of local node (i,j,k) of cell
 * (cx,cy,cz), or -1 if the node is on a Dirichlet face. */
static int64_t dof_of(const or_mesh *m, int cx, int cy, int cz, int i, int j, int k) {
    int64_t ix = axis_index(m, 0, (int64_t)cx * m->p + i);
    int64_t iy = axis_index(m, 1, (int64_t)cy * m->p + j);
    int64_t iz = axis_index(m, 2, (int64_t)cz * m->p + k);
    if (ix < 0 || iy < 0 || iz < 0) return -1;
    return ix + axis_free(m, 0) * (iy + axis_free(m, 1) * iz);
}

/* Cell->DoF map: map[c * nc + l], cells lexicographic (x fastest). */
void or_cell_dofs(const or_mesh *m, int64_t *map) {
    int n1 = m->p + 1, nc = n1 * n1 * n1;
    int64_t c = 0;
    for (int cz = 0; cz < m->ncell[2]; ++cz)
    for (int cy = 0; cy < m->ncell[1]; ++cy)
    for (int cx = 0; cx < m->ncell[0]; ++cx, ++c)
        for (int l = 0; l < nc; ++l)
            map[c * nc + l] = dof_of(m, cx, cy, cz, l % n1, (l / n1) % n1, l / (n1 * n1));
}

/* Coordinates of every cell-local GLL point, pts[(c*nc + l)*3 + a]. */
void or_quad_points(const or_mesh *m, double *pts) {
    int n1 = m->p + 1, nc = n1 * n1 * n1;
    double xi[16], w[16];
    or_gll(m->p, xi, w);
    int64_t c = 0;
    for (int cz = 0; cz < m->ncell[2]; ++cz)
    for (int cy = 0; cy < m->ncell[1]; ++cy)
    for (int cx = 0; cx < m->ncell[0]; ++cx, ++c)
        for (int l = 0; l < nc; ++l) {
            double *q = pts + (c * nc + l) * 3;
            q[0] = node_coord(m, 0, cx, l % n1, xi);
            q[1] = node_coord(m, 1, cy, (l / n1) % n1, xi);
            q[2] = node_coord(m, 2, cz, l / (n1 * n1), xi);
        }
}

/* GLL weight of cell-local node l times the Jacobian (h/2)^3:
 * the lumped cell mass (h^3/8) w_i w_j w_k. */
static double cell_mass(const or_mesh *m, const double *w, int l) {
    int n1 = m->p + 1;
    double j = 1.0;
    for (int a = 0; a < 3; ++a) j *= 0.5 * m->L[a] / m->ncell[a];
    return j * w[l % n1] * w[(l / n1) % n1] * w[l / (n1 * n1)];
}

/* Assembled diagonal mass M_I = sum over cells sharing I of the lumped cell mass. */
void or_mass(const or_mesh *m, double *M) {
    int n1 = m->p + 1, nc = n1 * n1 * n1;
    double xi[16], w[16];
    or_gll(m->p, xi, w);
    int64_t n = or_n_free(m);
    memset(M, 0, sizeof(double) * n);
    for (int cz = 0; cz < m->ncell[2]; ++cz)
    for (int cy = 0; cy < m->ncell[1]; ++cy)
    for (int cx = 0; cx < m->ncell[0]; ++cx)
        for (int l = 0; l < nc; ++l) {
            int64_t I = dof_of(m, cx, cy, cz, l % n1, (l / n1) % n1, l / (n1 * n1));
            if (I >= 0) M[I] += cell_mass(m, w, l);
        }
}

/* Coordinates of the free DoFs, xyz[I*3 + a]. */
void or_dof_coords(const or_mesh *m, double *xyz) {
    double xi[16], w[16];
    or_gll(m->p, xi, w);
    int64_t nf[3] = {axis_free(m, 0), axis_free(m, 1), axis_free(m, 2)};
    for (int64_t iz = 0; iz < nf[2]; ++iz)
    for (int64_t iy = 0; iy < nf[1]; ++iy)
    for (int64_t ix = 0; ix < nf[0]; ++ix) {
        int64_t t[3] = {ix, iy, iz};
        double *o = xyz + 3 * (ix + nf[0] * (iy + nf[1] * iz));
        for (int a = 0; a < 3; ++a) {
            int64_t g = axis_node(m, a, t[a]);
            int c = (int)(g / m->p), i = (int)(g % m->p);
            if (c == m->ncell[a]) { c -= 1; i = m->p; }
            o[a] = node_coord(m, a, c, i, xi);
        }
    }
}

/* ----------------------------------------------------------------- CSR */

typedef struct {
    int64_t n;
    int64_t *rowptr;
    int32_t *col;
    double *val;
} or_csr;

void or_csr_free(or_csr *A) {
    if (!A) return;
    free(A->rowptr); free(A->col); free(A->val);
    free(A);
}
int64_t or_csr_n(const or_csr *A) { return A->n; }
int64_t or_csr_nnz(const or_csr *A) { return A->rowptr[A->n]; }
void or_csr_export(const or_csr *A, int64_t *rowptr, int32_t *col, double *val) {
    memcpy(rowptr, A->rowptr, sizeof(int64_t) * (A->n + 1));
    memcpy(col, A->col, sizeof(int32_t) * A->rowptr[A->n]);
    memcpy(val, A->val, sizeof(double) * A->rowptr[A->n]);
}

typedef struct { int64_t j; double v; } entry;
static int entry_cmp(const void *a, const void *b) {
    int64_t x = ((const entry *)a)->j, y = ((const entry *)b)->j;
    return (x > y) - (x < y);
}

/* The cells that contain global node position g along axis a, with the
 * node's local index in each; returns how many (1 or 2). */
static int axis_cells(const or_mesh *m, int a, int64_t g, int *cell, int *loc) {
    int p = m->p, nca = m->ncell[a], k = 0;
    if (g % p != 0) { cell[0] = (int)(g / p); loc[0] = (int)(g % p); return 1; }
    int64_t c = g / p;
    /* as the upper node (local p) of cell c-1 */
    if (c - 1 >= 0) { cell[k] = (int)(c - 1); loc[k] = p; ++k; }
    else if (m->bc[a] == OR_PERIODIC) { cell[k] = nca - 1; loc[k] = p; ++k; }
    /* as the lower node (local 0) of cell c */
    if (c < nca) { cell[k] = (int)c; loc[k] = 0; ++k; }
    return k;
}

/*
 * Entries of one row I of the global matrix assembled from identical cell
 * matrices:
 *   A_IJ = sum_{cells c containing I and J} (alpha Kc + diag(mass_c V_c))[l_c(I), l_c(J)]
 * (before the M^-1/2 scaling), with V_total(x_q) = Vq[c][q] - E (z_q - z0)
 * at the GLL points (Vq may be NULL).  Writes the column/value pairs of
 * every contribution into buf (unsorted, duplicates kept) and returns their
 * number.
 */
static int row_contributions(const or_mesh *m, int64_t I, const double *Kc, double alpha, int with_potential,
                             const double *Vq, double E, double z0, const double *xi, const double *w, entry *buf) {
    int p = m->p, n1 = p + 1, nc = n1 * n1 * n1;
    int64_t nf0 = axis_free(m, 0), nf1 = axis_free(m, 1);
    int64_t t[3] = {I % nf0, (I / nf0) % nf1, I / (nf0 * nf1)};
    int cs[3][2], ls[3][2], nk[3];
    for (int a = 0; a < 3; ++a) nk[a] = axis_cells(m, a, axis_node(m, a, t[a]), cs[a], ls[a]);
    int ne = 0;
    for (int az = 0; az < nk[2]; ++az)
    for (int ay = 0; ay < nk[1]; ++ay)
    for (int ax = 0; ax < nk[0]; ++ax) {
        int cx = cs[0][ax], cy = cs[1][ay], cz = cs[2][az];
        int l = ls[0][ax] + n1 * (ls[1][ay] + n1 * ls[2][az]);
        int64_t cidx = cx + (int64_t)m->ncell[0] * (cy + (int64_t)m->ncell[1] * cz);
        for (int lp = 0; lp < nc; ++lp) {
            int64_t J = dof_of(m, cx, cy, cz, lp % n1, (lp / n1) % n1, lp / (n1 * n1));
            if (J < 0) continue;
            double v = alpha * Kc[(size_t)l * nc + lp];
            if (with_potential && lp == l) {
                double zq = node_coord(m, 2, cz, lp / (n1 * n1), xi);
                double V = (Vq ? Vq[cidx * nc + l] : 0.0) - E * (zq - z0);
                v += cell_mass(m, w, l) * V;
            }
            buf[ne].j = J; buf[ne].v = v; ++ne;
        }
    }
    return ne;
}

/*
 * Assemble a global matrix from identical cell matrices, row by row.
 * kind 0: A = K (stiffness, alpha = 1, no potential, s = 1);
 * kind 1: A = H~ = M^-1/2 (1/2 K + V) M^-1/2 with V the GLL-collocated
 *         potential matrix of V_total, s_I = M_I^-1/2.
 * Dirichlet rows/columns are dropped.  Returns NULL on allocation failure.
 */
or_csr *or_assemble(const or_mesh *m, int kind, const double *Vq, double E, double z0) {
    int p = m->p, n1 = p + 1, nc = n1 * n1 * n1;
    double xi[16], w[16];
    or_gll(p, xi, w);
    double h = m->L[0] / m->ncell[0];
    if (!(fabs(m->L[1] / m->ncell[1] - h) < 1e-12 * h && fabs(m->L[2] / m->ncell[2] - h) < 1e-12 * h))
        return NULL; /* cubic cells only */
    double *Kc = malloc(sizeof(double) * nc * nc);
    if (!Kc) return NULL;
    or_cell_stiffness(p, m->rule, h, Kc);
    double alpha = (kind == 0) ? 1.0 : 0.5;
    int64_t n = or_n_free(m);
    double *M = NULL;
    if (kind == 1) { M = malloc(sizeof(double) * n); or_mass(m, M); }

    /* pass 1: row lengths; pass 2: fill.  Rows are independent. */
    int64_t *rowlen = calloc(n + 1, sizeof(int64_t));
    or_csr *A = calloc(1, sizeof(or_csr));
    A->n = n;
    A->rowptr = malloc(sizeof(int64_t) * (n + 1));
    int maxent = 8 * nc;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            A->rowptr[0] = 0;
            for (int64_t I = 0; I < n; ++I) A->rowptr[I + 1] = A->rowptr[I] + rowlen[I];
            A->col = malloc(sizeof(int32_t) * A->rowptr[n]);
            A->val = malloc(sizeof(double) * A->rowptr[n]);
            if (!A->col || !A->val) { free(rowlen); free(Kc); free(M); or_csr_free(A); return NULL; }
        }
        #pragma omp parallel
        {
            entry *buf = malloc(sizeof(entry) * maxent);
            #pragma omp for schedule(dynamic, 256)
            for (int64_t I = 0; I < n; ++I) {
                int ne = row_contributions(m, I, Kc, alpha, kind == 1, Vq, E, z0, xi, w, buf);
                qsort(buf, ne, sizeof(entry), entry_cmp);
                int64_t len = 0;
                int64_t base = pass ? A->rowptr[I] : 0;
                for (int e = 0; e < ne; ++e) {
                    if (len > 0 && pass && A->col[base + len - 1] == buf[e].j) {
                        A->val[base + len - 1] += buf[e].v;
                    } else if (len > 0 && !pass && buf[e].j == buf[e - 1].j) {
                        /* duplicate column, counted once */
                    } else {
                        if (pass) { A->col[base + len] = (int32_t)buf[e].j; A->val[base + len] = buf[e].v; }
                        ++len;
                    }
                }
                if (!pass) rowlen[I] = len;
                else if (kind == 1) {
                    for (int64_t e = 0; e < len; ++e)
                        A->val[base + e] /= sqrt(M[I] * M[A->col[base + e]]);
                }
            }
            free(buf);
        }
    }
    free(rowlen); free(Kc); free(M);
    return A;
}

/* ------------------------------------------------ nonlocal (collocated) */

/* Real solid harmonics S_beta(d) for beta = 0..8: s; p_x, p_y, p_z;
 * d_xy, d_yz, d_zx, d_{x^2-y^2}, d_{3z^2-r^2} (unnormalised). */
static double solid_harmonic(int beta, double x, double y, double z) {
    switch (beta) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return y * z;
    case 6: return z * x;
    case 7: return x * x - y * y;
    default: return 3.0 * z * z - (x * x + y * y + z * z);
    }
}

/*
 * Projector coefficients of the separable nonlocal term (Sec. 2.1, Eq. V_nloc):
 *   p_beta(x) = S_beta(x - R) exp(-|x-R|^2 / (2 r_g^2)) [|x-R| < r_cut],
 * minimum image along periodic axes, normalised to unit discrete M-norm
 * sum_I M_I p_beta(x_I)^2 = 1, and carried to the standard form as
 *   C~_{I,(a,beta)} = M_I^{1/2} p_beta(x_I)
 * (collocation: int N_I p_beta ~= M_I p_beta(x_I) under GLL quadrature, then
 * the M^-1/2 similarity).  Stored by projector column (CSC): column 9*s+beta
 * holds the free DoFs of site s inside the cutoff ball, in increasing order.
 */
typedef struct {
    int64_t n, nproj;
    int64_t *colptr;
    int64_t *row;
    double *val;
} or_csc;

void or_csc_free(or_csc *C) {
    if (!C) return;
    free(C->colptr); free(C->row); free(C->val); free(C);
}
int64_t or_csc_nnz(const or_csc *C) { return C->colptr[C->nproj]; }
void or_csc_export(const or_csc *C, int64_t *colptr, int64_t *row, double *val) {
    memcpy(colptr, C->colptr, sizeof(int64_t) * (C->nproj + 1));
    memcpy(row, C->row, sizeof(int64_t) * C->colptr[C->nproj]);
    memcpy(val, C->val, sizeof(double) * C->colptr[C->nproj]);
}

static void site_offset(const or_mesh *m, const double *xyz, const double *R, double *d) {
    for (int a = 0; a < 3; ++a) {
        d[a] = xyz[a] - R[a];
        if (m->bc[a] == OR_PERIODIC) d[a] -= m->L[a] * nearbyint(d[a] / m->L[a]);
    }
}

or_csc *or_projectors(const or_mesh *m, int n_site, const double *centres, double r_cut, double r_g) {
    int64_t n = or_n_free(m);
    double *xyz = malloc(sizeof(double) * 3 * n);
    double *M = malloc(sizeof(double) * n);
    or_dof_coords(m, xyz);
    or_mass(m, M);
    or_csc *C = calloc(1, sizeof(or_csc));
    C->n = n; C->nproj = 9 * (int64_t)n_site;
    C->colptr = calloc(C->nproj + 1, sizeof(int64_t));
    int64_t *cnt = calloc(n_site, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < n_site; ++s) {
        int64_t k = 0;
        for (int64_t I = 0; I < n; ++I) {
            double d[3];
            site_offset(m, xyz + 3 * I, centres + 3 * s, d);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < r_cut * r_cut) ++k;
        }
        cnt[s] = k;
    }
    for (int s = 0; s < n_site; ++s)
        for (int beta = 0; beta < 9; ++beta)
            C->colptr[9 * s + beta + 1] = C->colptr[9 * s + beta] + cnt[s];
    C->row = malloc(sizeof(int64_t) * (C->colptr[C->nproj] + 1));
    C->val = malloc(sizeof(double) * (C->colptr[C->nproj] + 1));
    #pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < n_site; ++s) {
        double nrm[9] = {0};
        int64_t k = 0;
        for (int64_t I = 0; I < n; ++I) {
            double d[3];
            site_offset(m, xyz + 3 * I, centres + 3 * s, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < r_cut * r_cut)) continue;
            double rad = exp(-r2 / (2.0 * r_g * r_g));
            for (int beta = 0; beta < 9; ++beta) {
                int64_t e = C->colptr[9 * s + beta] + k;
                double v = solid_harmonic(beta, d[0], d[1], d[2]) * rad;
                C->row[e] = I;
                C->val[e] = v;
                nrm[beta] += M[I] * v * v;
            }
            ++k;
        }
        for (int beta = 0; beta < 9; ++beta) {
            double sc = nrm[beta] > 0 ? 1.0 / sqrt(nrm[beta]) : 0.0;
            for (int64_t e = C->colptr[9 * s + beta]; e < C->colptr[9 * s + beta + 1]; ++e)
                C->val[e] *= sc * sqrt(M[C->row[e]]);
        }
    }
    free(cnt); free(xyz); free(M);
    return C;
}

/* ------------------------------------------------------------ products */

typedef struct {
    const or_csr *A;
    const or_csc *C;      /* NULL: no nonlocal term */
    const double *Dnl;    /* nproj couplings */
} or_op;

/* Y = (A + C diag(Dnl) C^T) X for a row-major (n x N) block. */
static void op_apply(const or_op *op, const double *X, double *Y, int64_t N) {
    const or_csr *A = op->A;
    int64_t n = A->n;
    #pragma omp parallel for schedule(static)
    for (int64_t I = 0; I < n; ++I) {
        double *y = Y + I * N;
        for (int64_t j = 0; j < N; ++j) y[j] = 0.0;
        for (int64_t e = A->rowptr[I]; e < A->rowptr[I + 1]; ++e) {
            double a = A->val[e];
            const double *x = X + (int64_t)A->col[e] * N;
            for (int64_t j = 0; j < N; ++j) y[j] += a * x[j];
        }
    }
    const or_csc *C = op->C;
    if (C && C->nproj > 0) {
        double *W = calloc(C->nproj * N, sizeof(double));
        /* W = diag(Dnl) C^T X */
        #pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < C->nproj; ++b) {
            for (int64_t e = C->colptr[b]; e < C->colptr[b + 1]; ++e)
                for (int64_t j = 0; j < N; ++j) W[b * N + j] += C->val[e] * X[C->row[e] * N + j];
            for (int64_t j = 0; j < N; ++j) W[b * N + j] *= op->Dnl[b];
        }
        /* Y += C W, serial over projectors so that rows shared by sites add in a fixed order */
        for (int64_t b = 0; b < C->nproj; ++b) {
            #pragma omp parallel for schedule(static)
            for (int64_t e = C->colptr[b]; e < C->colptr[b + 1]; ++e)
                for (int64_t j = 0; j < N; ++j) Y[C->row[e] * N + j] += C->val[e] * W[b * N + j];
        }
        free(W);
    }
}

void or_apply(const or_csr *A, const or_csc *C, const double *Dnl, const double *X, double *Y, int64_t N) {
    or_op op = {A, C, Dnl};
    op_apply(&op, X, Y, N);
}

/*
 * Selected rows of Y = H~ X (plus the nonlocal term when C != NULL), without
 * assembling the whole matrix: each row is summed from its own cell
 * contributions by the same definition as or_assemble (kind 1).  X is the
 * full (n x N) block; Yr receives (nrows x N).  Used where the whole
 * operator is too large to assemble in test time.
 */
int or_apply_rows(const or_mesh *m, const double *Vq, double E, double z0, const or_csc *C, const double *Dnl,
                  const int64_t *rows, int64_t nrows, const double *X, int64_t N, double *Yr) {
    int p = m->p, n1 = p + 1, nc = n1 * n1 * n1;
    double xi[16], w[16];
    or_gll(p, xi, w);
    double h = m->L[0] / m->ncell[0];
    double *Kc = malloc(sizeof(double) * nc * nc);
    if (!Kc) return -2;
    or_cell_stiffness(p, m->rule, h, Kc);
    int64_t n = or_n_free(m);
    double *M = malloc(sizeof(double) * n);
    or_mass(m, M);
    #pragma omp parallel
    {
        entry *buf = malloc(sizeof(entry) * 8 * nc);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t I = rows[r];
            int ne = row_contributions(m, I, Kc, 0.5, 1, Vq, E, z0, xi, w, buf);
            double *y = Yr + r * N;
            for (int64_t j = 0; j < N; ++j) y[j] = 0.0;
            for (int e = 0; e < ne; ++e) {
                double a = buf[e].v / sqrt(M[I] * M[buf[e].j]);
                const double *x = X + buf[e].j * N;
                for (int64_t j = 0; j < N; ++j) y[j] += a * x[j];
            }
        }
        free(buf);
    }
    if (C && C->nproj > 0) {
        /* W = diag(D) C^T X over all projectors, then the selected rows of C W */
        double *W = calloc(C->nproj * N, sizeof(double));
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t b = 0; b < C->nproj; ++b) {
            for (int64_t e = C->colptr[b]; e < C->colptr[b + 1]; ++e)
                for (int64_t j = 0; j < N; ++j) W[b * N + j] += C->val[e] * X[C->row[e] * N + j];
            for (int64_t j = 0; j < N; ++j) W[b * N + j] *= Dnl[b];
        }
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t I = rows[r];
            for (int64_t b = 0; b < C->nproj; ++b) {
                /* the support of a projector is sorted: binary search for I */
                int64_t lo = C->colptr[b], hi = C->colptr[b + 1];
                while (lo < hi) {
                    int64_t mid = (lo + hi) / 2;
                    if (C->row[mid] < I) lo = mid + 1; else hi = mid;
                }
                if (lo < C->colptr[b + 1] && C->row[lo] == I)
                    for (int64_t j = 0; j < N; ++j) Yr[r * N + j] += C->val[lo] * W[b * N + j];
            }
        }
        free(W);
    }
    free(Kc); free(M);
    return 0;
}

/*
 * Recurrence coefficients of the Chebyshev filter on [a, b], e = (b-a)/2,
 * c = (b+a)/2:
 *   Y_1 = alpha_0 (H - c) Y_0,
 *   Y_{k+1} = alpha_k (H - c) Y_k - beta_k Y_{k-1},   k = 1..m-1.
 * Scaled form (a0 given): sigma_1 = e/(a0 - c), sigma_{k+1} = 1/(2/sigma_1 - sigma_k),
 *   alpha_0 = sigma_1/e, alpha_k = 2 sigma_{k+1}/e, beta_k = sigma_k sigma_{k+1},
 * so that Y_m = T_m((H-c)/e) X / T_m((a0-c)/e).
 * Unscaled form (a0 NaN): alpha_0 = 1/e, alpha_k = 2/e, beta_k = 1.
 */
void or_cheb_coeffs(int mdeg, double a, double b, double a0, double *alpha, double *beta, double *cshift) {
    double e = 0.5 * (b - a), c = 0.5 * (b + a);
    *cshift = c;
    if (isnan(a0)) {
        alpha[0] = 1.0 / e; beta[0] = 0.0;
        for (int k = 1; k < mdeg; ++k) { alpha[k] = 2.0 / e; beta[k] = 1.0; }
        return;
    }
    double s1 = e / (a0 - c), s = s1;
    alpha[0] = s1 / e; beta[0] = 0.0;
    for (int k = 1; k < mdeg; ++k) {
        double sn = 1.0 / (2.0 / s1 - s);
        alpha[k] = 2.0 * sn / e;
        beta[k] = s * sn;
        s = sn;
    }
}

/* Y = filter(X).  If Ystore != NULL it receives Y_0..Y_m (each n*N). */
int or_cheb_filter(const or_csr *A, const or_csc *C, const double *Dnl,
                   const double *X, double *Y, int64_t N, int mdeg, double a, double b, double a0,
                   double *Ystore) {
    if (mdeg < 1 || !(a < b)) return -1;
    or_op op = {A, C, Dnl};
    int64_t n = A->n, sz = n * N;
    double *alpha = malloc(sizeof(double) * mdeg), *beta = malloc(sizeof(double) * mdeg), c;
    or_cheb_coeffs(mdeg, a, b, a0, alpha, beta, &c);
    double *prev = malloc(sizeof(double) * sz), *cur = malloc(sizeof(double) * sz), *nxt = malloc(sizeof(double) * sz);
    double *HY = malloc(sizeof(double) * sz);
    if (!prev || !cur || !nxt || !HY) { free(prev); free(cur); free(nxt); free(HY); free(alpha); free(beta); return -2; }
    memcpy(cur, X, sizeof(double) * sz);
    if (Ystore) memcpy(Ystore, X, sizeof(double) * sz);
    for (int k = 0; k < mdeg; ++k) {
        op_apply(&op, cur, HY, N);
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < sz; ++t) {
            double v = alpha[k] * (HY[t] - c * cur[t]);
            if (k > 0) v -= beta[k] * prev[t];
            nxt[t] = v;
        }
        double *tmp = prev; prev = cur; cur = nxt; nxt = tmp;
        if (Ystore) memcpy(Ystore + (size_t)(k + 1) * sz, cur, sizeof(double) * sz);
    }
    memcpy(Y, cur, sizeof(double) * sz);
    free(prev); free(cur); free(nxt); free(HY); free(alpha); free(beta);
    return 0;
}

/*
 * Reverse-mode derivative of the filter for a cotangent G = dL/dY_m.
 * With all forward blocks stored, the adjoint runs k = m-1 .. 0:
 *   Ybar_k     += alpha_k (H - c) Ybar_{k+1}      (H symmetric),
 *   Ybar_{k-1} -= beta_k Ybar_{k+1}               (k >= 1),
 *   g_I        += alpha_k sum_j Ybar_{k+1}[I,j] Y_k[I,j],
 * where g = diag(dL/dH~) is the derivative with respect to the diagonal
 * potential term v of H~.  Returns Xbar = Ybar_0 and g.  The bounds a, b, a0
 * are held fixed.
 */
int or_cheb_filter_vjp(const or_csr *A, const or_csc *C, const double *Dnl,
                       const double *X, const double *G, int64_t N, int mdeg, double a, double b, double a0,
                       double *Xbar, double *g) {
    if (mdeg < 1 || !(a < b)) return -1;
    or_op op = {A, C, Dnl};
    int64_t n = A->n, sz = n * N;
    double *Ys = malloc(sizeof(double) * sz * (mdeg + 1));
    double *tmp = malloc(sizeof(double) * sz);
    double *Yb = calloc(sz * (mdeg + 1), sizeof(double));
    double *HB = malloc(sizeof(double) * sz);
    if (!Ys || !tmp || !Yb || !HB) { free(Ys); free(tmp); free(Yb); free(HB); return -2; }
    or_cheb_filter(A, C, Dnl, X, tmp, N, mdeg, a, b, a0, Ys);
    double *alpha = malloc(sizeof(double) * mdeg), *beta = malloc(sizeof(double) * mdeg), c;
    or_cheb_coeffs(mdeg, a, b, a0, alpha, beta, &c);
    memcpy(Yb + (size_t)mdeg * sz, G, sizeof(double) * sz);
    memset(g, 0, sizeof(double) * n);
    for (int k = mdeg - 1; k >= 0; --k) {
        const double *B1 = Yb + (size_t)(k + 1) * sz;
        const double *Yk = Ys + (size_t)k * sz;
        op_apply(&op, B1, HB, N);
        double *Bk = Yb + (size_t)k * sz;
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < sz; ++t) Bk[t] += alpha[k] * (HB[t] - c * B1[t]);
        if (k >= 1) {
            double *Bm = Yb + (size_t)(k - 1) * sz;
            #pragma omp parallel for schedule(static)
            for (int64_t t = 0; t < sz; ++t) Bm[t] -= beta[k] * B1[t];
        }
        #pragma omp parallel for schedule(static)
        for (int64_t I = 0; I < n; ++I) {
            double s = 0.0;
            for (int64_t j = 0; j < N; ++j) s += B1[I * N + j] * Yk[I * N + j];
            g[I] += alpha[k] * s;
        }
    }
    memcpy(Xbar, Yb, sizeof(double) * sz);
    free(Ys); free(tmp); free(Yb); free(HB); free(alpha); free(beta);
    return 0;
}

/*
 * Chain rule from g = dL/dv (v the diagonal potential term of H~) to the
 * potential at the quadrature points and to the field strength:
 *   v_I = sum_{(c,q) -> I} (mass_{c,q} / M_I) V_{c,q} - E (z_I - z0)
 *   dL/dV_{c,q} = (mass_{c,q} / M_I) g_I   (0 at Dirichlet points),
 *   dL/dE      = -sum_I g_I (z_I - z0).
 */
void or_potential_vjp(const or_mesh *m, const double *g, double z0, double *Vbar, double *Ebar) {
    int n1 = m->p + 1, nc = n1 * n1 * n1;
    double xi[16], w[16];
    or_gll(m->p, xi, w);
    int64_t n = or_n_free(m);
    double *M = malloc(sizeof(double) * n), *xyz = malloc(sizeof(double) * 3 * n);
    or_mass(m, M);
    or_dof_coords(m, xyz);
    int64_t c = 0;
    for (int cz = 0; cz < m->ncell[2]; ++cz)
    for (int cy = 0; cy < m->ncell[1]; ++cy)
    for (int cx = 0; cx < m->ncell[0]; ++cx, ++c)
        for (int l = 0; l < nc; ++l) {
            int64_t I = dof_of(m, cx, cy, cz, l % n1, (l / n1) % n1, l / (n1 * n1));
            Vbar[c * nc + l] = (I >= 0) ? cell_mass(m, w, l) / M[I] * g[I] : 0.0;
        }
    double s = 0.0;
    for (int64_t I = 0; I < n; ++I) s += g[I] * (xyz[3 * I + 2] - z0);
    *Ebar = -s;
    free(M); free(xyz);
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
