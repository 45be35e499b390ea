/*
 * Host sanitizer driver for the oracle's C code (test infrastructure).
 *
 * Compiled together with oracle/oracle.c (included below, one translation
 * unit) under AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py, it calls every exported routine on small meshes
 * of every boundary-condition kind and degree 1..7, so that an out-of-bounds
 * access, a use after free, a leak or undefined arithmetic in any of them
 * stops the run with a report.  The values are not checked here (the pinned
 * oracle tests do that); the driver only has to reach every code path.
 */
#include "../../oracle/oracle.c"

#include <stdio.h>

static double frand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0 - 0.5;
}

static void one_d(void) {
    for (int p = 1; p <= 7; ++p) {
        double xi[16], w[16], l[16], dl[16];
        if (or_gll(p, xi, w)) abort();
        if (or_gauss(p + 1, xi, w)) abort();
        for (int t = 0; t <= 4; ++t) or_lagrange_eval(p, -1.0 + 0.5 * t, l, dl);
        const int nc = (p + 1) * (p + 1) * (p + 1);
        double *K = malloc(sizeof(double) * nc * nc), *G = malloc(sizeof(double) * nc * nc);
        for (int rule = 0; rule < 2; ++rule) {
            if (or_cell_stiffness(p, rule, 1.0, K)) abort();
            for (int axis = 0; axis < 3; ++axis)
                if (or_cell_advection(p, rule, 1.0, axis, G)) abort();
        }
        free(K); free(G);
    }
}

static void mesh_case(int p, const int bc[3], const int ncell[3], unsigned seed) {
    or_mesh m;
    for (int a = 0; a < 3; ++a) { m.ncell[a] = ncell[a]; m.L[a] = ncell[a]; m.bc[a] = bc[a]; }
    m.p = p;
    m.rule = 0;
    const int nc = (p + 1) * (p + 1) * (p + 1);
    const int64_t cells = (int64_t)ncell[0] * ncell[1] * ncell[2];
    const int64_t n = or_n_free(&m);
    int64_t *map = malloc(sizeof(int64_t) * cells * nc);
    double *pts = malloc(sizeof(double) * cells * nc * 3), *M = malloc(sizeof(double) * n);
    double *xyz = malloc(sizeof(double) * n * 3), *Vq = malloc(sizeof(double) * cells * nc);
    or_cell_dofs(&m, map);
    or_quad_points(&m, pts);
    or_mass(&m, M);
    or_dof_coords(&m, xyz);
    for (int64_t i = 0; i < cells * nc; ++i) Vq[i] = frand(&seed);

    or_csr *K = or_assemble(&m, 0, NULL, 0.0, 0.0);
    or_csr *H = or_assemble(&m, 1, Vq, 0.01, 0.5 * m.L[2]);
    if (!K || !H) abort();
    {
        const int64_t nnz = or_csr_nnz(H);
        int64_t *rp = malloc(sizeof(int64_t) * (or_csr_n(H) + 1));
        int32_t *col = malloc(sizeof(int32_t) * nnz);
        double *val = malloc(sizeof(double) * nnz);
        or_csr_export(H, rp, col, val);
        free(rp); free(col); free(val);
    }
    const double centres[6] = {0.3 * m.L[0], 0.5 * m.L[1], 0.5 * m.L[2], 0.9 * m.L[0], 0.1 * m.L[1], 0.2 * m.L[2]};
    or_csc *C = or_projectors(&m, 2, centres, 1.5, 0.5);
    if (!C) abort();
    double *Dnl = malloc(sizeof(double) * C->nproj);
    for (int64_t j = 0; j < C->nproj; ++j) Dnl[j] = frand(&seed);
    {
        const int64_t nnz = or_csc_nnz(C);
        int64_t *cp = malloc(sizeof(int64_t) * (C->nproj + 1)), *row = malloc(sizeof(int64_t) * (nnz ? nnz : 1));
        double *val = malloc(sizeof(double) * (nnz ? nnz : 1));
        or_csc_export(C, cp, row, val);
        free(cp); free(row); free(val);
    }
    const int64_t N = 3;
    const int mdeg = 4;
    double *X = malloc(sizeof(double) * n * N), *Y = malloc(sizeof(double) * n * N);
    double *Ys = malloc(sizeof(double) * n * N * (mdeg + 1)), *G = malloc(sizeof(double) * n * N);
    double *Xb = malloc(sizeof(double) * n * N), *g = malloc(sizeof(double) * n);
    double *Vb = malloc(sizeof(double) * cells * nc);
    for (int64_t i = 0; i < n * N; ++i) { X[i] = frand(&seed); G[i] = frand(&seed); }
    or_apply(H, C, Dnl, X, Y, N);
    int64_t rows[3] = {0, n / 2, n - 1};
    double *Yr = malloc(sizeof(double) * 3 * N);
    if (or_apply_rows(&m, Vq, 0.01, 0.5 * m.L[2], C, Dnl, rows, 3, X, N, Yr)) abort();
    double alpha[8], beta[8], cs;
    or_cheb_coeffs(mdeg, 1.0, 50.0, -2.0, alpha, beta, &cs);
    or_cheb_coeffs(mdeg, 1.0, 50.0, NAN, alpha, beta, &cs);
    if (or_cheb_filter(H, C, Dnl, X, Y, N, mdeg, 1.0, 50.0, -2.0, Ys)) abort();
    if (or_cheb_filter(H, NULL, NULL, X, Y, N, mdeg, 1.0, 50.0, NAN, NULL)) abort();
    for (int64_t i = 0; i < n; ++i) g[i] = 0.0;
    if (or_cheb_filter_vjp(H, C, Dnl, X, G, N, mdeg, 1.0, 50.0, -2.0, Xb, g)) abort();
    double Eb;
    or_potential_vjp(&m, g, 0.5 * m.L[2], Vb, &Eb);
    or_csr_free(K); or_csr_free(H); or_csc_free(C);
    free(map); free(pts); free(M); free(xyz); free(Vq); free(Dnl);
    free(X); free(Y); free(Ys); free(G); free(Xb); free(g); free(Vb); free(Yr);
}

int main(void) {
    one_d();
    const int bcs[4][3] = {{OR_DIRICHLET, OR_DIRICHLET, OR_DIRICHLET}, {OR_PERIODIC, OR_PERIODIC, OR_DIRICHLET},
                           {OR_NEUMANN, OR_NEUMANN, OR_NEUMANN}, {OR_PERIODIC, OR_DIRICHLET, OR_NEUMANN}};
    const int ncell[3] = {3, 2, 4};
    unsigned seed = 12345u;
    for (int b = 0; b < 4; ++b)
        for (int p = 1; p <= 3; ++p) mesh_case(p, bcs[b], ncell, seed + 17u * (unsigned)(b * 8 + p));
    printf("oracle sanitizer driver: done\n");
    return 0;
}
