/*
 * Host sanitizer driver for the C ABI (test infrastructure).
 *
 * Linked by tests/test_sanitizers.py against a host-only build of the
 * library made with AddressSanitizer and UndefinedBehaviorSanitizer on the
 * host code, it runs the library's host paths that need no GPU: the
 * reference element (GLL rule and cell matrices) for every degree and
 * stiffness rule, and the argument checks of the entry points (bad
 * descriptors, NULL mesh and pointers).  Any out-of-bounds access, leak or
 * undefined arithmetic there stops the run with a report; a wrong status
 * code makes it exit non-zero.
 */
#include "fe.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

static int failures = 0;

static void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "capi driver: unexpected result: %s (last error: %s)\n", what, fe_last_error());
        ++failures;
    }
}

int main() {
    // reference element: every degree and rule, and refused degrees
    for (int p = 1; p <= 7; ++p)
        for (int rule = 0; rule < 2; ++rule) {
            const size_t nc = (size_t)(p + 1) * (p + 1) * (p + 1);
            std::vector<double> xi(p + 1), w(p + 1), A(nc * nc);
            expect(fe_reference_cell(p, rule, 1.0, xi.data(), w.data(), A.data()) == FE_OK, "fe_reference_cell");
            expect(fe_reference_cell(p, rule, 0.5, nullptr, nullptr, A.data()) == FE_OK, "fe_reference_cell A only");
        }
    {
        double A[64];
        expect(fe_reference_cell(0, 0, 1.0, nullptr, nullptr, A) != FE_OK, "p = 0 refused");
        expect(fe_reference_cell(8, 0, 1.0, nullptr, nullptr, A) != FE_OK, "p = 8 refused");
        expect(fe_reference_cell(2, 2, 1.0, nullptr, nullptr, A) != FE_OK, "unknown rule refused");
    }

    // descriptors refused before any device use
    const fe_mesh_desc good = {{4.0, 4.0, 4.0}, {2, 2, 2}, 3, {0, 0, 0}, 0};
    std::vector<fe_mesh_desc> bad(8, good);
    bad[0].p = 0;
    bad[1].p = 8;
    bad[2].ncell[0] = 0;
    bad[3].L[0] = 0.0;
    bad[4].L[2] = 5.0;
    bad[5].bc[0] = 1; bad[5].ncell[0] = 1; bad[5].L[0] = 2.0;
    bad[6].bc[0] = 3;
    bad[7].k_rule = 2;
    for (const fe_mesh_desc &d : bad) {
        fe_mesh *m = nullptr;
        expect(fe_mesh_create(&d, &m) == FE_EINVAL && m == nullptr, "bad descriptor refused");
        expect(std::strlen(fe_last_error()) > 0, "error message set");
    }
    expect(fe_mesh_create(nullptr, nullptr) == FE_EINVAL, "NULL descriptor");

    // every entry point refuses a NULL mesh
    double a0, b, mu, k2[2];
    int32_t it;
    double rel;
    expect(fe_mesh_destroy(nullptr) == FE_OK, "destroy NULL");
    expect(fe_mesh_set_kernel(nullptr, 0) == FE_EINVAL, "set_kernel");
    expect(fe_mesh_info(nullptr, nullptr, nullptr, nullptr) == FE_EINVAL, "info");
    expect(fe_mesh_quad_points(nullptr, nullptr) == FE_EINVAL, "quad_points");
    expect(fe_mesh_dof_coords(nullptr, nullptr) == FE_EINVAL, "dof_coords");
    expect(fe_set_potential(nullptr, nullptr, 0.0, 0.0, nullptr) == FE_EINVAL, "set_potential");
    expect(fe_set_nonlocal(nullptr, 0, nullptr, nullptr, 1.0, 0.5, nullptr) == FE_EINVAL, "set_nonlocal");
    expect(fe_hx_apply(nullptr, nullptr, nullptr, 1, 1, FE_F64, nullptr) == FE_EINVAL, "hx_apply");
    expect(fe_cheb_filter(nullptr, nullptr, nullptr, 1, 1, 3, 0.0, 1.0, NAN, FE_F64, nullptr, 0, nullptr) == FE_EINVAL,
           "cheb_filter");
    expect(fe_cheb_filter_vjp_work_bytes(nullptr, 1, 3, 1, 0) == 0, "vjp work bytes");
    expect(fe_cheb_filter_vjp(nullptr, nullptr, nullptr, 1, 1, 3, 0.0, 1.0, NAN, FE_F64, nullptr, nullptr, nullptr, 1, 0,
                              nullptr, 0, nullptr) == FE_EINVAL,
           "cheb_filter_vjp");
    expect(fe_lanczos_bounds(nullptr, nullptr, 10, &a0, &b, nullptr) == FE_EINVAL, "lanczos");
    expect(fe_cholqr2(nullptr, nullptr, 1, 1, nullptr) == FE_EINVAL, "cholqr2");
    expect(fe_rayleigh_ritz(nullptr, nullptr, nullptr, nullptr, 1, 1, nullptr, nullptr) == FE_EINVAL, "rayleigh_ritz");
    expect(fe_density(nullptr, nullptr, 1, 1, nullptr, nullptr, nullptr) == FE_EINVAL, "density");
    expect(fe_planar_average(nullptr, nullptr, 0, nullptr, nullptr) == FE_EINVAL, "planar_average");
    expect(fe_dipole(nullptr, nullptr, 0.0, &mu, nullptr) == FE_EINVAL, "dipole");
    expect(fe_poisson_work_bytes(nullptr) == 0, "poisson work bytes");
    expect(fe_poisson_solve(nullptr, nullptr, nullptr, 1e-10, 10, nullptr, 0, &it, &rel, nullptr) == FE_EINVAL,
           "poisson_solve");
    expect(fe_set_kpoint(nullptr, 0.0, 0.0) == FE_EINVAL, "set_kpoint");
    expect(fe_get_kpoint(nullptr, k2) == FE_EINVAL, "get_kpoint");
    expect(fe_hx_apply_k(nullptr, nullptr, nullptr, 1, 1, nullptr) == FE_EINVAL, "hx_apply_k");
    expect(fe_cheb_filter_k(nullptr, nullptr, nullptr, 1, 1, 3, 0.0, 1.0, NAN, nullptr, 0, nullptr) == FE_EINVAL,
           "cheb_filter_k");
    expect(fe_cholqr2_k(nullptr, nullptr, 1, 1, nullptr) == FE_EINVAL, "cholqr2_k");
    expect(fe_rayleigh_ritz_k(nullptr, nullptr, nullptr, nullptr, 1, 1, nullptr, nullptr) == FE_EINVAL,
           "rayleigh_ritz_k");
    if (failures) return 1;
    std::printf("capi sanitizer driver: done\n");
    return 0;
}
