// C ABI of the gfx950 FE Hamiltonian filter: argument checks, mesh set-up,
// the filter and adjoint drivers, and the dense steps of subspace iteration.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "fe_internal.h"

namespace fe {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

fe_status fail(fe_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

static fe_status hip_fail(hipError_t e, const char *what) {
    return fail(FE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define FE_HIP(call, what)                              \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

static bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Byte range [lo, hi) touched by an (n x N) block with leading dimension ld.
static void block_range(const double *p, int64_t n, int64_t N, int64_t ld, uintptr_t &lo, uintptr_t &hi) {
    lo = reinterpret_cast<uintptr_t>(p);
    hi = lo + (uintptr_t)(((n - 1) * ld + N) * (int64_t)sizeof(double));
}

bool overlap(const double *a, int64_t na, int64_t Na, int64_t lda, const double *b, int64_t nb, int64_t Nb,
             int64_t ldb) {
    uintptr_t a0, a1, b0, b1;
    block_range(a, na, Na, lda, a0, a1);
    block_range(b, nb, Nb, ldb, b0, b1);
    return a0 < b1 && b0 < a1;
}

static fe_status check_block(const fe_mesh *m, const double *p, int64_t N, int64_t ld, const char *name) {
    if (!p) return fail(FE_EINVAL, std::string(name) + " is NULL");
    if (!aligned8(p)) return fail(FE_EINVAL, std::string(name) + " is not 8-byte aligned");
    if (ld < N) return fail(FE_EINVAL, std::string("ld < N for ") + name);
    (void)m;
    return FE_OK;
}

static fe_status check_prec(fe_dtype prec) {
    if (prec != FE_F64 && prec != FE_F32 && prec != FE_BF16) return fail(FE_EINVAL, "unknown fe_dtype");
    return FE_OK;
}

fe_status validate_filter_args(fe_mesh *m, int64_t N, int32_t mdeg, double a, double b, double a0, fe_dtype prec) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (N < 0) return fail(FE_EINVAL, "N must be >= 0");
    if (mdeg < 1) return fail(FE_EINVAL, "m must be >= 1");
    if (!(a < b) || !std::isfinite(a) || !std::isfinite(b)) return fail(FE_EINVAL, "need finite a < b");
    if (!std::isnan(a0) && !(std::isfinite(a0) && a0 < a))
        return fail(FE_EINVAL, "a0 must be NaN or finite and below a");
    return check_prec(prec);
}

static fe_status ensure_scratch(fe_mesh *m, size_t bytes) {
    if (m->scratch_bytes >= bytes) return FE_OK;
    if (m->d_scratch) {
        FE_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        FE_HIP(hipFree(m->d_scratch), "hipFree");
        m->d_scratch = nullptr;
        m->scratch_bytes = 0;
    }
    if (hipMalloc(&m->d_scratch, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FE_ENOMEM, "scratch allocation failed");
    }
    m->scratch_bytes = bytes;
    return FE_OK;
}

// Filter coefficients (scaled when a0 is finite).
void cheb_coefficients(int mdeg, double a, double b, double a0, std::vector<double> &al, std::vector<double> &be,
                        double &c) {
    double e = 0.5 * (b - a);
    c = 0.5 * (b + a);
    al.assign(mdeg, 0.0);
    be.assign(mdeg, 0.0);
    if (std::isnan(a0)) {
        al[0] = 1.0 / e;
        for (int k = 1; k < mdeg; ++k) { al[k] = 2.0 / e; be[k] = 1.0; }
        return;
    }
    double s1 = e / (a0 - c), s = s1;
    al[0] = s1 / e;
    for (int k = 1; k < mdeg; ++k) {
        double sn = 1.0 / (2.0 / s1 - s);
        al[k] = 2.0 * sn / e;
        be[k] = s * sn;
        s = sn;
    }
}

// One recurrence step Y = alpha (H~ - c) X - beta Ym1, nonlocal term included.
fe_status filter_step(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, const double *Ym1,
                      int64_t ldm, double alpha, double beta, double shift, int64_t N, fe_dtype prec, hipStream_t s,
                      double *nlW) {
    StepArgs a{X, ldx, Y, ldy, Ym1, ldm, alpha, beta, shift, N};
    FE_HIP(launch_step(m, a, prec, s), "step kernel launch");
    // the nonlocal term after all colour passes: they write the base values
    if (m->nl.n_site > 0) FE_HIP(launch_nonlocal(m, X, ldx, Y, ldy, N, alpha, s, nlW), "nonlocal kernel launch");
    return FE_OK;
}

static int axis_colours(int ncell, int bc) {
    if (bc == FE_BC_PERIODIC && (ncell & 1)) return 3;
    return ncell >= 2 ? 2 : 1;
}

// A fragments of the padded cell matrix for each MFMA shape:
//   f64/f32 16x16x4 : frag[t][s][lane]    = A[16t + lane%16][4s + lane/16]
//   bf16 16x16x32   : frag[t][s][lane][j] = A[16t + lane%16][32s + 8(lane/16) + j]
void swizzle_f64(const fe_mesh *m, const std::vector<double> &A, std::vector<double> &f64) {
    const int ncp = m->ncp, nc = m->nc, NT = ncp / 16, nks4 = ncp / 4;
    f64.assign((size_t)NT * nks4 * 64, 0.0);
    for (int t = 0; t < NT; ++t)
        for (int s = 0; s < nks4; ++s)
            for (int lane = 0; lane < 64; ++lane) {
                const int r = 16 * t + lane % 16, c = 4 * s + lane / 16;
                f64[((size_t)t * nks4 + s) * 64 + lane] = (r < nc && c < nc) ? A[(size_t)r * nc + c] : 0.0;
            }
}

static void swizzle_fragments(const fe_mesh *m, std::vector<double> &f64, std::vector<float> &f32,
                              std::vector<uint16_t> &bf) {
    int ncp = m->ncp, nc = m->nc, NT = ncp / 16;
    auto A = [&](int r, int c) -> double { return (r < nc && c < nc) ? m->cellA[(size_t)r * nc + c] : 0.0; };
    int nks32 = ncp / 32;
    swizzle_f64(m, m->cellA, f64);
    f32.resize(f64.size());
    for (size_t i = 0; i < f64.size(); ++i) f32[i] = (float)f64[i];
    bf.assign((size_t)NT * nks32 * 64 * 8, 0);
    for (int t = 0; t < NT; ++t)
        for (int s = 0; s < nks32; ++s)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    float f = (float)A(16 * t + lane % 16, 32 * s + 8 * (lane / 16) + j);
                    uint32_t u;
                    std::memcpy(&u, &f, 4);
                    u += 0x7FFFu + ((u >> 16) & 1u);
                    bf[(((size_t)t * nks32 + s) * 64 + lane) * 8 + j] = (uint16_t)(u >> 16);
                }
}

// Swizzled FP64 fragments of D^ A D^ for a cell matrix A (nc x nc), with D^
// the per-local-index M^-1/2 of a node inside the mesh: (h/2) w_i per cell,
// summed over the two cells at a cell face (i = 0 or p), the same sums as the
// assembled masses.  It equals every free node's scale unless an axis is
// zero-Neumann (a boundary face node there has one cell's mass only).  With
// perm (the table kernel's output-row order), row r of the fragments holds
// node perm[r] (-1: zeros).
void fold_swizzle(const fe_mesh *m, const std::vector<double> &A, const std::vector<int32_t> *perm,
                  std::vector<double> &f64) {
    const int nc = m->nc, n1 = m->n1, p = m->p;
    std::vector<double> dh(n1);
    for (int i = 0; i <= p; ++i) {
        const double mi = (i == 0 || i == p) ? 0.5 * m->h * m->w[p] + 0.5 * m->h * m->w[0] : 0.5 * m->h * m->w[i];
        dh[i] = 1.0 / std::sqrt(mi);
    }
    auto dl = [&](int l) { return (dh[l % n1] * dh[(l / n1) % n1]) * dh[l / (n1 * n1)]; };
    const int nks4 = m->ncp / 4;
    f64.assign((size_t)(m->ncp / 16) * nks4 * 64, 0.0);
    // fragment layout of swizzle_f64: frag[t][s][lane] = row 16t + lane % 16, column 4s + lane / 16
    for (int r = 0; r < m->ncp; ++r) {
        const int l = perm ? (*perm)[r] : (r < nc ? r : -1);
        if (l < 0) continue;
        for (int c = 0; c < nc; ++c) {
            const int t = r / 16, sk = c / 4, lane = r % 16 + 16 * (c % 4);
            f64[((size_t)t * nks4 + sk) * 64 + lane] = dl(l) * A[(size_t)l * nc + c] * dl(c);
        }
    }
}

static void free_mesh(fe_mesh *m) {
    if (!m) return;
    (void)hipFree(m->d_axis);
    (void)hipFree(m->d_zcoord);
    (void)hipFree(m->d_Af64);
    (void)hipFree(m->d_Af64s);
    (void)hipFree(m->d_Af32s);
    (void)hipFree(m->d_tabperm);
    (void)hipFree(m->d_zero);
    (void)hipFree(m->d_segtab);
    (void)hipFree(m->d_segtab1);
    (void)hipFree(m->d_Af32);
    (void)hipFree(m->d_Abf16);
    (void)hipFree(m->d_v);
    (void)hipFree(m->d_wrel);
    (void)hipFree(m->d_Sf64);
    (void)hipFree(m->d_Sf64s);
    (void)hipFree(m->d_scratch);
    nonlocal_release(m);
    if (m->blas) rocblas_destroy_handle(static_cast<rocblas_handle>(m->blas));
    delete m;
}

}  // namespace fe

using namespace fe;

extern "C" {

const char *fe_last_error(void) { return g_err.c_str(); }

fe_status fe_mesh_create(const fe_mesh_desc *d, fe_mesh **out) {
    if (!d || !out) return fail(FE_EINVAL, "NULL descriptor or output");
    *out = nullptr;
    if (d->p < 1 || d->p > kMaxP) return fail(FE_EINVAL, "p must be in 1..7");
    for (int a = 0; a < 3; ++a) {
        if (!(d->L[a] > 0.0) || !std::isfinite(d->L[a])) return fail(FE_EINVAL, "L must be positive");
        if (d->ncell[a] < 1) return fail(FE_EINVAL, "ncell must be >= 1");
        if (d->bc[a] < 0 || d->bc[a] > 2) return fail(FE_EINVAL, "unknown boundary condition");
        if (d->bc[a] == FE_BC_PERIODIC && d->ncell[a] < 2) return fail(FE_EINVAL, "a periodic axis needs >= 2 cells");
    }
    if (d->k_rule != FE_RULE_EXACT && d->k_rule != FE_RULE_GLL) return fail(FE_EINVAL, "unknown stiffness rule");
    double h = d->L[0] / d->ncell[0];
    for (int a = 1; a < 3; ++a)
        if (std::fabs(d->L[a] / d->ncell[a] - h) > 1e-12 * h) return fail(FE_EINVAL, "cells must be cubes");

    int dev = 0;
    FE_HIP(hipGetDevice(&dev), "hipGetDevice");
    // the device address of the allocation-free entry point's scratch, once per device
    fe_status sst = static_scratch_init(dev);
    if (sst != FE_OK) return sst;
    fe_mesh *m = new fe_mesh();
    m->device = dev;
    m->h = h;
    m->p = d->p;
    m->n1 = d->p + 1;
    m->nc = m->n1 * m->n1 * m->n1;
    m->ncp = padded_nc(d->p);
    m->rule = d->k_rule;
    m->n = 1;
    m->ncells = 1;
    for (int a = 0; a < 3; ++a) {
        m->L[a] = d->L[a];
        m->ncell[a] = d->ncell[a];
        m->bc[a] = d->bc[a];
        int64_t k = (int64_t)d->ncell[a] * d->p;
        m->nf[a] = d->bc[a] == FE_BC_DIRICHLET ? k - 1 : d->bc[a] == FE_BC_PERIODIC ? k : k + 1;
        if (m->nf[a] < 1) { delete m; return fail(FE_EINVAL, "an axis has no free nodes"); }
        m->n *= m->nf[a];
        m->ncells *= d->ncell[a];
        m->ncol[a] = axis_colours(d->ncell[a], d->bc[a]);
    }
    if (m->n > (int64_t)INT32_MAX) { delete m; return fail(FE_EINVAL, "more than 2^31-1 DoFs"); }

    gll_rule(m->p, m->xi, m->w);
    cell_matrix_half(m->p, m->rule, h, m->cellA);

    // per-axis coordinates and assembled lumped masses of the free positions
    m->maxf = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t k = (int64_t)m->ncell[a] * m->p;
        std::vector<double> mass(k + 1, 0.0), coord(k + 1, 0.0);
        for (int c = 0; c < m->ncell[a]; ++c)
            for (int i = 0; i <= m->p; ++i) {
                mass[(int64_t)c * m->p + i] += 0.5 * h * m->w[i];
                coord[(int64_t)c * m->p + i] = c * h + 0.5 * h * (m->xi[i] + 1.0);
            }
        coord[k] = m->ncell[a] * h;
        if (m->bc[a] == FE_BC_PERIODIC) mass[0] += mass[k];
        m->axis_mass[a].clear();
        m->axis_coord[a].clear();
        for (int64_t t = 0; t < m->nf[a]; ++t) {
            int64_t g = m->bc[a] == FE_BC_DIRICHLET ? t + 1 : t;
            m->axis_mass[a].push_back(mass[g]);
            m->axis_coord[a].push_back(coord[g]);
        }
        m->maxf = std::max<int>(m->maxf, (int)m->nf[a]);
    }
    std::vector<double> axis(9 * (size_t)m->maxf, 0.0);
    for (int a = 0; a < 3; ++a)
        for (int64_t t = 0; t < m->nf[a]; ++t) {
            axis[(size_t)a * m->maxf + t] = 1.0 / std::sqrt(m->axis_mass[a][t]);
            axis[(size_t)(3 + a) * m->maxf + t] = 1.0 / m->axis_mass[a][t];
            axis[(size_t)(6 + a) * m->maxf + t] = m->axis_mass[a][t];
        }
    std::vector<double> wrel(3 * (size_t)m->n1);
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i <= m->p; ++i) wrel[(size_t)a * m->n1 + i] = 0.5 * h * m->w[i];

    std::vector<double> f64;
    std::vector<float> f32;
    std::vector<uint16_t> bf;
    swizzle_fragments(m, f64, f32, bf);
    // D^ (1/2 Kc) D^ with D^ the per-local-index M^-1/2 of a node inside the
    // mesh: (h/2) w_i per cell, summed over the two cells at a cell face
    // (i = 0 or p), the same sums as the assembled masses above.  It equals
    // every free node's scale unless an axis is zero-Neumann (a boundary face
    // node there has one cell's mass only).
    const bool fold = m->bc[0] != FE_BC_NEUMANN && m->bc[1] != FE_BC_NEUMANN && m->bc[2] != FE_BC_NEUMANN;
    // the table kernel (p = 3, 4, 5 with the folded matrix; it indexes DoFs
    // in 32 bits) takes the rows of the folded matrix in its own order
    const bool table = fold && m->p >= 3 && m->p <= 5 && m->n < INT32_MAX;
    std::vector<int32_t> perm;
    if (table) build_table_row_perm(m->p, table_tiles_per_wave(m->p), perm);
    m->tab_perm = perm;
    std::vector<double> f64s;
    std::vector<float> f32s;
    if (fold) {
        fold_swizzle(m, m->cellA, table ? &perm : nullptr, f64s);
        f32s.assign(f64s.begin(), f64s.end());
    }
    const double zeros[32] = {};
    std::vector<int32_t> segtab, segtab1;
    if (table) {
        build_segment_table(m, 2, segtab, m->seg_off, m->seg_zl, m->seg_bx, m->seg_by);
        int zl1 = 1, bx1 = 1, by1 = 1;
        if (m->seg_by > 1) build_segment_table(m, 1, segtab1, m->seg_off1, zl1, bx1, by1);
    }

    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = up((void **)&m->d_axis, axis.data(), axis.size() * sizeof(double)) &&
              up((void **)&m->d_zcoord, m->axis_coord[2].data(), m->axis_coord[2].size() * sizeof(double)) &&
              up((void **)&m->d_wrel, wrel.data(), wrel.size() * sizeof(double)) &&
              up((void **)&m->d_Af64, f64.data(), f64.size() * sizeof(double)) &&
              (!fold || up((void **)&m->d_Af64s, f64s.data(), f64s.size() * sizeof(double))) &&
              (!fold || up((void **)&m->d_Af32s, f32s.data(), f32s.size() * sizeof(float))) &&
              up((void **)&m->d_zero, zeros, sizeof(zeros)) &&
              (segtab.empty() || up((void **)&m->d_segtab, segtab.data(), segtab.size() * sizeof(int32_t))) &&
              (segtab1.empty() || up((void **)&m->d_segtab1, segtab1.data(), segtab1.size() * sizeof(int32_t))) &&
              (perm.empty() || up((void **)&m->d_tabperm, perm.data(), perm.size() * sizeof(int32_t))) &&
              up((void **)&m->d_Af32, f32.data(), f32.size() * sizeof(float)) &&
              up((void **)&m->d_Abf16, bf.data(), bf.size() * sizeof(uint16_t)) &&
              hipMalloc((void **)&m->d_v, (size_t)m->n * sizeof(double)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_mesh(m);
        return fail(FE_ENOMEM, "device allocation failed in fe_mesh_create");
    }
    fe_status st = ensure_scratch(m, 1024 * sizeof(double));
    if (st != FE_OK) { free_mesh(m); return st; }
    *out = m;
    return FE_OK;
}

fe_status fe_reference_cell(int32_t p, int32_t k_rule, double h, double *xi, double *w, double *A) {
    if (p < 1 || p > kMaxP) return fail(FE_EINVAL, "p must be in 1..7");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(FE_EINVAL, "h must be positive");
    if (k_rule != FE_RULE_EXACT && k_rule != FE_RULE_GLL) return fail(FE_EINVAL, "unknown stiffness rule");
    std::vector<double> x, wt, Ac;
    gll_rule(p, x, wt);
    if (xi) std::copy(x.begin(), x.end(), xi);
    if (w) std::copy(wt.begin(), wt.end(), w);
    if (A) {
        cell_matrix_half(p, k_rule, h, Ac);
        std::copy(Ac.begin(), Ac.end(), A);
    }
    return FE_OK;
}

fe_status fe_mesh_destroy(fe_mesh *mesh) {
    if (!mesh) return FE_OK;
    (void)hipDeviceSynchronize();
    free_mesh(mesh);
    return FE_OK;
}

fe_status fe_mesh_set_kernel(fe_mesh *m, int32_t variant) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (variant < 0 || variant > 10 || variant == 2 || variant == 5 || variant == 8)
        return fail(FE_EINVAL, "kernel variant must be 0, 1, 3, 4, 6, 7, 9 or 10 (2, 5 and 8 were removed)");
    m->kernel_variant = variant;
    return FE_OK;
}

fe_status fe_mesh_info(const fe_mesh *m, int64_t *n_dof, int64_t *n_cell, int32_t *n_c) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (n_dof) *n_dof = m->n;
    if (n_cell) *n_cell = m->ncells;
    if (n_c) *n_c = m->nc;
    return FE_OK;
}

fe_status fe_mesh_quad_points(const fe_mesh *m, double *xyz) {
    if (!m || !xyz) return fail(FE_EINVAL, "NULL argument");
    int n1 = m->n1;
    int64_t c = 0;
    for (int cz = 0; cz < m->ncell[2]; ++cz)
        for (int cy = 0; cy < m->ncell[1]; ++cy)
            for (int cx = 0; cx < m->ncell[0]; ++cx, ++c)
                for (int l = 0; l < m->nc; ++l) {
                    int li[3] = {l % n1, (l / n1) % n1, l / (n1 * n1)};
                    int cc[3] = {cx, cy, cz};
                    for (int a = 0; a < 3; ++a)
                        xyz[(c * m->nc + l) * 3 + a] = cc[a] * m->h + 0.5 * m->h * (m->xi[li[a]] + 1.0);
                }
    return FE_OK;
}

fe_status fe_mesh_dof_coords(const fe_mesh *m, double *xyz) {
    if (!m || !xyz) return fail(FE_EINVAL, "NULL argument");
    for (int64_t iz = 0; iz < m->nf[2]; ++iz)
        for (int64_t iy = 0; iy < m->nf[1]; ++iy)
            for (int64_t ix = 0; ix < m->nf[0]; ++ix) {
                int64_t I = ix + m->nf[0] * (iy + m->nf[1] * iz);
                xyz[I * 3 + 0] = m->axis_coord[0][ix];
                xyz[I * 3 + 1] = m->axis_coord[1][iy];
                xyz[I * 3 + 2] = m->axis_coord[2][iz];
            }
    return FE_OK;
}

fe_status fe_set_potential(fe_mesh *m, const double *Vq, double E, double z0, hipStream_t s) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (Vq && !aligned8(Vq)) return fail(FE_EINVAL, "V_quad is not 8-byte aligned");
    if (!std::isfinite(E) || !std::isfinite(z0)) return fail(FE_EINVAL, "E and z0 must be finite");
    FE_HIP(launch_potential(m, Vq, E, z0, s), "potential kernel launch");
    m->potential_set = true;
    m->E = E;
    m->z0 = z0;
    return FE_OK;
}

fe_status fe_hx_apply(fe_mesh *m, const double *X, double *Y, int64_t N, int64_t ld, fe_dtype prec,
                      hipStream_t s) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (N == 0) return FE_OK;
    if (N < 0) return fail(FE_EINVAL, "N must be >= 0");
    fe_status st;
    if ((st = check_prec(prec)) != FE_OK) return st;
    if ((st = check_block(m, X, N, ld, "X")) != FE_OK) return st;
    if ((st = check_block(m, Y, N, ld, "Y")) != FE_OK) return st;
    if (overlap(X, m->n, N, ld, Y, m->n, N, ld)) return fail(FE_EINVAL, "X and Y overlap");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    return filter_step(m, X, ld, Y, ld, nullptr, 0, 1.0, 0.0, 0.0, N, prec, s);
}

fe_status fe_hx_apply_noalloc(fe_mesh *m, const double *X, double *Y, int64_t N, int64_t ld, fe_dtype prec,
                              hipStream_t s) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (N == 0) return FE_OK;
    if (N < 0) return fail(FE_EINVAL, "N must be >= 0");
    fe_status st;
    if ((st = check_prec(prec)) != FE_OK) return st;
    if ((st = check_block(m, X, N, ld, "X")) != FE_OK) return st;
    if ((st = check_block(m, Y, N, ld, "Y")) != FE_OK) return st;
    if (overlap(X, m->n, N, ld, Y, m->n, N, ld)) return fail(FE_EINVAL, "X and Y overlap");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    double *W = nullptr;
    if (m->nl.n_site > 0) {
        // the projections of the nonlocal term go to the device's static
        // scratch instead of the mesh's buffer grown on demand
        if (nonlocal_work_doubles(m, N) > kStaticScratchDoubles)
            return fail(FE_ENOMEM, "9 * n_site * N = " + std::to_string(nonlocal_work_doubles(m, N)) +
                                       " doubles exceeds the static scratch of " +
                                       std::to_string(kStaticScratchDoubles) + " doubles");
        W = static_scratch(m->device);
        if (!W) return fail(FE_EDEVICE, "static scratch not resolved on the mesh's device");
    }
    return filter_step(m, X, ld, Y, ld, nullptr, 0, 1.0, 0.0, 0.0, N, prec, s, W);
}

fe_status fe_cheb_filter(fe_mesh *m, const double *X, double *Y, int64_t N, int64_t ld, int32_t mdeg, double a,
                         double b, double a0, fe_dtype prec, double *work, size_t work_bytes, hipStream_t s) {
    fe_status st = validate_filter_args(m, N, mdeg, a, b, a0, prec);
    if (st != FE_OK) return st;
    if (N == 0) return FE_OK;
    if ((st = check_block(m, X, N, ld, "X")) != FE_OK) return st;
    if ((st = check_block(m, Y, N, ld, "Y")) != FE_OK) return st;
    if (mdeg >= 2) {
        if ((st = check_block(m, work, N, N, "work")) != FE_OK) return st;
        if (work_bytes < (size_t)m->n * N * sizeof(double)) return fail(FE_ENOMEM, "work smaller than n*N doubles");
        if (overlap(X, m->n, N, ld, work, m->n, N, N) || overlap(Y, m->n, N, ld, work, m->n, N, N))
            return fail(FE_EINVAL, "work overlaps X or Y");
    }
    if (overlap(X, m->n, N, ld, Y, m->n, N, ld)) return fail(FE_EINVAL, "X and Y overlap");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    std::vector<double> al, be;
    double c;
    cheb_coefficients(mdeg, a, b, a0, al, be, c);
    // Y_k for odd k lives in one buffer and even k >= 2 in the other, so that
    // Y_{k+1} overwrites Y_{k-1} in place and Y_m lands in Y.
    double *odd = (mdeg & 1) ? Y : work;
    double *even = (mdeg & 1) ? work : Y;
    int64_t ldo = (mdeg & 1) ? ld : N, lde = (mdeg & 1) ? N : ld;
    auto buf = [&](int k) -> double * { return k == 0 ? const_cast<double *>(X) : (k & 1) ? odd : even; };
    auto ldb = [&](int k) -> int64_t { return k == 0 ? ld : (k & 1) ? ldo : lde; };
    st = filter_step(m, X, ld, buf(1), ldb(1), nullptr, 0, al[0], 0.0, c, N, prec, s);
    if (st != FE_OK) return st;
    for (int k = 1; k < mdeg; ++k) {
        st = filter_step(m, buf(k), ldb(k), buf(k + 1), ldb(k + 1), buf(k - 1), ldb(k - 1), al[k], be[k], c, N, prec,
                         s);
        if (st != FE_OK) return st;
    }
    return FE_OK;
}


// ---------------------------------------------------------------- Bloch-k mode

fe_status fe_set_kpoint(fe_mesh *m, double kx, double ky) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (!std::isfinite(kx) || !std::isfinite(ky)) return fail(FE_EINVAL, "k must be finite");
    if ((kx != 0.0 && m->bc[0] != FE_BC_PERIODIC) || (ky != 0.0 && m->bc[1] != FE_BC_PERIODIC))
        return fail(FE_EINVAL, "a nonzero Bloch wave number needs a periodic axis");
    FE_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
    const double old[2] = {m->kvec[0], m->kvec[1]};
    if (kx != 0.0 || ky != 0.0) {
        std::vector<double> S, f, fs;
        cell_matrix_bloch(m->p, m->rule, m->h, kx, ky, S);
        swizzle_f64(m, S, f);
        // the table kernel's copy (FP64 at p = 3, 4): folded, rows in its order
        const bool table = m->d_Af64s && !m->tab_perm.empty() && m->p <= 4;
        if (table) fold_swizzle(m, S, &m->tab_perm, fs);
        if (!m->d_Sf64 && hipMalloc(&m->d_Sf64, f.size() * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            m->d_Sf64 = nullptr;
            return fail(FE_ENOMEM, "device allocation failed in fe_set_kpoint");
        }
        if (table && !m->d_Sf64s && hipMalloc(&m->d_Sf64s, fs.size() * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            m->d_Sf64s = nullptr;
            return fail(FE_ENOMEM, "device allocation failed in fe_set_kpoint");
        }
        FE_HIP(hipMemcpy(m->d_Sf64, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
        if (table)
            FE_HIP(hipMemcpy(m->d_Sf64s, fs.data(), fs.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
    }
    m->kvec[0] = kx;
    m->kvec[1] = ky;
    fe_status st = nonlocal_set_phase(m);
    if (st != FE_OK) {
        m->kvec[0] = old[0];
        m->kvec[1] = old[1];
    }
    return st;
}

fe_status fe_get_kpoint(const fe_mesh *m, double *k_host) {
    if (!m || !k_host) return fail(FE_EINVAL, "NULL argument");
    k_host[0] = m->kvec[0];
    k_host[1] = m->kvec[1];
    return FE_OK;
}

}  // extern "C"

namespace fe {

// One step of the recurrence on complex blocks (n x N complex, interleaved
// re/im, leading dimensions in complex elements): the real kernels on the
// 2N real columns, plus the k.G product and the phase-twisted projectors
// when k != 0.  |k|^2 / 2 enters through the shift.
fe_status filter_step_k(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, const double *Ym1,
                        int64_t ldm, double alpha, double beta, double shift, int64_t N, hipStream_t s) {
    const bool gamma = m->kvec[0] == 0.0 && m->kvec[1] == 0.0;
    const double kk = 0.5 * (m->kvec[0] * m->kvec[0] + m->kvec[1] * m->kvec[1]);
    StepArgs a{X, 2 * ldx, Y, 2 * ldy, Ym1, 2 * ldm, alpha, beta, shift - kk, 2 * N};
    a.S = gamma ? nullptr : m->d_Sf64;
    FE_HIP(launch_step(m, a, FE_F64, s), "step kernel launch");
    if (m->nl.n_site > 0) {
        if (gamma) FE_HIP(launch_nonlocal(m, X, 2 * ldx, Y, 2 * ldy, 2 * N, alpha, s), "nonlocal kernel launch");
        else FE_HIP(launch_nonlocal_k(m, X, 2 * ldx, Y, 2 * ldy, N, alpha, s), "nonlocal kernel launch");
    }
    return FE_OK;
}

}  // namespace fe

extern "C" {

fe_status fe_hx_apply_k(fe_mesh *m, const double *X, double *Y, int64_t N, int64_t ld, hipStream_t s) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (N == 0) return FE_OK;
    if (N < 0) return fail(FE_EINVAL, "N must be >= 0");
    fe_status st;
    if ((st = check_block(m, X, N, ld, "X")) != FE_OK) return st;
    if ((st = check_block(m, Y, N, ld, "Y")) != FE_OK) return st;
    if (overlap(X, m->n, 2 * N, 2 * ld, Y, m->n, 2 * N, 2 * ld)) return fail(FE_EINVAL, "X and Y overlap");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    return filter_step_k(m, X, ld, Y, ld, nullptr, 0, 1.0, 0.0, 0.0, N, s);
}

fe_status fe_cheb_filter_k(fe_mesh *m, const double *X, double *Y, int64_t N, int64_t ld, int32_t mdeg, double a,
                           double b, double a0, double *work, size_t work_bytes, hipStream_t s) {
    fe_status st = validate_filter_args(m, N, mdeg, a, b, a0, FE_F64);
    if (st != FE_OK) return st;
    if (N == 0) return FE_OK;
    if ((st = check_block(m, X, N, ld, "X")) != FE_OK) return st;
    if ((st = check_block(m, Y, N, ld, "Y")) != FE_OK) return st;
    if (mdeg >= 2) {
        if ((st = check_block(m, work, N, N, "work")) != FE_OK) return st;
        if (work_bytes < (size_t)m->n * N * 2 * sizeof(double))
            return fail(FE_ENOMEM, "work smaller than 2*n*N doubles");
        if (overlap(X, m->n, 2 * N, 2 * ld, work, m->n, 2 * N, 2 * N) ||
            overlap(Y, m->n, 2 * N, 2 * ld, work, m->n, 2 * N, 2 * N))
            return fail(FE_EINVAL, "work overlaps X or Y");
    }
    if (overlap(X, m->n, 2 * N, 2 * ld, Y, m->n, 2 * N, 2 * ld)) return fail(FE_EINVAL, "X and Y overlap");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    std::vector<double> al, be;
    double c;
    cheb_coefficients(mdeg, a, b, a0, al, be, c);
    // the buffer rotation of fe_cheb_filter: Y_m lands in Y
    double *odd = (mdeg & 1) ? Y : work;
    double *even = (mdeg & 1) ? work : Y;
    int64_t ldo = (mdeg & 1) ? ld : N, lde = (mdeg & 1) ? N : ld;
    auto buf = [&](int k) -> double * { return k == 0 ? const_cast<double *>(X) : (k & 1) ? odd : even; };
    auto ldb = [&](int k) -> int64_t { return k == 0 ? ld : (k & 1) ? ldo : lde; };
    st = filter_step_k(m, X, ld, buf(1), ldb(1), nullptr, 0, al[0], 0.0, c, N, s);
    if (st != FE_OK) return st;
    for (int k = 1; k < mdeg; ++k) {
        st = filter_step_k(m, buf(k), ldb(k), buf(k + 1), ldb(k + 1), buf(k - 1), ldb(k - 1), al[k], be[k], c, N, s);
        if (st != FE_OK) return st;
    }
    return FE_OK;
}

}  // extern "C"
