// Electrostatics on the same finite-element space (paper Sec. 2.2, Eq. for the
// Poisson problem, -lap(phi) / 4 pi = rho + b).
//
// The Galerkin system is K phi = 4 pi M s for the nodal charge density s
// (GLL-collocated right-hand side, M the lumped mass).  With phi = M^-1/2 x it
// reads  H0 x = 2 pi M^1/2 s,  H0 = M^-1/2 (1/2 K) M^-1/2,  which is the
// filter's operator H~ with a zero diagonal term, so the colour-pass step
// kernel serves as the matrix-vector product.  Dirichlet axes of the mesh give
// phi = 0 on those faces; with none (periodic / zero-Neumann only, the
// constant-field setup of Sec. 2.2.1) H0 has the null vector M^1/2 1, which is
// projected out of the right-hand side and of every search direction, so the
// solution has zero mean (integral of phi = 0).  Conjugate gradients with a
// Jacobi preconditioner (the assembled diagonal of H0); dot products by
// rocBLAS.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <string>
#include <vector>

#include "fe_internal.h"

namespace fe {

namespace {

__global__ void mass_sqrt_kernel(const double *massax, int maxf, int nfx, int nfy, int64_t n, double *out) {
    const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (I >= n) return;
    const int tx = (int)(I % nfx), ty = (int)((I / nfx) % nfy), tz = (int)(I / ((int64_t)nfx * nfy));
    out[I] = std::sqrt((massax[tx] * massax[maxf + ty]) * massax[2 * maxf + tz]);
}

// out_I = x_I M_I^-1/2 (per-axis factors, multiplied in the order the step
// kernels use)
__global__ void dscale_kernel(const double *axisD, int maxf, int nfx, int nfy, int64_t n, const double *x,
                              double *out) {
    const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (I >= n) return;
    const int tx = (int)(I % nfx), ty = (int)((I / nfx) % nfy), tz = (int)(I / ((int64_t)nfx * nfy));
    out[I] = x[I] * ((axisD[tx] * axisD[maxf + ty]) * axisD[2 * maxf + tz]);
}

__global__ void vmul_kernel(double *z, const double *a, const double *b, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) z[i] = a[i] * b[i];
}

__global__ void xpby_kernel(double *p, const double *z, double beta, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + beta * p[i];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

#define FE_HIPP(call, what)                                                                          \
    do {                                                                                             \
        hipError_t _e = (call);                                                                      \
        if (_e != hipSuccess) return fail(FE_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)
#define FE_BLASP(call, what)                                                                         \
    do {                                                                                             \
        rocblas_status _b = (call);                                                                  \
        if (_b != rocblas_status_success)                                                            \
            return fail(FE_EDEVICE, std::string(what) + ": " + rocblas_status_to_string(_b));         \
    } while (0)

// free index of global position g along an axis (-1 on a Dirichlet face)
int64_t free_index(int bc, int64_t K, int64_t g) {
    if (bc == FE_BC_DIRICHLET) return (g == 0 || g == K) ? -1 : g - 1;
    if (bc == FE_BC_PERIODIC) return g == K ? 0 : g;
    return g;
}

// 1 / diag(H0): the diagonal of the assembled (1/2) K from the cell matrix,
// scaled by 1 / M_I (host, once per mesh size).
void jacobi_inverse(const fe_mesh *m, std::vector<double> &pinv) {
    const int n1 = m->p + 1;
    const int64_t K[3] = {(int64_t)m->ncell[0] * m->p, (int64_t)m->ncell[1] * m->p, (int64_t)m->ncell[2] * m->p};
    std::vector<double> dg((size_t)m->n, 0.0);
    for (int cz = 0; cz < m->ncell[2]; ++cz)
        for (int cy = 0; cy < m->ncell[1]; ++cy)
            for (int cx = 0; cx < m->ncell[0]; ++cx)
                for (int k = 0; k < n1; ++k)
                    for (int j = 0; j < n1; ++j)
                        for (int i = 0; i < n1; ++i) {
                            const int64_t tx = free_index(m->bc[0], K[0], (int64_t)cx * m->p + i);
                            const int64_t ty = free_index(m->bc[1], K[1], (int64_t)cy * m->p + j);
                            const int64_t tz = free_index(m->bc[2], K[2], (int64_t)cz * m->p + k);
                            if (tx < 0 || ty < 0 || tz < 0) continue;
                            const int l = i + n1 * (j + n1 * k);
                            dg[(size_t)(tx + m->nf[0] * (ty + m->nf[1] * tz))] += m->cellA[(size_t)l * m->nc + l];
                        }
    pinv.resize((size_t)m->n);
    for (int64_t tz = 0; tz < m->nf[2]; ++tz)
        for (int64_t ty = 0; ty < m->nf[1]; ++ty)
            for (int64_t tx = 0; tx < m->nf[0]; ++tx) {
                const int64_t I = tx + m->nf[0] * (ty + m->nf[1] * tz);
                const double M = m->axis_mass[0][tx] * m->axis_mass[1][ty] * m->axis_mass[2][tz];
                pinv[(size_t)I] = M / dg[(size_t)I];
            }
}

}  // namespace

hipError_t launch_mass_sqrt(const fe_mesh *m, double *out, hipStream_t s) {
    hipLaunchKernelGGL(mass_sqrt_kernel, dim3(blocks(m->n)), dim3(256), 0, s, m->d_axis + 6 * m->maxf, m->maxf,
                       (int)m->nf[0], (int)m->nf[1], m->n, out);
    return hipGetLastError();
}

hipError_t launch_vmul(double *z, const double *a, const double *b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(vmul_kernel, dim3(blocks(n)), dim3(256), 0, s, z, a, b, n);
    return hipGetLastError();
}

hipError_t launch_xpby(double *p, const double *z, double beta, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(xpby_kernel, dim3(blocks(n)), dim3(256), 0, s, p, z, beta, n);
    return hipGetLastError();
}

}  // namespace fe

using namespace fe;

extern "C" {

size_t fe_poisson_work_bytes(const fe_mesh *m) {
    if (!m) return 0;
    return (size_t)8 * (size_t)m->n * sizeof(double);
}

fe_status fe_poisson_solve(fe_mesh *m, const double *charge, double *phi, double tol, int32_t maxit,
                           double *work, size_t work_bytes, int32_t *iters_host, double *relres_host,
                           hipStream_t st) {
    if (!m || !charge || !phi || !work) return fail(FE_EINVAL, "NULL argument");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FE_EINVAL, "tol must be positive");
    if (maxit < 1) return fail(FE_EINVAL, "maxit must be >= 1");
    if (work_bytes < fe_poisson_work_bytes(m))
        return fail(FE_ENOMEM, "work smaller than fe_poisson_work_bytes");
    FE_HIPP(hipSetDevice(m->device), "hipSetDevice");
    const int64_t n = m->n;
    const int ni = (int)n;
    double *x = work, *r = x + n, *z = r + n, *p = z + n, *q = p + n, *e = q + n, *pinv = e + n, *zero = pinv + n;
    const bool singular = m->bc[0] != FE_BC_DIRICHLET && m->bc[1] != FE_BC_DIRICHLET && m->bc[2] != FE_BC_DIRICHLET;

    void *hv = nullptr;
    fe_status stt = blas_handle(m, st, &hv);
    if (stt != FE_OK) return stt;
    rocblas_handle h = static_cast<rocblas_handle>(hv);

    std::vector<double> pinv_h;
    jacobi_inverse(m, pinv_h);
    FE_HIPP(hipMemcpyAsync(pinv, pinv_h.data(), n * sizeof(double), hipMemcpyHostToDevice, st), "copy pinv");
    FE_HIPP(launch_fill(zero, n, 0.0, st), "fill");
    FE_HIPP(launch_fill(x, n, 0.0, st), "fill");
    // e = M^1/2 1 / |M^1/2 1| (the null vector when no axis is Dirichlet)
    FE_HIPP(launch_mass_sqrt(m, e, st), "mass sqrt");
    // r = b = 2 pi M^1/2 s
    FE_HIPP(launch_vmul(r, e, charge, n, st), "rhs");
    const double twopi = 2.0 * M_PI;
    FE_BLASP(rocblas_dscal(h, ni, &twopi, r, 1), "dscal");
    double enrm = 0.0;
    FE_BLASP(rocblas_dnrm2(h, ni, e, 1, &enrm), "dnrm2");
    const double ie = 1.0 / enrm;
    FE_BLASP(rocblas_dscal(h, ni, &ie, e, 1), "dscal");
    auto project = [&](double *v) -> fe_status {
        if (!singular) return FE_OK;
        double c = 0.0;
        FE_BLASP(rocblas_ddot(h, ni, e, 1, v, 1, &c), "ddot");
        c = -c;
        FE_BLASP(rocblas_daxpy(h, ni, &c, e, 1, v, 1), "daxpy");
        return FE_OK;
    };
    if ((stt = project(r)) != FE_OK) return stt;
    double bnrm = 0.0;
    FE_BLASP(rocblas_dnrm2(h, ni, r, 1, &bnrm), "dnrm2");
    int it = 0;
    double rel = 0.0;
    if (bnrm > 0.0) {
        FE_HIPP(launch_vmul(z, pinv, r, n, st), "precondition");
        if ((stt = project(z)) != FE_OK) return stt;
        FE_HIPP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
        double rz = 0.0;
        FE_BLASP(rocblas_ddot(h, ni, r, 1, z, 1, &rz), "ddot");
        rel = 1.0;
        while (it < maxit) {
            StepArgs a{p, 1, q, 1, nullptr, 0, 1.0, 0.0, 0.0, 1, zero};
            FE_HIPP(launch_step(m, a, FE_F64, st), "step kernel launch");
            double pq = 0.0;
            FE_BLASP(rocblas_ddot(h, ni, p, 1, q, 1, &pq), "ddot");
            if (!(pq > 0.0)) return fail(FE_EDEVICE, "CG breakdown: p^T H0 p <= 0");
            double al = rz / pq, mal = -al;
            FE_BLASP(rocblas_daxpy(h, ni, &al, p, 1, x, 1), "daxpy");
            FE_BLASP(rocblas_daxpy(h, ni, &mal, q, 1, r, 1), "daxpy");
            ++it;
            double rn = 0.0;
            FE_BLASP(rocblas_dnrm2(h, ni, r, 1, &rn), "dnrm2");
            rel = rn / bnrm;
            if (rel <= tol) break;
            FE_HIPP(launch_vmul(z, pinv, r, n, st), "precondition");
            if ((stt = project(z)) != FE_OK) return stt;
            double rz2 = 0.0;
            FE_BLASP(rocblas_ddot(h, ni, r, 1, z, 1, &rz2), "ddot");
            FE_HIPP(launch_xpby(p, z, rz2 / rz, n, st), "xpby");
            rz = rz2;
        }
        if ((stt = project(x)) != FE_OK) return stt;
    }
    // phi = M^-1/2 x
    hipLaunchKernelGGL(dscale_kernel, dim3(blocks(n)), dim3(256), 0, st, m->d_axis, m->maxf, (int)m->nf[0],
                       (int)m->nf[1], n, x, phi);
    FE_HIPP(hipGetLastError(), "scale");
    if (iters_host) *iters_host = it;
    if (relres_host) *relres_host = rel;
    return FE_OK;
}

}  // extern "C"
