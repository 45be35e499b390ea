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
// Jacobi preconditioner (the assembled diagonal of H0); the product is the
// two-launch single-vector form (all cell products, then fixed-order nodal
// sums) for p <= 5.  The iteration runs on
// the device: its dot products are fixed-order two-pass reductions whose
// results, and the CG scalars computed from them, stay in device memory; the
// host reads the convergence state once per batch of iterations, and
// iterations queued after convergence leave the iterate untouched.
//
// The constrained-potential-difference setup (Sec. 2.2.2) prescribes phi in
// the two conductor regions, Omega_0 = {z <= z_lo} and Omega_1 = {z >= z_hi}:
// phi = -w there, plus dV in Omega_1 (w = V_loc - V_sm at the nodes), so the
// total potential phi + w is 0 and dV inside the conductors.  The same CG runs
// on the free block: the constrained entries of x start at M^1/2 g, the
// initial residual b - H0 x0 is taken on the free nodes only, and the Jacobi
// preconditioner is zero on constrained nodes, which keeps every search
// direction and the residual zero there; the constrained phi are written as
// the data themselves at the end.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
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

// ---------------------------------------------------------------- device CG
// Scalars of the device iteration (doubles in the work buffer).
enum : int {
    S_RZ = 0,     // r.z of the current iterate (z = projected P r)
    S_ALPHA,      // rz / p.Hp
    S_BETA,       // rz_new / rz
    S_EZ,         // e.(P r): the null-space component removed from z
    S_BNRM,       // |b|
    S_REL,        // |r| / |b| after the last update
    S_DONE,       // 1 once converged (or broken down): later iterations do nothing
    S_IT,         // updates made
    S_TOL,
    S_SING,       // 1 when e spans the null space
    S_BREAK,      // 1 when p.Hp <= 0 was met
    S_COUNT
};
constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;  // partial sums per reduction (fixed: the summation order does not depend on timing)

// Fixed-order sum of the block's per-thread values for C components.
template <int C> __device__ __forceinline__ void block_sum(double (&v)[C], double *lds) {
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < C; ++c) lds[c * kRedThreads + t] = v[c];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int c = 0; c < C; ++c) lds[c * kRedThreads + t] += lds[c * kRedThreads + t + w];
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = lds[c * kRedThreads];
}

// part[blk] = sum over the block's grid-stride elements of p_i q_i
__global__ __launch_bounds__(kRedThreads) void cg_pq_kernel(const double *p, const double *q, int64_t n,
                                                            const double *sc, double *part) {
    __shared__ double lds[kRedThreads];
    if (sc[S_DONE] != 0.0) return;
    double v[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
        v[0] += p[i] * q[i];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// alpha = rz / p.Hp (one block); a non-positive p.Hp stops the iteration
__global__ __launch_bounds__(kRedThreads) void cg_alpha_kernel(const double *part, int nb, double *sc) {
    __shared__ double lds[kRedThreads];
    if (sc[S_DONE] != 0.0) return;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads) v[0] += part[b];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) {
        const double pq = v[0];
        if (!(pq > 0.0)) {
            sc[S_BREAK] = 1.0;
            sc[S_DONE] = 1.0;
            sc[S_ALPHA] = 0.0;
        } else {
            sc[S_ALPHA] = sc[S_RZ] / pq;
        }
    }
}

// x += alpha p, r -= alpha q, and the partial sums r.r, r.z, e.z, r.e with
// z = pinv r (before the null-space projection)
__global__ __launch_bounds__(kRedThreads) void cg_update_kernel(double *x, double *r, const double *p,
                                                                const double *q, const double *pinv,
                                                                const double *e, int64_t n, const double *sc,
                                                                double *part) {
    __shared__ double lds[4 * kRedThreads];
    if (sc[S_DONE] != 0.0) return;
    const double al = sc[S_ALPHA];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
        x[i] += al * p[i];
        // a zero preconditioner entry marks a constrained node: no equation there
        const double ri = pinv[i] != 0.0 ? r[i] - al * q[i] : 0.0;
        r[i] = ri;
        const double zi = pinv[i] * ri;
        v[0] += ri * ri;
        v[1] += ri * zi;
        v[2] += e[i] * zi;
        v[3] += ri * e[i];
    }
    block_sum<4>(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) part[c * kRedBlocks + blockIdx.x] = v[c];
}

// |r| / |b|, convergence, and beta with the projected z:
//   z' = z - (e.z) e,  r.z' = r.z - (e.z)(r.e)
__global__ __launch_bounds__(kRedThreads) void cg_beta_kernel(const double *part, int nb, double *sc) {
    __shared__ double lds[4 * kRedThreads];
    if (sc[S_DONE] != 0.0) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads)
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] += part[c * kRedBlocks + b];
    block_sum<4>(v, lds);
    if (threadIdx.x == 0) {
        sc[S_IT] += 1.0;
        const double rel = sqrt(v[0]) / sc[S_BNRM];
        sc[S_REL] = rel;
        if (rel <= sc[S_TOL]) {
            sc[S_DONE] = 1.0;
            return;
        }
        const double ez = sc[S_SING] != 0.0 ? v[2] : 0.0;
        const double rz = v[1] - ez * (sc[S_SING] != 0.0 ? v[3] : 0.0);
        sc[S_EZ] = ez;
        sc[S_BETA] = rz / sc[S_RZ];
        sc[S_RZ] = rz;
    }
}

// p = (pinv r - ez e) + beta p
__global__ void cg_direction_kernel(double *p, const double *r, const double *pinv, const double *e, int64_t n,
                                    const double *sc) {
    if (sc[S_DONE] != 0.0) return;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = (pinv[i] * r[i] - sc[S_EZ] * e[i]) + sc[S_BETA] * p[i];
}

// Region of a node for the constrained setup: 0 free, 1 Omega_0, 2 Omega_1.
__device__ __forceinline__ int cpd_region(double z, double z_lo, double z_hi) {
    return z <= z_lo ? 1 : (z >= z_hi ? 2 : 0);
}

// x = M^1/2 g on constrained nodes (g = -w, plus dV in Omega_1), 0 elsewhere
__global__ void cpd_start_kernel(double *x, const double *msqrt, const double *w, const double *zcoord, int nfx,
                                 int nfy, int64_t n, double z_lo, double z_hi, double dV) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int reg = cpd_region(zcoord[i / ((int64_t)nfx * nfy)], z_lo, z_hi);
    const double g = (reg == 2 ? dV : 0.0) - (w ? w[i] : 0.0);
    x[i] = reg ? msqrt[i] * g : 0.0;
}

// r = b - q on free nodes, 0 on constrained ones
__global__ void cpd_residual_kernel(double *r, const double *q, const double *pinv, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    r[i] = pinv[i] != 0.0 ? r[i] - q[i] : 0.0;
}

// phi = g on constrained nodes (the data, exactly)
__global__ void cpd_fix_kernel(double *phi, const double *w, const double *zcoord, int nfx, int nfy, int64_t n,
                               double z_lo, double z_hi, double dV) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int reg = cpd_region(zcoord[i / ((int64_t)nfx * nfy)], z_lo, z_hi);
    if (reg) phi[i] = (reg == 2 ? dV : 0.0) - (w ? w[i] : 0.0);
}

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

extern "C" size_t fe_poisson_work_bytes(const fe_mesh *m) {
    if (!m) return 0;
    return ((size_t)8 * (size_t)m->n + 4 * (size_t)kRedBlocks + 16 + assembled_scratch_doubles(m)) * sizeof(double);
}

namespace fe {

// The conductor regions of the constrained setup (null: the mesh's own
// boundary conditions only).
struct CpdSpec {
    const double *w;
    double z_lo, z_hi, dV;
};

fe_status poisson_solve(fe_mesh *m, const double *charge, double *phi, double tol, int32_t maxit, double *work,
                        size_t work_bytes, int32_t *iters_host, double *relres_host, hipStream_t st,
                        const CpdSpec *cpd) {
    if (!m || !charge || !phi || !work) return fail(FE_EINVAL, "NULL argument");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FE_EINVAL, "tol must be positive");
    if (maxit < 1) return fail(FE_EINVAL, "maxit must be >= 1");
    if (work_bytes < fe_poisson_work_bytes(m))
        return fail(FE_ENOMEM, "work smaller than fe_poisson_work_bytes");
    FE_HIPP(hipSetDevice(m->device), "hipSetDevice");
    const int64_t n = m->n;
    const int ni = (int)n;
    double *x = work, *r = x + n, *z = r + n, *p = z + n, *q = p + n, *e = q + n, *pinv = e + n, *zero = pinv + n;
    const bool singular =
        !cpd && m->bc[0] != FE_BC_DIRICHLET && m->bc[1] != FE_BC_DIRICHLET && m->bc[2] != FE_BC_DIRICHLET;

    void *hv = nullptr;
    fe_status stt = blas_handle(m, st, &hv);
    if (stt != FE_OK) return stt;
    rocblas_handle h = static_cast<rocblas_handle>(hv);

    std::vector<double> pinv_h;
    jacobi_inverse(m, pinv_h);
    if (cpd) {
        // no equation on constrained nodes: a zero preconditioner entry marks them
        int64_t nc = 0;
        const int64_t plane = m->nf[0] * m->nf[1];
        for (int64_t tz = 0; tz < m->nf[2]; ++tz) {
            const double zz = m->axis_coord[2][(size_t)tz];
            if (zz > cpd->z_lo && zz < cpd->z_hi) continue;
            std::fill(pinv_h.begin() + tz * plane, pinv_h.begin() + (tz + 1) * plane, 0.0);
            nc += plane;
        }
        if (nc == 0) return fail(FE_EINVAL, "no node lies in a conductor region (z <= z_lo or z >= z_hi)");
        if (nc == n) return fail(FE_EINVAL, "every node lies in a conductor region: nothing to solve");
    }
    FE_HIPP(hipMemcpyAsync(pinv, pinv_h.data(), n * sizeof(double), hipMemcpyHostToDevice, st), "copy pinv");
    FE_HIPP(launch_fill(zero, n, 0.0, st), "fill");
    // e = M^1/2 1 / |M^1/2 1| (the null vector when no axis is Dirichlet)
    FE_HIPP(launch_mass_sqrt(m, e, st), "mass sqrt");
    if (cpd) {
        hipLaunchKernelGGL(cpd_start_kernel, dim3(blocks(n)), dim3(256), 0, st, x, e, cpd->w, m->d_zcoord,
                           (int)m->nf[0], (int)m->nf[1], n, cpd->z_lo, cpd->z_hi, cpd->dV);
        FE_HIPP(hipGetLastError(), "cpd start");
    } else {
        FE_HIPP(launch_fill(x, n, 0.0, st), "fill");
    }
    // r = b = 2 pi M^1/2 s
    FE_HIPP(launch_vmul(r, e, charge, n, st), "rhs");
    const double twopi = 2.0 * M_PI;
    FE_BLASP(rocblas_dscal(h, ni, &twopi, r, 1), "dscal");
    if (cpd) {
        // r = b - H0 x0 on the free nodes (the prescribed values moved to the right-hand side)
        double *Zc = zero + n + 4 * kRedBlocks + 16;
        StepArgs a{x, 1, q, 1, nullptr, 0, 1.0, 0.0, 0.0, 1, zero};
        FE_HIPP(launch_step_assembled(m, a, Zc, st), "product");
        hipLaunchKernelGGL(cpd_residual_kernel, dim3(blocks(n)), dim3(256), 0, st, r, q, pinv, n);
        FE_HIPP(hipGetLastError(), "cpd residual");
    }
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
        // the iteration itself on the device; the host looks at its state
        // once per batch
        double *part = zero + n, *sc = part + 4 * kRedBlocks, *Zc = sc + 16;
        const double sc0[S_COUNT] = {rz, 0.0, 0.0, 0.0, bnrm, 1.0, 0.0, 0.0, tol, singular ? 1.0 : 0.0, 0.0};
        FE_HIPP(hipMemcpyAsync(sc, sc0, sizeof(sc0), hipMemcpyHostToDevice, st), "copy scalars");
        const int nb = (int)std::min<int64_t>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads);
        constexpr int kBatch = 8;
        // one CG iteration: seven launches on fixed buffers
        auto iteration = [&](hipStream_t ss) -> hipError_t {
            StepArgs a{p, 1, q, 1, nullptr, 0, 1.0, 0.0, 0.0, 1, zero};
            hipError_t e2 = launch_step_assembled(m, a, Zc, ss);
            if (e2 != hipSuccess) return e2;
            hipLaunchKernelGGL(cg_pq_kernel, dim3(nb), dim3(kRedThreads), 0, ss, p, q, n, sc, part);
            hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(kRedThreads), 0, ss, part, nb, sc);
            hipLaunchKernelGGL(cg_update_kernel, dim3(nb), dim3(kRedThreads), 0, ss, x, r, p, q, pinv, e, n, sc, part);
            hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kRedThreads), 0, ss, part, nb, sc);
            hipLaunchKernelGGL(cg_direction_kernel, dim3(blocks(n)), dim3(256), 0, ss, p, r, pinv, e, n, sc);
            return hipGetLastError();
        };
        // After the first batch (direct launches, which also set the kernels'
        // launch attributes) a full batch is captured once, on a private
        // stream so that the caller's stream may be the null stream, into a
        // HIP graph of kernel nodes only, and replayed on the caller's stream:
        // the same launches in the same order, without the per-launch host
        // overhead of 56 short kernels.  If the capture or instantiation
        // fails the batches stay direct launches.
        hipGraphExec_t exec = nullptr;
        bool graph_tried = false;
        auto capture = [&]() {
            graph_tried = true;
            hipStream_t cs = nullptr;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return;
            hipGraph_t graph = nullptr;
            bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess;
            if (ok) {
                for (int j = 0; j < kBatch && ok; ++j) ok = iteration(cs) == hipSuccess;
                ok = (hipStreamEndCapture(cs, &graph) == hipSuccess) && ok && graph;
            }
            if (ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipStreamDestroy(cs);
            (void)hipGetLastError();  // a failed capture leaves no error behind
        };
        double sh[S_COUNT] = {};
        int queued = 0;
        fe_status loop_st = FE_OK;
        while (queued < maxit) {
            const int nbatch = std::min(kBatch, maxit - queued);
            if (queued > 0 && nbatch == kBatch && !graph_tried) capture();
            if (exec && nbatch == kBatch) {
                if (hipGraphLaunch(exec, st) != hipSuccess) { loop_st = fail(FE_EDEVICE, "CG graph launch"); break; }
            } else {
                for (int j = 0; j < nbatch; ++j)
                    if (iteration(st) != hipSuccess) { loop_st = fail(FE_EDEVICE, "CG kernel launch"); break; }
                if (loop_st != FE_OK) break;
            }
            queued += nbatch;
            if (hipMemcpyAsync(sh, sc, sizeof(sh), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                loop_st = fail(FE_EDEVICE, "read CG state");
                break;
            }
            if (sh[S_DONE] != 0.0) break;
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (loop_st != FE_OK) return loop_st;
        if (sh[S_BREAK] != 0.0) return fail(FE_EDEVICE, "CG breakdown: p^T H0 p <= 0");
        it = (int)sh[S_IT];
        rel = sh[S_REL];
        if ((stt = project(x)) != FE_OK) return stt;
    }
    // phi = M^-1/2 x
    hipLaunchKernelGGL(dscale_kernel, dim3(blocks(n)), dim3(256), 0, st, m->d_axis, m->maxf, (int)m->nf[0],
                       (int)m->nf[1], n, x, phi);
    FE_HIPP(hipGetLastError(), "scale");
    if (cpd) {
        hipLaunchKernelGGL(cpd_fix_kernel, dim3(blocks(n)), dim3(256), 0, st, phi, cpd->w, m->d_zcoord,
                           (int)m->nf[0], (int)m->nf[1], n, cpd->z_lo, cpd->z_hi, cpd->dV);
        FE_HIPP(hipGetLastError(), "cpd data");
    }
    if (iters_host) *iters_host = it;
    if (relres_host) *relres_host = rel;
    return FE_OK;
}

}  // namespace fe

extern "C" {

fe_status fe_poisson_solve(fe_mesh *m, const double *charge, double *phi, double tol, int32_t maxit,
                           double *work, size_t work_bytes, int32_t *iters_host, double *relres_host,
                           hipStream_t st) {
    return fe::poisson_solve(m, charge, phi, tol, maxit, work, work_bytes, iters_host, relres_host, st, nullptr);
}

fe_status fe_poisson_solve_cpd(fe_mesh *m, const double *charge, const double *w, double z_lo, double z_hi,
                               double dV, double *phi, double tol, int32_t maxit, double *work, size_t work_bytes,
                               int32_t *iters_host, double *relres_host, hipStream_t st) {
    if (!m) return fail(FE_EINVAL, "NULL argument");
    if (!std::isfinite(z_lo) || !std::isfinite(z_hi) || !std::isfinite(dV) || !(z_lo < z_hi))
        return fail(FE_EINVAL, "z_lo < z_hi and dV must be finite");
    if (m->bc[2] == FE_BC_PERIODIC) return fail(FE_EINVAL, "the z axis of a CPD mesh cannot be periodic");
    if (phi && ((charge && fe::overlap(phi, m->n, 1, 1, charge, m->n, 1, 1)) ||
                (w && fe::overlap(phi, m->n, 1, 1, w, m->n, 1, 1))))
        return fail(FE_EINVAL, "phi overlaps charge or w");
    const fe::CpdSpec cpd{w, z_lo, z_hi, dV};
    return fe::poisson_solve(m, charge, phi, tol, maxit, work, work_bytes, iters_host, relres_host, st, &cpd);
}

}  // extern "C"
