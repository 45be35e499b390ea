// Electron density and planar integrals/averages over x-y node planes.
//
// rho_I = 2 sum_n f_n |psi_n(x_I)|^2 with psi_n = M^-1/2 x_n, i.e. the
// density of the occupied orbitals (paper Sec. 2.1) evaluated at the GLL
// nodes, where the orbitals of the lumped-mass discretisation are nodal
// values (the collocated GLL quadrature used throughout).  The planar
// integral over the plane S_z through a row of z nodes (paper Sec. 3.2) is
// the x-y GLL quadrature of the nodal field: sum_ij m_x(i) m_y(j) F(i,j,k),
// with m_a the assembled 1-D lumped masses; the planar average divides it by
// the plane area sum_i m_x(i) sum_j m_y(j).  Reductions run in a fixed
// order, so results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "fe_internal.h"

namespace fe {

namespace {

// 16 lanes per DoF: lane j sums f_n X[I,n]^2 over n = j, j+16, ..., then the
// 16 partial sums are combined in a fixed butterfly order.  V2 (N even, X, f
// 16-byte aligned, ld even): lane j takes the column pairs 2j + 32i, 2j + 1 +
// 32i with one 16-byte load each, even and odd columns summed apart and then
// added.
template <bool V2>
__global__ void density_kernel(const double *X, int64_t ld, int64_t N, const double *f, int64_t n, int nfx, int nfy,
                               const double *invM, int maxf, double *rho) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t I = gid >> 4;
    const int j = (int)(gid & 15);
    double s = 0.0;
    if (I < n) {
        const double *row = X + I * ld;
        if constexpr (V2) {
            double s1 = 0.0;
            for (int64_t c = 2 * j; c < N; c += 32) {
                const double2 x = *reinterpret_cast<const double2 *>(row + c);
                const double2 w = *reinterpret_cast<const double2 *>(f + c);
                s += w.x * (x.x * x.x);
                s1 += w.y * (x.y * x.y);
            }
            s += s1;
        } else {
            for (int64_t c = j; c < N; c += 16) {
                const double x = row[c];
                s += f[c] * (x * x);
            }
        }
    }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off, 16);
    if (I < n && j == 0) {
        const int tx = (int)(I % nfx);
        const int ty = (int)((I / nfx) % nfy);
        const int tz = (int)(I / ((int64_t)nfx * nfy));
        const double im = (invM[tx] * invM[maxf + ty]) * invM[2 * maxf + tz];
        rho[I] = 2.0 * s * im;
    }
}

// one workgroup per free z plane k
__global__ __launch_bounds__(256) void planar_kernel(const double *F, int nfx, int nfy, const double *mass, int maxf,
                                                     double scale, double *out) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    const int64_t plane = (int64_t)nfx * nfy;
    const double *Fk = F + (int64_t)k * plane;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < plane; e += 256) {
        const int tx = (int)(e % nfx), ty = (int)(e / nfx);
        s += (mass[tx] * mass[maxf + ty]) * Fk[e];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0] * scale;
}

// planar average of V_bare = (phi + w) + vapp (w, vapp may be null: 0),
// one workgroup per free z plane k, the order of planar_kernel
__global__ __launch_bounds__(256) void planar_bare_kernel(const double *phi, const double *w, const double *vapp,
                                                          int nfx, int nfy, const double *mass, int maxf,
                                                          double scale, double *out) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    const int64_t plane = (int64_t)nfx * nfy, off = (int64_t)k * plane;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < plane; e += 256) {
        const int tx = (int)(e % nfx), ty = (int)(e / nfx);
        double v = phi[off + e];
        if (w) v += w[off + e];
        if (vapp) v += vapp[off + e];
        s += (mass[tx] * mass[maxf + ty]) * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int wd = 128; wd >= 1; wd >>= 1) {
        if ((int)threadIdx.x < wd) red[threadIdx.x] += red[threadIdx.x + wd];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0] * scale;
}

// mu = sum_k m_z(k) (z_k - z0) P[k] over the free z positions, one workgroup,
// fixed order
__global__ __launch_bounds__(256) void zmoment_kernel(const double *P, int nz, const double *massz, const double *zc,
                                                      double z0, double *out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int kk = threadIdx.x; kk < nz; kk += 256) s += (massz[kk] * (zc[kk] - z0)) * P[kk];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

#define FE_HIPD(call, what)                                                                          \
    do {                                                                                             \
        hipError_t _e = (call);                                                                      \
        if (_e != hipSuccess) return fail(FE_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

}  // namespace

}  // namespace fe

using namespace fe;

extern "C" {

fe_status fe_density(fe_mesh *m, const double *X, int64_t N, int64_t ld, const double *f, double *rho,
                     hipStream_t st) {
    if (!m || !rho) return fail(FE_EINVAL, "NULL argument");
    if (N < 0) return fail(FE_EINVAL, "N must be >= 0");
    if (N > 0 && (!X || !f)) return fail(FE_EINVAL, "NULL X or f");
    if (ld < N) return fail(FE_EINVAL, "ld < N");
    FE_HIPD(hipSetDevice(m->device), "hipSetDevice");
    if (N == 0) {
        FE_HIPD(launch_fill(rho, m->n, 0.0, st), "fill");
        return FE_OK;
    }
    const int64_t threads = m->n * 16;
    const bool v2 = N % 2 == 0 && ld % 2 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(f) & 15) == 0;
    if (v2)
        hipLaunchKernelGGL(density_kernel<true>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, X, ld, N, f,
                           m->n, (int)m->nf[0], (int)m->nf[1], m->d_axis + 3 * m->maxf, m->maxf, rho);
    else
        hipLaunchKernelGGL(density_kernel<false>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, X, ld, N,
                           f, m->n, (int)m->nf[0], (int)m->nf[1], m->d_axis + 3 * m->maxf, m->maxf, rho);
    FE_HIPD(hipGetLastError(), "density kernel");
    return FE_OK;
}

fe_status fe_planar_average(fe_mesh *m, const double *field, int32_t normalize, double *out, hipStream_t st) {
    if (!m || !field || !out) return fail(FE_EINVAL, "NULL argument");
    if (normalize != 0 && normalize != 1) return fail(FE_EINVAL, "normalize must be 0 or 1");
    FE_HIPD(hipSetDevice(m->device), "hipSetDevice");
    double scale = 1.0;
    if (normalize) {
        double ax = 0.0, ay = 0.0;
        for (double v : m->axis_mass[0]) ax += v;
        for (double v : m->axis_mass[1]) ay += v;
        scale = 1.0 / (ax * ay);
    }
    hipLaunchKernelGGL(planar_kernel, dim3((unsigned)m->nf[2]), dim3(256), 0, st, field, (int)m->nf[0], (int)m->nf[1],
                       m->d_axis + 6 * m->maxf, m->maxf, scale, out);
    FE_HIPD(hipGetLastError(), "planar kernel");
    return FE_OK;
}

fe_status fe_bare_potential_planar(fe_mesh *m, const double *phi, const double *w, const double *vapp, double *out,
                                   hipStream_t st) {
    if (!m || !phi || !out) return fail(FE_EINVAL, "NULL argument");
    FE_HIPD(hipSetDevice(m->device), "hipSetDevice");
    double ax = 0.0, ay = 0.0;
    for (double v : m->axis_mass[0]) ax += v;
    for (double v : m->axis_mass[1]) ay += v;
    hipLaunchKernelGGL(planar_bare_kernel, dim3((unsigned)m->nf[2]), dim3(256), 0, st, phi, w, vapp, (int)m->nf[0],
                       (int)m->nf[1], m->d_axis + 6 * m->maxf, m->maxf, 1.0 / (ax * ay), out);
    FE_HIPD(hipGetLastError(), "planar kernel");
    return FE_OK;
}

fe_status fe_dipole(fe_mesh *m, const double *rho, double z0, double *mu_host, hipStream_t st) {
    if (!m || !rho || !mu_host) return fail(FE_EINVAL, "NULL argument");
    if (!std::isfinite(z0)) return fail(FE_EINVAL, "z0 must be finite");
    FE_HIPD(hipSetDevice(m->device), "hipSetDevice");
    const int nz = (int)m->nf[2];
    fe_status rc = ensure_scratch_dense(m, (size_t)(nz + 8) * sizeof(double));
    if (rc != FE_OK) return rc;
    double *planes = m->d_scratch, *res = m->d_scratch + nz;
    hipLaunchKernelGGL(planar_kernel, dim3((unsigned)nz), dim3(256), 0, st, rho, (int)m->nf[0], (int)m->nf[1],
                       m->d_axis + 6 * m->maxf, m->maxf, 1.0, planes);
    FE_HIPD(hipGetLastError(), "planar kernel");
    hipLaunchKernelGGL(zmoment_kernel, dim3(1), dim3(256), 0, st, planes, nz, m->d_axis + 8 * m->maxf, m->d_zcoord, z0,
                       res);
    FE_HIPD(hipGetLastError(), "z-moment kernel");
    FE_HIPD(hipMemcpyAsync(mu_host, res, sizeof(double), hipMemcpyDeviceToHost, st), "copy");
    FE_HIPD(hipStreamSynchronize(st), "hipStreamSynchronize");
    return FE_OK;
}

}  // extern "C"
