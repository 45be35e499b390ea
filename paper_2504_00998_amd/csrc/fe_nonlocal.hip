// Separable nonlocal pseudopotential term (paper Sec. 2.1, Eq. V_nloc and the
// action of H_nloc):
//
//   H~ += C~ diag(D) C~^T,   C~_{I,(s,beta)} = M_I^{1/2} p_{s,beta}(x_I),
//
// with p_{s,beta}(x) = S_beta(x - R_s) exp(-|x - R_s|^2 / (2 r_g^2)) inside the
// cutoff ball |x - R_s| < r_cut (minimum image on periodic axes), normalised
// to sum_I M_I p(x_I)^2 = 1, and S_beta the real solid harmonics 1; x, y, z;
// xy, yz, zx, x^2 - y^2, 3z^2 - r^2 (s, p, d channels).  The host builds the
// per-site supports and a colouring of the sites (sites that share a node
// differ in colour, found from the node -> site incidence), so that the
// application  Y += alpha C~ D C~^T X  runs on the device without atomics and
// gives the same bits on every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "fe_internal.h"

namespace fe {

// support entries per workgroup of the expansion kernel
constexpr int64_t kNlChunk = 64;
// rows loaded ahead of their products in the projection and expansion loops
constexpr int kNlBatch = 8;

// Device-resident scratch of the allocation-free H~X entry point
// (fe_hx_apply_noalloc): the nonlocal projections W = D C~^T X of one call,
// 9 n_site N doubles, at most kStaticScratchDoubles (32 MiB) per device.  Each
// device that loads the library holds its own copy until the process ends;
// every call on a device shares it, so calls that overlap on one device race.
// Host code never uses the array's name as an address: the device address is
// resolved once per device (static_scratch_init, from fe_mesh_create) and
// kept in g_scratch_ptr.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

fe_status static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(FE_EDEVICE, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return FE_OK;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    double *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(reinterpret_cast<void **>(&ptr), HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(FE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
    return FE_OK;
}

double *static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

namespace {

double solid_harmonic(int beta, double x, double y, double z) {
    switch (beta) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return y * z;
    case 6: return z * x;
    case 7: return x * x - y * y;
    default: return 2.0 * z * z - x * x - y * y;  // 3 z^2 - r^2
    }
}

void free_nl(NonlocalData &nl) {
    (void)hipFree(nl.d_supp_ptr);
    (void)hipFree(nl.d_supp_dof);
    (void)hipFree(nl.d_vals);
    (void)hipFree(nl.d_D);
    (void)hipFree(nl.d_W);
    (void)hipFree(nl.d_phase);
    (void)hipFree(nl.d_chunk_site);
    (void)hipFree(nl.d_chunk_e0);
    nl = NonlocalData();
}

}  // namespace

void nonlocal_release(fe_mesh *m) { free_nl(m->nl); }

// the value a double register holds in lane l (l uniform)
__device__ __forceinline__ double lane_double(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// W[(s*9+beta)][j] = D_{s,beta} sum_{e in supp(s)} C~[e][beta] X[dof(e)][j]
// One workgroup per site and 64 columns; its kNlWaves waves take contiguous
// parts of the support, and the partial sums meet in LDS in wave
// order, so the result does not depend on timing.
constexpr int kNlWaves = 8;
__global__ void __launch_bounds__(64 * kNlWaves)
    nl_project_kernel(const double *__restrict__ X, int64_t ldx, int64_t N, const int64_t *__restrict__ supp_ptr,
                      const int32_t *__restrict__ supp_dof, const double *__restrict__ vals,
                      const double *__restrict__ D, double *__restrict__ W) {
    __shared__ double part[kNlWaves][9][64];
    // workgroups of one site are consecutive (its matrix rows stay in cache)
    const int64_t ncb = (N + 63) / 64;
    const int s = (int)(blockIdx.x / ncb);
    const int64_t cb = blockIdx.x % ncb;
    // the wave index is uniform over the wave: the entry loop runs on scalar
    // registers
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t j = cb * 64 + lane;
    const int64_t s0 = supp_ptr[s], len = supp_ptr[s + 1] - s0;
    const int64_t e0 = s0 + len * wv / kNlWaves, e1 = s0 + len * (wv + 1) / kNlWaves;
    // every lane takes part in the loads that are broadcast; a lane past the
    // last column reads column N - 1 and its sums are dropped
    const int64_t jl = j < N ? j : N - 1;
    double acc[9];
#pragma unroll
    for (int b = 0; b < 9; ++b) acc[b] = 0.0;
    int64_t e = e0;
    if (e + kNlBatch <= e1) {
        // batches of kNlBatch rows: the batch's row indices come through one
        // scalar load, made while the previous batch is in flight; its 9
        // kNlBatch matrix entries through two vector loads spread over the
        // lanes (issued with the rows of X) and broadcast with readlane
        static_assert(kNlBatch == 8, "72 matrix entries in two loads of 64 and 8");
        int d[kNlBatch];
#pragma unroll
        for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[e + t];
        for (; e + kNlBatch <= e1; e += kNlBatch) {
            const double va = vals[e * 9 + lane], vb = vals[e * 9 + 64 + (lane & 7)];
            double x[kNlBatch];
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) x[t] = X[(int64_t)d[t] * ldx + jl];
            // indices of the next full batch (this one's again after the last)
            const int64_t en = e + 2 * kNlBatch <= e1 ? e + kNlBatch : e;
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[en + t];
            // keep all loads of the batch ahead of its products
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) {
#pragma unroll
                for (int b = 0; b < 9; ++b) {
                    const int q = t * 9 + b;
                    acc[b] += (q < 64 ? lane_double(va, q) : lane_double(vb, q - 64)) * x[t];
                }
            }
        }
    }
    for (; e < e1; ++e) {
        const double x = X[(int64_t)supp_dof[e] * ldx + jl];
        const double *v = vals + e * 9;
#pragma unroll
        for (int b = 0; b < 9; ++b) acc[b] += v[b] * x;
    }
#pragma unroll
    for (int b = 0; b < 9; ++b) part[wv][b][lane] = acc[b];
    __syncthreads();
    for (int q = threadIdx.x; q < 9 * 64; q += 64 * kNlWaves) {
        const int b = q >> 6, c = q & 63;
        const int64_t jc = cb * 64 + c;
        if (jc >= N) continue;
        double t = part[0][b][c];
#pragma unroll
        for (int w = 1; w < kNlWaves; ++w) t += part[w][b][c];
        W[((int64_t)s * 9 + b) * N + jc] = D[s * 9 + b] * t;
    }
}

// Y[dof(e)][j] += alpha sum_beta C~[e][beta] W[(site(e)*9+beta)][j], entry
// by entry, over chunks of the supports of the sites of one colour (disjoint
// supports, so no two workgroups of a launch touch one row of Y), the site's
// nine W values held in registers.  A node in the supports of sites of
// several colours takes their terms colour by colour.
__global__ void nl_expand_chunk_kernel(double *__restrict__ Y, int64_t ldy, int64_t N, double alpha,
                                       const int32_t *__restrict__ chunk_site, const int64_t *__restrict__ chunk_e0,
                                       const int64_t *__restrict__ supp_ptr, const int32_t *__restrict__ supp_dof,
                                       const double *__restrict__ vals, const double *__restrict__ W) {
    // workgroups of one chunk are consecutive (its matrix rows stay in cache)
    const int64_t ncb = (N + blockDim.x - 1) / blockDim.x;
    const int64_t q = blockIdx.x / ncb, cb = blockIdx.x % ncb;
    const int s = chunk_site[q];
    const int lane = threadIdx.x & 63;
    const int64_t j = cb * blockDim.x + threadIdx.x;
    // a wave whose 64 columns all exist takes the batched path below, which
    // broadcasts loads across the lanes; a wave at the ragged end of the
    // columns goes entry by entry
    const int64_t wave_end = cb * blockDim.x + (threadIdx.x & ~63) + 64;
    const bool full = wave_end <= N;
    if (!full && j >= N) return;
    double w[9];
#pragma unroll
    for (int b = 0; b < 9; ++b) w[b] = W[((int64_t)s * 9 + b) * N + j];
    const int64_t e0 = chunk_e0[q];
    const int64_t e1 = min(e0 + (int64_t)kNlChunk, supp_ptr[s + 1]);
    int64_t e = e0;
    if (full && e + kNlBatch <= e1) {
        // batches of kNlBatch entries (distinct rows of Y): the row indices
        // through one scalar load, made while the previous batch is in
        // flight; the 9 kNlBatch matrix entries through two vector loads
        // spread over the lanes and broadcast with readlane; all loads of a
        // batch ahead of its stores
        int d[kNlBatch];
#pragma unroll
        for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[e + t];
        for (; e + kNlBatch <= e1; e += kNlBatch) {
            const double va = vals[e * 9 + lane], vb = vals[e * 9 + 64 + (lane & 7)];
            double y[kNlBatch];
            double *yp[kNlBatch];
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) {
                yp[t] = Y + (int64_t)d[t] * ldy + j;
                y[t] = *yp[t];
            }
            const int64_t en = e + 2 * kNlBatch <= e1 ? e + kNlBatch : e;
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[en + t];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) {
                double acc = 0.0;
#pragma unroll
                for (int b = 0; b < 9; ++b) {
                    const int q = t * 9 + b;
                    acc += (q < 64 ? lane_double(va, q) : lane_double(vb, q - 64)) * w[b];
                }
                *yp[t] = y[t] + alpha * acc;
            }
        }
    }
    for (; e < e1; ++e) {
        const double *v = vals + e * 9;
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < 9; ++b) acc += v[b] * w[b];
        double *y = Y + (int64_t)supp_dof[e] * ldy + j;
        *y += alpha * acc;
    }
}

// Bloch mode (paper Sec. 2.3 with k-point sampling): with u = exp(-i k.r) psi
// the projectors become C^k_I = exp(-i k.d_I) C~_I, d_I = x_I - R_s the
// minimum-image displacement (the cutoff ball never wraps onto itself, so one
// image per entry), and H~^k gains C^k diag(D) C^k^H.  Complex columns are
// interleaved (re, im); ph[e] = (cos k.d_e, sin k.d_e).
// W[(s*9+beta)][j] = D_{s,beta} sum_e exp(+i k.d_e) C~[e][beta] X[dof(e)][j],
// the projection kernel's layout and batching with complex columns: one lane
// per complex column (16 B), each batch's 16 phase values through one more
// vector load broadcast with readlane.
__global__ void __launch_bounds__(64 * kNlWaves)
    nl_project_k_kernel(const double *__restrict__ X, int64_t ldx, int64_t N, const int64_t *__restrict__ supp_ptr,
                        const int32_t *__restrict__ supp_dof, const double *__restrict__ vals,
                        const double *__restrict__ ph, const double *__restrict__ D, double *__restrict__ W) {
    __shared__ double part[kNlWaves][9][64][2];
    const int64_t ncb = (N + 63) / 64;
    const int s = (int)(blockIdx.x / ncb);
    const int64_t cb = blockIdx.x % ncb;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t j = cb * 64 + lane;
    const int64_t jl = j < N ? j : N - 1;
    const int64_t s0 = supp_ptr[s], len = supp_ptr[s + 1] - s0;
    const int64_t e0 = s0 + len * wv / kNlWaves, e1 = s0 + len * (wv + 1) / kNlWaves;
    double ar[9], ai[9];
#pragma unroll
    for (int b = 0; b < 9; ++b) ar[b] = ai[b] = 0.0;
    int64_t e = e0;
    if (e + kNlBatch <= e1) {
        static_assert(kNlBatch == 8, "72 matrix entries in two loads of 64 and 8, 16 phases in one");
        int d[kNlBatch];
#pragma unroll
        for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[e + t];
        for (; e + kNlBatch <= e1; e += kNlBatch) {
            const double va = vals[e * 9 + lane], vb = vals[e * 9 + 64 + (lane & 7)];
            const double vp = ph[2 * e + (lane & 15)];
            double xr[kNlBatch], xi[kNlBatch];  // complex blocks are only 8-byte aligned
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) {
                const double *xp = X + (int64_t)d[t] * ldx + 2 * jl;
                xr[t] = xp[0];
                xi[t] = xp[1];
            }
            const int64_t en = e + 2 * kNlBatch <= e1 ? e + kNlBatch : e;
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[en + t];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) {
                const double c = lane_double(vp, 2 * t), sn = lane_double(vp, 2 * t + 1);
                const double tr = c * xr[t] - sn * xi[t], ti = sn * xr[t] + c * xi[t];
#pragma unroll
                for (int b = 0; b < 9; ++b) {
                    const int q = t * 9 + b;
                    const double v = q < 64 ? lane_double(va, q) : lane_double(vb, q - 64);
                    ar[b] += v * tr;
                    ai[b] += v * ti;
                }
            }
        }
    }
    for (; e < e1; ++e) {
        const double *x = X + (int64_t)supp_dof[e] * ldx + 2 * jl;
        const double c = ph[2 * e], sn = ph[2 * e + 1];
        const double tr = c * x[0] - sn * x[1], ti = sn * x[0] + c * x[1];
        const double *v = vals + e * 9;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            ar[b] += v[b] * tr;
            ai[b] += v[b] * ti;
        }
    }
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        part[wv][b][lane][0] = ar[b];
        part[wv][b][lane][1] = ai[b];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 9 * 64; q += 64 * kNlWaves) {
        const int b = q >> 6, c = q & 63;
        const int64_t jc = cb * 64 + c;
        if (jc >= N) continue;
        double tr = part[0][b][c][0], ti = part[0][b][c][1];
#pragma unroll
        for (int w = 1; w < kNlWaves; ++w) {
            tr += part[w][b][c][0];
            ti += part[w][b][c][1];
        }
        double *o = W + ((int64_t)s * 9 + b) * 2 * N + 2 * jc;
        o[0] = D[s * 9 + b] * tr;
        o[1] = D[s * 9 + b] * ti;
    }
}

// Y[dof(e)][j] += alpha exp(-i k.d_e) sum_beta C~[e][beta] W[(site(e)*9+beta)][j],
// the expansion kernel's chunks, colours and batching with complex columns.
__global__ void nl_expand_k_kernel(double *__restrict__ Y, int64_t ldy, int64_t N, double alpha,
                                   const int32_t *__restrict__ chunk_site, const int64_t *__restrict__ chunk_e0,
                                   const int64_t *__restrict__ supp_ptr, const int32_t *__restrict__ supp_dof,
                                   const double *__restrict__ vals, const double *__restrict__ ph,
                                   const double *__restrict__ W) {
    const int64_t ncb = (N + blockDim.x - 1) / blockDim.x;
    const int64_t q = blockIdx.x / ncb, cb = blockIdx.x % ncb;
    const int s = chunk_site[q];
    const int lane = threadIdx.x & 63;
    const int64_t j = cb * blockDim.x + threadIdx.x;
    const int64_t wave_end = cb * blockDim.x + (threadIdx.x & ~63) + 64;
    const bool full = wave_end <= N;
    if (!full && j >= N) return;
    double wr[9], wi[9];
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        const double *w = W + ((int64_t)s * 9 + b) * 2 * N + 2 * j;
        wr[b] = w[0];
        wi[b] = w[1];
    }
    const int64_t e0 = chunk_e0[q];
    const int64_t e1 = min(e0 + (int64_t)kNlChunk, supp_ptr[s + 1]);
    int64_t e = e0;
    if (full && e + kNlBatch <= e1) {
        int d[kNlBatch];
#pragma unroll
        for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[e + t];
        for (; e + kNlBatch <= e1; e += kNlBatch) {
            const double va = vals[e * 9 + lane], vb = vals[e * 9 + 64 + (lane & 7)];
            const double vp = ph[2 * e + (lane & 15)];
            double yr[kNlBatch], yi[kNlBatch];
            double *yp[kNlBatch];
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) {
                yp[t] = Y + (int64_t)d[t] * ldy + 2 * j;
                yr[t] = yp[t][0];
                yi[t] = yp[t][1];
            }
            const int64_t en = e + 2 * kNlBatch <= e1 ? e + kNlBatch : e;
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) d[t] = supp_dof[en + t];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < kNlBatch; ++t) {
                double tr = 0.0, ti = 0.0;
#pragma unroll
                for (int b = 0; b < 9; ++b) {
                    const int qq = t * 9 + b;
                    const double v = qq < 64 ? lane_double(va, qq) : lane_double(vb, qq - 64);
                    tr += v * wr[b];
                    ti += v * wi[b];
                }
                const double c = lane_double(vp, 2 * t), sn = lane_double(vp, 2 * t + 1);
                yp[t][0] = yr[t] + alpha * (c * tr + sn * ti);
                yp[t][1] = yi[t] + alpha * (c * ti - sn * tr);
            }
        }
    }
    for (; e < e1; ++e) {
        const double *v = vals + e * 9;
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            tr += v[b] * wr[b];
            ti += v[b] * wi[b];
        }
        const double c = ph[2 * e], sn = ph[2 * e + 1];
        double *y = Y + (int64_t)supp_dof[e] * ldy + 2 * j;
        y[0] += alpha * (c * tr + sn * ti);
        y[1] += alpha * (c * ti - sn * tr);
    }
}

size_t nonlocal_work_doubles(const fe_mesh *m, int64_t N) { return (size_t)m->nl.n_site * 9 * (size_t)N; }

static hipError_t ensure_nl_work(fe_mesh *m, int64_t N) {
    size_t need = nonlocal_work_doubles(m, N);
    if (need <= m->nl.W_cap) return hipSuccess;
    if (m->nl.d_W) {
        hipError_t e = hipFree(m->nl.d_W);  // synchronises the device
        if (e != hipSuccess) return e;
        m->nl.d_W = nullptr;
        m->nl.W_cap = 0;
    }
    hipError_t e = hipMalloc(&m->nl.d_W, need * sizeof(double));
    if (e != hipSuccess) return e;
    m->nl.W_cap = need;
    return hipSuccess;
}

hipError_t launch_nonlocal(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t N,
                           double alpha, hipStream_t s, double *W) {
    if (m->nl.n_site == 0 || N <= 0) return hipSuccess;
    if (!W) {
        hipError_t e = ensure_nl_work(m, N);
        if (e != hipSuccess) return e;
        W = m->nl.d_W;
    }
    hipError_t e;
    const int TB = 128;
    const int64_t nb1 = (int64_t)m->nl.n_site * ((N + 63) / 64);
    if (nb1 > INT32_MAX) return hipErrorInvalidConfiguration;
    dim3 g1((unsigned)nb1);
    hipLaunchKernelGGL(nl_project_kernel, g1, dim3(64 * kNlWaves), 0, s, X, ldx, N, (const int64_t *)m->nl.d_supp_ptr,
                       (const int32_t *)m->nl.d_supp_dof, (const double *)m->nl.d_vals, (const double *)m->nl.d_D,
                       W);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m->nl.n_node == 0) return hipSuccess;
    // one launch per site colour, one workgroup per support chunk and column block
    const std::vector<int64_t> &cp = m->nl.chunk_col_ptr;
    for (size_t c = 0; c + 1 < cp.size(); ++c) {
        const int64_t nq = cp[c + 1] - cp[c];
        if (nq == 0) continue;
        const int64_t nb2 = nq * ((N + TB - 1) / TB);
        if (nb2 > INT32_MAX) return hipErrorInvalidConfiguration;
        dim3 g2((unsigned)nb2);
        hipLaunchKernelGGL(nl_expand_chunk_kernel, g2, dim3(TB), 0, s, Y, ldy, N, alpha,
                           (const int32_t *)m->nl.d_chunk_site + cp[c], (const int64_t *)m->nl.d_chunk_e0 + cp[c],
                           (const int64_t *)m->nl.d_supp_ptr, (const int32_t *)m->nl.d_supp_dof,
                           (const double *)m->nl.d_vals, (const double *)W);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// complex blocks: N complex columns, ldx / ldy in doubles
hipError_t launch_nonlocal_k(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t N,
                             double alpha, hipStream_t s) {
    if (m->nl.n_site == 0 || N <= 0) return hipSuccess;
    if (!m->nl.d_phase) return hipErrorInvalidValue;
    hipError_t e = ensure_nl_work(m, 2 * N);
    if (e != hipSuccess) return e;
    const int TB = 128;
    const int64_t nb1 = (int64_t)m->nl.n_site * ((N + 63) / 64);
    if (nb1 > INT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(nl_project_k_kernel, dim3((unsigned)nb1), dim3(64 * kNlWaves), 0, s, X, ldx, N,
                       (const int64_t *)m->nl.d_supp_ptr, (const int32_t *)m->nl.d_supp_dof,
                       (const double *)m->nl.d_vals, (const double *)m->nl.d_phase, (const double *)m->nl.d_D,
                       m->nl.d_W);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const std::vector<int64_t> &cp = m->nl.chunk_col_ptr;
    for (size_t c = 0; c + 1 < cp.size(); ++c) {
        const int64_t nq = cp[c + 1] - cp[c];
        if (nq == 0) continue;
        const int64_t nb2 = nq * ((N + TB - 1) / TB);
        if (nb2 > INT32_MAX) return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL(nl_expand_k_kernel, dim3((unsigned)nb2), dim3(TB), 0, s, Y, ldy, N, alpha,
                           (const int32_t *)m->nl.d_chunk_site + cp[c], (const int64_t *)m->nl.d_chunk_e0 + cp[c],
                           (const int64_t *)m->nl.d_supp_ptr, (const int32_t *)m->nl.d_supp_dof,
                           (const double *)m->nl.d_vals, (const double *)m->nl.d_phase, (const double *)m->nl.d_W);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// (cos, sin) of k.d for every support entry, for the mesh's current k
// (host build, synchronous upload; nothing to do without sites).
fe_status nonlocal_set_phase(fe_mesh *m) {
    NonlocalData &nl = m->nl;
    if (nl.n_site == 0 || nl.nnz == 0) return FE_OK;
    std::vector<double> ph(2 * (size_t)nl.nnz);
    for (int64_t e = 0; e < nl.nnz; ++e) {
        const double t = m->kvec[0] * nl.disp[2 * e] + m->kvec[1] * nl.disp[2 * e + 1];
        ph[2 * e] = std::cos(t);
        ph[2 * e + 1] = std::sin(t);
    }
    if (!nl.d_phase && hipMalloc(&nl.d_phase, ph.size() * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        nl.d_phase = nullptr;
        return fail(FE_ENOMEM, "device allocation failed for the projector phases");
    }
    if (hipMemcpy(nl.d_phase, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FE_EDEVICE, "hipMemcpy of the projector phases failed");
    return FE_OK;
}

}  // namespace fe

using namespace fe;

extern "C" {

fe_status fe_set_nonlocal(fe_mesh *m, int32_t n_site, const double *centres, const double *D, double r_cut,
                          double r_g, hipStream_t st) {
    if (!m) return fail(FE_EINVAL, "NULL mesh");
    if (n_site < 0) return fail(FE_EINVAL, "n_site must be >= 0");
    if (n_site > 0) {
        if (!centres || !D) return fail(FE_EINVAL, "NULL centres or D");
        if (!(r_cut > 0.0) || !(r_g > 0.0) || !std::isfinite(r_cut) || !std::isfinite(r_g))
            return fail(FE_EINVAL, "r_cut and r_g must be positive");
        for (int a = 0; a < 3; ++a)
            if (m->bc[a] == FE_BC_PERIODIC && 2.0 * r_cut >= m->L[a])
                return fail(FE_EINVAL, "cutoff ball wraps onto itself on a periodic axis");
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(FE_EDEVICE, "stream synchronisation failed");
    free_nl(m->nl);
    if (n_site == 0) return FE_OK;

    // per-axis free positions within r_cut of each centre coordinate
    std::vector<int64_t> supp_ptr(1, 0);
    std::vector<int32_t> supp_dof;
    std::vector<double> vals, disp;
    for (int s = 0; s < n_site; ++s) {
        std::vector<std::pair<int64_t, double>> cand[3];  // (free index, signed offset)
        for (int a = 0; a < 3; ++a) {
            for (int64_t t = 0; t < m->nf[a]; ++t) {
                double d = m->axis_coord[a][t] - centres[3 * s + a];
                if (m->bc[a] == FE_BC_PERIODIC) d -= m->L[a] * std::nearbyint(d / m->L[a]);
                if (std::fabs(d) < r_cut) cand[a].push_back({t, d});
            }
        }
        std::vector<std::pair<int32_t, double>> pts;  // (dof, M_I)
        std::vector<double> pv, pd;                   // projector values; in-plane offsets
        double nrm[9] = {0};
        for (auto &z : cand[2])
            for (auto &y : cand[1])
                for (auto &x : cand[0]) {
                    double r2 = x.second * x.second + y.second * y.second + z.second * z.second;
                    if (!(r2 < r_cut * r_cut)) continue;
                    int64_t I = x.first + m->nf[0] * (y.first + m->nf[1] * z.first);
                    double M = m->axis_mass[0][x.first] * m->axis_mass[1][y.first] * m->axis_mass[2][z.first];
                    double rad = std::exp(-r2 / (2.0 * r_g * r_g));
                    pts.push_back({(int32_t)I, M});
                    pd.push_back(x.second);
                    pd.push_back(y.second);
                    for (int b = 0; b < 9; ++b) {
                        double p = solid_harmonic(b, x.second, y.second, z.second) * rad;
                        pv.push_back(p);
                        nrm[b] += M * p * p;
                    }
                }
        // increasing DoF order within the support
        std::vector<size_t> order(pts.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](size_t u, size_t v) { return pts[u].first < pts[v].first; });
        for (size_t oi : order) {
            supp_dof.push_back(pts[oi].first);
            disp.push_back(pd[2 * oi]);
            disp.push_back(pd[2 * oi + 1]);
            double sq = std::sqrt(pts[oi].second);
            for (int b = 0; b < 9; ++b) {
                double sc = nrm[b] > 0.0 ? 1.0 / std::sqrt(nrm[b]) : 0.0;
                vals.push_back(pv[oi * 9 + b] * sc * sq);
            }
        }
        supp_ptr.push_back((int64_t)supp_dof.size());
    }
    // node -> incident support entries, nodes ascending, entries by site then position
    std::vector<std::pair<int32_t, int64_t>> inc;  // (dof, entry)
    inc.reserve(supp_dof.size());
    for (int64_t e = 0; e < (int64_t)supp_dof.size(); ++e) inc.push_back({supp_dof[e], e});
    std::stable_sort(inc.begin(), inc.end(), [](const auto &u, const auto &v) { return u.first < v.first; });
    std::vector<int32_t> node;
    std::vector<int64_t> inc_ptr(1, 0), inc_entry;
    std::vector<int32_t> entry_site(supp_dof.size());
    for (int s = 0; s < n_site; ++s)
        for (int64_t e = supp_ptr[s]; e < supp_ptr[s + 1]; ++e) entry_site[e] = s;
    for (size_t i = 0; i < inc.size(); ++i) {
        if (node.empty() || node.back() != inc[i].first) {
            if (!node.empty()) inc_ptr.push_back((int64_t)inc_entry.size());
            node.push_back(inc[i].first);
        }
        inc_entry.push_back(inc[i].second);
    }
    inc_ptr.push_back((int64_t)inc_entry.size());
    // site colours: sites that share a node get different colours (greedy,
    // in site order), so that the sites of one colour can add to Y at once
    std::vector<std::vector<int>> nbr(n_site);
    for (size_t u = 0; u + 1 < inc_ptr.size(); ++u)
        for (int64_t a = inc_ptr[u]; a < inc_ptr[u + 1]; ++a)
            for (int64_t b = a + 1; b < inc_ptr[u + 1]; ++b) {
                const int sa = entry_site[inc_entry[a]], sb = entry_site[inc_entry[b]];
                if (sa != sb) {
                    nbr[sa].push_back(sb);
                    nbr[sb].push_back(sa);
                }
            }
    for (auto &v : nbr) {
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    std::vector<int> colour(n_site, -1);
    int ncol = 0;
    for (int s = 0; s < n_site; ++s) {
        std::vector<char> used(ncol + 1, 0);
        for (int t : nbr[s])
            if (colour[t] >= 0) used[colour[t]] = 1;
        int c = 0;
        while (used[c]) ++c;
        colour[s] = c;
        ncol = std::max(ncol, c + 1);
    }
    std::vector<int32_t> chunk_site;
    std::vector<int64_t> chunk_e0, chunk_col_ptr(1, 0);
    for (int c = 0; c < ncol; ++c) {
        for (int s = 0; s < n_site; ++s)
            if (colour[s] == c)
                for (int64_t e = supp_ptr[s]; e < supp_ptr[s + 1]; e += kNlChunk) {
                    chunk_site.push_back(s);
                    chunk_e0.push_back(e);
                }
        chunk_col_ptr.push_back((int64_t)chunk_site.size());
    }

    NonlocalData &nl = m->nl;
    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (bytes == 0) bytes = 8;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = up((void **)&nl.d_supp_ptr, supp_ptr.data(), supp_ptr.size() * sizeof(int64_t)) &&
              up((void **)&nl.d_supp_dof, supp_dof.data(), supp_dof.size() * sizeof(int32_t)) &&
              up((void **)&nl.d_vals, vals.data(), vals.size() * sizeof(double)) &&
              up((void **)&nl.d_D, D, (size_t)n_site * 9 * sizeof(double)) &&
              up((void **)&nl.d_chunk_site, chunk_site.data(), chunk_site.size() * sizeof(int32_t)) &&
              up((void **)&nl.d_chunk_e0, chunk_e0.data(), chunk_e0.size() * sizeof(int64_t));
    if (!ok) {
        (void)hipGetLastError();
        free_nl(nl);
        return fail(FE_ENOMEM, "device allocation failed in fe_set_nonlocal");
    }
    nl.n_site = n_site;
    nl.nnz = (int64_t)supp_dof.size();
    nl.n_node = (int64_t)node.size();
    nl.disp.swap(disp);
    nl.chunk_col_ptr.swap(chunk_col_ptr);
    const fe_status ps = nonlocal_set_phase(m);
    if (ps != FE_OK) free_nl(nl);
    return ps;
}

}  // extern "C"
