// gfx950 kernels of the FE Hamiltonian filter.
//
// One application of H~ = M^-1/2 (1/2 K + V) M^-1/2 (paper Sec. 2.3 with the
// Hamiltonian of Sec. 2.1 and the field term of Sec. 2.2.1) is
//
//   (H~ X)_I = D_I sum_{c containing I} [A (D X)_c]_{l_c(I)} + v_I X_I,
//
// with A = 1/2 Kc the dense cell matrix shared by every (cubic) cell and
// D = M^-1/2 separable over the axes.  The fused step kernel computes, for a
// Chebyshev step,
//
//   Y_{k+1} = alpha (H~ - c) Y_k - beta Y_{k-1}
//
// as: gather (D Y_k)_c for a cell and 16 vectors into LDS -> dense
// A (D Y_k)_c on MFMA -> scatter each row to its node with the recurrence
// epilogue.  Cells are coloured (parity per axis; a third colour on a
// periodic axis with an odd cell count) so that cells of one colour share no
// node; one launch per colour, in a fixed order.  The first colour to reach
// a node writes  alpha (v_I - c) Y_k - beta Y_{k-1} + its contribution;
// later colours add theirs.  The sum order is therefore fixed and the result
// bitwise reproducible, with no atomics.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fe_internal.h"

namespace fe {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int64_t axis_free_index(const AxisInfo &a, int p, int64_t g) {
    int64_t k = (int64_t)a.ncell * p;
    if (a.bc == FE_BC_DIRICHLET) return (g == 0 || g == k) ? -1 : g - 1;
    if (a.bc == FE_BC_PERIODIC) return g % k;
    return g;
}

__device__ __forceinline__ int axis_colour(const AxisInfo &a, int c) {
    return (a.ncol == 3 && c == a.ncell - 1) ? 2 : (c & 1);
}

// Neighbour cell along the axis that shares local node i of cell c, or -1.
__device__ __forceinline__ int axis_neighbour(const AxisInfo &a, int p, int c, int i) {
    if (i == 0) {
        if (c > 0) return c - 1;
        return a.bc == FE_BC_PERIODIC ? a.ncell - 1 : -1;
    }
    if (i == p) {
        if (c < a.ncell - 1) return c + 1;
        return a.bc == FE_BC_PERIODIC ? 0 : -1;
    }
    return -1;
}

// k-th cell of colour col along an axis.
__device__ __forceinline__ int colour_cell(const AxisInfo &a, int col, int k) {
    return col == 2 ? a.ncell - 1 : col + 2 * k;
}

// FP64 -> FP32 (RNE) -> BF16 (RNE), returned as raw bits.
__device__ __forceinline__ uint16_t to_bf16_bits(double x) {
    float f = (float)x;
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct StepParams {
    const double *X;
    int64_t ldx;
    double *Y;
    int64_t ldy;
    const double *Ym1;
    int64_t ldm;
    double alpha, beta, shift;
    int64_t N;
    int nchunk;
    const double *axisD;  // [3][maxf]
    int maxf;
    const double *v;
    const void *A;
    AxisInfo ax[3];
    int col[3];
    int cnt[3];
    int64_t nfx, nfy;
};

template <int PREC> struct PrecTraits;
template <> struct PrecTraits<0> { typedef double T; static constexpr int KSTEP = 4; };
template <> struct PrecTraits<1> { typedef float T; static constexpr int KSTEP = 4; };
template <> struct PrecTraits<2> { typedef uint16_t T; static constexpr int KSTEP = 32; };

// LDS row stride (elements) of the transposed bf16 operand: pad by 8 to
// spread the 16 column reads of a fragment over the banks.
template <int NCP> struct Bf16Stride { static constexpr int value = NCP + 8; };

template <int P, int PREC>
__global__ __launch_bounds__(256) void step_kernel(StepParams k) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32, NT = NCP / 16;
    constexpr int KSTEP = PrecTraits<PREC>::KSTEP, NKS = NCP / KSTEP;
    typedef typename PrecTraits<PREC>::T T;
    extern __shared__ __align__(16) unsigned char smem[];
    T *xs = reinterpret_cast<T *>(smem);
    constexpr size_t xs_bytes = (PREC == 2 ? (size_t)16 * Bf16Stride<NCP>::value : (size_t)NCP * 16) * sizeof(T);
    int64_t *dof = reinterpret_cast<int64_t *>(smem + ((xs_bytes + 15) / 16) * 16);
    double *dsc = reinterpret_cast<double *>(dof + NCP);
    unsigned char *first = reinterpret_cast<unsigned char *>(dsc + NCP);

    const int tid = threadIdx.x;
    const int chunk = blockIdx.x % k.nchunk;
    int cidx = blockIdx.x / k.nchunk;
    const int ix = cidx % k.cnt[0];
    cidx /= k.cnt[0];
    const int iy = cidx % k.cnt[1];
    const int iz = cidx / k.cnt[1];
    const int cx = colour_cell(k.ax[0], k.col[0], ix);
    const int cy = colour_cell(k.ax[1], k.col[1], iy);
    const int cz = colour_cell(k.ax[2], k.col[2], iz);

    // node table of the cell: DoF, D scale, and whether this colour is the
    // first to write the node
    for (int l = tid; l < NCP; l += 256) {
        int64_t I = -1;
        double d = 0.0;
        unsigned char f = 1;
        if (l < NC) {
            int li[3] = {l % N1, (l / N1) % N1, l / (N1 * N1)};
            int cc[3] = {cx, cy, cz};
            int64_t t[3];
            bool ok = true;
            d = 1.0;
            for (int a = 0; a < 3; ++a) {
                t[a] = axis_free_index(k.ax[a], P, (int64_t)cc[a] * P + li[a]);
                if (t[a] < 0) { ok = false; break; }
                d *= k.axisD[a * k.maxf + t[a]];
                int nb = axis_neighbour(k.ax[a], P, cc[a], li[a]);
                if (nb >= 0 && axis_colour(k.ax[a], nb) < axis_colour(k.ax[a], cc[a])) f = 0;
            }
            if (ok) I = t[0] + k.nfx * (t[1] + k.nfy * t[2]);
            else d = 0.0;
        }
        dof[l] = I;
        dsc[l] = d;
        first[l] = f;
    }
    __syncthreads();

    // gather (D X)_c for this chunk of 16 vectors into LDS (rounded per PREC)
    const int64_t vec0 = (int64_t)chunk * 16;
    for (int e = tid; e < NCP * 16; e += 256) {
        int l = e >> 4, c = e & 15;
        int64_t I = dof[l];
        double x = 0.0;
        if (I >= 0 && vec0 + c < k.N) x = dsc[l] * k.X[I * k.ldx + vec0 + c];
        if constexpr (PREC == 0) xs[e] = x;
        else if constexpr (PREC == 1) xs[e] = (float)x;
        else xs[c * Bf16Stride<NCP>::value + l] = to_bf16_bits(x);
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int col = lane & 15;
    const int64_t vec = vec0 + col;
    for (int t = wave; t < NT; t += 4) {
        double acc[4];
        if constexpr (PREC == 0) {
            const double *A = reinterpret_cast<const double *>(k.A) + (size_t)t * NKS * 64 + lane;
            d4 c4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int s = 0; s < NKS; ++s) {
                double a = A[s * 64];
                double b = xs[(4 * s + (lane >> 4)) * 16 + col];
                c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c4, 0, 0, 0);
            }
            for (int i = 0; i < 4; ++i) acc[i] = c4[i];
        } else if constexpr (PREC == 1) {
            const float *A = reinterpret_cast<const float *>(k.A) + (size_t)t * NKS * 64 + lane;
            f4 c4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int s = 0; s < NKS; ++s) {
                float a = A[s * 64];
                float b = xs[(4 * s + (lane >> 4)) * 16 + col];
                c4 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c4, 0, 0, 0);
            }
            for (int i = 0; i < 4; ++i) acc[i] = (double)c4[i];
        } else {
            const uint4 *A = reinterpret_cast<const uint4 *>(k.A) + (size_t)t * NKS * 64 + lane;
            f4 c4 = {0.f, 0.f, 0.f, 0.f};
            const uint16_t *xrow = xs + col * Bf16Stride<NCP>::value + 8 * (lane >> 4);
#pragma unroll 2
            for (int s = 0; s < NKS; ++s) {
                uint4 av = A[s * 64];
                uint4 bv = *reinterpret_cast<const uint4 *>(xrow + 32 * s);
                bf8 a = __builtin_bit_cast(bf8, av);
                bf8 b = __builtin_bit_cast(bf8, bv);
                c4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c4, 0, 0, 0);
            }
            for (int i = 0; i < 4; ++i) acc[i] = (double)c4[i];
        }
        if (vec >= k.N) continue;
        for (int i = 0; i < 4; ++i) {
            // output row of accumulator i: f64 16x16x4 puts row (lane/16) + 4i
            // in lane's slot i; the f32 and bf16 shapes put row 4(lane/16) + i.
            int r = 16 * t + (PREC == 0 ? (lane >> 4) + 4 * i : 4 * (lane >> 4) + i);
            if (r >= NC) continue;
            int64_t I = dof[r];
            if (I < 0) continue;
            double contrib = k.alpha * dsc[r] * acc[i];
            double *y = k.Y + I * k.ldy + vec;
            if (first[r]) {
                double base = k.alpha * (k.v[I] - k.shift) * k.X[I * k.ldx + vec];
                if (k.Ym1) base -= k.beta * k.Ym1[I * k.ldm + vec];
                *y = base + contrib;
            } else {
                *y += contrib;
            }
        }
    }
}

template <int P, int PREC>
static size_t step_smem() {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32;
    typedef typename PrecTraits<PREC>::T T;
    size_t xs_bytes = (PREC == 2 ? (size_t)16 * Bf16Stride<NCP>::value : (size_t)NCP * 16) * sizeof(T);
    return ((xs_bytes + 15) / 16) * 16 + NCP * (sizeof(int64_t) + sizeof(double) + 1);
}

template <int P, int PREC>
static hipError_t launch_step_p(const fe_mesh *m, StepParams prm, hipStream_t s) {
    size_t smem = step_smem<P, PREC>();
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_kernel<P, PREC>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    // colours in lexicographic order (x fastest): the order the first-writer rule assumes
    for (int c2 = 0; c2 < m->ncol[2]; ++c2)
        for (int c1 = 0; c1 < m->ncol[1]; ++c1)
            for (int c0 = 0; c0 < m->ncol[0]; ++c0) {
                int col[3] = {c0, c1, c2};
                int64_t cells = 1;
                for (int a = 0; a < 3; ++a) {
                    const AxisInfo &ax = prm.ax[a];
                    int cnt;
                    if (col[a] == 2) cnt = 1;
                    else {
                        int limit = ax.ncol == 3 ? ax.ncell - 1 : ax.ncell;
                        cnt = limit > col[a] ? (limit - col[a] + 1) / 2 : 0;
                    }
                    prm.col[a] = col[a];
                    prm.cnt[a] = cnt;
                    cells *= cnt;
                }
                if (cells == 0) continue;
                int64_t blocks = cells * prm.nchunk;
                hipLaunchKernelGGL((step_kernel<P, PREC>), dim3((unsigned)blocks), dim3(256), smem, s, prm);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

hipError_t launch_step(const fe_mesh *m, const StepArgs &a, fe_dtype prec, hipStream_t s) {
    StepParams prm;
    prm.X = a.X; prm.ldx = a.ldx;
    prm.Y = a.Y; prm.ldy = a.ldy;
    prm.Ym1 = a.Ym1; prm.ldm = a.ldm;
    prm.alpha = a.alpha; prm.beta = a.beta; prm.shift = a.shift;
    prm.N = a.N;
    prm.nchunk = (int)((a.N + 15) / 16);
    prm.axisD = m->d_axis;
    prm.maxf = m->maxf;
    prm.v = m->d_v;
    prm.A = prec == FE_F64 ? (const void *)m->d_Af64 : prec == FE_F32 ? (const void *)m->d_Af32 : (const void *)m->d_Abf16;
    for (int d = 0; d < 3; ++d) {
        prm.ax[d].ncell = m->ncell[d];
        prm.ax[d].nfree = (int)m->nf[d];
        prm.ax[d].bc = m->bc[d];
        prm.ax[d].ncol = m->ncol[d];
    }
    prm.nfx = m->nf[0];
    prm.nfy = m->nf[1];
#define FE_DISPATCH(PP)                                                        \
    case PP:                                                                   \
        if (prec == FE_F64) return launch_step_p<PP, 0>(m, prm, s);            \
        if (prec == FE_F32) return launch_step_p<PP, 1>(m, prm, s);            \
        return launch_step_p<PP, 2>(m, prm, s);
    switch (m->p) {
        FE_DISPATCH(1)
        FE_DISPATCH(2)
        FE_DISPATCH(3)
        FE_DISPATCH(4)
        FE_DISPATCH(5)
        FE_DISPATCH(6)
        FE_DISPATCH(7)
    default: return hipErrorInvalidValue;
    }
#undef FE_DISPATCH
}

// ------------------------------------------------------- potential update

struct PotParams {
    const double *Vq;
    double E, z0;
    double *v;
    const double *axisMinv;  // [3][maxf] 1 / (assembled 1-D lumped mass)
    const double *wrel;      // [3][p+1] (h/2) w_i
    const double *zcoord;    // [nf_z]
    int maxf, p, nc;
    AxisInfo ax[3];
    int64_t nfx, nfy, n;
};

// Cells containing free position t along an axis, with local indices.
__device__ __forceinline__ int axis_cells_of(const AxisInfo &a, int p, int64_t t, int *cell, int *loc) {
    int64_t g = a.bc == FE_BC_DIRICHLET ? t + 1 : t;
    int n = 0;
    if (g % p != 0) { cell[0] = (int)(g / p); loc[0] = (int)(g % p); return 1; }
    int64_t c = g / p;
    if (c - 1 >= 0) { cell[n] = (int)(c - 1); loc[n] = p; ++n; }
    else if (a.bc == FE_BC_PERIODIC) { cell[n] = a.ncell - 1; loc[n] = p; ++n; }
    if (c < a.ncell) { cell[n] = (int)c; loc[n] = 0; ++n; }
    return n;
}

// v_I = sum_{(c,q)->I} (|J| w_q / M_I) V[c][q] - E (z_I - z0); the weight is
// separable: prod_a (h/2) w_{i_a} / M1_a.
__global__ void potential_kernel(PotParams k) {
    int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (I >= k.n) return;
    int64_t t[3] = {I % k.nfx, (I / k.nfx) % k.nfy, I / (k.nfx * k.nfy)};
    double acc = 0.0;
    if (k.Vq) {
        int cs[3][2], ls[3][2], nk[3];
        for (int a = 0; a < 3; ++a) nk[a] = axis_cells_of(k.ax[a], k.p, t[a], cs[a], ls[a]);
        int n1 = k.p + 1;
        for (int az = 0; az < nk[2]; ++az)
            for (int ay = 0; ay < nk[1]; ++ay)
                for (int axx = 0; axx < nk[0]; ++axx) {
                    int64_t cell = cs[0][axx] + (int64_t)k.ax[0].ncell * (cs[1][ay] + (int64_t)k.ax[1].ncell * cs[2][az]);
                    int l = ls[0][axx] + n1 * (ls[1][ay] + n1 * ls[2][az]);
                    double wgt = k.wrel[0 * n1 + ls[0][axx]] * k.axisMinv[0 * k.maxf + t[0]] *
                                 k.wrel[1 * n1 + ls[1][ay]] * k.axisMinv[1 * k.maxf + t[1]] *
                                 k.wrel[2 * n1 + ls[2][az]] * k.axisMinv[2 * k.maxf + t[2]];
                    acc += wgt * k.Vq[cell * k.nc + l];
                }
    }
    k.v[I] = acc - k.E * (k.zcoord[t[2]] - k.z0);
}

static PotParams pot_params(const fe_mesh *m) {
    PotParams k;
    k.axisMinv = m->d_axis + 3 * m->maxf;
    k.wrel = m->d_wrel;
    k.zcoord = m->d_zcoord;
    k.maxf = m->maxf;
    k.p = m->p;
    k.nc = m->nc;
    for (int d = 0; d < 3; ++d) {
        k.ax[d].ncell = m->ncell[d];
        k.ax[d].nfree = (int)m->nf[d];
        k.ax[d].bc = m->bc[d];
        k.ax[d].ncol = m->ncol[d];
    }
    k.nfx = m->nf[0];
    k.nfy = m->nf[1];
    k.n = m->n;
    return k;
}

hipError_t launch_potential(const fe_mesh *m, const double *Vq, double E, double z0, hipStream_t s) {
    PotParams k = pot_params(m);
    k.Vq = Vq; k.E = E; k.z0 = z0; k.v = m->d_v;
    int64_t blocks = (m->n + 255) / 256;
    hipLaunchKernelGGL(potential_kernel, dim3((unsigned)blocks), dim3(256), 0, s, k);
    return hipGetLastError();
}

// Vbar[c][q] = (|J| w_q / M_I) g_I for the point's DoF I (0 at Dirichlet points).
struct PotVjpParams {
    const double *g;
    double *Vbar;
    const double *axisMinv, *wrel;
    int maxf, p, nc;
    AxisInfo ax[3];
    int64_t nfx, nfy, ncells;
};

__global__ void potential_vjp_kernel(PotVjpParams k) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= k.ncells * k.nc) return;
    int64_t c = e / k.nc;
    int l = (int)(e % k.nc);
    int n1 = k.p + 1;
    int li[3] = {l % n1, (l / n1) % n1, l / (n1 * n1)};
    int64_t cc[3] = {c % k.ax[0].ncell, (c / k.ax[0].ncell) % k.ax[1].ncell, c / ((int64_t)k.ax[0].ncell * k.ax[1].ncell)};
    double wgt = 1.0;
    int64_t t[3];
    for (int a = 0; a < 3; ++a) {
        t[a] = axis_free_index(k.ax[a], k.p, cc[a] * k.p + li[a]);
        if (t[a] < 0) { k.Vbar[e] = 0.0; return; }
        wgt *= k.wrel[a * n1 + li[a]] * k.axisMinv[a * k.maxf + t[a]];
    }
    int64_t I = t[0] + k.nfx * (t[1] + k.nfy * t[2]);
    k.Vbar[e] = wgt * k.g[I];
}

// Ebar = -sum_I g_I (z_I - z0): one block per slab of rows, then a second pass.
__global__ void ebar_partial_kernel(const double *g, const double *zcoord, double z0, int64_t n, int64_t nxy,
                                    double *partial) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < n; I += (int64_t)gridDim.x * blockDim.x)
        s += g[I] * (zcoord[I / nxy] - z0);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void ebar_final_kernel(const double *partial, int nb, double *Ebar) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *Ebar = -red[0];
}

hipError_t launch_potential_vjp(const fe_mesh *m, const double *g, double z0, double *Vbar, double *Ebar,
                                hipStream_t s) {
    PotParams b = pot_params(m);
    PotVjpParams k;
    k.g = g; k.Vbar = Vbar; k.axisMinv = b.axisMinv; k.wrel = b.wrel;
    k.maxf = b.maxf; k.p = b.p; k.nc = b.nc;
    for (int d = 0; d < 3; ++d) k.ax[d] = b.ax[d];
    k.nfx = b.nfx; k.nfy = b.nfy; k.ncells = m->ncells;
    int64_t tot = m->ncells * m->nc;
    hipLaunchKernelGGL(potential_vjp_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // partial sums live at the end of the mesh scratch (1024 doubles reserved)
    const int nb = 1024;
    double *partial = m->d_scratch;
    hipLaunchKernelGGL(ebar_partial_kernel, dim3(nb), dim3(256), 0, s, g, (const double *)m->d_zcoord, z0, m->n,
                       m->nf[0] * m->nf[1], partial);
    hipLaunchKernelGGL(ebar_final_kernel, dim3(1), dim3(256), 0, s, (const double *)partial, nb, Ebar);
    return hipGetLastError();
}

// g_I += scale * sum_j U[I,j] V[I,j]; one wave per row, fixed reduction order.
__global__ void rowdot_kernel(const double *U, const double *V, int64_t ld, int64_t N, int64_t n, double scale,
                              double *g) {
    int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (I >= n) return;
    double s = 0.0;
    for (int64_t j = lane; j < N; j += 64) s += U[I * ld + j] * V[I * ld + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) g[I] += scale * s;
}

hipError_t launch_rowdot_accum(const fe_mesh *m, const double *U, const double *V, int64_t ld, int64_t N,
                               double scale, double *g, hipStream_t s) {
    int64_t threads = m->n * 64;
    hipLaunchKernelGGL(rowdot_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, U, V, ld, N, m->n,
                       scale, g);
    return hipGetLastError();
}

// Y = a X + b Y over an (n x N) block (b == 0 overwrites Y).
__global__ void axpby_kernel(double *Y, int64_t ldy, const double *X, int64_t ldx, int64_t n, int64_t N, double a,
                             double b) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * N) return;
    int64_t I = e / N, j = e % N;
    double y = a * X[I * ldx + j];
    if (b != 0.0) y += b * Y[I * ldy + j];
    Y[I * ldy + j] = y;
}

hipError_t launch_axpby(double *Y, int64_t ldy, const double *X, int64_t ldx, int64_t n, int64_t N, double a,
                        double b, hipStream_t s) {
    int64_t tot = n * N;
    hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Y, ldy, X, ldx, n, N, a,
                       b);
    return hipGetLastError();
}

}  // namespace fe
