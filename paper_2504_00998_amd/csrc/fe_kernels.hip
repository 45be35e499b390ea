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

#include <algorithm>
#include <type_traits>
#include <cstdint>

#include "fe_internal.h"

namespace fe {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
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
    const double *S;  // FP64 fragments of k.G_c (Bloch mode), else null
    AxisInfo ax[3];
    int col[3];
    int cnt[3];
    int64_t nfx, nfy;
    AxisInfo zs;  // z axis in segments of zl cells (the pipelined kernel's z segments; zl = 1: cells)
    int zl;
    const double *zero;  // >= 32 zero doubles (source of padded and absent rows)
    int nfz;
};

template <int PREC> struct PrecTraits;
template <> struct PrecTraits<0> { typedef double T; static constexpr int KSTEP = 4; };
template <> struct PrecTraits<1> { typedef float T; static constexpr int KSTEP = 4; };
template <> struct PrecTraits<2> { typedef uint16_t T; static constexpr int KSTEP = 32; };

// LDS row stride (elements) of the transposed bf16 operand: pad by 8 to
// spread the 16 column reads of a fragment over the banks.
template <int NCP> struct Bf16Stride { static constexpr int value = NCP + 8; };

// FP64 cell product on v_mfma_f64_4x4x4f64 (four 4x4x4 blocks per wave).
// Lane l of a block instruction carries A[4b + l%4][l/16] and B[l/16][l%4]
// of block b = (l/4)%4 and returns D[l/16][l%4] of that block.  The blocks
// are taken as the four 4-row groups of a 16-row tile of (1/2)K_c, so the A
// operand is exactly the 16x16x4 fragment A[l%16][l/16].  The four blocks
// share one 4-column slice of B; instruction q = 0..3 gives lane l the slice
// of vectors {4j + q}, j = l%4, so lane l accumulates row 4((l/4)%4) + l/16
// of the tile for the four consecutive vectors 4(l%4) .. 4(l%4)+3, read from
// a row of 16 vectors in LDS as 32 contiguous bytes.
__device__ __forceinline__ void f64_quad_b(const double *xs, int s, int lane, double b[4]) {
    const double2 *p = reinterpret_cast<const double2 *>(xs + (4 * s + (lane >> 4)) * 16 + 4 * (lane & 3));
    double2 u = p[0], v = p[1];
    b[0] = u.x;
    b[1] = u.y;
    b[2] = v.x;
    b[3] = v.y;
}

// Row (within the 16-row tile) and vector (within the 16-vector chunk) of
// accumulator i of a lane: FP64 4x4x4 blocks as above; the FP32 and BF16
// 16x16 shapes put row 4(l/16) + i, vector l%16.
template <int PREC> __device__ __forceinline__ void acc_position(int lane, int i, int &r, int &cv) {
    if constexpr (PREC == 0) {
        r = 4 * ((lane >> 2) & 3) + (lane >> 4);
        cv = 4 * (lane & 3) + i;
    } else {
        r = 4 * (lane >> 4) + i;
        cv = lane & 15;
    }
}

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
    for (int t = wave; t < NT; t += 4) {
        double acc[4];
        if constexpr (PREC == 0) {
            const double *A = reinterpret_cast<const double *>(k.A) + (size_t)t * NKS * 64 + lane;
            double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
            for (int s = 0; s < NKS; ++s) {
                double a = A[s * 64];
                double b[4];
                f64_quad_b(xs, s, lane, b);
#pragma unroll
                for (int q = 0; q < 4; ++q) c[q] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b[q], c[q], 0, 0, 0);
            }
            for (int i = 0; i < 4; ++i) acc[i] = c[i];
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
        for (int i = 0; i < 4; ++i) {
            int r, cv;
            acc_position<PREC>(lane, i, r, cv);
            r += 16 * t;
            const int64_t vec = vec0 + cv;
            if (r >= NC || vec >= k.N) continue;
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

// ------------------------------------------------------------------------
// Helpers of the persistent kernels: the A-fragment type per precision, the
// cell of a work item, node references and first-writer tests.
template <int PREC> struct FragOf;
template <> struct FragOf<0> { typedef double T; };
template <> struct FragOf<1> { typedef float T; };
template <> struct FragOf<2> { typedef uint4 T; };

struct ItemCell {
    int cx, cy, cz, chunk;
};

// Free index of node position g in [0, ncell*p] along an axis (-1 on a
// Dirichlet face); 32-bit and division-free.
__device__ __forceinline__ int axis_free_index32(const AxisInfo &a, int p, int g) {
    int k = a.ncell * p;
    if (a.bc == FE_BC_DIRICHLET) return (g == 0 || g == k) ? -1 : g - 1;
    if (a.bc == FE_BC_PERIODIC) return g == k ? 0 : g;
    return g;
}

__device__ __forceinline__ ItemCell item_cell(const StepParams &k, int64_t item) {
    ItemCell r;
    const int it = (int)item;  // items per launch < 2^31
    r.chunk = it % k.nchunk;
    int cidx = it / k.nchunk;
    int ix = cidx % k.cnt[0];
    cidx /= k.cnt[0];
    int iy = cidx % k.cnt[1];
    int iz = cidx / k.cnt[1];
    r.cx = colour_cell(k.ax[0], k.col[0], ix);
    r.cy = colour_cell(k.ax[1], k.col[1], iy);
    r.cz = colour_cell(k.ax[2], k.col[2], iz);
    return r;
}

// DoF and D scale of local node l of a cell (-1 / 0 when on a Dirichlet face).
// The three per-axis factors are fetched unconditionally (clamped index), so
// their loads are independent and in flight together.
template <int P>
__device__ __forceinline__ int node_dof(const StepParams &k, const ItemCell &c, int l, double &d) {
    constexpr int N1 = P + 1;
    const int t0 = axis_free_index32(k.ax[0], P, c.cx * P + l % N1);
    const int t1 = axis_free_index32(k.ax[1], P, c.cy * P + (l / N1) % N1);
    const int t2 = axis_free_index32(k.ax[2], P, c.cz * P + l / (N1 * N1));
    const bool ok = t0 >= 0 && t1 >= 0 && t2 >= 0;
    const double d0 = k.axisD[max(t0, 0)];
    const double d1 = k.axisD[k.maxf + max(t1, 0)];
    const double d2 = k.axisD[2 * k.maxf + max(t2, 0)];
    d = ok ? (d0 * d1) * d2 : 0.0;
    return ok ? t0 + (int)k.nfx * (t1 + (int)k.nfy * t2) : -1;
}

// Branch-free form for any padded row r < NCP: DoF (-1 off the cell or on a
// Dirichlet face) and the three per-axis D factors, loaded here but combined
// only by node_scale, so that nothing waits on them before the caller's
// other loads are in flight.
struct NodeRef {
    int I;
    double f[3];
};

template <int P>
__device__ __forceinline__ NodeRef node_ref(const StepParams &k, const ItemCell &c, int r) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1;
    const int l = min(r, NC - 1);
    const int t0 = axis_free_index32(k.ax[0], P, c.cx * P + l % N1);
    const int t1 = axis_free_index32(k.ax[1], P, c.cy * P + (l / N1) % N1);
    const int t2 = axis_free_index32(k.ax[2], P, c.cz * P + l / (N1 * N1));
    const bool ok = r < NC && t0 >= 0 && t1 >= 0 && t2 >= 0;
    NodeRef n;
    n.I = ok ? t0 + (int)k.nfx * (t1 + (int)k.nfy * t2) : -1;
    n.f[0] = k.axisD[max(t0, 0)];
    n.f[1] = k.axisD[k.maxf + max(t1, 0)];
    n.f[2] = k.axisD[2 * k.maxf + max(t2, 0)];
    return n;
}

// D factor of the node (same rounding as node_dof: (d0 d1) d2).
__device__ __forceinline__ double node_scale(const NodeRef &n) {
    return n.I >= 0 ? (n.f[0] * n.f[1]) * n.f[2] : 0.0;
}

// Whether columns [c0, c0 + ncols) lie inside N and every block a step
// touches (X, Y, the previous iterate) allows 16-byte accesses at any row:
// then each lane's four consecutive values move as two 16-byte loads or
// stores.  The same for all lanes of a workgroup item.
__device__ __forceinline__ bool wide_ok(const StepParams &k, int64_t c0, int ncols) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(k.X) | reinterpret_cast<uintptr_t>(k.Y) |
                        reinterpret_cast<uintptr_t>(k.Ym1 ? k.Ym1 : k.X);
    const int64_t ld = k.ldx | k.ldy | (k.Ym1 ? k.ldm : k.ldx);
    return (a & 15) == 0 && (ld & 1) == 0 && c0 + ncols <= k.N;
}

__device__ __forceinline__ void load4(const double *p, double (&v)[4]) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

__device__ __forceinline__ void store4(double *p, double v0, double v1, double v2, double v3) {
    reinterpret_cast<double2 *>(p)[0] = double2{v0, v1};
    reinterpret_cast<double2 *>(p)[1] = double2{v2, v3};
}

template <int P>
__device__ __forceinline__ bool node_first(const StepParams &k, const ItemCell &c, int l) {
    constexpr int N1 = P + 1;
    int li[3] = {l % N1, (l / N1) % N1, l / (N1 * N1)};
    int cc[3] = {c.cx, c.cy, c.cz};
    for (int a = 0; a < 3; ++a) {
        int nb = axis_neighbour(k.ax[a], P, cc[a], li[a]);
        if (nb >= 0 && axis_colour(k.ax[a], nb) < axis_colour(k.ax[a], cc[a])) return false;
    }
    return true;
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

// ------------------------------------------------------------------------
// Multi-chunk variant: one cell and G chunks of 16 vectors per workgroup,
// one row tile of the cell matrix per wave.  Each A fragment read from L2
// feeds G MFMAs, so the cell-matrix traffic falls by G while many
// independent workgroups stay resident to hide memory latency.
template <int P> struct McShape {
    static constexpr int NCP = ((P + 1) * (P + 1) * (P + 1) + 31) / 32 * 32, NT = NCP / 16;
    static constexpr int TPW = NT > 16 ? 2 : 1;  // row tiles per wave (<= 16 waves per block)
    static constexpr int W = NT / TPW;
};

template <int P, int PREC, int G>
__global__ __launch_bounds__(64 * McShape<P>::W) void step_mc_kernel(StepParams k) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32, NT = NCP / 16;
    constexpr int KSTEP = PrecTraits<PREC>::KSTEP, NKS = NCP / KSTEP;
    constexpr int TPW = McShape<P>::TPW, W = McShape<P>::W;
    static_assert(NT % TPW == 0, "row tiles must divide evenly among waves");
    constexpr int NTHR = 64 * W;
    typedef typename PrecTraits<PREC>::T T;
    typedef typename FragOf<PREC>::T FragT;
    constexpr int XS = PREC == 2 ? 16 * Bf16Stride<NCP>::value : NCP * 16;
    extern __shared__ __align__(16) unsigned char smem[];
    T *xs = reinterpret_cast<T *>(smem);  // [G][XS]
    constexpr size_t xs_bytes = ((size_t)G * XS * sizeof(T) + 15) / 16 * 16;
    int32_t *dof = reinterpret_cast<int32_t *>(smem + xs_bytes);
    double *dsc = reinterpret_cast<double *>(dof + NCP);
    unsigned char *first = reinterpret_cast<unsigned char *>(dsc + NCP);

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15;
    const int ngroups = (k.nchunk + G - 1) / G;
    const int grp = blockIdx.x % ngroups;
    const ItemCell c = item_cell(k, (int64_t)(blockIdx.x / ngroups) * k.nchunk);

    for (int l = tid; l < NCP; l += NTHR) {
        double d = 0.0;
        int I = l < NC ? node_dof<P>(k, c, l, d) : -1;
        dof[l] = I;
        dsc[l] = d;
        first[l] = (l < NC && node_first<P>(k, c, l)) ? 1 : 0;
    }
    __syncthreads();
    const int64_t vbase = (int64_t)grp * G * 16;
    for (int e = tid; e < G * NCP * 16; e += NTHR) {
        int g = e / (NCP * 16), r = e % (NCP * 16);
        int l = r >> 4, cc = r & 15;
        int I = dof[l];
        int64_t vv = vbase + g * 16 + cc;
        double x = 0.0;
        if (I >= 0 && vv < k.N) x = dsc[l] * k.X[(int64_t)I * k.ldx + vv];
        if constexpr (PREC == 0) xs[g * XS + r] = x;
        else if constexpr (PREC == 1) xs[g * XS + r] = (float)x;
        else xs[g * XS + cc * Bf16Stride<NCP>::value + l] = to_bf16_bits(x);
    }
    __syncthreads();

#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const int t = wave + tt * W;
        const FragT *A = reinterpret_cast<const FragT *>(k.A) + (size_t)t * NKS * 64 + lane;
        double acc[G][4];
        if constexpr (PREC == 0) {
            double c[G][4];
#pragma unroll
            for (int g = 0; g < G; ++g)
                for (int q = 0; q < 4; ++q) c[g][q] = 0.0;
            // all A fragments of the row tile issued at once (one L2 round trip)
            // up to p = 5; in batches of 8 above that (register budget)
            constexpr int UNR = NKS <= 40 ? NKS : 8;
#pragma unroll UNR
            for (int s = 0; s < NKS; ++s) {
                double a = A[s * 64];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    double b[4];
                    f64_quad_b(xs + g * XS, s, lane, b);
#pragma unroll
                    for (int q = 0; q < 4; ++q) c[g][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b[q], c[g][q], 0, 0, 0);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                for (int i = 0; i < 4; ++i) acc[g][i] = c[g][i];
        } else if constexpr (PREC == 1) {
            f4 c4[G];
#pragma unroll
            for (int g = 0; g < G; ++g) c4[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
            for (int s = 0; s < NKS; ++s) {
                float a = A[s * 64];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    float b = xs[g * XS + (4 * s + (lane >> 4)) * 16 + col];
                    c4[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c4[g], 0, 0, 0);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                for (int i = 0; i < 4; ++i) acc[g][i] = (double)c4[g][i];
        } else {
            f4 c4[G];
#pragma unroll
            for (int g = 0; g < G; ++g) c4[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int s = 0; s < NKS; ++s) {
                bf8 a = __builtin_bit_cast(bf8, A[s * 64]);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const uint16_t *xrow = xs + g * XS + col * Bf16Stride<NCP>::value + 8 * (lane >> 4);
                    bf8 b = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4 *>(xrow + 32 * s));
                    c4[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c4[g], 0, 0, 0);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                for (int i = 0; i < 4; ++i) acc[g][i] = (double)c4[g][i];
        }

#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int r, cv;
                acc_position<PREC>(lane, i, r, cv);
                r += 16 * t;
                const int64_t vec = vbase + g * 16 + cv;
                if (r >= NC || vec >= k.N) continue;
                int I = dof[r];
                if (I < 0) continue;
                double contrib = k.alpha * dsc[r] * acc[g][i];
                double *y = k.Y + (int64_t)I * k.ldy + vec;
                if (first[r]) {
                    double base = k.alpha * (k.v[I] - k.shift) * k.X[(int64_t)I * k.ldx + vec];
                    if (k.Ym1) base -= k.beta * k.Ym1[(int64_t)I * k.ldm + vec];
                    *y = base + contrib;
                } else {
                    *y += contrib;
                }
            }
        }
    }
}

template <int P, int PREC, int G>
static hipError_t launch_mc_p(StepParams prm, const fe_mesh *m, hipStream_t s) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32, W = McShape<P>::W;
    typedef typename PrecTraits<PREC>::T T;
    constexpr int XS = PREC == 2 ? 16 * Bf16Stride<NCP>::value : NCP * 16;
    size_t smem = ((size_t)G * XS * sizeof(T) + 15) / 16 * 16 + NCP * (sizeof(int32_t) + sizeof(double) + 1);
    // a block that would not fit the 160 KiB of LDS runs the one-chunk kernel
    if (smem > 160 * 1024) return launch_step_p<P, PREC>(m, prm, s);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_mc_kernel<P, PREC, G>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int ngroups = (prm.nchunk + G - 1) / G;
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
                hipLaunchKernelGGL((step_mc_kernel<P, PREC, G>), dim3((unsigned)(cells * ngroups)), dim3(64 * W), smem,
                                   s, prm);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

// ------------------------------------------------------------------------
// Row-owner variant: one cell x G chunks of 16 vectors per workgroup, one
// 16-row tile of (1/2)K_c per wave (TPW tiles where the tiles outnumber 16
// waves), and each thread owns the outputs its accumulators hold: one row of
// the cell per tile, four consecutive vectors per chunk.
//   FP64: 4x4x4 blocks (see f64_quad_b): lane l owns row 4((l/4)%4) + l/16,
//         vectors 4(l%4) .. 4(l%4)+3.
//   FP32 / BF16: the 16x16 products are taken transposed, Y_c^T = X_c^T A^T,
//         i.e. with the X slice as the first operand and the cell-matrix
//         fragment as the second (both operands keep their 16x16 fragment
//         layouts); lane l then owns row l%16, vectors 4(l/16) .. 4(l/16)+3.
// Everything those outputs need from HBM (X for D X and the base term, the
// previous iterate or the old Y, v) is loaded in one round trip at the start,
// before the barrier; the cell-matrix fragments stream from L2 in batches of
// BK k-steps; each thread then writes its outputs without reading memory
// again.
template <int P, int TPW> struct RowShape {
    static constexpr int NCP = ((P + 1) * (P + 1) * (P + 1) + 31) / 32 * 32, NT = NCP / 16, W = NT / TPW;
    static_assert(NT % TPW == 0, "row tiles must divide evenly among waves");
};

// largest divisor of nks not above bk
constexpr int batch_size(int nks, int bk) {
    for (int b = bk < nks ? bk : nks; b > 1; --b)
        if (nks % b == 0) return b;
    return 1;
}

template <int PREC, int G, int NCP> struct RowLds {
    typedef typename PrecTraits<PREC>::T T;
    static constexpr int XS = PREC == 2 ? 16 * Bf16Stride<NCP>::value : NCP * 16;  // per chunk
    static constexpr size_t bytes = ((size_t)G * XS * sizeof(T) + 15) / 16 * 16;
};

// G chunks of 16 vectors per workgroup, TPW row tiles per wave, OCC waves
// per SIMD the register allocation aims at, cell-matrix fragments fetched in
// batches of BK k-steps (0: one k-step at a time).
// CPX (FP64 only): Bloch-k mode.  The columns are complex vectors stored as
// interleaved (re, im) pairs, so the four consecutive columns of a lane are
// two complex vectors, and the operator gains -i M^-1/2 (k.G) M^-1/2 with the
// real cell matrix S_c = k.G_c (fragments in k.S, same layout as k.A).  As
// -i S (x_r + i x_i) = S x_i - i S x_r, each k-step adds S_c times the
// operand (x_i, -x_r, x_i', -x_r') to the same accumulators; the diagonal
// part (v - shift, with |k|^2/2 folded into shift by the caller) acts on
// each real column as in the real mode.
template <int P, int PREC, int G, int TPW, int OCC, int BK, bool CPX = false>
__global__ __launch_bounds__((64 * RowShape<P, TPW>::W)) __attribute__((amdgpu_waves_per_eu(OCC)))
void step_row_kernel(StepParams k) {
    static_assert(!CPX || PREC == 0, "the Bloch mode is FP64 only");
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32;
    constexpr int KSTEP = PrecTraits<PREC>::KSTEP, NKS = NCP / KSTEP;
    constexpr int W = RowShape<P, TPW>::W, XS = RowLds<PREC, G, NCP>::XS;
    typedef typename PrecTraits<PREC>::T T;
    typedef typename FragOf<PREC>::T FragT;
    extern __shared__ __align__(16) unsigned char smem[];
    T *xs = reinterpret_cast<T *>(smem);  // [G][XS], D X rounded to the product precision

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ngroups = (k.nchunk + G - 1) / G;
    const int grp = blockIdx.x % ngroups;
    const ItemCell c = item_cell(k, (int64_t)(blockIdx.x / ngroups) * k.nchunk);
    const int rl = PREC == 0 ? 4 * ((lane >> 2) & 3) + (lane >> 4) : (lane & 15);  // row within a tile
    const int vq = PREC == 0 ? 4 * (lane & 3) : 4 * (lane >> 4);                   // first vector in a chunk
    const int64_t v0 = (int64_t)grp * G * 16 + vq;

    // cell-matrix fragments: the first batch is requested before the HBM
    // loads so that it has arrived when the product starts
    const FragT *A = reinterpret_cast<const FragT *>(k.A) + (size_t)wave * NKS * 64 + lane;
    constexpr size_t TS = (size_t)W * NKS * 64;  // fragment stride between the wave's tiles
    constexpr int BKE = batch_size(NKS, BK > 0 ? BK : 1), NB = NKS / BKE;
    static_assert(NKS % BKE == 0, "k-steps must split into batches");
    const double *Sf = CPX ? k.S + (size_t)wave * NKS * 64 + lane : nullptr;
    constexpr int NS = CPX ? 2 : 1;  // fragment streams: (1/2)K_c, and S_c in the Bloch mode
    auto load_batch = [&](FragT (&ab)[BKE][NS][TPW], int sb) {
#pragma unroll
        for (int j = 0; j < BKE; ++j)
#pragma unroll
            for (int tt = 0; tt < TPW; ++tt) {
                ab[j][0][tt] = A[tt * TS + (size_t)(sb * BKE + j) * 64];
                if constexpr (CPX) ab[j][NS - 1][tt] = Sf[tt * TS + (size_t)(sb * BKE + j) * 64];
            }
    };
    FragT ab0[BKE][NS][TPW], ab1[BKE][NS][TPW];
    if constexpr (BK > 0) load_batch(ab0, 0);

    int I[TPW];
    double d[TPW];
    // per output: the first writer's base term alpha (v - c) X - beta Y_{k-1},
    // or the Y already there.  All addresses first, then every load of the
    // thread's rows as one straight run (unconditional, from clamped valid
    // addresses, masked afterwards), then the consumers.
    double bo[TPW][G][4];
    NodeRef nr[TPW];
    bool fst[TPW];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const int r = 16 * (wave + tt * W) + rl;
        nr[tt] = node_ref<P>(k, c, r);
        fst[tt] = r < NC && node_first<P>(k, c, r);
    }
    double xv[TPW][G][4], ov[TPW][G][4], vraw[TPW];
    const bool wide = wide_ok(k, (int64_t)grp * G * 16, 16 * G);
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const int64_t Ic = max(nr[tt].I, 0);
        const double *orow =
            !fst[tt] ? k.Y + Ic * k.ldy : (k.Ym1 ? k.Ym1 + Ic * k.ldm : k.X + Ic * k.ldx);
        const double *xrow = k.X + Ic * k.ldx;
        vraw[tt] = k.v[Ic];
        if (wide) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                load4(xrow + v0 + 16 * g, xv[tt][g]);
                load4(orow + v0 + 16 * g, ov[tt][g]);
            }
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t vc = min(v0 + 16 * g + q, k.N - 1);
                    xv[tt][g][q] = xrow[vc];
                    ov[tt][g][q] = orow[vc];
                }
        }
    }
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        const int r = 16 * (wave + tt * W) + rl;
        I[tt] = nr[tt].I;
        const bool useo = !fst[tt] || k.Ym1 != nullptr;
        const double vI = (nr[tt].I >= 0 && fst[tt]) ? vraw[tt] : 0.0;
        const double sc = k.alpha * (vI - k.shift);
        d[tt] = node_scale(nr[tt]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double dx[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = nr[tt].I >= 0 && v0 + 16 * g + q < k.N;
                const double x = ok ? xv[tt][g][q] : 0.0;
                const double o = (ok && useo) ? ov[tt][g][q] : 0.0;
                double base = sc * x;
                if (k.Ym1) base -= k.beta * o;
                bo[tt][g][q] = fst[tt] ? base : o;
                dx[q] = d[tt] * x;
            }
            if constexpr (PREC == 0) {
                double2 *dst = reinterpret_cast<double2 *>(xs + g * XS + r * 16 + vq);
                dst[0] = double2{dx[0], dx[1]};
                dst[1] = double2{dx[2], dx[3]};
            } else if constexpr (PREC == 1) {
                *reinterpret_cast<f4 *>(xs + g * XS + r * 16 + vq) =
                    f4{(float)dx[0], (float)dx[1], (float)dx[2], (float)dx[3]};
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) xs[g * XS + (vq + q) * Bf16Stride<NCP>::value + r] = to_bf16_bits(dx[q]);
            }
        }
    }
    __syncthreads();

    // the wave's TPW row tiles share each B read from LDS
    double acc[TPW][G][4];
    {
        typedef typename std::conditional<PREC == 0, double, f4>::type AccT;
        AccT cacc[TPW][G][PREC == 0 ? 4 : 1];
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int q = 0; q < (PREC == 0 ? 4 : 1); ++q) {
                    if constexpr (PREC == 0) cacc[tt][g][q] = 0.0;
                    else cacc[tt][g][q] = f4{0.f, 0.f, 0.f, 0.f};
                }
        auto mul_step = [&](const FragT (&af)[NS][TPW], int s) {
            const FragT(&a)[TPW] = af[0];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if constexpr (PREC == 0) {
                    double b[4];
                    f64_quad_b(xs + g * XS, s, lane, b);
#pragma unroll
                    for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            cacc[tt][g][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[tt], b[q], cacc[tt][g][q], 0, 0, 0);
                    if constexpr (CPX) {
                        const double bs[4] = {b[1], -b[0], b[3], -b[2]};
#pragma unroll
                        for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                cacc[tt][g][q] =
                                    __builtin_amdgcn_mfma_f64_4x4x4f64(af[NS - 1][tt], bs[q], cacc[tt][g][q], 0, 0, 0);
                    }
                } else if constexpr (PREC == 1) {
                    const float b = xs[g * XS + (4 * s + (lane >> 4)) * 16 + (lane & 15)];
#pragma unroll
                    for (int tt = 0; tt < TPW; ++tt)
                        cacc[tt][g][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(b, a[tt], cacc[tt][g][0], 0, 0, 0);
                } else {
                    const uint16_t *xcol = xs + g * XS + (lane & 15) * Bf16Stride<NCP>::value + 8 * (lane >> 4);
                    const bf8 b = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4 *>(xcol + 32 * s));
#pragma unroll
                    for (int tt = 0; tt < TPW; ++tt)
                        cacc[tt][g][0] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, __builtin_bit_cast(bf8, a[tt]), cacc[tt][g][0], 0, 0, 0);
                }
            }
        };
        if constexpr (BK == 0) {
            constexpr int UNR = NKS <= 40 ? NKS : 8;
#pragma unroll UNR
            for (int s = 0; s < NKS; ++s) {
                FragT a[NS][TPW];
#pragma unroll
                for (int tt = 0; tt < TPW; ++tt) {
                    a[0][tt] = A[tt * TS + (size_t)s * 64];
                    if constexpr (CPX) a[NS - 1][tt] = Sf[tt * TS + (size_t)s * 64];
                }
                mul_step(a, s);
            }
        } else {
            // batch j + 1 in flight while batch j is multiplied (loads complete
            // in issue order, so a wait for batch j leaves the later batch
            // outstanding); batch 0 was requested at the start
            auto mul_batch = [&](const FragT (&ab)[BKE][NS][TPW], int sb) {
#pragma unroll
                for (int j = 0; j < BKE; ++j) mul_step(ab[j], sb * BKE + j);
            };
constexpr int UNRB = NB <= 8 ? NB : 1;
#pragma unroll UNRB
            for (int sb = 0; sb < NB; sb += 2) {
                if (sb + 1 < NB) load_batch(ab1, sb + 1);
                mul_batch(ab0, sb);
                if (sb + 1 < NB) {
                    if (sb + 2 < NB) load_batch(ab0, sb + 2);
                    mul_batch(ab1, sb + 1);
                }
            }
        }
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (PREC == 0) acc[tt][g][q] = cacc[tt][g][q];
                    else acc[tt][g][q] = (double)cacc[tt][g][0][q];
                }
    }
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
        if (I[tt] < 0) continue;
        double *yrow = k.Y + (int64_t)I[tt] * k.ldy;
        if (wide) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double o4[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) o4[q] = bo[tt][g][q] + k.alpha * d[tt] * acc[tt][g][q];
                store4(yrow + v0 + 16 * g, o4[0], o4[1], o4[2], o4[3]);
            }
            continue;
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t vec = v0 + 16 * g + q;
                if (vec >= k.N) continue;
                yrow[vec] = bo[tt][g][q] + k.alpha * d[tt] * acc[tt][g][q];
            }
    }
}

template <int P, int PREC, int G, int TPW, int OCC, int BK, bool CPX = false>
static hipError_t launch_row_p(StepParams prm, const fe_mesh *m, hipStream_t s) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32, W = RowShape<P, TPW>::W;
    const size_t smem = RowLds<PREC, G, NCP>::bytes;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_row_kernel<P, PREC, G, TPW, OCC, BK, CPX>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int ngroups = (prm.nchunk + G - 1) / G;
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
                hipLaunchKernelGGL((step_row_kernel<P, PREC, G, TPW, OCC, BK, CPX>), dim3((unsigned)(cells * ngroups)),
                                   dim3(64 * W), smem, s, prm);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

// ------------------------------------------------------------------------
// Single-vector step (N = 1, FP64): the 16 columns of the MFMA tile carry 16
// cells of the colour instead of 16 vectors, so one cell-matrix fragment
// multiplies 16 cells at once.  A workgroup takes 16 cells; each wave a 16-row
// tile; lane l owns row 4((l/4)%4) + l/16 of the four cells 4(l%4) .. +3 of
// the batch (the FP64 4x4x4 layout of the row-owner kernel with cells in
// place of vectors).  Cells of one colour share no node, so every output is
// written by one lane.  Same arithmetic, in the same order, as the other
// FP64 variants at N = 1.
template <int P, int BK>
__global__ __launch_bounds__((64 * RowShape<P, 1>::W)) __attribute__((amdgpu_waves_per_eu(5)))
void step_cells_kernel(StepParams k, int64_t ncells) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32, NKS = NCP / 4;
    extern __shared__ __align__(16) unsigned char smem[];
    double *xs = reinterpret_cast<double *>(smem);  // [NCP][16 cells], D X

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rl = 4 * ((lane >> 2) & 3) + (lane >> 4);
    const int cq = 4 * (lane & 3);  // first of the lane's four cells in the batch
    const int r = 16 * wave + rl;
    const int64_t cell0 = (int64_t)blockIdx.x * 16 + cq;

    const double *A = reinterpret_cast<const double *>(k.A) + (size_t)wave * NKS * 64 + lane;
    constexpr int BKE = batch_size(NKS, BK), NB = NKS / BKE;
    static_assert(NKS % BKE == 0, "k-steps must split into batches");
    auto load_batch = [&](double (&ab)[BKE], int sb) {
#pragma unroll
        for (int j = 0; j < BKE; ++j) ab[j] = A[(size_t)(sb * BKE + j) * 64];
    };
    double ab0[BKE], ab1[BKE];
    load_batch(ab0, 0);

    NodeRef nr[4];
    bool fst[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t ci = min(cell0 + q, ncells - 1);
        const ItemCell c = item_cell(k, ci);
        nr[q] = node_ref<P>(k, c, r);
        if (cell0 + q >= ncells) nr[q].I = -1;
        fst[q] = r < NC && node_first<P>(k, c, r);
    }
    double xv[4], ov[4], vraw[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t Ic = max(nr[q].I, 0);
        xv[q] = k.X[Ic * k.ldx];
        ov[q] = !fst[q] ? k.Y[Ic * k.ldy] : (k.Ym1 ? k.Ym1[Ic * k.ldm] : 0.0);
        vraw[q] = k.v[Ic];
    }
    double bo[4], d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool ok = nr[q].I >= 0;
        const bool useo = !fst[q] || k.Ym1 != nullptr;
        const double vI = (ok && fst[q]) ? vraw[q] : 0.0;
        const double sc = k.alpha * (vI - k.shift);
        d[q] = node_scale(nr[q]);
        const double x = ok ? xv[q] : 0.0;
        const double o = (ok && useo) ? ov[q] : 0.0;
        double base = sc * x;
        if (k.Ym1) base -= k.beta * o;
        bo[q] = fst[q] ? base : o;
        xv[q] = d[q] * x;
    }
    {
        double2 *dst = reinterpret_cast<double2 *>(xs + r * 16 + cq);
        dst[0] = double2{xv[0], xv[1]};
        dst[1] = double2{xv[2], xv[3]};
    }
    __syncthreads();

    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto mul_batch = [&](const double (&ab)[BKE], int sb) {
#pragma unroll
        for (int j = 0; j < BKE; ++j) {
            double b[4];
            f64_quad_b(xs, sb * BKE + j, lane, b);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f64_4x4x4f64(ab[j], b[q], acc[q], 0, 0, 0);
        }
    };
    constexpr int UNRB = NB <= 8 ? NB : 1;
#pragma unroll UNRB
    for (int sb = 0; sb < NB; sb += 2) {
        if (sb + 1 < NB) load_batch(ab1, sb + 1);
        mul_batch(ab0, sb);
        if (sb + 1 < NB) {
            if (sb + 2 < NB) load_batch(ab0, sb + 2);
            mul_batch(ab1, sb + 1);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (nr[q].I >= 0) k.Y[(int64_t)nr[q].I * k.ldy] = bo[q] + k.alpha * d[q] * acc[q];
}

// ------------------------------------------------------------------------
// Single-vector product in two launches (the CG iteration of the Poisson
// solve): every cell's product at once into a cell-local buffer, then each
// free DoF sums its (at most eight) cell rows in a fixed order.  No colour
// passes, so one launch covers all cells; deterministic, but the nodal sums
// are associated differently from the colour-pass kernels.
//   cell_apply_kernel: 16 cells per workgroup (the MFMA vector columns carry
//   cells, as in step_cells_kernel); Zc[cell][r] = d_r ((1/2)K_c (D x)_c)_r.
template <int P, int BK>
__global__ __launch_bounds__((64 * RowShape<P, 1>::W)) __attribute__((amdgpu_waves_per_eu(5)))
void cell_apply_kernel(StepParams k, int64_t ncells, double *Zc) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32, NKS = NCP / 4;
    extern __shared__ __align__(16) unsigned char smem[];
    double *xs = reinterpret_cast<double *>(smem);  // [NCP][16 cells], D x

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rl = 4 * ((lane >> 2) & 3) + (lane >> 4);
    const int cq = 4 * (lane & 3);
    const int r = 16 * wave + rl;
    const int64_t cell0 = (int64_t)blockIdx.x * 16 + cq;

    const double *A = reinterpret_cast<const double *>(k.A) + (size_t)wave * NKS * 64 + lane;
    constexpr int BKE = batch_size(NKS, BK), NB = NKS / BKE;
    static_assert(NKS % BKE == 0, "k-steps must split into batches");
    auto load_batch = [&](double (&ab)[BKE], int sb) {
#pragma unroll
        for (int j = 0; j < BKE; ++j) ab[j] = A[(size_t)(sb * BKE + j) * 64];
    };
    double ab0[BKE], ab1[BKE];
    load_batch(ab0, 0);

    NodeRef nr[4];
    const int ncx = k.ax[0].ncell, ncy = k.ax[1].ncell;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ci = (int)min(cell0 + q, ncells - 1);
        ItemCell c;
        c.cx = ci % ncx;
        c.cy = (ci / ncx) % ncy;
        c.cz = ci / (ncx * ncy);
        c.chunk = 0;
        nr[q] = node_ref<P>(k, c, r);
        if (cell0 + q >= ncells) nr[q].I = -1;
    }
    double xv[4], d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) xv[q] = k.X[(int64_t)max(nr[q].I, 0) * k.ldx];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        d[q] = node_scale(nr[q]);
        xv[q] = nr[q].I >= 0 ? d[q] * xv[q] : 0.0;
    }
    {
        double2 *dst = reinterpret_cast<double2 *>(xs + r * 16 + cq);
        dst[0] = double2{xv[0], xv[1]};
        dst[1] = double2{xv[2], xv[3]};
    }
    __syncthreads();

    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto mul_batch = [&](const double (&ab)[BKE], int sb) {
#pragma unroll
        for (int j = 0; j < BKE; ++j) {
            double b[4];
            f64_quad_b(xs, sb * BKE + j, lane, b);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f64_4x4x4f64(ab[j], b[q], acc[q], 0, 0, 0);
        }
    };
    constexpr int UNRB = NB <= 8 ? NB : 1;
#pragma unroll UNRB
    for (int sb = 0; sb < NB; sb += 2) {
        if (sb + 1 < NB) load_batch(ab1, sb + 1);
        mul_batch(ab0, sb);
        if (sb + 1 < NB) {
            if (sb + 2 < NB) load_batch(ab0, sb + 2);
            mul_batch(ab1, sb + 1);
        }
    }
    if (r < NC) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (cell0 + q < ncells) Zc[(cell0 + q) * NCP + r] = d[q] * acc[q];
    }
}

// Cells containing global node position g along an axis (left one first) and
// the node's local index in each; returns how many (1 or 2).
__device__ __forceinline__ int axis_cells(const AxisInfo &a, int p, int g, int (&c)[2], int (&l)[2]) {
    const int K = a.ncell * p;
    if (g % p != 0) {
        c[0] = g / p;
        l[0] = g % p;
        return 1;
    }
    int n = 0;
    if (g > 0) {
        c[n] = g / p - 1;
        l[n++] = p;
    } else if (a.bc == FE_BC_PERIODIC) {
        c[n] = a.ncell - 1;
        l[n++] = p;
    }
    if (g < K) {
        c[n] = g / p;
        l[n++] = 0;
    }
    return n;
}

// y_I = alpha ((v_I - shift) x_I + sum over the cells containing I of Zc)
//       - beta Ym1_I,  summed over the cells z-, y-, x-outermost, left first.
template <int P>
__global__ void assemble_kernel(StepParams k, const double *Zc) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, NCP = (NC + 31) / 32 * 32;
    const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = k.nfx * k.nfy * (int64_t)k.ax[2].nfree;
    if (I >= n) return;
    const int t[3] = {(int)(I % k.nfx), (int)((I / k.nfx) % k.nfy), (int)(I / (k.nfx * k.nfy))};
    int cs[3][2], ls[3][2], nc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int g = k.ax[a].bc == FE_BC_DIRICHLET ? t[a] + 1 : t[a];
        nc[a] = axis_cells(k.ax[a], P, g, cs[a], ls[a]);
    }
    const int ncx = k.ax[0].ncell, ncy = k.ax[1].ncell;
    double sum = 0.0;
    for (int iz = 0; iz < nc[2]; ++iz)
        for (int iy = 0; iy < nc[1]; ++iy)
            for (int ix = 0; ix < nc[0]; ++ix) {
                const int64_t cell = cs[0][ix] + (int64_t)ncx * (cs[1][iy] + (int64_t)ncy * cs[2][iz]);
                const int l = ls[0][ix] + N1 * (ls[1][iy] + N1 * ls[2][iz]);
                sum += Zc[cell * NCP + l];
            }
    double base = k.alpha * (k.v[I] - k.shift) * k.X[I * k.ldx];
    if (k.Ym1) base -= k.beta * k.Ym1[I * k.ldm];
    k.Y[I * k.ldy] = base + k.alpha * sum;
}

template <int P>
static hipError_t launch_assembled_p(StepParams prm, const fe_mesh *m, double *Zc, hipStream_t s) {
    constexpr int NCP = RowShape<P, 1>::NCP, W = RowShape<P, 1>::W;
    static_assert(RowShape<P, 1>::NT <= 16, "one wave per row tile");
    const size_t smem = (size_t)NCP * 16 * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&cell_apply_kernel<P, 4>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int64_t ncells = m->ncells;
    hipLaunchKernelGGL((cell_apply_kernel<P, 4>), dim3((unsigned)((ncells + 15) / 16)), dim3(64 * W), smem, s, prm,
                       ncells, Zc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((assemble_kernel<P>), dim3((unsigned)((m->n + 255) / 256)), dim3(256), 0, s, prm,
                       (const double *)Zc);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_cells_p(StepParams prm, const fe_mesh *m, hipStream_t s) {
    constexpr int NCP = RowShape<P, 1>::NCP, W = RowShape<P, 1>::W;
    static_assert(RowShape<P, 1>::NT <= 16, "one wave per row tile");
    const size_t smem = (size_t)NCP * 16 * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_cells_kernel<P, 4>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    prm.nchunk = 1;
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
                hipLaunchKernelGGL((step_cells_kernel<P, 4>), dim3((unsigned)((cells + 15) / 16)), dim3(64 * W), smem,
                                   s, prm, cells);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

// ------------------------------------------------------------------------
// Pipelined row-owner variant (p <= 4): persistent workgroups walk the items
// (cell or z segment of cells, group of G chunks of 16 vectors) of a colour
// with stride gridDim.x, one wave per 16-row tile of (1/2)K_c with the tile's
// fragments held in registers for the whole launch, each thread owning one
// row for four vectors per chunk.  Products: FP64 on 4x4x4 blocks, FP32 on
// transposed 16x16x4 and BF16 on transposed 16x16x32 products (X operand
// first), FP32 accumulation below FP64.  The product loop issues no
// vector-memory instruction, so the HBM loads of the next cells (X, the
// previous iterate or the old Y, v; from clamped addresses) stay in flight
// while it runs.  After the product the next cell is staged into the other
// LDS buffer -- the only wait on those loads -- and only then are the
// current cell's outputs stored, so the wait never includes the stores.  The
// B (FP64) or X (FP32) operand is read from LDS one k-step ahead of its
// products.  Without z segments: the same arithmetic, in the same order, as
// the other FP64 and FP32 variants.
template <int P, int PREC = 0> struct PipeShape {
    typedef typename PrecTraits<PREC>::T T;
    static constexpr int NCP = ((P + 1) * (P + 1) * (P + 1) + 31) / 32 * 32, NT = NCP / 16;
    static constexpr int NKS = NCP / PrecTraits<PREC>::KSTEP;  // k-steps of the product
    // BF16 keeps each chunk transposed (vector-major, rows padded to
    // Bf16Stride) for the 8-element operand reads of the 16x16x32 product
    static constexpr int STR = PREC == 2 ? Bf16Stride<NCP>::value : 16;
    static constexpr int W = NT, G = 2, XS = PREC == 2 ? 16 * STR : NCP * 16;  // waves; chunks; elements per chunk
    static constexpr size_t bytes = ((size_t)2 * G * XS * sizeof(T) + 15) / 16 * 16;
};

// Row within the 16-row tile and the vectors a lane owns.  The four lanes
// sharing a row own the vector pairs {2j, 2j+1} and {8+2j, 9+2j} of each
// 16-vector chunk (j = 0..3), so that each 16-byte load or store of the four
// covers one contiguous 64-byte run of the row.  FP64: 4x4x4 blocks, lane l
// owns row 4((l/4)%4) + l/16 with j = l%4; instruction q multiplies the
// B slice of vectors {pipe_off(q) + 2j}.  FP32: the transposed 16x16x4
// product, lane l owns row l%16 with j = l/16, the X operand's vector
// index permuted to match (pipe_perm).
template <int PREC> __device__ __forceinline__ int pipe_row(int lane) {
    return PREC == 0 ? 4 * ((lane >> 2) & 3) + (lane >> 4) : (lane & 15);
}
template <int PREC> __device__ __forceinline__ int pipe_vec(int lane) {
    return PREC == 0 ? 2 * (lane & 3) : 2 * (lane >> 4);
}
// Offset of a lane's q-th owned vector from pipe_vec: q = 0, 1 the first
// pair, q = 2, 3 the pair 8 vectors on.
__device__ __forceinline__ constexpr int pipe_off(int q) { return (q & 1) + 8 * (q >> 1); }
// Vector carried by row i of the X operand of the transposed FP32 and BF16
// products, so that lane l's accumulator q holds vector pipe_vec(l) +
// pipe_off(q).
__device__ __forceinline__ int pipe_perm(int i) { return 2 * (i >> 2) + pipe_off(i & 3); }

// B operand of the FP64 4x4x4 product at k-step s for the pipelined layout:
// row 4s + l/16 of the chunk, vectors 2(l%4) + pipe_off(q), as two 16-byte
// LDS reads.
__device__ __forceinline__ void f64_pair_b(const double *xs, int s, int lane, double b[4]) {
    const double *row = xs + (4 * s + (lane >> 4)) * 16 + 2 * (lane & 3);
    const double2 u = reinterpret_cast<const double2 *>(row)[0], v = reinterpret_cast<const double2 *>(row + 8)[0];
    b[0] = u.x;
    b[1] = u.y;
    b[2] = v.x;
    b[3] = v.y;
}

// Whether local node i of cell c is not shared, along this axis, with a cell
// of a lower colour: node_first for one axis, as selects only (no branches).
// An i outside [0, p] (the z-segment kernel passes -1 for a face inside a
// segment) counts as interior: true.
__device__ __forceinline__ bool axis_first_sel(const AxisInfo &a, int p, int c, int i) {
    const bool lo = i == 0, hi = i == p;
    const bool wrap_lo = lo && c == 0, wrap_hi = hi && c == a.ncell - 1;
    int nb = lo ? c - 1 : c + 1;
    nb = wrap_lo ? a.ncell - 1 : nb;
    nb = wrap_hi ? 0 : nb;
    const bool exists = (lo || hi) && (!(wrap_lo || wrap_hi) || a.bc == FE_BC_PERIODIC);
    const int cn = (a.ncol == 3 && nb == a.ncell - 1) ? 2 : (nb & 1);
    const int cc = (a.ncol == 3 && c == a.ncell - 1) ? 2 : (c & 1);
    return !(exists && cn < cc);
}

// The loads of one thread for one cell of an item, and what the epilogue
// needs.  With z segments (ZS), bot marks a row on the bottom face of a cell
// after the segment's first: it loads nothing (X comes from the previous
// cell's staged top face, the old value from the LDS hold); top marks a row on
// the top face of a cell before the segment's last, whose output goes to the
// hold instead of Y.
template <int G> struct PipeRow {
    NodeRef n;
    bool fst, bot, top;
    double vraw;
    double x[G][4], o[G][4];
    int64_t v0;
};

// Cell of cell index ci of the launch's colour: along z, segment s of the
// colour and cell c within it (c = 0 without segments).
__device__ __forceinline__ ItemCell seg_cell(const StepParams &k, int ci, int c, int &seg) {
    ItemCell r;
    r.chunk = 0;
    const int ix = ci % k.cnt[0];
    ci /= k.cnt[0];
    const int iy = ci % k.cnt[1];
    const int iz = ci / k.cnt[1];
    r.cx = colour_cell(k.ax[0], k.col[0], ix);
    r.cy = colour_cell(k.ax[1], k.col[1], iy);
    seg = colour_cell(k.zs, k.col[2], iz);
    r.cz = seg * k.zl + c;
    return r;
}

template <int P, int PREC, bool ZS>
__device__ __forceinline__ void pipe_issue(const StepParams &k, int64_t item, int c, int ngroups, int wave, int lane,
                                           PipeRow<PipeShape<P>::G> &L) {
    constexpr int N1 = P + 1, NC = N1 * N1 * N1, G = PipeShape<P>::G;
    const int it = (int)item;  // items per launch < 2^31: 32-bit division
    const int grp = it % ngroups;
    int seg;
    const ItemCell cc = seg_cell(k, it / ngroups, c, seg);
    const int r = 16 * wave + pipe_row<PREC>(lane);
    L.v0 = (int64_t)grp * G * 16 + pipe_vec<PREC>(lane);
    L.n = node_ref<P>(k, cc, r);
    const int l = min(r, NC - 1);
    const int lz = l / (N1 * N1);
    const bool f0 = axis_first_sel(k.ax[0], P, cc.cx, l % N1);
    const bool f1 = axis_first_sel(k.ax[1], P, cc.cy, (l / N1) % N1);
    bool f2;
    if constexpr (ZS) {
        // along z only the segment's end faces meet other workgroups
        const int iz = lz == 0 ? (c == 0 ? 0 : -1) : lz == P ? (c == k.zl - 1 ? P : -1) : -1;
        f2 = axis_first_sel(k.zs, P, seg, iz);
        L.bot = r < NC && lz == 0 && c > 0;
        L.top = r < NC && lz == P && c < k.zl - 1;
    } else {
        f2 = axis_first_sel(k.ax[2], P, cc.cz, lz);
        L.bot = L.top = false;
    }
    L.fst = (r < NC) & f0 & f1 & f2;
    const int64_t Ic = max(L.n.I, 0);
    // the old value: Y where an earlier colour has written the node, else the
    // previous iterate (or X when there is none, unused then); the two base
    // pointers are uniform, only the choice between them is per lane
    const double *ob = k.Ym1 ? k.Ym1 : k.X;
    const int64_t ol = k.Ym1 ? k.ldm : k.ldx;
    const double *orow = L.fst ? ob + Ic * ol : k.Y + Ic * k.ldy;
    const double *xrow = k.X + Ic * k.ldx;
    L.vraw = k.v[Ic];
    // a bottom-face row of a segment's later cell loads nothing; its x and o
    // are left unset (never read), so that no register a load in flight
    // targets is written by the other lanes
    const bool skip = ZS && L.bot;
    if (wide_ok(k, (int64_t)grp * G * 16, 16 * G)) {
        // the item's columns are all inside N and the blocks 16-byte aligned:
        // each lane's four values as two 16-byte loads
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (skip) continue;
            const double *xp = xrow + L.v0 + 16 * g, *op = orow + L.v0 + 16 * g;
            const double2 x01 = *reinterpret_cast<const double2 *>(xp);
            const double2 x23 = *reinterpret_cast<const double2 *>(xp + 8);
            const double2 o01 = *reinterpret_cast<const double2 *>(op);
            const double2 o23 = *reinterpret_cast<const double2 *>(op + 8);
            L.x[g][0] = x01.x; L.x[g][1] = x01.y; L.x[g][2] = x23.x; L.x[g][3] = x23.y;
            L.o[g][0] = o01.x; L.o[g][1] = o01.y; L.o[g][2] = o23.x; L.o[g][3] = o23.y;
        }
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (skip) continue;
                const int64_t vc = min(L.v0 + 16 * g + pipe_off(q), k.N - 1);
                L.x[g][q] = xrow[vc];
                L.o[g][q] = orow[vc];
            }
    }
}

// D X of the cell into an LDS buffer; per output the first writer's base term
// alpha (v - c) X - beta Y_{k-1}, or the old Y, into bo.  A bottom-face row of
// a segment's later cell copies D X from the previous cell's top face in xp
// (the same node) and takes its base from the hold later (hf bit 0); hf bit 1
// sends the row's output to the hold.
template <int P, int PREC, bool ZS>
__device__ __forceinline__ void pipe_stage(const StepParams &k, const PipeRow<PipeShape<P>::G> &L,
                                           typename PipeShape<P, PREC>::T *xs,
                                           const typename PipeShape<P, PREC>::T *xp, int wave, int lane,
                                           double (&bo)[PipeShape<P>::G][4], int &I, double &d, int64_t &v0,
                                           int &hf) {
    constexpr int N1 = P + 1, G = PipeShape<P>::G, XS = PipeShape<P, PREC>::XS, STR = PipeShape<P, PREC>::STR;
    typedef typename PipeShape<P, PREC>::T T;
    const int r = 16 * wave + pipe_row<PREC>(lane);
    const int vq = pipe_vec<PREC>(lane);
    const bool useo = !L.fst || k.Ym1 != nullptr;
    const double vI = (L.n.I >= 0 && L.fst) ? L.vraw : 0.0;
    const double sc = k.alpha * (vI - k.shift);
    d = node_scale(L.n);
    I = L.n.I;
    v0 = L.v0;
    hf = (L.bot ? 1 : 0) | (L.top ? 2 : 0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (ZS && L.bot) {
            if constexpr (PREC == 2) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int v = vq + pipe_off(q);
                    xs[g * XS + v * STR + r] = xp[g * XS + v * STR + r + P * N1 * N1];
                }
            } else {
                const T *src = xp + g * XS + (r + P * N1 * N1) * 16 + vq;
                T *dst = xs + g * XS + r * 16 + vq;
                if constexpr (PREC == 0) {
                    *reinterpret_cast<double2 *>(dst) = *reinterpret_cast<const double2 *>(src);
                    *reinterpret_cast<double2 *>(dst + 8) = *reinterpret_cast<const double2 *>(src + 8);
                } else {
                    *reinterpret_cast<f2 *>(dst) = *reinterpret_cast<const f2 *>(src);
                    *reinterpret_cast<f2 *>(dst + 8) = *reinterpret_cast<const f2 *>(src + 8);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) bo[g][q] = 0.0;
            continue;
        }
        double dx[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool ok = L.n.I >= 0 && L.v0 + 16 * g + pipe_off(q) < k.N;
            const double x = ok ? L.x[g][q] : 0.0;
            const double o = (ok && useo) ? L.o[g][q] : 0.0;
            double base = sc * x;
            if (k.Ym1) base -= k.beta * o;
            bo[g][q] = L.fst ? base : o;
            dx[q] = d * x;
        }
        if constexpr (PREC == 2) {
            // transposed: element (row r, vector v) at v * STR + r
#pragma unroll
            for (int q = 0; q < 4; ++q) xs[g * XS + (vq + pipe_off(q)) * STR + r] = to_bf16_bits(dx[q]);
        } else {
            T *dst = xs + g * XS + r * 16 + vq;
            if constexpr (PREC == 0) {
                *reinterpret_cast<double2 *>(dst) = double2{dx[0], dx[1]};
                *reinterpret_cast<double2 *>(dst + 8) = double2{dx[2], dx[3]};
            } else {
                *reinterpret_cast<f2 *>(dst) = f2{(float)dx[0], (float)dx[1]};
                *reinterpret_cast<f2 *>(dst + 8) = f2{(float)dx[2], (float)dx[3]};
            }
        }
    }
}

// Walk of a workgroup: its items blockIdx.x, blockIdx.x + gridDim.x, ...,
// each taken as ZL consecutive cells of a z segment (ZL = 1 without
// segments); position t of the walk is cell t % ZL of the workgroup's item
// t / ZL.  One body call handles one position: the product from xbuf[cur];
// the next position (loaded into Ln) staged into the other buffer, with the
// loads of the position after it requested into Lf first (index clamped to
// the last position, so the loads are unconditional and the wait for Ln's
// loads leaves them in flight); then this position's outputs are stored (to
// the hold for the top face of a segment's non-last cell).
template <int P, int PREC, int PD, bool ZS>
__global__ __launch_bounds__(64 * PipeShape<P>::W) __attribute__((amdgpu_waves_per_eu(1, 2)))
void step_pipe_kernel(StepParams k, int64_t nitems) {
    static_assert(PD == 2 || !ZS, "z segments need the two-deep pipeline");
    constexpr int N1 = P + 1, NKS = PipeShape<P, PREC>::NKS, G = PipeShape<P>::G, XS = PipeShape<P, PREC>::XS;
    constexpr int HS = N1 * N1 * 16 * G;  // doubles per hold buffer
    typedef typename PipeShape<P, PREC>::T T;
    typedef typename FragOf<PREC>::T FragT;
    extern __shared__ __align__(16) unsigned char smem[];
    T *xbuf = reinterpret_cast<T *>(smem);                                      // [2][G][XS]
    double *hold = reinterpret_cast<double *>(smem + PipeShape<P, PREC>::bytes);  // [2][N1*N1][16G] (ZS)

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ngroups = (k.nchunk + G - 1) / G;
    const int64_t stride = gridDim.x;
    if ((int64_t)blockIdx.x >= nitems) return;  // whole workgroup
    const int zl = ZS ? k.zl : 1;
    const int npos = (int)((nitems - 1 - blockIdx.x) / stride + 1) * zl;  // < 2^31, as items per launch
    auto item_of = [&](int t) { return (int64_t)blockIdx.x + (int64_t)(ZS ? t / zl : t) * stride; };
    auto cell_of = [&](int t) { return ZS ? t % zl : 0; };
    // the wave's row tile of (1/2)K_c, resident for the launch
    FragT ar[NKS];
    {
        const FragT *A = reinterpret_cast<const FragT *>(k.A) + (size_t)wave * NKS * 64 + lane;
#pragma unroll
        for (int s = 0; s < NKS; ++s) ar[s] = A[s * 64];
    }
    const int r = 16 * wave + pipe_row<PREC>(lane);
    const int vq = pipe_vec<PREC>(lane);
    double bo[G][4], d;
    int I, hf = 0;
    int64_t v0;
    int cur = 0;
    int t = 0;
    auto body = [&](PipeRow<G> &Ln, PipeRow<G> &Lf) -> bool {
        const bool more = t + 1 < npos;  // uniform over the workgroup
        if constexpr (PD == 2) {
            const int tf = min(t + 2, npos - 1);
            pipe_issue<P, PREC, ZS>(k, item_of(tf), cell_of(tf), ngroups, wave, lane, Lf);
        } else if (more) {
            pipe_issue<P, PREC, ZS>(k, item_of(t + 1), cell_of(t + 1), ngroups, wave, lane, Ln);
        }
        const T *xs = xbuf + cur * G * XS;
        double acc[G][4];
        if constexpr (PREC == 0) {
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[g][q] = 0.0;
            double bc[G][4], bn[G][4];
#pragma unroll
            for (int g = 0; g < G; ++g) f64_pair_b(xs + g * XS, 0, lane, bc[g]);
#pragma unroll
            for (int s = 0; s < NKS; ++s) {
                if (s + 1 < NKS)
#pragma unroll
                    for (int g = 0; g < G; ++g) f64_pair_b(xs + g * XS, s + 1, lane, bn[g]);
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[g][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[s], bc[g][q], acc[g][q], 0, 0, 0);
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) bc[g][q] = bn[g][q];
            }
        } else if constexpr (PREC == 2) {
            // transposed 16x16x32 products: 8 consecutive rows of one vector of
            // X from the vector-major buffer, the cell-matrix fragment second
            constexpr int STR = PipeShape<P, PREC>::STR;
            const T *xa = xs + pipe_perm(lane & 15) * STR + 8 * (lane >> 4);
            f4 c4[G];
#pragma unroll
            for (int g = 0; g < G; ++g) c4[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < NKS; ++s)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const bf8 a = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4 *>(xa + g * XS + 32 * s));
                    c4[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf8, ar[s]), c4[g], 0, 0, 0);
                }
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[g][q] = (double)c4[g][q];
        } else {
            // transposed 16x16x4 products: X slice first, cell-matrix fragment second
            f4 c4[G];
            float bc[G], bn[G];
            const int bo0 = (lane >> 4) * 16 + pipe_perm(lane & 15);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                c4[g] = f4{0.f, 0.f, 0.f, 0.f};
                bc[g] = xs[g * XS + bo0];
            }
#pragma unroll
            for (int s = 0; s < NKS; ++s) {
                if (s + 1 < NKS)
#pragma unroll
                    for (int g = 0; g < G; ++g) bn[g] = xs[g * XS + (4 * (s + 1)) * 16 + bo0];
#pragma unroll
                for (int g = 0; g < G; ++g) c4[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(bc[g], ar[s], c4[g], 0, 0, 0);
#pragma unroll
                for (int g = 0; g < G; ++g) bc[g] = bn[g];
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[g][q] = (double)c4[g][q];
        }
        if constexpr (ZS) {
            // a bottom-face row of a later cell continues the previous cell's
            // output for the same node, left in the hold
            if (hf & 1) {
                const double *h = hold + ((t - 1) & 1) * HS + r * 16 * G + vq;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const double2 u = *reinterpret_cast<const double2 *>(h + 16 * g);
                    const double2 w = *reinterpret_cast<const double2 *>(h + 16 * g + 8);
                    bo[g][0] = u.x; bo[g][1] = u.y; bo[g][2] = w.x; bo[g][3] = w.y;
                }
            }
        }
        // outputs of this position, kept while the next one is staged
        double out[G][4];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q) out[g][q] = bo[g][q] + k.alpha * d * acc[g][q];
        const int Io = I, hfo = hf;
        const int64_t v0o = v0;
        if (more)
            pipe_stage<P, PREC, ZS>(k, Ln, xbuf + (cur ^ 1) * G * XS, xs, wave, lane, bo, I, d, v0, hf);
        if (ZS && (hfo & 2)) {
            double *h = hold + (t & 1) * HS + (r - P * N1 * N1) * 16 * G + vq;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                *reinterpret_cast<double2 *>(h + 16 * g) = double2{out[g][0], out[g][1]};
                *reinterpret_cast<double2 *>(h + 16 * g + 8) = double2{out[g][2], out[g][3]};
            }
        } else if (Io >= 0) {
            double *yrow = k.Y + (int64_t)Io * k.ldy;
            if (wide_ok(k, v0o - vq, 16 * G)) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    double *yp = yrow + v0o + 16 * g;
                    *reinterpret_cast<double2 *>(yp) = double2{out[g][0], out[g][1]};
                    *reinterpret_cast<double2 *>(yp + 8) = double2{out[g][2], out[g][3]};
                }
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t vec = v0o + 16 * g + pipe_off(q);
                        if (vec < k.N) yrow[vec] = out[g][q];
                    }
            }
        }
        if (!more) return false;
        cur ^= 1;
        __syncthreads();
        ++t;
        return true;
    };
    PipeRow<G> LA, LB;
    pipe_issue<P, PREC, ZS>(k, item_of(0), 0, ngroups, wave, lane, LA);
    pipe_stage<P, PREC, ZS>(k, LA, xbuf, xbuf, wave, lane, bo, I, d, v0, hf);  // cell 0: no bottom copy
    __syncthreads();
    if constexpr (PD == 2) {
        const int t1 = min(1, npos - 1);
        pipe_issue<P, PREC, ZS>(k, item_of(t1), cell_of(t1), ngroups, wave, lane, LA);
        for (;;) {
            if (!body(LA, LB)) break;
            if (!body(LB, LA)) break;
        }
    } else {
        while (body(LA, LB)) {
        }
    }
}

// Cells per z segment for the segmented pipelined kernel: the largest length
// up to 6 that divides the cell count along z and leaves a periodic axis at
// least two segments; 1 (no segments) when there is none above 1.
static int zseg_length(const fe_mesh *m) {
    const int nz = m->ncell[2];
    for (int L = 6; L >= 2; --L)
        if (nz % L == 0 && (m->bc[2] != FE_BC_PERIODIC || nz / L >= 2)) return L;
    return 1;
}

template <int P, int PREC, int PD, bool ZS>
static hipError_t launch_pipe_p(StepParams prm, const fe_mesh *m, hipStream_t s) {
    constexpr int W = PipeShape<P>::W, G = PipeShape<P>::G, N1 = P + 1;
    const size_t smem = PipeShape<P, PREC>::bytes + (ZS ? (size_t)2 * N1 * N1 * 16 * G * sizeof(double) : 0);
    static bool attr = false;
    static int resident = 0;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_pipe_kernel<P, PREC, PD, ZS>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        int per_cu = 0, dev = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&step_pipe_kernel<P, PREC, PD, ZS>), 64 * W, smem);
        if (e != hipSuccess) return e;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        resident = std::max(1, per_cu) * std::max(1, cus);
        attr = true;
    }
    // along z the colours are those of segments of zl cells (of cells when
    // zl = 1): segments of one colour share no node, as cells do
    prm.zl = ZS ? zseg_length(m) : 1;
    prm.zs = prm.ax[2];
    prm.zs.ncell = prm.ax[2].ncell / prm.zl;
    prm.zs.ncol = (prm.zs.bc == FE_BC_PERIODIC && (prm.zs.ncell & 1)) ? 3 : prm.zs.ncell >= 2 ? 2 : 1;
    const int ngroups = (prm.nchunk + G - 1) / G;
    for (int c2 = 0; c2 < prm.zs.ncol; ++c2)
        for (int c1 = 0; c1 < m->ncol[1]; ++c1)
            for (int c0 = 0; c0 < m->ncol[0]; ++c0) {
                int col[3] = {c0, c1, c2};
                int64_t cells = 1;
                for (int a = 0; a < 3; ++a) {
                    const AxisInfo &ax = a == 2 ? prm.zs : prm.ax[a];
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
                const int64_t nitems = cells * ngroups;
                const int64_t grid = std::min<int64_t>(nitems, resident);
                hipLaunchKernelGGL((step_pipe_kernel<P, PREC, PD, ZS>), dim3((unsigned)grid), dim3(64 * W), smem, s,
                                   prm, nitems);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

// ------------------------------------------------------------------------
// Step kernel with direct-to-LDS prefetch and a brick table (p = 3, 4, and
// p = 5 with FP32 products; meshes without a zero-Neumann axis, where M^-1/2
// of a free node depends
// only on its local index and folds into the cell matrix:
// A' = D^ (1/2 Kc) D^), with FP64 cell products (PREC 0) or FP32 ones
// (PREC 1: A' rounded to FP32, each X element rounded to FP32 as the
// product reads it from the FP64 buffer, FP32 accumulation; everything
// else, the buffers and the epilogue, in FP64 as for PREC 0).
//
// On gfx950 the FP64 4x4x4 MFMA and every other vector instruction share the
// SIMD's vector ALU (an FP64 MFMA holds it as long as 16 wave-wide FMA
// instructions would), and a wave issues about one instruction per four
// cycles, so every instruction a wave spends per cell position besides its
// products is taken from them.  This kernel keeps that count small:
// - the X rows go from HBM straight into LDS with 16-byte global-to-LDS
//   requests, two positions ahead, into three LDS buffers (no staging
//   arithmetic; with the folded cell matrix they need no scaling);
// - everything a position needs to know about its cell comes from one 8-byte
//   entry per brick of a colour, built on the host: the DoF of the brick's
//   first node and masks of the cell faces that are shared with a
//   cell of an earlier colour, lie on a Dirichlet face, or wrap on a periodic
//   axis.  A row's DoF is then the cell's first DoF plus a per-lane constant
//   (minus a per-lane wrap correction where the mask says so), and its
//   first-writer and validity tests are its per-lane face bits against those
//   masks: no per-row index arithmetic, no colour logic, no divisions.
// Persistent workgroups walk the items (brick of BX x BY x zl cells, 32
// vectors (16 at p = 5); the launcher hands the columns past the last whole
// group to another kernel) of a colour with stride gridDim.x, cell by cell
// (x fastest, then y, then z), one wave per 16-row tile of A' with the
// tile's fragments in registers.  A position's old values and v are
// loaded to registers at its start and used after its product; the partial
// sums of a brick's inner faces pass from cell to cell through LDS holds
// (the X rows of those faces are read again, mostly from the caches).
//
// Per position t: the old values and v of t are requested, then the X rows of
// t + 2 (into buffer (t + 2) % 3, free since the barrier that ended t - 1);
// the product reads buffer t % 3; one wait for the memory counter down to the
// four newest requests (the X rows of t + 2) covers both the old values of t
// and the X rows of t + 1 (requested before them); then the epilogue, the
// stores, and one barrier that makes every wave's X rows of t + 1 visible.
// Shape: TPW row tiles of A' per wave (tiles wave + W j), G 16-vector groups
// per item; W waves; XS doubles per group of an X buffer; DMA requests per
// position and wave (one per 8 rows and group).
template <int P, int TPW, int NGRP> struct TabShape {
    static constexpr int NCP = ((P + 1) * (P + 1) * (P + 1) + 31) / 32 * 32, NT = NCP / 16, NKS = NCP / 4;
    static constexpr int W = NT / TPW, G = NGRP, XS = NCP * 16, NDMA = 2 * TPW * G;
    static_assert(NT % TPW == 0, "row tiles split evenly over the waves");
};

// Brick-table entry: .x the DoF of local node 0 of the brick's first cell
// (its free-index arithmetic extended below 0 on a Dirichlet face), .y face
// masks of the brick (bit order lo x, hi x, lo y, hi y, lo z, hi z):
//   bits 0-5   faces shared with a brick of an earlier colour
//   bits 6-11  faces on a Dirichlet boundary
//   bits 12-17 faces that wrap on a periodic axis (hi faces only)
// A cell of the brick takes a lo bit only in the brick's first cell along
// that axis and a hi bit only in its last.
enum : int { SEG_FM = 0, SEG_DM = 6, SEG_WM = 12 };

// Buffer descriptors of the table kernel's X requests: byte range (offsets
// at or past it read zeros) and the fourth descriptor word of a raw buffer
// on this architecture family.
constexpr uint32_t kTabRange = 0x7FFFFFFFu;
constexpr int kBufferWord3 = 0x00020000;

// s_waitcnt immediates: vector-memory counter <= n, the other counters free;
// LDS counter 0, the other counters free
__device__ __forceinline__ constexpr int vmcnt_imm(int n) { return (n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8); }
__device__ __forceinline__ constexpr int lgkmcnt0_imm() { return 0xF | (0x3 << 14) | (0x7 << 4); }

// 16-byte LDS store written out as the instruction itself, so that the
// compiler's wait analysis does not order it behind the global-to-LDS
// requests in flight (it cannot tell that they write other buffers); the
// caller drains the LDS counter before the barrier that publishes it.
__device__ __forceinline__ void lds_store16(double *p, double a, double b) {
    const uint32_t off = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) double *)p;
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const dv2 v = {a, b};
    asm volatile("ds_write_b128 %0, %1" : : "v"(off), "v"(v) : "memory");
}

// a where c, else b, as two lane selects written out, so that the compiler
// keeps a select of request addresses a select instead of splitting the
// request under two execution masks (then it can no longer count the
// requests in flight and waits for all of them); all lanes active
__device__ __forceinline__ const double *select_ptr(bool c, const double *a, const double *b) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(c);
    const uint64_t pa = reinterpret_cast<uint64_t>(a), pb = reinterpret_cast<uint64_t>(b);
    uint32_t lo, hi;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(lo) : "v"((uint32_t)pb), "v"((uint32_t)pa), "s"(m));
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(hi) : "v"((uint32_t)(pb >> 32)), "v"((uint32_t)(pa >> 32)), "s"(m));
    return reinterpret_cast<const double *>(((uint64_t)hi << 32) | lo);
}

// a where c, else b, as one lane select written out (see select_ptr)
__device__ __forceinline__ uint32_t select_u32(bool c, uint32_t a, uint32_t b) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(c);
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(m));
    return r;
}

// Launch constants of one padded row r of the cell for one lane: element
// offset of the row within a block relative to the cell's local node 0
// (in-order DoF offset times the leading dimension, plus the lane's column),
// DoF offset, and face bits (bit 6: a padding row past (p+1)^3).
template <int P> struct TabRow {
    int64_t e;
    int off, faces;
    uint32_t eb;  // e in bytes (the request offset of a cell without Dirichlet or wrapping faces)
    __device__ __forceinline__ void init(const StepParams &k, int r, int col) {
        constexpr int N1 = P + 1, NC = N1 * N1 * N1;
        const int l = min(r, NC - 1);
        const int i = l % N1, j = (l / N1) % N1, kk = l / (N1 * N1);
        off = i + (int)k.nfx * (j + (int)k.nfy * kk);
        e = (int64_t)off * k.ldx + col;
        eb = (uint32_t)(e * 8);
        faces = r < NC ? ((i == 0 ? 1 : 0) | (i == P ? 2 : 0) | (j == 0 ? 4 : 0) | (j == P ? 8 : 0) |
                          (kk == 0 ? 16 : 0) | (kk == P ? 32 : 0))
                       : 64;
    }
    // DoF correction of a row on a wrapping hi face (wm: the position's wrap mask)
    __device__ __forceinline__ int wrap(const StepParams &k, int wm) const {
        const int w = faces & wm;
        return ((w & 2) ? (int)k.nfx : 0) + ((w & 8) ? (int)(k.nfx * k.nfy) : 0) +
               ((w & 32) ? (int)(k.nfx * k.nfy) * k.nfz : 0);
    }
};

// Shapes of the table kernel: one 16-row tile of A' per wave; p = 3, 4: 4 / 8
// tiles and 32 vectors per item; with FP32 products at p = 4 two waves per
// tile, one 16-vector group each (16 waves, up to 4 per SIMD within 128
// registers: 3-5 % faster than one wave per tile; no faster at p = 3; with
// FP64 products the same split spills at 128 registers and was 4.7 %
// slower); p = 5 (FP32
// products only: 224 padded rows): 14 waves (up to 4 per SIMD; 56 fragment
// registers each) and 16 vectors per item, so that three X buffers of 224
// rows fit the LDS (7 waves of two tiles each, 2 per SIMD, were 7 % slower)
template <int P, int PREC = 0> struct TabCfg {
    static constexpr int TPW = 1, G = P == 5 ? 1 : 2, GS = (PREC == 1 && P == 4) ? 2 : 1;
};

// (at most 2 waves per SIMD, or as many as the workgroup puts on one)
// CPX (FP64 only): the Bloch-k mode, columns complex vectors stored as
// interleaved (re, im) pairs; the operator gains -i D^ (k.G_c) D^ (folded
// fragments in k.S, rows in the same order as k.A).  As -i S (x_r + i x_i) =
// S x_i - i S x_r, each k-step adds S times the lane's im column to its re
// accumulator and S times the negated re column (the product's B-operand
// negation) to its im accumulator.
// GS waves per row tile, each taking NGRP / GS of the item's 16-vector groups
// (GS = 2: twice the waves, each with half the accumulators and requests).
template <int P, int PREC, int TPW, int NGRP, int BX, int BY, bool CPX = false, int GS = 1>
__global__ __launch_bounds__((64 * GS * TabShape<P, TPW, NGRP>::W))
__attribute__((amdgpu_waves_per_eu(1, GS * TabShape<P, TPW, NGRP>::W > 8 ? (GS * TabShape<P, TPW, NGRP>::W + 3) / 4 : 2)))
void step_tab_kernel(StepParams k, const int2 *__restrict__ segtab, const int *__restrict__ rowperm, int64_t nitems) {
    static_assert(PREC == 0 || PREC == 1, "FP64 or FP32 cell products");
    static_assert(!CPX || PREC == 0, "the Bloch mode is FP64 only");
    typedef typename FragOf<PREC>::T AT;
    typedef TabShape<P, TPW, NGRP> S;
    static_assert(NGRP % GS == 0, "groups split evenly over a tile's waves");
    // GI groups per item, G per wave
    constexpr int N1 = P + 1, NKS = S::NKS, GI = S::G, G = GI / GS, XS = S::XS, W = S::W, NDMA = 2 * TPW * G;
    // LDS holds (doubles), each node once: the x face between consecutive
    // cells of a brick row (N1 x N1 nodes), the back faces of a brick row
    // ((BX p + 1) x N1 nodes: x by z), the top faces of a brick layer
    // ((BX p + 1) x (BY p + 1) nodes: x by y); each slot is read and written
    // at one position by two rows of the same wave (see build_table_row_perm)
    constexpr int ZW = BX * P + 1, V = 16 * GI;
    constexpr int XHS = BX > 1 ? N1 * N1 * V : 0, YHS = BY > 1 ? ZW * N1 * V : 0, ZHS = ZW * (BY * P + 1) * V;
    constexpr int YH0 = XHS, ZH0 = YH0 + YHS, ZERO0 = ZH0 + ZHS;
    // three X buffers [G][NCP][16] as distinct arrays, each named at compile
    // time by the position it serves, so that the compiler sees that a
    // product's LDS reads and the X requests in flight touch different
    // buffers; the holds followed by 32 zeros (the hold term of rows that
    // take none) in one array, so that every hold read is based on it and the
    // compiler sees it apart from the X requests in flight
    __shared__ __align__(16) double xb0[GI * XS], xb1[GI * XS], xb2[GI * XS];
    __shared__ __align__(16) double hold[ZERO0 + 32];
    static_assert(sizeof(double) * (3 * GI * XS + ZERO0 + 32) <= 160 * 1024, "LDS of one workgroup");

    const int tid = threadIdx.x, lane = tid & 63;
    // the wave's row tile(s), and g0 the item's group of its first group
    const int wall = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wave = GS == 1 ? wall : wall % W, g0 = GS == 1 ? 0 : (wall / W) * G;
    if ((int64_t)blockIdx.x >= nitems) return;  // whole workgroup
    if (tid < 32) hold[ZERO0 + tid] = 0.0;
    const int ngroups = (k.nchunk + GI - 1) / GI;
    const int stride = (int)gridDim.x;
    const int sdiv = stride / ngroups, smod = stride % ngroups;
    const int zl = k.zl;
    const int npos = (int)((nitems - 1 - blockIdx.x) / stride + 1) * zl * BX * BY;  // < 2^31, as items per launch
    const int ystep = P * (int)k.nfx, zstep = P * (int)(k.nfx * k.nfy);  // DoF steps to the next cell along y, z
    const int64_t ld = k.ldx;  // one leading dimension for X, Y and the previous iterate
    // the wave's row tiles of A' (tiles wave + W j), and in the Bloch mode
    // of S', resident for the launch
    AT ar[TPW][NKS], sr[CPX ? TPW : 1][CPX ? NKS : 1];
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const AT *A = reinterpret_cast<const AT *>(k.A) + (size_t)(wave + W * j) * NKS * 64 + lane;
#pragma unroll
        for (int s = 0; s < NKS; ++s) ar[j][s] = A[s * 64];
        if constexpr (CPX) {
            const double *Sf = k.S + (size_t)(wave + W * j) * NKS * 64 + lane;
#pragma unroll
            for (int s = 0; s < NKS; ++s) sr[j][s] = Sf[s * 64];
        }
    }
    // per tile: the node whose output row this lane's accumulators hold
    // (row pipe_row of the tile, vectors vq + pipe_off(q) of each 16-vector
    // group; the rows of A' are the cell's nodes in the order rowperm gives)
    // and the two rows it requests X for (rows 16 tile + 8 h + l / 8, in
    // node order, vectors 2 (l % 8) + {0, 1} of each group)
    const int vq = pipe_vec<PREC>(lane);
    TabRow<P> R[TPW], Q[TPW][2];
    int xo[TPW], xh[TPW], yh[TPW], zh[TPW];  // offsets in an X buffer and in the three holds
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int tile = wave + W * j, node = rowperm[16 * tile + pipe_row<PREC>(lane)];
        R[j].init(k, node < 0 ? N1 * N1 * N1 : node, vq);
        Q[j][0].init(k, 16 * tile + (lane >> 3), 2 * (lane & 7));
        Q[j][1].init(k, 16 * tile + 8 + (lane >> 3), 2 * (lane & 7));
        const int l = node < 0 ? 0 : node, i = l % N1, jy = (l / N1) % N1, kk = l / (N1 * N1);
        xo[j] = l * 16 + vq;
        xh[j] = (jy + N1 * kk) * V + vq;
        yh[j] = YH0 + (i + ZW * kk) * V + vq;
        zh[j] = ZH0 + (i + ZW * jy) * V + vq;
    }
    const double *ob = k.Ym1 ? k.Ym1 : k.X;
    const double nbeta = k.Ym1 ? -k.beta : 0.0;

    // a walk position: brick s of the colour, vector group grp, cell
    // (bx, by, c) of the brick (bx along x, fastest; by along y; c along z);
    // e its table entry
    struct Pos {
        int s, grp, c, bx, by;
        int2 e;
    };
    auto advance = [&](Pos p) {
        if (++p.bx == BX) {
            p.bx = 0;
            if (++p.by == BY) {
                p.by = 0;
                if (++p.c == zl) {
                    p.c = 0;
                    p.s += sdiv;
                    p.grp += smod;
                    if (p.grp >= ngroups) {
                        p.grp -= ngroups;
                        ++p.s;
                    }
                    p.e = segtab[p.s];
                }
            }
        }
        return p;
    };
    // what a position needs (uniform): element offset of its cell's node 0
    // and first vector, DoF of node 0, face masks with the bits that apply
    // at its place in the brick
    struct Cell {
        int64_t U;
        int I0, fm, dm, wm;
    };
    auto cell = [&](const Pos &p) {
        Cell q;
        q.I0 = p.e.x + p.bx * P + p.by * ystep + p.c * zstep;
        q.U = (int64_t)q.I0 * ld + (int64_t)p.grp * GI * 16 + g0 * 16;
        const int hi = (p.bx == BX - 1 ? 2 : 0) | (p.by == BY - 1 ? 8 : 0) | (p.c == zl - 1 ? 32 : 0);
        const int m = hi | (p.bx == 0 ? 1 : 0) | (p.by == 0 ? 4 : 0) | (p.c == 0 ? 16 : 0);
        q.fm = (p.e.y >> SEG_FM) & m;
        q.dm = (p.e.y >> SEG_DM) & m;
        q.wm = (p.e.y >> SEG_WM) & hi;
        return q;
    };
    // X rows of a position into buffer bufp, as buffer requests (a global
    // request that writes LDS would make the compiler drain the LDS counter
    // at every wait of the product loop): the buffer starts at the cell's
    // first row, less the largest wrap correction of the position, so that
    // every row's byte offset is a non-negative 32-bit value, a launch
    // constant for cells without Dirichlet or wrapping faces.  Padding rows
    // take the row of the cell's last node (their columns of A' are zero),
    // which exists when no face of the cell is on a Dirichlet boundary or
    // wraps; otherwise they, and the rows on a Dirichlet face, take an offset
    // past the buffer's range, which reads zeros.
    auto prefetch = [&](const Cell &q, double *__restrict__ bufp) {
        int64_t wt = 0;  // uniform: the wrap corrections that apply to the position
        if (q.wm)
            wt = ((q.wm & 2) ? k.nfx : 0) + ((q.wm & 8) ? k.nfx * k.nfy : 0) +
                 ((q.wm & 32) ? k.nfx * k.nfy * (int64_t)k.nfz : 0);
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(k.X + (q.U - wt * ld)), (short)0, kTabRange, kBufferWord3);
        uint32_t vo[TPW][2];
#pragma unroll
        for (int j = 0; j < TPW; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h) vo[j][h] = Q[j][h].eb;
        if (q.dm | q.wm) {  // uniform: a cell on a Dirichlet face or a periodic wrap
#pragma unroll
            for (int j = 0; j < TPW; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const TabRow<P> &T = Q[j][h];
                    vo[j][h] = select_u32((T.faces & (q.dm | 64)) == 0,
                                          (uint32_t)((T.e + (wt - T.wrap(k, q.wm)) * ld) * 8), kTabRange + 1u);
                }
        }
        // one join before the requests, so that both paths issue them in the
        // same block (the compiler counts the requests in flight only there)
#pragma unroll
        for (int j = 0; j < TPW; ++j) asm volatile("" : "+v"(vo[j][0]), "+v"(vo[j][1]));
#pragma unroll
        for (int j = 0; j < TPW; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    // (the offset goes through a scalar local: an array element
                    // as the argument leaves the kernel without its host stub)
                    const uint32_t voff = vo[j][h];
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs, (__attribute__((address_space(3))) void *)(bufp + (g0 + g) * XS + (16 * (wave + W * j) + 8 * h) * 16),
                        16u, voff, 128u * (unsigned)g, 0, 0);
                }
        asm volatile("" ::: "memory");
    };

    // position t (cell cur): product from xs, X rows of t + 2 (n2, the
    // position after n1) into xn; false after the last position
    auto body = [&](int t, const Pos &cur, const Pos &n1, Pos &n2, const double *__restrict__ xs,
                    double *__restrict__ xn, double *__restrict__ hd) -> bool {
        const Cell e = cell(cur);
        const bool slow = (e.dm | e.wm) != 0;  // uniform
        int64_t E[TPW];
        bool valid[TPW], fst[TPW], left[TPW], right[TPW], front[TPW], back[TPW], bot[TPW], top[TPW];
        double vraw[TPW], o[TPW][G][4];
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            // the accumulator row: DoF, element offset, validity, first writer
            int I = e.I0 + R[j].off;
            E[j] = e.U + R[j].e;
            valid[j] = R[j].faces < 64;
            if (slow) {
                const int w = R[j].wrap(k, e.wm);
                I -= w;
                E[j] -= (int64_t)w * ld;
                valid[j] = (R[j].faces & (e.dm | 64)) == 0;
            }
            // faces shared with the brick's previous / next cell along x
            // (the x-face hold), along y (the back-face hold) and along z
            // (the top-face hold)
            left[j] = BX > 1 && (R[j].faces & 1) != 0 && cur.bx > 0;
            right[j] = BX > 1 && (R[j].faces & 2) != 0 && cur.bx < BX - 1;
            front[j] = BY > 1 && (R[j].faces & 4) != 0 && cur.by > 0;
            back[j] = BY > 1 && (R[j].faces & 8) != 0 && cur.by < BY - 1;
            bot[j] = (R[j].faces & 16) != 0 && cur.c > 0;
            top[j] = (R[j].faces & 32) != 0 && cur.c < zl - 1;
            const bool held = left[j] || front[j] || bot[j];
            fst[j] = valid[j] && (R[j].faces & e.fm) == 0 && !held;
            // old values: the previous iterate for a first writer, else Y
            // (an earlier colour has written the node); none for rows off the
            // cell, rows whose partial sum a hold carries, or a first writer
            // without a previous iterate
            const bool none = !valid[j] || held || (fst[j] && !k.Ym1);
            const double *orow = none ? k.zero : (fst[j] ? ob : k.Y) + E[j];
            vraw[j] = k.v[valid[j] ? I : 0];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double2 a = *reinterpret_cast<const double2 *>(orow + 16 * g);
                const double2 b = *reinterpret_cast<const double2 *>(orow + 16 * g + 8);
                o[j][g][0] = a.x; o[j][g][1] = a.y; o[j][g][2] = b.x; o[j][g][3] = b.y;
            }
        }
        asm volatile("" ::: "memory");  // these requests go out before the X rows of t + 2
        // X rows two positions ahead (past the walk's end the last position's
        // rows again, into the free buffer, which nobody reads afterwards)
        n2 = t + 2 < npos ? advance(n1) : n1;
        prefetch(cell(n2), xn);
        double acc[TPW][G][4];
        if constexpr (PREC == 0) {
#pragma unroll
            for (int j = 0; j < TPW; ++j)
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[j][g][q] = 0.0;
            double bc[G][4], bn[G][4];
#pragma unroll
            for (int g = 0; g < G; ++g) f64_pair_b(xs + (g0 + g) * XS, 0, lane, bc[g]);
#pragma unroll
            for (int s = 0; s < NKS; ++s) {
                if (s + 1 < NKS)
#pragma unroll
                    for (int g = 0; g < G; ++g) f64_pair_b(xs + (g0 + g) * XS, s + 1, lane, bn[g]);
#pragma unroll
                for (int j = 0; j < TPW; ++j)
#pragma unroll
                    for (int g = 0; g < G; ++g)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[j][g][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[j][s], bc[g][q], acc[j][g][q], 0, 0, 0);
                if constexpr (CPX) {
                    // columns q = 0, 2 are re, q = 1, 3 the im of the same
                    // complex vectors; the last argument 2 negates B
#pragma unroll
                    for (int j = 0; j < TPW; ++j)
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            acc[j][g][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(sr[j][s], bc[g][1], acc[j][g][0], 0, 0, 0);
                            acc[j][g][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(sr[j][s], bc[g][0], acc[j][g][1], 0, 0, 2);
                            acc[j][g][2] = __builtin_amdgcn_mfma_f64_4x4x4f64(sr[j][s], bc[g][3], acc[j][g][2], 0, 0, 0);
                            acc[j][g][3] = __builtin_amdgcn_mfma_f64_4x4x4f64(sr[j][s], bc[g][2], acc[j][g][3], 0, 0, 2);
                        }
                }
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) bc[g][q] = bn[g][q];
            }
        } else {
            // transposed 16x16x4 products: the X slice (row 4s + l / 16,
            // vector pipe_perm(l % 16), rounded from the buffer's f64 to f32)
            // first, the fragment second; lane l's accumulator q then holds
            // row pipe_row(l), vector vq + pipe_off(q)
            const int bo = (lane >> 4) * 16 + pipe_perm(lane & 15);
            f4 c4[TPW][G];
            float bc[G], bn[G];
#pragma unroll
            for (int g = 0; g < G; ++g) bc[g] = (float)xs[(g0 + g) * XS + bo];
#pragma unroll
            for (int j = 0; j < TPW; ++j)
#pragma unroll
                for (int g = 0; g < G; ++g) c4[j][g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < NKS; ++s) {
                if (s + 1 < NKS)
#pragma unroll
                    for (int g = 0; g < G; ++g) bn[g] = (float)xs[(g0 + g) * XS + 64 * (s + 1) + bo];
#pragma unroll
                for (int j = 0; j < TPW; ++j)
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        c4[j][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(bc[g], ar[j][s], c4[j][g], 0, 0, 0);
#pragma unroll
                for (int g = 0; g < G; ++g) bc[g] = bn[g];
            }
#pragma unroll
            for (int j = 0; j < TPW; ++j)
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[j][g][q] = (double)c4[j][g][q];
        }
        // the old values and v of t, and the X rows of t + 1 (both requested
        // before the NDMA X requests of t + 2)
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(NDMA));
        asm volatile("" ::: "memory");
        // the loaded values are used only from here on (not inside the product)
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            asm volatile("" : "+v"(vraw[j]));
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int q = 0; q < 4; ++q) asm volatile("" : "+v"(o[j][g][q]));
        }
        // this cell's offsets in the back-face hold (x) and the top-face hold (x, y)
        const int yoff = cur.bx * P * V, zoff = yoff + cur.by * P * ZW * V;
        // epilogue, one form for every row:
        //   out = alpha acc + (s x + (gamma o + h))
        // first writer: s = alpha (v - c), gamma = -beta, h = 0 (x raw from
        // the buffer); a row whose partial sum a hold carries (from the
        // previous cell along x, else along y, else along z): s = 0, o = 0,
        // h = the hold; any other row: s = 0, gamma = 1, h = 0.  Every hold
        // read of the wave comes before its hold writes (a slot read at this
        // position is written at it only by a row of the same wave).
        double out[TPW][G][4];
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const double sl = fst[j] ? k.alpha * (vraw[j] - k.shift) : 0.0;
            const double gl = fst[j] ? nbeta : 1.0;
            const int hoff = left[j] ? xh[j] : front[j] ? yh[j] + yoff : bot[j] ? zh[j] + zoff : ZERO0;
            const double *hrow = hd + hoff;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double2 x01 = *reinterpret_cast<const double2 *>(xs + (g0 + g) * XS + xo[j]);
                const double2 x23 = *reinterpret_cast<const double2 *>(xs + (g0 + g) * XS + xo[j] + 8);
                const double2 h01 = *reinterpret_cast<const double2 *>(hrow + 16 * (g0 + g));
                const double2 h23 = *reinterpret_cast<const double2 *>(hrow + 16 * (g0 + g) + 8);
                const double xv[4] = {x01.x, x01.y, x23.x, x23.y}, hv[4] = {h01.x, h01.y, h23.x, h23.y};
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    out[j][g][q] = __builtin_fma(k.alpha, acc[j][g][q],
                                                 __builtin_fma(sl, xv[q], __builtin_fma(gl, o[j][g][q], hv[q])));
            }
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            // the partial sum goes on to the next cell along x, else along y,
            // else along z, else to Y
            if (right[j] || back[j] || top[j]) {
                double *h = hd + (right[j] ? xh[j] : back[j] ? yh[j] + yoff : zh[j] + zoff);
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    lds_store16(h + 16 * (g0 + g), out[j][g][0], out[j][g][1]);
                    lds_store16(h + 16 * (g0 + g) + 8, out[j][g][2], out[j][g][3]);
                }
            } else if (valid[j]) {
                double *yrow = k.Y + E[j];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    *reinterpret_cast<double2 *>(yrow + 16 * g) = double2{out[j][g][0], out[j][g][1]};
                    *reinterpret_cast<double2 *>(yrow + 16 * g + 8) = double2{out[j][g][2], out[j][g][3]};
                }
            }
        }
        // every wave's LDS writes done, then the barrier; the X rows of t + 1
        // were waited for above, those of t + 2 stay in flight
        __builtin_amdgcn_s_waitcnt(lgkmcnt0_imm());
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        return t + 1 < npos;
    };

    Pos p0, p1, p2;
    {
        const int it = (int)blockIdx.x;
        p0.s = it / ngroups;
        p0.grp = it % ngroups;
        p0.c = 0;
        p0.bx = 0;
        p0.by = 0;
        p0.e = segtab[p0.s];
    }
    p1 = npos > 1 ? advance(p0) : p0;
    prefetch(cell(p0), xb0);
    prefetch(cell(p1), xb1);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    asm volatile("" ::: "memory");
    __syncthreads();
    // the walk, three positions per round so that each buffer is named
    for (int t = 0;; t += 3) {
        if (!body(t, p0, p1, p2, xb0, xb2, hold)) break;
        if (!body(t + 1, p1, p2, p0, xb1, xb0, hold)) break;
        if (!body(t + 2, p2, p0, p1, xb2, xb1, hold)) break;
    }
    // the requests of the last positions (rows past the walk's end, into free
    // buffers) land before the workgroup's LDS is released
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
}

template <int P, int PREC, int TPW, int G, int BX, int BY, bool CPX, int GS>
static hipError_t launch_tab_p(StepParams prm, const fe_mesh *m, hipStream_t s) {
    typedef TabShape<P, TPW, G> S;
    constexpr int W = GS * S::W;
    static bool attr = false;
    static int resident = 0;
    if (!attr) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&step_tab_kernel<P, PREC, TPW, G, BX, BY, CPX, GS>), 64 * W, 0);
        if (e != hipSuccess) return e;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        resident = std::max(1, per_cu) * std::max(1, cus);
        attr = true;
    }
    prm.A = PREC == 0 ? (const void *)m->d_Af64s : (const void *)m->d_Af32s;
    prm.S = CPX ? m->d_Sf64s : nullptr;
    prm.zl = m->seg_zl;
    prm.nfz = (int)m->nf[2];
    const int ngroups = (prm.nchunk + G - 1) / G;
    // the table of this brick shape (y bricks: the first table)
    const std::vector<int64_t> &off = BY > 1 || m->seg_by == 1 ? m->seg_off : m->seg_off1;
    const int32_t *tab0 = BY > 1 || m->seg_by == 1 ? m->d_segtab : m->d_segtab1;
    for (size_t col = 0; col + 1 < off.size(); ++col) {
        const int64_t segs = off[col + 1] - off[col];
        if (segs == 0) continue;
        const int2 *tab = reinterpret_cast<const int2 *>(tab0) + off[col];
        const int64_t nitems = segs * ngroups;
        const int64_t grid = std::min<int64_t>(nitems, resident);
        hipLaunchKernelGGL((step_tab_kernel<P, PREC, TPW, G, BX, BY, CPX, GS>), dim3((unsigned)grid), dim3(64 * W), 0, s, prm,
                           tab, m->d_tabperm, nitems);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int P, int PREC, int BY, bool CPX>
static hipError_t launch_tab_y(StepParams prm, const fe_mesh *m, hipStream_t s) {
    typedef TabCfg<P, PREC> C;
    switch (m->seg_bx) {
    case 3: return launch_tab_p<P, PREC, C::TPW, C::G, 3, BY, CPX, C::GS>(prm, m, s);
    case 2: return launch_tab_p<P, PREC, C::TPW, C::G, 2, BY, CPX, C::GS>(prm, m, s);
    default: return launch_tab_p<P, PREC, C::TPW, C::G, 1, BY, CPX, C::GS>(prm, m, s);
    }
}

// FP64 products walk the bricks with y extent (2 cells where the mesh
// allows): fewer bytes, and faster where the products dominate; FP32
// products, HBM-bound, were measured faster on bricks one cell deep in y
// (the second table), where a brick's cells are closer together in memory.
template <int P, int PREC, bool CPX = false>
static hipError_t launch_tab(StepParams prm, const fe_mesh *m, hipStream_t s) {
    if constexpr (PREC == 0)
        if (m->seg_by == 2) return launch_tab_y<P, PREC, 2, CPX>(prm, m, s);
    return launch_tab_y<P, PREC, 1, CPX>(prm, m, s);
}

// Cells per brick along an axis of the table kernel (x: up to 3, y: up to
// 2): the largest length that divides the axis' cell count and leaves a
// periodic axis at least two bricks; 1 when there is none above 1.
static int brick_length(const fe_mesh *m, int axis, int most) {
    const int n = m->ncell[axis];
    for (int L = most; L >= 2; --L)
        if (n % L == 0 && (m->bc[axis] != FE_BC_PERIODIC || n / L >= 2)) return L;
    return 1;
}

// Output-row order of the table kernel's cell matrix (host): rowperm[r] is
// the local node whose output row r of A' holds (-1: a padding row), so that
// the rows a wave owns (its tiles wave + W j, 16 rows each) hold whole
// classes of nodes linked by the holds: the two nodes of a cell at i = 0 and
// i = p with the same (j, k) read and write the same x-face hold slot at one
// position, those at j = 0, p with the same (i, k) the same back-face slot,
// those at k = 0, p with the same (i, j) the same top-face slot.  The
// classes (8 corners; 4 nodes of an edge; 2 of a face; 1 inside) are placed
// largest first into the first wave with room (their sizes divide a wave's
// rows, so they always fit).
void build_table_row_perm(int p, int tiles_per_wave, std::vector<int32_t> &perm) {
    const int n1 = p + 1, nc = n1 * n1 * n1, ncp = padded_nc(p), nt = ncp / 16, nw = nt / tiles_per_wave;
    std::vector<int> cls(nc);
    for (int l = 0; l < nc; ++l) {
        // the class representative: each coordinate at p folded onto 0
        int i = l % n1, j = (l / n1) % n1, kk = l / (n1 * n1);
        i = i == p ? 0 : i;
        j = j == p ? 0 : j;
        kk = kk == p ? 0 : kk;
        cls[l] = i + n1 * (j + n1 * kk);
    }
    std::vector<std::vector<int>> classes(nc);
    for (int l = 0; l < nc; ++l) classes[cls[l]].push_back(l);
    std::vector<int> order;
    for (int c = 0; c < nc; ++c)
        if (!classes[c].empty()) order.push_back(c);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return classes[a].size() > classes[b].size(); });
    std::vector<std::vector<int>> waves(nw);
    const size_t cap = 16 * (size_t)tiles_per_wave;
    for (int c : order) {
        size_t w = 0;
        while (waves[w].size() + classes[c].size() > cap) ++w;  // the sizes are powers of 2 dividing cap
        waves[w].insert(waves[w].end(), classes[c].begin(), classes[c].end());
    }
    perm.assign(ncp, -1);
    for (int w = 0; w < nw; ++w)
        for (size_t q = 0; q < waves[w].size(); ++q) {
            const int tile = w + nw * (int)(q / 16);
            perm[16 * tile + q % 16] = waves[w][q];
        }
}

int table_tiles_per_wave(int p) { return p == 5 ? TabCfg<5>::TPW : TabCfg<4>::TPW; }

// Segment table of the table kernel (host): for every colour pass, in launch
// order, the bricks of that colour (BX cells along x by BY along y by zl
// along z), in the order the kernel walks them, one entry each (see SEG_FM /
// SEG_DM / SEG_WM; the bits describe the brick's outer faces).  Bricks are
// coloured along each axis as cells are.
void build_segment_table(const fe_mesh *m, int by_most, std::vector<int32_t> &tab, std::vector<int64_t> &off,
                         int &zl_out, int &bx_out, int &by_out) {
    tab.clear();
    off.assign(1, 0);
    const int P = m->p;
    const int zl = zseg_length(m), bxl = brick_length(m, 0, 3), byl = brick_length(m, 1, by_most);
    zl_out = zl;
    bx_out = bxl;
    by_out = byl;
    AxisInfo ax[3];
    for (int d = 0; d < 3; ++d) {
        ax[d].ncell = m->ncell[d];
        ax[d].nfree = (int)m->nf[d];
        ax[d].bc = m->bc[d];
        ax[d].ncol = m->ncol[d];
    }
    // the brick axes: x in runs of bxl cells, y of byl, z of zl
    AxisInfo bk[3] = {ax[0], ax[1], ax[2]};
    const int len[3] = {bxl, byl, zl};
    for (int a = 0; a < 3; ++a) {
        bk[a].ncell = ax[a].ncell / len[a];
        bk[a].ncol = (bk[a].bc == FE_BC_PERIODIC && (bk[a].ncell & 1)) ? 3 : bk[a].ncell >= 2 ? 2 : 1;
    }
    auto colour_of = [](const AxisInfo &a, int c) { return (a.ncol == 3 && c == a.ncell - 1) ? 2 : (c & 1); };
    // whether the neighbour across face lo or hi of brick (cell) c exists and has a lower colour
    auto shared_earlier = [&](const AxisInfo &a, int c, bool hi) {
        int nb = hi ? c + 1 : c - 1;
        bool wrap = false;
        if (nb < 0) { nb = a.ncell - 1; wrap = true; }
        if (nb >= a.ncell) { nb = 0; wrap = true; }
        const bool exists = !wrap || a.bc == FE_BC_PERIODIC;
        return exists && colour_of(a, nb) < colour_of(a, c);
    };
    auto first_free = [&](const AxisInfo &a, int c) { return c * P - (a.bc == FE_BC_DIRICHLET ? 1 : 0); };
    for (int c2 = 0; c2 < bk[2].ncol; ++c2)
        for (int c1 = 0; c1 < bk[1].ncol; ++c1)
            for (int c0 = 0; c0 < bk[0].ncol; ++c0) {
                const int col[3] = {c0, c1, c2};
                int cnt[3];
                for (int a = 0; a < 3; ++a) {
                    const AxisInfo &A = bk[a];
                    if (col[a] == 2) cnt[a] = 1;
                    else {
                        const int limit = A.ncol == 3 ? A.ncell - 1 : A.ncell;
                        cnt[a] = limit > col[a] ? (limit - col[a] + 1) / 2 : 0;
                    }
                }
                for (int iz = 0; iz < cnt[2]; ++iz)
                    for (int iy = 0; iy < cnt[1]; ++iy)
                        for (int ix = 0; ix < cnt[0]; ++ix) {
                            const int ic[3] = {iz, iy, ix};
                            int b[3];  // brick index along each axis
                            for (int a = 0; a < 3; ++a)
                                b[a] = col[a] == 2 ? bk[a].ncell - 1 : col[a] + 2 * ic[2 - a];
                            const int I0 = first_free(ax[0], b[0] * bxl) +
                                           (int)m->nf[0] * (first_free(ax[1], b[1] * byl) +
                                                            (int)m->nf[1] * first_free(ax[2], b[2] * zl));
                            int fm = 0, dm = 0, wm = 0;
                            for (int a = 0; a < 3; ++a) {
                                fm |= (shared_earlier(bk[a], b[a], false) ? 1 : 0) << (2 * a);
                                fm |= (shared_earlier(bk[a], b[a], true) ? 2 : 0) << (2 * a);
                                if (bk[a].bc == FE_BC_DIRICHLET) {
                                    dm |= (b[a] == 0 ? 1 : 0) << (2 * a);
                                    dm |= (b[a] == bk[a].ncell - 1 ? 2 : 0) << (2 * a);
                                }
                                if (bk[a].bc == FE_BC_PERIODIC) wm |= (b[a] == bk[a].ncell - 1 ? 2 : 0) << (2 * a);
                            }
                            tab.push_back(I0);
                            tab.push_back((fm << SEG_FM) | (dm << SEG_DM) | (wm << SEG_WM));
                        }
                off.push_back((int64_t)tab.size() / 2);
            }
}

// Whether the table kernel applies: FP64 (p = 3, 4) or FP32 (p = 3, 4, 5)
// products, real mode, folded cell matrix and segment table (no Neumann
// axis), one leading
// dimension for X, Y and the previous iterate, 16-byte requests at every row
// and column pair (blocks 16-byte aligned, even leading dimension), and X
// request offsets within the 31-bit range of its buffer requests.
static bool dma_applies(const fe_mesh *m, const StepArgs &a, fe_dtype prec) {
    if (!m->d_segtab || m->p < 3 || m->p > 5 || (m->p == 5 && prec != FE_F32)) return false;
    // the Bloch mode: FP64 at p = 3, 4, with the folded k.G fragments
    if (a.S && (prec != FE_F64 || m->p > 4 || !m->d_Sf64s)) return false;
    if (!(prec == FE_F64 ? m->d_Af64s != nullptr : prec == FE_F32 && m->d_Af32s != nullptr)) return false;
    const uintptr_t ptrs = reinterpret_cast<uintptr_t>(a.X) | reinterpret_cast<uintptr_t>(a.Y) |
                           reinterpret_cast<uintptr_t>(a.Ym1 ? a.Ym1 : a.X);
    const bool same_ld = a.ldy == a.ldx && (!a.Ym1 || a.ldm == a.ldx);
    // every X request's byte offset from its position's buffer start (the
    // largest in-cell offset plus the largest wrap correction) below 2^31
    const int64_t P = m->p;
    const int64_t offmax = P * (1 + m->nf[0] * (1 + m->nf[1]));
    const int64_t wrapmax = (m->bc[0] == FE_BC_PERIODIC ? m->nf[0] : 0) +
                            (m->bc[1] == FE_BC_PERIODIC ? m->nf[0] * m->nf[1] : 0) +
                            (m->bc[2] == FE_BC_PERIODIC ? m->n : 0);
    const bool in_range = ((offmax + wrapmax + 1) * a.ldx + 64) * 8 < (int64_t)kTabRange;
    return (ptrs & 15) == 0 && (a.ldx & 1) == 0 && same_ld && in_range;
}

size_t assembled_scratch_doubles(const fe_mesh *m) {
    return m->p <= 5 ? (size_t)m->ncells * (size_t)padded_nc(m->p) : 0;
}

// N = 1, FP64: the two-launch form above for p <= 5 (Zc: device scratch of
// assembled_scratch_doubles), the colour passes otherwise.
hipError_t launch_step_assembled(const fe_mesh *m, const StepArgs &a, double *Zc, hipStream_t s) {
    if (a.N != 1 || m->p > 5 || !Zc) return launch_step(m, a, FE_F64, s);
    StepParams prm;
    prm.X = a.X; prm.ldx = a.ldx;
    prm.Y = a.Y; prm.ldy = a.ldy;
    prm.Ym1 = a.Ym1; prm.ldm = a.ldm;
    prm.alpha = a.alpha; prm.beta = a.beta; prm.shift = a.shift;
    prm.N = 1;
    prm.nchunk = 1;
    prm.axisD = m->d_axis;
    prm.maxf = m->maxf;
    prm.v = a.v ? a.v : m->d_v;
    prm.A = m->d_Af64;
    prm.S = nullptr;
    prm.zero = m->d_zero;
    for (int d = 0; d < 3; ++d) {
        prm.ax[d].ncell = m->ncell[d];
        prm.ax[d].nfree = (int)m->nf[d];
        prm.ax[d].bc = m->bc[d];
        prm.ax[d].ncol = m->ncol[d];
        prm.col[d] = 0;
        prm.cnt[d] = m->ncell[d];
    }
    prm.nfx = m->nf[0];
    prm.nfy = m->nf[1];
    switch (m->p) {
    case 1: return launch_assembled_p<1>(prm, m, Zc, s);
    case 2: return launch_assembled_p<2>(prm, m, Zc, s);
    case 3: return launch_assembled_p<3>(prm, m, Zc, s);
    case 4: return launch_assembled_p<4>(prm, m, Zc, s);
    default: return launch_assembled_p<5>(prm, m, Zc, s);
    }
}

static hipError_t launch_step_v(const fe_mesh *m, const StepArgs &a, fe_dtype prec, hipStream_t s, int variant);

hipError_t launch_step(const fe_mesh *m, const StepArgs &a, fe_dtype prec, hipStream_t s) {
    return launch_step_v(m, a, prec, s, m->kernel_variant);
}

static hipError_t launch_step_v(const fe_mesh *m, const StepArgs &a, fe_dtype prec, hipStream_t s, int variant) {
    StepParams prm;
    prm.X = a.X; prm.ldx = a.ldx;
    prm.Y = a.Y; prm.ldy = a.ldy;
    prm.Ym1 = a.Ym1; prm.ldm = a.ldm;
    prm.alpha = a.alpha; prm.beta = a.beta; prm.shift = a.shift;
    prm.N = a.N;
    prm.nchunk = (int)((a.N + 15) / 16);
    prm.axisD = m->d_axis;
    prm.maxf = m->maxf;
    prm.v = a.v ? a.v : m->d_v;
    prm.A = prec == FE_F64 ? (const void *)m->d_Af64 : prec == FE_F32 ? (const void *)m->d_Af32 : (const void *)m->d_Abf16;
    prm.S = a.S;
    prm.zero = m->d_zero;
    for (int d = 0; d < 3; ++d) {
        prm.ax[d].ncell = m->ncell[d];
        prm.ax[d].nfree = (int)m->nf[d];
        prm.ax[d].bc = m->bc[d];
        prm.ax[d].ncol = m->ncol[d];
    }
    prm.nfx = m->nf[0];
    prm.nfy = m->nf[1];
    prm.zs = prm.ax[2];
    prm.zl = 1;
    if (a.S) {
        if (prec != FE_F64) return hipErrorInvalidValue;
        // Bloch mode: the table kernel with the k.G product (p = 3, 4) on the
        // whole 32-column groups (16 complex vectors), the rest in the
        // row-owner kernel
        if ((variant == 0 || variant == 10) && a.N >= 32 && dma_applies(m, a, prec)) {
            const int64_t Nf = a.N / 32 * 32;
            prm.N = Nf;
            prm.nchunk = (int)(Nf / 16);
            const hipError_t e = m->p == 3 ? launch_tab<3, 0, true>(prm, m, s) : launch_tab<4, 0, true>(prm, m, s);
            if (e != hipSuccess || Nf == a.N) return e;
            StepArgs rest = a;
            rest.X += Nf;
            rest.Y += Nf;
            if (rest.Ym1) rest.Ym1 += Nf;
            rest.N = a.N - Nf;
            return launch_step_v(m, rest, prec, s, 6);
        }
        // the FP64 row-owner kernel in the configurations of the real mode,
        // with one wave less per SIMD for the second fragment stream
        switch (m->p) {
        case 1: return launch_row_p<1, 0, 2, 1, 4, 4, true>(prm, m, s);
        case 2: return launch_row_p<2, 0, 2, 1, 4, 4, true>(prm, m, s);
        case 3: return launch_row_p<3, 0, 2, 1, 4, 4, true>(prm, m, s);
        case 4: return launch_row_p<4, 0, 2, 1, 4, 4, true>(prm, m, s);
        case 5: return launch_row_p<5, 0, 2, 1, 4, 4, true>(prm, m, s);
        case 6: return launch_row_p<6, 0, 1, 2, 4, 2, true>(prm, m, s);
        case 7: return launch_row_p<7, 0, 1, 2, 4, 2, true>(prm, m, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (variant == 0 && prec == FE_F64 && prm.N == 1 && m->p <= 5) {
        switch (m->p) {
        case 1: return launch_cells_p<1>(prm, m, s);
        case 2: return launch_cells_p<2>(prm, m, s);
        case 3: return launch_cells_p<3>(prm, m, s);
        case 4: return launch_cells_p<4>(prm, m, s);
        case 5: return launch_cells_p<5>(prm, m, s);
        default: break;
        }
    }
    // variant 10: the table kernel with direct-to-LDS prefetch (bricks) on
    // the whole 32-vector groups, FP64 (p = 3, 4) or FP32 (p = 3, 4, 5) cell
    // products; the columns past the last whole group (fewer than 32) go to
    // the z-segment pipelined kernel (the default wherever it applies, where
    // it was measured fastest: FP64 4.48 against 5.75, FP32 3.26 against
    // 4.17 ms per H~X for the z-segment kernel on the 24x24x48-cell p = 4
    // slab, 256 vectors)
    const bool tab = variant == 10 || (variant == 0 && (prec == FE_F64 || prec == FE_F32));
    if (tab && a.N >= 32 && dma_applies(m, a, prec)) {
        const int64_t Nf = a.N / 32 * 32;
        prm.N = Nf;
        prm.nchunk = (int)(Nf / 16);
        hipError_t e = hipErrorInvalidValue;
        if (prec == FE_F64) e = m->p == 3 ? launch_tab<3, 0>(prm, m, s) : launch_tab<4, 0>(prm, m, s);
        else e = m->p == 3 ? launch_tab<3, 1>(prm, m, s) : m->p == 4 ? launch_tab<4, 1>(prm, m, s) : launch_tab<5, 1>(prm, m, s);
        if (e != hipSuccess || Nf == a.N) return e;
        StepArgs rest = a;
        rest.X += Nf;
        rest.Y += Nf;
        if (rest.Ym1) rest.Ym1 += Nf;
        rest.N = a.N - Nf;
        return launch_step_v(m, rest, prec, s, 9);
    }
    // the pipelined kernel walking z segments is the default at p = 4 for all
    // three product precisions, where it was measured fastest (FP64 5.7-6.0
    // against 5.9-6.1 for the one-cell pipelined kernel, FP32 4.24 against
    // 5.8, BF16 3.84 against 5.0 for the multi-chunk kernel, ms per H~X on
    // the 24x24x48-cell slab, 256 vectors)
    const bool zseg = variant == 9 || (variant == 0 && m->p == 4);
    if (variant == 7 && prec != FE_BF16) {
#define FE_PIPE(PP)                                                                       \
    case PP:                                                                              \
        return prec == FE_F64 ? launch_pipe_p<PP, 0, 2, false>(prm, m, s) : launch_pipe_p<PP, 1, 2, false>(prm, m, s);
        switch (m->p) {
            FE_PIPE(1)
            FE_PIPE(2)
            FE_PIPE(3)
            FE_PIPE(4)
        default: break;
        }
#undef FE_PIPE
    }
    // variant 9: the pipelined kernel walking z segments of cells, the shared
    // faces inside a segment kept in LDS
    if (zseg) {
#define FE_ZSEG(PP)                                                                       \
    case PP:                                                                              \
        if (prec == FE_F64) return launch_pipe_p<PP, 0, 2, true>(prm, m, s);              \
        if (prec == FE_F32) return launch_pipe_p<PP, 1, 2, true>(prm, m, s);              \
        return launch_pipe_p<PP, 2, 2, true>(prm, m, s);
        switch (m->p) {
            FE_ZSEG(1)
            FE_ZSEG(2)
            FE_ZSEG(3)
            FE_ZSEG(4)
        default: break;
        }
#undef FE_ZSEG
    }
    if ((variant == 0 && prec == FE_F64) || variant == 6 ||
        ((variant == 7 || variant == 9) && prec == FE_F64)) {
        // 32 vectors per workgroup and one row tile per wave measured best
        // where the tiles fit one workgroup (p <= 5); above that two tiles
        // per wave keep the workgroup within 1024 threads (p = 6: 32 vectors
        // per workgroup, three waves per SIMD, 5.78 ms per H~X on the
        // 16x16x32-cell slab against 6.32 for 16 vectors; fragment batches of
        // 4 k-steps, 168 VGPRs with 4 spilled, 5.42 ms against 5.75 for 2
        // with 158 and none on one box; at p = 7, 4 k-steps were slower:
        // 5.28 against 4.82 ms on a 12x12x24-cell slab)
        // BK / BKL: fragment batch (k-steps) for FP64 / for FP32 and BF16
#define FE_ROW(PP, G, TPW, OCC, BK, BKL)                                                     \
    case PP:                                                                                 \
        if (prec == FE_F64) return launch_row_p<PP, 0, G, TPW, OCC, BK>(prm, m, s);          \
        if (prec == FE_F32) return launch_row_p<PP, 1, G, TPW, OCC, BKL>(prm, m, s);         \
        return launch_row_p<PP, 2, G, TPW, OCC, BKL>(prm, m, s);
        switch (m->p) {
            FE_ROW(1, 2, 1, 5, 4, 4)
            FE_ROW(2, 2, 1, 5, 4, 4)
            FE_ROW(3, 2, 1, 5, 4, 4)
            FE_ROW(4, 2, 1, 5, 4, 4)
            FE_ROW(5, 2, 1, 5, 4, 4)
            FE_ROW(6, 2, 2, 3, 4, 2)
            FE_ROW(7, 1, 2, 5, 2, 2)
        default: break;
        }
#undef FE_ROW
    }
    // variant 3/4: one cell x 2/4 chunks per workgroup; variant 0 picks the
    // multi-chunk kernel with the chunk count measured best for the precision
    // (bf16 with p >= 6 is fastest with one chunk per workgroup)
    if ((variant == 0 && !(prec == FE_BF16 && m->p >= 6)) || variant == 3 ||
        variant == 4 || variant == 7 || variant == 9) {
        const int G = variant == 4 ? 4 : variant == 3 ? 2 : (prec == FE_BF16 ? 4 : 2);
#define FE_MC(PP)                                                                                   \
    case PP:                                                                                        \
        if (prec == FE_F64) return G == 4 ? launch_mc_p<PP, 0, 4>(prm, m, s) : launch_mc_p<PP, 0, 2>(prm, m, s); \
        if (prec == FE_F32) return G == 4 ? launch_mc_p<PP, 1, 4>(prm, m, s) : launch_mc_p<PP, 1, 2>(prm, m, s); \
        return G == 4 ? launch_mc_p<PP, 2, 4>(prm, m, s) : launch_mc_p<PP, 2, 2>(prm, m, s);
        switch (m->p) {
            FE_MC(1)
            FE_MC(2)
            FE_MC(3)
            FE_MC(4)
            FE_MC(5)
            FE_MC(6)
            FE_MC(7)
        default: break;
        }
#undef FE_MC
    }
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

// g_I += scale * sum_j U[I,j] V[I,j]; 16 lanes per row, fixed reduction order.
// V2 (N even, U and V 16-byte aligned, even leading dimensions): lane l takes
// the column pairs 2l + 32i, 2l + 1 + 32i with one 16-byte request per block,
// even and odd columns summed apart and then added.
template <bool V2>
__global__ void rowdot_kernel(const double *U, int64_t ldu, const double *V, int64_t ldv, int64_t N, int64_t n,
                              double scale, double *g) {
    int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
    int lane = threadIdx.x & 15;
    if (I >= n) return;
    double s = 0.0;
    if constexpr (V2) {
        double s1 = 0.0;
        for (int64_t j = 2 * lane; j < N; j += 32) {
            const double2 u = *reinterpret_cast<const double2 *>(U + I * ldu + j);
            const double2 v = *reinterpret_cast<const double2 *>(V + I * ldv + j);
            s += u.x * v.x;
            s1 += u.y * v.y;
        }
        s += s1;
    } else {
        for (int64_t j = lane; j < N; j += 16) s += U[I * ldu + j] * V[I * ldv + j];
    }
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
    if (lane == 0) g[I] += scale * s;
}

hipError_t launch_rowdot_accum(const fe_mesh *m, const double *U, int64_t ldu, const double *V, int64_t ldv,
                               int64_t N, double scale, double *g, hipStream_t s) {
    int64_t threads = m->n * 16;
    const bool v2 = N % 2 == 0 && ldu % 2 == 0 && ldv % 2 == 0 && (reinterpret_cast<uintptr_t>(U) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(V) & 15) == 0;
    if (v2)
        hipLaunchKernelGGL(rowdot_kernel<true>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, U, ldu, V,
                           ldv, N, m->n, scale, g);
    else
        hipLaunchKernelGGL(rowdot_kernel<false>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, U, ldu, V,
                           ldv, N, m->n, scale, g);
    return hipGetLastError();
}

// p[0..n) = v (a kernel rather than a memset, so the call is safe inside a
// captured graph).
__global__ void fill_kernel(double *p, int64_t n, double v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// S[i] = sum_b P[b * len + i] for i < len, b in order (deterministic reduction
// of split-K partial products).
__global__ void sum_partials_kernel(const double *P, int64_t nb, int64_t len, double *S) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int64_t b = 0; b < nb; ++b) s += P[b * len + i];
    S[i] = s;
}

hipError_t launch_sum_partials(const double *P, int64_t nb, int64_t len, double *S, hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, P, nb, len, S);
    return hipGetLastError();
}

// Zero the strictly lower triangle of a column-major N x N matrix.
__global__ void zero_lower_kernel(double *A, int N) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    int col = (int)(e / N), row = (int)(e % N);
    if (row > col) A[e] = 0.0;
}

// complex N x N column-major matrix stored as (re, im) pairs
__global__ void zero_lower_z_kernel(double *A, int N) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    int col = (int)(e / N), row = (int)(e % N);
    if (row > col) {
        A[2 * e] = 0.0;
        A[2 * e + 1] = 0.0;
    }
}

hipError_t launch_zero_lower_z(double *A, int N, hipStream_t s) {
    int64_t tot = (int64_t)N * N;
    hipLaunchKernelGGL(zero_lower_z_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, A, N);
    return hipGetLastError();
}

hipError_t launch_zero_lower(double *A, int N, hipStream_t s) {
    int64_t tot = (int64_t)N * N;
    hipLaunchKernelGGL(zero_lower_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, A, N);
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
