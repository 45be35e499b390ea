// Internal structures of the gfx950 FE Hamiltonian library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fe.h"

namespace fe {

constexpr int kMaxP = 7;
constexpr int kVec = 16;  // vectors per MFMA column tile (one workgroup chunk)

// Cell products are padded to a multiple of 32 rows/columns so that every
// MFMA shape used (f64 16x16x4, f32 16x16x4, bf16 16x16x32) tiles them.
inline int padded_nc(int p) {
    int nc = (p + 1) * (p + 1) * (p + 1);
    return (nc + 31) / 32 * 32;
}

// Per-axis description passed by value to kernels.
struct AxisInfo {
    int ncell;   // cells along the axis
    int nfree;   // free node positions
    int bc;      // fe_bc
    int ncol;    // colours along the axis (1, 2 or 3)
};

struct NonlocalData {
    int n_site = 0;
    int64_t nnz = 0;                 // support entries over all sites
    int64_t n_node = 0;              // DoFs inside at least one support
    int64_t *d_supp_ptr = nullptr;   // [n_site + 1]
    int32_t *d_supp_dof = nullptr;   // [nnz] DoF of each support entry
    double *d_vals = nullptr;        // [nnz][9] C~ values per projector
    double *d_D = nullptr;           // [n_site][9] couplings
    double *d_W = nullptr;           // projections C~^T X, grown on demand
    size_t W_cap = 0;                // doubles
    std::vector<double> disp;        // [nnz][2] in-plane x_I - R_s of each entry (minimum image)
    // chunks of at most kNlChunk support entries of one site, grouped by
    // site colour (sites of one colour have disjoint supports): colour c holds
    // chunks chunk_col_ptr[c] .. chunk_col_ptr[c + 1], chunk q being entries
    // d_chunk_e0[q] .. min(d_chunk_e0[q] + kNlChunk, end of site d_chunk_site[q])
    int32_t *d_chunk_site = nullptr;
    int64_t *d_chunk_e0 = nullptr;
    std::vector<int64_t> chunk_col_ptr;
    double *d_phase = nullptr;       // [nnz][2] cos, sin of k.(x_I - R_s) (Bloch mode)
};

}  // namespace fe

struct fe_mesh {
    int device = 0;
    double L[3];
    double h;
    int ncell[3];
    int p, n1, nc, ncp;
    int bc[3];
    int rule;
    int64_t nf[3];
    int64_t n;      // free DoFs
    int64_t ncells;
    int ncol[3];

    // host copies
    std::vector<double> xi, w;          // GLL nodes/weights on [-1,1]
    std::vector<double> cellA;          // 1/2 Kc, nc x nc, row-major
    std::vector<double> axis_coord[3];  // coordinate of each free node position
    std::vector<double> axis_mass[3];   // assembled 1-D lumped mass per free position

    // device
    // [9][maxf]: per axis a, rows a / 3 + a / 6 + a hold M^-1/2, M^-1 and M of
    // the assembled 1-D lumped mass at each free position
    double *d_axis = nullptr;
    double *d_zcoord = nullptr;   // [nf_z] z coordinate of free z positions
    int maxf = 0;
    double *d_Af64 = nullptr;     // swizzled A fragments of 1/2 Kc (f64)
    // with no Neumann axis every free node's M^-1/2 is the product of per-axis
    // factors that depend only on its local index in any cell containing it,
    // so D Kc D folds into one cell matrix: swizzled f64 fragments of
    // D^ (1/2 Kc) D^ (null with a Neumann axis), and the same rounded to f32;
    // where the table kernel applies (p = 3, 4, 5) their rows are in the
    // order of d_tabperm (row r: local node d_tabperm[r], -1 a zero row)
    double *d_Af64s = nullptr;
    float *d_Af32s = nullptr;
    int32_t *d_tabperm = nullptr;
    std::vector<int32_t> tab_perm;  // its host copy
    double *d_zero = nullptr;     // 32 zero doubles (source of padded / absent rows)
    // segment table of the table kernel (p = 3, 4, 5 with the folded cell
    // matrix): per colour pass, per z segment, first DoF and face masks
    int32_t *d_segtab = nullptr;
    std::vector<int64_t> seg_off;  // entries of colour pass c: [seg_off[c], seg_off[c+1])
    // the same for bricks one cell deep in y, where seg_by > 1 (else null)
    int32_t *d_segtab1 = nullptr;
    std::vector<int64_t> seg_off1;
    int seg_zl = 1, seg_bx = 1, seg_by = 1;  // cells of a brick along z, x and y
    float *d_Af32 = nullptr;      // f32
    uint16_t *d_Abf16 = nullptr;  // bf16 bits
    double *d_v = nullptr;        // [n] diagonal potential term of H~
    double *d_wrel = nullptr;     // [3][p+1]: (h/2) w_i per axis (for v and Vbar)
    double kvec[2] = {0.0, 0.0};  // Bloch wave vector (k_x, k_y) of the complex entry points
    double *d_Sf64 = nullptr;     // swizzled FP64 fragments of k.G_c (null while k = 0)
    double *d_Sf64s = nullptr;    // the same folded as d_Af64s, for the table kernel (p = 3, 4)
    bool potential_set = false;
    int kernel_variant = 0;  // 0: fastest available, 1: generic colour-pass kernel
    double E = 0.0, z0 = 0.0;

    fe::NonlocalData nl;
    // scratch for Lanczos / dense steps (grown on demand)
    double *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    void *blas = nullptr;  // rocblas_handle
};

namespace fe {

// thread-local error message
void set_error(const std::string &msg);
fe_status fail(fe_status s, const std::string &msg);
// whether two row-major blocks (n x N doubles, leading dimension ld) share a byte
bool overlap(const double *a, int64_t na, int64_t Na, int64_t lda, const double *b, int64_t nb, int64_t Nb,
             int64_t ldb);

// reference element (host, FP64)
void gll_rule(int p, std::vector<double> &x, std::vector<double> &w);
void ref_matrices(int p, int rule, std::vector<double> &Khat, std::vector<double> &Mhat);
void cell_matrix_half(int p, int rule, double h, std::vector<double> &A);
void cell_matrix_bloch(int p, int rule, double h, double kx, double ky, std::vector<double> &S);

// kernels (fe_kernels.hip)
struct StepArgs {
    const double *X;    // Y_k (gathered operand)
    int64_t ldx;
    double *Y;          // Y_{k+1}
    int64_t ldy;
    const double *Ym1;  // Y_{k-1} (may alias Y); null when beta == 0
    int64_t ldm;
    double alpha, beta, shift;
    int64_t N;
    const double *v = nullptr;  // diagonal term of H~; null: the mesh's potential
    const double *S = nullptr;  // Bloch mode: FP64 fragments of k.G_c (interleaved complex columns)
};

hipError_t launch_step(const fe_mesh *m, const StepArgs &a, fe_dtype prec, hipStream_t s);
// single-vector FP64 product in two launches (cell products, then nodal sums)
size_t assembled_scratch_doubles(const fe_mesh *m);
hipError_t launch_step_assembled(const fe_mesh *m, const StepArgs &a, double *Zc, hipStream_t s);
hipError_t launch_potential(const fe_mesh *m, const double *Vq, double E, double z0, hipStream_t s);
hipError_t launch_potential_vjp(const fe_mesh *m, const double *g, double z0, double *Vbar, double *Ebar,
                                hipStream_t s);
hipError_t launch_rowdot_accum(const fe_mesh *m, const double *U, int64_t ldu, const double *V, int64_t ldv,
                               int64_t N, double scale, double *g, hipStream_t s);
fe_status filter_step(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, const double *Ym1,
                      int64_t ldm, double alpha, double beta, double shift, int64_t N, fe_dtype prec, hipStream_t s,
                      double *nlW = nullptr);
void cheb_coefficients(int mdeg, double a, double b, double a0, std::vector<double> &al, std::vector<double> &be,
                       double &c);
fe_status validate_filter_args(fe_mesh *m, int64_t N, int32_t mdeg, double a, double b, double a0, fe_dtype prec);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);
fe_status ensure_scratch_dense(fe_mesh *m, size_t bytes);
fe_status blas_handle(fe_mesh *m, hipStream_t s, void **h);
// Poisson helpers (fe_poisson.hip)
hipError_t launch_mass_sqrt(const fe_mesh *m, double *out, hipStream_t s);
hipError_t launch_vmul(double *z, const double *a, const double *b, int64_t n, hipStream_t s);
hipError_t launch_xpby(double *p, const double *z, double beta, int64_t n, hipStream_t s);
hipError_t launch_sum_partials(const double *P, int64_t nb, int64_t len, double *S, hipStream_t s);
hipError_t launch_zero_lower(double *A, int N, hipStream_t s);
hipError_t launch_zero_lower_z(double *A, int N, hipStream_t s);
// one Bloch-mode recurrence step on complex blocks (leading dimensions in
// complex elements); fe_api.cpp
fe_status filter_step_k(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, const double *Ym1,
                        int64_t ldm, double alpha, double beta, double shift, int64_t N, hipStream_t s);
hipError_t launch_axpby(double *Y, int64_t ldy, const double *X, int64_t ldx, int64_t n, int64_t N, double a,
                        double b, hipStream_t s);
// W: the projection buffer (9 n_site N doubles); null: the mesh's own, grown on demand
hipError_t launch_nonlocal(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t N,
                           double alpha, hipStream_t s, double *W = nullptr);
// device scratch of the allocation-free entry point (fe_nonlocal.hip)
constexpr size_t kStaticScratchDoubles = (size_t)4 << 20;
fe_status static_scratch_init(int device);
double *static_scratch(int device);
size_t nonlocal_work_doubles(const fe_mesh *m, int64_t N);
hipError_t launch_nonlocal_k(fe_mesh *m, const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t N,
                             double alpha, hipStream_t s);
fe_status nonlocal_set_phase(fe_mesh *m);
void swizzle_f64(const fe_mesh *m, const std::vector<double> &A, std::vector<double> &f64);
void fold_swizzle(const fe_mesh *m, const std::vector<double> &A, const std::vector<int32_t> *perm,
                  std::vector<double> &f64);
// segment table, output-row order and row tiles per wave of the table
// kernel (fe_kernels.hip)
void build_segment_table(const fe_mesh *m, int by_most, std::vector<int32_t> &tab, std::vector<int64_t> &off,
                         int &zl, int &bx, int &by);
void build_table_row_perm(int p, int tiles_per_wave, std::vector<int32_t> &perm);
int table_tiles_per_wave(int p);
void nonlocal_release(fe_mesh *m);

}  // namespace fe
