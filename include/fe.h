/*
 * fe.h -- C ABI of the MI355X (gfx950) finite-element Hamiltonian filter.
 *
 * The library applies the GLL spectral-element Kohn-Sham Hamiltonian of a
 * slab under a constant external field, in the symmetric standard form
 *
 *     H~ = M^-1/2 ( 1/2 K + V ) M^-1/2  (+ C~ diag(D) C~^T, optional),
 *
 * to blocks of wavefunction coefficients, and runs the Chebyshev filter
 * Y = T_m((H~ - c)/e) X built on it.  K is the FE stiffness
 * K_IJ = int grad N_I . grad N_J and M the GLL-lumped overlap of the
 * C0 Lagrange basis on GLL nodes (paper Sec. 2.3); V is the effective
 * potential V_eff + V_app at the cell GLL points, with V_app the linear
 * field term of slope -E (Sec. 2.1, Eq. for H_loc and V_eff; Sec. 2.2.1);
 * the optional term is the separable nonlocal pseudopotential (Sec. 2.1,
 * Eq. V_nloc).  The filter is the kernel of Chebyshev-filtered subspace
 * iteration for the discrete eigenproblem H u = eps M u (Sec. 2.3).
 *
 * Conventions (all entry points):
 *   - Every function returns fe_status; FE_OK is 0.  On failure nothing has
 *     been enqueued and fe_last_error() returns a message (thread-local).
 *   - The library never aborts, prints or exits.
 *   - Array arguments are DEVICE pointers owned by the caller unless a
 *     parameter says "host".  The library owns only what fe_mesh_create and
 *     fe_set_* allocate (cell matrices, scales, potential, projectors,
 *     scratch), released by fe_mesh_destroy.
 *   - Work is enqueued on the caller's stream; calls return without a device
 *     synchronisation unless the description says otherwise.
 *   - A mesh is not thread-safe; distinct meshes are independent.
 *   - Hartree atomic units (bohr, Ha).
 *   - Wavefunction blocks are FP64, (n x N) row-major with leading dimension
 *     ld >= N: the N values of one degree of freedom are contiguous.  Free
 *     DoFs are numbered x fastest, z slowest, after periodic identification
 *     and removal of homogeneous-Dirichlet nodes.
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FE_OK = 0,
    FE_EINVAL = 1,  /* bad argument (range, null, alignment, overlap)      */
    FE_ENOMEM = 2,  /* device allocation failed or workspace too small     */
    FE_EDEVICE = 3, /* a HIP call failed                                    */
    FE_ESTATE = 4,  /* call out of order (e.g. no potential set yet)       */
    FE_ENOTSUP = 5  /* valid request the library does not implement        */
} fe_status;

typedef enum { FE_BC_DIRICHLET = 0, FE_BC_PERIODIC = 1, FE_BC_NEUMANN = 2 } fe_bc;

/* Integration of the stiffness: EXACT integrates int grad N_I . grad N_J
 * exactly (the paper's definition, Sec. 2.3); GLL uses the collocated GLL
 * rule (the classic spectral-element stiffness). */
typedef enum { FE_RULE_EXACT = 0, FE_RULE_GLL = 1 } fe_rule;

/* Precision of the cell products only; the recurrence, the nodal sums and
 * all inputs/outputs stay FP64.  F32: operands rounded to FP32 (RNE), FP32
 * accumulation.  BF16: operands rounded FP64->FP32->BF16 (RNE each), FP32
 * accumulation. */
typedef enum { FE_F64 = 0, FE_F32 = 1, FE_BF16 = 2 } fe_dtype;

typedef struct {
    double L[3];       /* box edge lengths; cells must be cubes L[a]/ncell[a] = h */
    int32_t ncell[3];  /* cells per axis, >= 1 (>= 2 on a periodic axis)          */
    int32_t p;         /* GLL degree, 1..7                                         */
    int32_t bc[3];     /* fe_bc per axis                                           */
    int32_t k_rule;    /* fe_rule                                                  */
} fe_mesh_desc;

typedef struct fe_mesh fe_mesh;

/* Message describing the last failure on this thread ("" if none). */
const char *fe_last_error(void);

/* Build the mesh, reference element and cell matrices (Sec. 2.3) on the
 * current HIP device and upload them.  Errors: FE_EINVAL for p outside 1..7,
 * ncell < 1 (or < 2 on a periodic axis), L <= 0, non-cubic cells, unknown bc
 * or rule; FE_ENOMEM / FE_EDEVICE from the device.  *out is owned by the
 * caller and released with fe_mesh_destroy. Synchronous. */
fe_status fe_mesh_create(const fe_mesh_desc *desc, fe_mesh **out);

/* Release everything the mesh owns (synchronises the device first).
 * NULL is accepted. */
fe_status fe_mesh_destroy(fe_mesh *mesh);

/* Select the implementation of the step kernel: 0 = the fastest measured
 * for the degree and precision (default); 1 = one cell x 16 vectors per
 * workgroup, cell matrix streamed from L2 (the plain reference form);
 * 3 / 4 = one cell x 32 / 64 vectors per workgroup, so each cell-matrix
 * fragment read from L2 feeds 2 / 4 products (falls back to 1 when the block
 * would exceed the LDS); 6 = row-owner kernel (each thread loads
 * everything its outputs need in one round trip before the cell product;
 * the FP64 default for p = 1, 2 and p >= 5); 7 = persistent pipelined
 * row-owner kernel with the cell matrix in registers and the loads of the
 * next two items in flight during each cell product (FP64 and FP32, p <= 4;
 * else 6; BF16: 3); 9 = the pipelined kernel of 7 walking z segments of up
 * to 6 cells (the largest length that divides the z cell count, at least
 * two segments on a periodic z axis), the faces shared inside a segment
 * kept in LDS instead of being read and written in HBM (FP64, FP32 and BF16
 * products, p <= 4; the BF16 default at p = 4; else as 7);
 * 10 = the table kernel: the walk of 9 with the X rows copied from HBM
 * straight into LDS two positions ahead, each position's cell read from a
 * per-segment table of first DoF and face masks built at mesh creation, and
 * the cell matrix pre-scaled by M^-1/2 (FP64 products at p = 3 and 4, FP32
 * products at p = 3, 4 and 5; no zero-Neumann axis, one leading dimension
 * for X, Y and the previous iterate, 16-byte aligned blocks with an even
 * leading dimension; applied to the whole 32-vector groups of N, the
 * columns past the last whole group run variant 9; the default wherever it
 * applies; else as 0).
 * Variants 0, 1, 3, 4, 6 and 7 give bitwise-identical results (variant 0
 * wherever it is not variant 9 or 10); variants 9 and 10 sum each node's
 * contributions in other fixed orders (equal to rounding, reproducible).
 * In the Bloch mode (the _k entry points at k != 0) variants 0 and 10 run
 * the table kernel with the k.G product at p = 3, 4 on the whole groups of
 * 16 complex vectors, the row-owner kernel elsewhere; the other variants
 * run the row-owner kernel.
 * Variants 2 (register-resident), 5 (tiles of cells) and 8
 * (warp-specialised), slower than the defaults everywhere, were removed:
 * FE_EINVAL for them and for values outside 0..10. */
fe_status fe_mesh_set_kernel(fe_mesh *mesh, int32_t variant);

/* Sizes: free DoFs n, cells, and points per cell n_c = (p+1)^3.  Any output
 * pointer may be NULL.  Host pointers. */
fe_status fe_mesh_info(const fe_mesh *mesh, int64_t *n_dof, int64_t *n_cell, int32_t *n_c);

/* Host copies of geometry: the cell GLL points xyz[(c*n_c + l)*3 + a]
 * (cells lexicographic, x fastest; local index l = i + (p+1)(j + (p+1)k))
 * and the free-DoF coordinates xyz[I*3 + a].  Host pointers, caller-owned,
 * sized n_cell*n_c*3 and n*3 doubles. */
fe_status fe_mesh_quad_points(const fe_mesh *mesh, double *xyz_host);
fe_status fe_mesh_dof_coords(const fe_mesh *mesh, double *xyz_host);

/* Host copy of the reference element of degree p (Sec. 2.3): GLL nodes
 * xi[p+1] and weights w[p+1] on [-1, 1], and the half cell stiffness
 * A = 1/2 Kc ((p+1)^3 x (p+1)^3, row-major, local index i + (p+1)(j + (p+1)k))
 * of a cube of edge h under the given rule.  Pure host computation; any
 * output may be NULL.  FE_EINVAL for p outside 1..7, h <= 0 or an unknown
 * rule. */
fe_status fe_reference_cell(int32_t p, int32_t k_rule, double h, double *xi_host, double *w_host, double *A_host);

/* Set the potential (Sec. 2.1 V_eff, Sec. 2.2.1 V_app):
 *   v_I = sum_{(c,q) -> I} (|J| w_q / M_I) V_quad[c][q]  -  E (z_I - z0),
 * the diagonal of H~ from GLL-collocated quadrature of V at the cell GLL
 * points.  V_quad: device, [n_cell][n_c] as in fe_mesh_quad_points; values at
 * Dirichlet points are ignored.  May be NULL (V_loc = 0).  Enqueued on stream;
 * V_quad must stay valid until the stream reaches this call. */
fe_status fe_set_potential(fe_mesh *mesh, const double *V_quad, double E, double z0, hipStream_t stream);

/* Separable nonlocal term (Sec. 2.1, Eq. V_nloc, and Eq. for H_nloc): per site
 * s, nine projectors p_beta = S_beta(x - R_s) exp(-|x-R_s|^2/(2 r_g^2)) for
 * |x - R_s| < r_cut (S: 1; x, y, z; xy, yz, zx, x^2-y^2, 3z^2-r^2), minimum
 * image on periodic axes, each normalised to sum_I M_I p(x_I)^2 = 1 and
 * collocated as C~_I = M_I^1/2 p(x_I); H~ gains C~ diag(D) C~^T.
 * centres_host [n_site][3], D_host [n_site][9] (Ha), host pointers.
 * n_site = 0 clears the term.  Synchronous. */
fe_status fe_set_nonlocal(fe_mesh *mesh, int32_t n_site, const double *centres_host, const double *D_host,
                          double r_cut, double r_g, hipStream_t stream);

/* Y = H~ X.  X, Y: device FP64 (n x N), leading dimension ld >= N, must not
 * overlap.  prec selects the cell-product precision.  FE_ESTATE if no
 * potential has been set; FE_EINVAL for N < 1, ld < N, NULL or overlapping
 * blocks, or misalignment (8 bytes).  N = 0 is a no-op. */
fe_status fe_hx_apply(fe_mesh *mesh, const double *X, double *Y, int64_t N, int64_t ld, fe_dtype prec,
                      hipStream_t stream);

/* Y = H~ X exactly as fe_hx_apply (same kernels, same results bit for bit),
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The only
 * scratch of H~X, the nonlocal projections W = diag(D) C~^T X (9 * n_site * N
 * doubles, needed when fe_set_nonlocal has set sites), lives in a static
 * device array of 4,194,304 doubles (32 MiB) per device, instead of the
 * mesh's buffer that fe_hx_apply grows with hipMalloc / hipFree (hipFree
 * synchronises the device).  This call allocates and frees nothing.  Every
 * call on one device shares that array: calls that overlap on a device (on
 * concurrent streams or threads) race and must be serialised by the caller.
 * Errors as for fe_hx_apply, plus FE_ENOMEM (nothing enqueued) when
 * 9 * n_site * N exceeds 4,194,304, and FE_EDEVICE if the array's device
 * address could not be resolved when the mesh was created. */
fe_status fe_hx_apply_noalloc(fe_mesh *mesh, const double *X, double *Y, int64_t N, int64_t ld, fe_dtype prec,
                              hipStream_t stream);

/* Chebyshev filter of degree m on the unwanted interval [a, b]
 * (e = (b-a)/2, c = (b+a)/2), by the three-term recurrence
 *   Y_1 = alpha_0 (H~ - c) X,   Y_{k+1} = alpha_k (H~ - c) Y_k - beta_k Y_{k-1}.
 * Scaled (a0 finite, a0 < a): sigma_1 = e/(a0-c), sigma_{k+1} = 1/(2/sigma_1 -
 * sigma_k), alpha_0 = sigma_1/e, alpha_k = 2 sigma_{k+1}/e, beta_k =
 * sigma_k sigma_{k+1}, giving Y = T_m((H~-c)/e) X / T_m((a0-c)/e).
 * Unscaled (a0 NaN): alpha_0 = 1/e, alpha_k = 2/e, beta_k = 1.
 * X is read-only; Y receives the result; work is caller-owned device scratch
 * of at least n*N doubles (work_bytes) holding one recurrence block.  X, Y and
 * work must not overlap.  Requires a < b and m >= 1 (FE_EINVAL); FE_ENOMEM
 * if work_bytes is too small. */
fe_status fe_cheb_filter(fe_mesh *mesh, const double *X, double *Y, int64_t N, int64_t ld, int32_t m, double a,
                         double b, double a0, fe_dtype prec, double *work, size_t work_bytes, hipStream_t stream);

/* Bytes of `work` fe_cheb_filter_vjp needs for these arguments (host call). */
size_t fe_cheb_filter_vjp_work_bytes(const fe_mesh *mesh, int64_t N, int32_t m, int32_t ckpt_stride,
                                     int32_t col_chunk);

/* Reverse-mode derivative of fe_cheb_filter with respect to X and to the
 * potential, for a cotangent G = dL/dY (bounds a, b, a0 held fixed):
 *   Xbar = dL/dX  (n x N, ld),
 *   Vbar_quad[c][q] = dL/dV_quad[c][q] = (|J| w_q / M_I) g_I,
 *   *Ebar = dL/dE = -sum_I g_I (z_I - z0)  (device scalar),
 * with g_I = sum_k alpha_k sum_j Ybar_{k+1}[I,j] Y_k[I,j] from the reverse
 * three-term sweep (H~ symmetric, so the same operator is applied).
 * Forward blocks are kept every ckpt_stride steps and recomputed in between
 * (ckpt_stride = 1 stores all); columns are processed in chunks of col_chunk
 * (0 = all N at once).  The nonlocal couplings are held fixed.  work and
 * work_bytes as returned by fe_cheb_filter_vjp_work_bytes (FE_ENOMEM if
 * smaller).  Vbar_quad and Ebar are overwritten. */
fe_status fe_cheb_filter_vjp(fe_mesh *mesh, const double *X, const double *G, int64_t N, int64_t ld, int32_t m,
                             double a, double b, double a0, fe_dtype prec, double *Xbar, double *Vbar_quad,
                             double *Ebar, int32_t ckpt_stride, int32_t col_chunk, double *work,
                             size_t work_bytes, hipStream_t stream);

/* Spectrum bounds by k-step Lanczos on H~ with full reorthogonalisation
 * from the device start vector v0 (n doubles): *a0 = smallest Ritz value,
 * *b = largest Ritz value + |beta_k| (an upper bound of the spectrum).
 * Host outputs; synchronises the stream.  k in 1..64. */
fe_status fe_lanczos_bounds(fe_mesh *mesh, const double *v0, int32_t k, double *a0_host, double *b_host,
                            hipStream_t stream);

/* Two passes of Cholesky-QR on a device block Y (n x N, ld): Y <- Q with
 * Q^T Q = I (FP64 throughout).  FE_EDEVICE if the Gram matrix is not
 * numerically positive definite.  Synchronises the stream. */
fe_status fe_cholqr2(fe_mesh *mesh, double *Y, int64_t N, int64_t ld, hipStream_t stream);

/* Rayleigh-Ritz on an orthonormal block Q (n x N, ld): Hs = Q^T H~ Q
 * (symmetrised, FP64 products), Hs = W diag(theta) W^T, X <- Q W.
 * theta_host receives the N Ritz values ascending; P is caller scratch of n x N
 * doubles (ld).  Q, X and P must not overlap (FE_EINVAL).  Synchronises the
 * stream. */
fe_status fe_rayleigh_ritz(fe_mesh *mesh, const double *Q, double *X, double *P, int64_t N, int64_t ld,
                           double *theta_host, hipStream_t stream);

/* Electron density at the free nodes (Sec. 2.1, rho = 2 sum_n f_n |psi_n|^2):
 *   rho[I] = 2 sum_n f[n] X[I,n]^2 / M_I,
 * i.e. the density of the orbitals psi_n = M^-1/2 x_n (the vectors this
 * library filters are M^1/2-scaled nodal coefficients) at the GLL nodes,
 * where the lumped-mass orbitals are collocated.  X: device, (n, N)
 * row-major, leading dimension ld >= N; f: device, N occupation weights;
 * rho: device, n doubles, overwritten.  N = 0 writes zeros (X, f may then be
 * NULL).  The sum over n runs in a fixed order (reproducible).  Enqueued on
 * stream.  FE_EINVAL for NULL arguments, N < 0 or ld < N. */
fe_status fe_density(fe_mesh *mesh, const double *X, int64_t N, int64_t ld, const double *f, double *rho,
                     hipStream_t stream);

/* Planar integral (normalize = 0) or planar average (normalize = 1) of a
 * nodal field over the x-y plane through each row of free z nodes
 * (Sec. 3.2, rho^0(z) and V^0_bare(z)):
 *   out[k] = s * sum_{i,j} m_x(i) m_y(j) field[i + n_x (j + n_y k)],
 * with m_a the assembled 1-D GLL lumped masses of the free positions,
 * s = 1 or 1 / (sum_i m_x(i) sum_j m_y(j)) (the plane area when x and y are
 * periodic).  field: device, n doubles in DoF order; out: device, n_z
 * doubles (one per free z position, ascending z).  Fixed reduction order.
 * Enqueued on stream.  FE_EINVAL for NULL arguments or normalize not 0/1. */
fe_status fe_planar_average(fe_mesh *mesh, const double *field, int32_t normalize, double *out,
                            hipStream_t stream);

/* Planar average of the bare potential (Sec. 3.2): V_bare = phi~ + V_app
 * with phi~ = phi + (V_loc - V_self) the total electrostatic potential, so
 *   out[k] = (1 / A) sum over the free nodes of z plane k of
 *            m_x m_y ((phi + w) + vapp),
 * with w = V_loc - V_self at the nodes and vapp the applied potential at the
 * nodes (the sawtooth of the constant-field setup; zero in the
 * constrained-potential setup, where the bias sits in phi), A the plane
 * area; the quadrature and fixed reduction order of fe_planar_average.
 * phi: device, n doubles; w, vapp: device, n doubles or NULL (0); out:
 * device, n_z doubles (ascending z).  Enqueued on stream.  FE_EINVAL for a
 * NULL mesh, phi or out. */
fe_status fe_bare_potential_planar(fe_mesh *mesh, const double *phi, const double *w, const double *vapp,
                                   double *out, hipStream_t stream);

/* Electronic dipole about z0 (Sec. 3.1, mu_z = int rho (z - z0) for the
 * electron density; the nuclear part is the caller's):
 *   *mu_host = sum_I M_I rho[I] (z_I - z0),
 * the GLL quadrature of the nodal density, computed as the z moment of the
 * planar integrals (fe_planar_average) in a fixed order.  By the
 * Hellmann-Feynman relation for v containing -E (z - z0), the band-energy
 * derivative 2 sum f_n d eps_n / dE at eigenvectors equals -mu.  rho: device,
 * n doubles.  Synchronous with stream (uses the mesh's scratch).  FE_EINVAL
 * for NULL arguments or non-finite z0. */
fe_status fe_dipole(fe_mesh *mesh, const double *rho, double z0, double *mu_host, hipStream_t stream);

/* Electrostatic potential on the mesh's finite-element space (Sec. 2.2, the
 * Poisson problem -lap(phi) / 4 pi = rho + b): solves K phi = 4 pi M s for
 * the nodal charge density s, by Jacobi-preconditioned conjugate gradients
 * on M^-1/2 (1/2 K) M^-1/2 (the step kernel with a zero diagonal term; any
 * potential set on the mesh is ignored).  Boundary conditions are the
 * mesh's: phi = 0 on Dirichlet faces; with no Dirichlet axis (periodic x-y
 * and zero-Neumann z, Sec. 2.2.1) the constant null space is projected out
 * and phi has zero mean (the charge's mean is removed, i.e. a neutral slab
 * is assumed).  The constrained-potential setup of Sec. 2.2.2 is
 * fe_poisson_solve_cpd below.  charge, phi: device, n doubles;
 * work: device, >= fe_poisson_work_bytes(mesh) bytes.  Stops when
 * |r| / |b| <= tol or after maxit iterations (r, b: residual and right-hand
 * side of the scaled system in x = M^1/2 phi); *iters_host and *relres_host
 * (may be NULL) receive the iteration count and the final |r| / |b|.  The
 * iteration runs on the device (fixed-order reductions, so results are
 * reproducible); the host reads its state once per 8 iterations and returns
 * after the stream has drained.  Full batches of 8 after the first are
 * replayed from a HIP graph (captured once per call on a private stream,
 * kernel nodes only; direct launches if the capture fails), so the stream
 * may be the null stream.  FE_EINVAL for NULL arguments, tol <= 0 or
 * maxit < 1; FE_ENOMEM if work is too small; FE_EDEVICE for a failed
 * launch. */
size_t fe_poisson_work_bytes(const fe_mesh *mesh);
fe_status fe_poisson_solve(fe_mesh *mesh, const double *charge, double *phi, double tol, int32_t maxit,
                           double *work, size_t work_bytes, int32_t *iters_host, double *relres_host,
                           hipStream_t stream);

/* Electrostatics of the constrained-potential-difference setup (Sec. 2.2.2,
 * its governing equations): K phi = 4 pi M s at the nodes between the two
 * metal conductors, and phi prescribed inside them,
 *   phi = -w       on Omega_0 = {z <= z_lo},
 *   phi = dV - w   on Omega_1 = {z >= z_hi},
 * where w = V_loc - V_sm at the nodes (NULL: 0), so that the total
 * electrostatic potential phi + w is 0 in one conductor and dV in the other
 * (no field inside them).  x and y keep the mesh's boundary conditions
 * (periodic for the paper's slabs); the z faces lie inside the conductors.
 * The same device CG as fe_poisson_solve runs on the free nodes: the
 * constrained values start at their data, enter the right-hand side through
 * one product, and carry a zero preconditioner entry, so search directions
 * never touch them; on return phi holds the data there exactly.  The
 * relative residual is measured against the reduced right-hand side
 * (2 pi M^1/2 s - H0 M^1/2 g on the free nodes).  charge, w, phi: device,
 * n doubles (phi may not alias charge or w); work, tol, maxit, iters_host,
 * relres_host, stream as for fe_poisson_solve.  FE_EINVAL for NULL mesh,
 * charge, phi or work, non-finite z_lo / z_hi / dV, z_lo >= z_hi, a
 * periodic z axis, or when no node (or every node) lies in a conductor;
 * FE_ENOMEM if work is too small; FE_EDEVICE for a failed launch. */
fe_status fe_poisson_solve_cpd(fe_mesh *mesh, const double *charge, const double *w, double z_lo, double z_hi,
                               double dV, double *phi, double tol, int32_t maxit, double *work, size_t work_bytes,
                               int32_t *iters_host, double *relres_host, hipStream_t stream);

/* ---------------------------------------------------------------- Bloch-k
 * Bloch form of the Hamiltonian over the periodic x-y directions (Sec. 2.1,
 * governing equations for u_nk = exp(-i k.x) psi_nk): H~^k = H~ + |k|^2/2
 * - i M^-1/2 (k_x G_x + k_y G_y) M^-1/2, G_a the assembled matrices
 * int N_I dN_J/dx_a (antisymmetric on periodic axes, so H~^k is Hermitian),
 * and the projectors of fe_set_nonlocal twisted to
 * C^k_I = exp(-i k.(x_I - R_s)) C~_I (minimum-image displacement), so the
 * nonlocal term becomes C^k diag(D) C^k^H.  Products in FP64 only.
 *
 * Complex blocks: device, n x N complex FP64 stored row-major as interleaved
 * (re, im) pairs (the layout of C99 double _Complex / std::complex<double>),
 * leading dimension ld >= N in complex elements, 8-byte aligned. */

/* Set the wave vector (k_x, k_y) (bohr^-1) used by the _k entry points;
 * (0, 0) is the Gamma point, where they equal the real entry points applied
 * to the real and imaginary parts (bitwise).  FE_EINVAL for a non-finite k
 * or a nonzero component along a non-periodic axis.  Waits for the device,
 * then builds the k.G cell fragments and projector phases (synchronous). */
fe_status fe_set_kpoint(fe_mesh *mesh, double kx, double ky);

/* The current wave vector, k_host[2] (host pointer). */
fe_status fe_get_kpoint(const fe_mesh *mesh, double *k_host);

/* Y = H~^k X on complex blocks.  X, Y must not overlap.  Errors as for
 * fe_hx_apply (FE_ESTATE without a potential).  N = 0 is a no-op. */
fe_status fe_hx_apply_k(fe_mesh *mesh, const double *X, double *Y, int64_t N, int64_t ld, hipStream_t stream);

/* Chebyshev filter of fe_cheb_filter (same coefficients, same recurrence)
 * with H~^k on complex blocks.  work: device scratch of at least 2*n*N
 * doubles (one complex recurrence block, leading dimension N); X, Y and work
 * must not overlap. */
fe_status fe_cheb_filter_k(fe_mesh *mesh, const double *X, double *Y, int64_t N, int64_t ld, int32_t m, double a,
                           double b, double a0, double *work, size_t work_bytes, hipStream_t stream);

/* Two passes of Cholesky-QR on a complex block: Y <- Y R^-1 with
 * Y^H Y = R^H R, so that the columns become orthonormal in the complex inner
 * product (the dense step of subspace iteration at a k-point; the real
 * fe_cholqr2 for Bloch vectors).  Y: device complex n x N, ld >= N (complex
 * elements), overwritten.  FE_EDEVICE if the Gram matrix is not positive
 * definite; synchronous with stream. */
fe_status fe_cholqr2_k(fe_mesh *mesh, double *Y, int64_t N, int64_t ld, hipStream_t stream);

/* Rayleigh-Ritz with H~^k on span(Q) (Q complex n x N with orthonormal
 * columns): P = H~^k Q, the Hermitian projection (Q^H P + P^H Q) / 2 =
 * W diag(theta) W^H, X = Q W.  Q, X, P: device complex n x N with leading
 * dimension ld (X and P caller-owned outputs, P scratch); theta_host: N
 * doubles, ascending.  Synchronous with stream.  FE_ESTATE without a
 * potential; FE_EINVAL if Q, X and P overlap. */
fe_status fe_rayleigh_ritz_k(fe_mesh *mesh, const double *Q, double *X, double *P, int64_t N, int64_t ld,
                             double *theta_host, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* FE_H */
