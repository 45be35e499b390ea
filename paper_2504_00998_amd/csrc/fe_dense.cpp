// Dense steps of Chebyshev-filtered subspace iteration on the device, FP64:
// spectrum bounds by Lanczos (Zhou & Li 2011 upper bound), Cholesky-QR in two
// passes, and Rayleigh-Ritz.  Tall-skinny products go through rocBLAS, the
// N x N factorisations through rocSOLVER; the Hamiltonian applications are
// the library's own kernels.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fe_internal.h"

namespace fe {

static fe_status blas_fail(rocblas_status s, const char *what) {
    return fail(FE_EDEVICE, std::string(what) + ": " + rocblas_status_to_string(s));
}

#define FE_BLAS(call, what)                                   \
    do {                                                      \
        rocblas_status _s = (call);                           \
        if (_s != rocblas_status_success) return blas_fail(_s, what); \
    } while (0)

#define FE_HIPD(call, what)                                                                        \
    do {                                                                                           \
        hipError_t _e = (call);                                                                    \
        if (_e != hipSuccess) return fail(FE_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

static fe_status handle(fe_mesh *m, hipStream_t s, rocblas_handle &h) {
    if (!m->blas) {
        rocblas_handle hh;
        FE_BLAS(rocblas_create_handle(&hh), "rocblas_create_handle");
        m->blas = hh;
    }
    h = static_cast<rocblas_handle>(m->blas);
    FE_BLAS(rocblas_set_stream(h, s), "rocblas_set_stream");
    FE_BLAS(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host), "rocblas_set_pointer_mode");
    return FE_OK;
}

fe_status blas_handle(fe_mesh *m, hipStream_t s, void **h) {
    rocblas_handle hh;
    fe_status st = handle(m, s, hh);
    *h = hh;
    return st;
}

// Eigenvalues of a small symmetric matrix (row-major, n x n) by cyclic Jacobi.
static void jacobi_eigvals(std::vector<double> A, int n, std::vector<double> &ev) {
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-300) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    ev.resize(n);
    for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
    std::sort(ev.begin(), ev.end());
}

fe_status ensure_scratch_dense(fe_mesh *m, size_t bytes) {
    if (m->scratch_bytes >= bytes) return FE_OK;
    if (m->d_scratch) {
        FE_HIPD(hipDeviceSynchronize(), "hipDeviceSynchronize");
        FE_HIPD(hipFree(m->d_scratch), "hipFree");
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

// Rows per split-K slice of the tall-skinny products, and rows per block of
// the in-place right multiplication.
constexpr int64_t kSliceRows = 8192;
constexpr int64_t kBlockRows = 65536;

// out (N x N, column-major) = A^T B for row-major (n x N) blocks A, B with
// leading dimension ld, i.e. Acm Bcm^T.  The long dimension n is split into
// slices (strided-batched GEMM) whose partial products are summed in slice
// order, so the result is deterministic.  part: scratch of
// (n / kSliceRows + 1) * N * N doubles.
static fe_status tsgram(rocblas_handle h, const double *A, const double *B, int64_t n, int64_t N, int64_t ld,
                        double *part, double *out, hipStream_t s) {
    int64_t nfull = n / kSliceRows, rem = n - nfull * kSliceRows;
    double one = 1.0, zero = 0.0;
    int Ni = (int)N, ldi = (int)ld, kb = (int)kSliceRows;
    if (nfull > 0)
        FE_BLAS(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, Ni, Ni, kb, &one,
                                              A, ldi, kSliceRows * ld, B, ldi, kSliceRows * ld, &zero, part, Ni, N * N,
                                              (int)nfull),
                "dgemm_strided_batched (gram)");
    if (rem > 0)
        FE_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, Ni, Ni, (int)rem, &one,
                              A + nfull * kSliceRows * ld, ldi, B + nfull * kSliceRows * ld, ldi, &zero,
                              part + nfull * N * N, Ni),
                "dgemm (gram tail)");
    FE_HIPD(launch_sum_partials(part, nfull + (rem > 0 ? 1 : 0), N * N, out, s), "sum partials");
    return FE_OK;
}

static size_t tsgram_doubles(int64_t n, int64_t N) { return (size_t)(n / kSliceRows + 1) * N * N; }

// Complex blocks (interleaved re/im, ld in complex elements): out (N x N,
// column-major complex) = Acm Bcm^H, which is conj(A^H B) for the row-major
// blocks; the same deterministic split-K as tsgram.  part: scratch of
// 2 * tsgram_doubles(n, N) doubles.
static fe_status tsgram_z(rocblas_handle h, const double *A, const double *B, int64_t n, int64_t N, int64_t ld,
                          double *part, double *out, hipStream_t s) {
    int64_t nfull = n / kSliceRows, rem = n - nfull * kSliceRows;
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
    int Ni = (int)N, ldi = (int)ld, kb = (int)kSliceRows;
    auto z = [](const double *p) { return reinterpret_cast<const rocblas_double_complex *>(p); };
    auto zw = [](double *p) { return reinterpret_cast<rocblas_double_complex *>(p); };
    if (nfull > 0)
        FE_BLAS(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_conjugate_transpose, Ni, Ni,
                                              kb, &one, z(A), ldi, kSliceRows * ld, z(B), ldi, kSliceRows * ld, &zero,
                                              zw(part), Ni, N * N, (int)nfull),
                "zgemm_strided_batched (gram)");
    if (rem > 0)
        FE_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_conjugate_transpose, Ni, Ni, (int)rem, &one,
                              z(A + 2 * nfull * kSliceRows * ld), ldi, z(B + 2 * nfull * kSliceRows * ld), ldi, &zero,
                              zw(part + 2 * nfull * N * N), Ni),
                "zgemm (gram tail)");
    FE_HIPD(launch_sum_partials(part, nfull + (rem > 0 ? 1 : 0), 2 * N * N, out, s), "sum partials");
    return FE_OK;
}

}  // namespace fe

using namespace fe;

extern "C" {

fe_status fe_lanczos_bounds(fe_mesh *m, const double *v0, int32_t k, double *a0, double *b, hipStream_t s) {
    if (!m || !v0 || !a0 || !b) return fail(FE_EINVAL, "NULL argument");
    if (k < 1 || k > 64) return fail(FE_EINVAL, "k must be in 1..64");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    int64_t n = m->n;
    // scratch: V [n x (k+1)] column-major, w [n], h [k+1]
    size_t need = ((size_t)n * (k + 2) + (k + 1) + 1024) * sizeof(double);
    fe_status st = ensure_scratch_dense(m, need);
    if (st != FE_OK) return st;
    double *V = m->d_scratch + 1024, *w = V + (size_t)n * (k + 1), *hv = w + n;
    rocblas_handle h;
    if ((st = handle(m, s, h)) != FE_OK) return st;
    int ni = (int)n;
    double nrm;
    FE_BLAS(rocblas_dnrm2(h, ni, v0, 1, &nrm), "dnrm2");
    if (!(nrm > 0.0)) return fail(FE_EINVAL, "start vector is zero");
    FE_HIPD(hipMemcpyAsync(V, v0, n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy v0");
    double inv = 1.0 / nrm;
    FE_BLAS(rocblas_dscal(h, ni, &inv, V, 1), "dscal");
    std::vector<double> alpha(k), beta(k);
    int kk = k;
    for (int j = 0; j < k; ++j) {
        double *vj = V + (size_t)j * n;
        StepArgs a{vj, 1, w, 1, nullptr, 0, 1.0, 0.0, 0.0, 1};
        FE_HIPD(launch_step(m, a, FE_F64, s), "step kernel launch");
        if (m->nl.n_site > 0) FE_HIPD(launch_nonlocal(m, vj, 1, w, 1, 1, 1.0, s), "nonlocal");
        FE_BLAS(rocblas_ddot(h, ni, vj, 1, w, 1, &alpha[j]), "ddot");
        // full reorthogonalisation, twice: w -= V (V^T w)
        for (int pass = 0; pass < 2; ++pass) {
            double one = 1.0, zero = 0.0, mone = -1.0;
            FE_BLAS(rocblas_dgemv(h, rocblas_operation_transpose, ni, j + 1, &one, V, ni, w, 1, &zero, hv, 1), "dgemv T");
            FE_BLAS(rocblas_dgemv(h, rocblas_operation_none, ni, j + 1, &mone, V, ni, hv, 1, &one, w, 1), "dgemv N");
        }
        FE_BLAS(rocblas_dnrm2(h, ni, w, 1, &beta[j]), "dnrm2");
        if (beta[j] == 0.0) { kk = j + 1; break; }
        if (j + 1 < k) {
            double ib = 1.0 / beta[j];
            FE_HIPD(hipMemcpyAsync(V + (size_t)(j + 1) * n, w, n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
            FE_BLAS(rocblas_dscal(h, ni, &ib, V + (size_t)(j + 1) * n, 1), "dscal");
        }
    }
    std::vector<double> T((size_t)kk * kk, 0.0), ev;
    for (int i = 0; i < kk; ++i) {
        T[i * kk + i] = alpha[i];
        if (i + 1 < kk) T[i * kk + i + 1] = T[(i + 1) * kk + i] = beta[i];
    }
    jacobi_eigvals(T, kk, ev);
    *a0 = ev.front();
    *b = ev.back() + std::fabs(beta[kk - 1]);
    return FE_OK;
}

fe_status fe_cholqr2(fe_mesh *m, double *Y, int64_t N, int64_t ld, hipStream_t s) {
    if (!m || !Y) return fail(FE_EINVAL, "NULL argument");
    if (N < 1 || ld < N) return fail(FE_EINVAL, "need N >= 1 and ld >= N");
    if (N > m->n) return fail(FE_EINVAL, "N exceeds the number of DoFs");
    int64_t n = m->n;
    int64_t nb = std::min(kBlockRows, n);
    // scratch: [1024 reserved][S: N*N][partials][T: nb*N][info]
    size_t need = (1024 + (size_t)N * N + tsgram_doubles(n, N) + (size_t)nb * N + 64) * sizeof(double);
    fe_status st = ensure_scratch_dense(m, need);
    if (st != FE_OK) return st;
    double *S = m->d_scratch + 1024, *part = S + (size_t)N * N, *T = part + tsgram_doubles(n, N);
    rocblas_int *info = reinterpret_cast<rocblas_int *>(T + (size_t)nb * N);
    rocblas_handle h;
    if ((st = handle(m, s, h)) != FE_OK) return st;
    int Ni = (int)N, ldi = (int)ld;
    for (int pass = 0; pass < 2; ++pass) {
        // S = Y^T Y, S = U^T U (Cholesky), Y <- Y U^-1
        if ((st = tsgram(h, Y, Y, n, N, ld, part, S, s)) != FE_OK) return st;
        FE_BLAS(rocsolver_dpotrf(h, rocblas_fill_upper, Ni, S, Ni, info), "dpotrf");
        rocblas_int hinfo = 0;
        FE_HIPD(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s), "copy info");
        FE_HIPD(hipStreamSynchronize(s), "sync");
        if (hinfo != 0) return fail(FE_EDEVICE, "Gram matrix not positive definite (potrf info " + std::to_string(hinfo) + ")");
        FE_BLAS(rocsolver_dtrtri(h, rocblas_fill_upper, rocblas_diagonal_non_unit, Ni, S, Ni, info), "dtrtri");
        FE_HIPD(launch_zero_lower(S, Ni, s), "zero lower");
        double one = 1.0, zero = 0.0;
        for (int64_t r0 = 0; r0 < n; r0 += nb) {
            int64_t rows = std::min(nb, n - r0);
            double *Yb = Y + r0 * ld;
            FE_HIPD(hipMemcpy2DAsync(T, N * sizeof(double), Yb, ld * sizeof(double), N * sizeof(double), rows,
                                     hipMemcpyDeviceToDevice, s),
                    "stage block");
            // (Y_b U^-1) in column-major form: Ycm_b = U^-T Tcm
            FE_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, Ni, (int)rows, Ni, &one, S,
                                  Ni, T, Ni, &zero, Yb, ldi),
                    "dgemm (Y U^-1)");
        }
    }
    return FE_OK;
}

fe_status fe_rayleigh_ritz(fe_mesh *m, const double *Q, double *X, double *P, int64_t N, int64_t ld, double *theta,
                           hipStream_t s) {
    if (!m || !Q || !X || !P || !theta) return fail(FE_EINVAL, "NULL argument");
    if (N < 1 || ld < N) return fail(FE_EINVAL, "need N >= 1 and ld >= N");
    if (overlap(Q, m->n, N, ld, X, m->n, N, ld) || overlap(Q, m->n, N, ld, P, m->n, N, ld) ||
        overlap(X, m->n, N, ld, P, m->n, N, ld))
        return fail(FE_EINVAL, "Q, X and P must not overlap");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    int64_t n = m->n;
    // P = H~ Q (FP64 cell products)
    StepArgs a{Q, ld, P, ld, nullptr, 0, 1.0, 0.0, 0.0, N};
    FE_HIPD(launch_step(m, a, FE_F64, s), "step kernel launch");
    size_t need = (1024 + 2 * (size_t)N * N + 2 * (size_t)N + 64 + tsgram_doubles(n, N)) * sizeof(double);
    fe_status st = ensure_scratch_dense(m, need);
    if (st != FE_OK) return st;
    double *Hs = m->d_scratch + 1024, *Ht = Hs + (size_t)N * N, *d = Ht + (size_t)N * N, *e = d + N;
    rocblas_int *info = reinterpret_cast<rocblas_int *>(e + N);
    double *part = reinterpret_cast<double *>(info + 128);
    if (m->nl.n_site > 0) FE_HIPD(launch_nonlocal(m, Q, ld, P, ld, N, 1.0, s), "nonlocal");
    rocblas_handle h;
    if ((st = handle(m, s, h)) != FE_OK) return st;
    int Ni = (int)N, ni = (int)n, ldi = (int)ld;
    double one = 1.0, zero = 0.0, half = 0.5;
    // Hs = Q^T P (split-K over the DoFs), then symmetrise Hs = (Hs + Hs^T)/2
    if ((st = tsgram(h, Q, P, n, N, ld, part, Hs, s)) != FE_OK) return st;
    FE_BLAS(rocblas_dgeam(h, rocblas_operation_none, rocblas_operation_transpose, Ni, Ni, &half, Hs, Ni, &half, Hs, Ni,
                          Ht, Ni),
            "dgeam");
    FE_BLAS(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, Ni, Ht, Ni, d, e, info), "dsyevd");
    rocblas_int hinfo = 0;
    FE_HIPD(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s), "copy info");
    FE_HIPD(hipMemcpyAsync(theta, d, N * sizeof(double), hipMemcpyDeviceToHost, s), "copy theta");
    FE_HIPD(hipStreamSynchronize(s), "sync");
    if (hinfo != 0) return fail(FE_EDEVICE, "syevd failed (info " + std::to_string(hinfo) + ")");
    // X = Q W  (column-major: Xcm = W^T Qcm)
    FE_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, Ni, ni, Ni, &one, Ht, Ni, Q, ldi,
                          &zero, X, ldi),
            "dgemm QW");
    return FE_OK;
}

// ------------------------------------------------------------ Bloch-k blocks

fe_status fe_cholqr2_k(fe_mesh *m, double *Y, int64_t N, int64_t ld, hipStream_t s) {
    if (!m || !Y) return fail(FE_EINVAL, "NULL argument");
    if (N < 1 || ld < N) return fail(FE_EINVAL, "need N >= 1 and ld >= N");
    if (N > m->n) return fail(FE_EINVAL, "N exceeds the number of DoFs");
    int64_t n = m->n;
    int64_t nb = std::min(kBlockRows, n);
    // scratch: [1024 reserved][D: N*N complex][partials][T: nb*N complex][info]
    size_t need = (1024 + 2 * (size_t)N * N + 2 * tsgram_doubles(n, N) + 2 * (size_t)nb * N + 64) * sizeof(double);
    fe_status st = ensure_scratch_dense(m, need);
    if (st != FE_OK) return st;
    double *D = m->d_scratch + 1024, *part = D + 2 * (size_t)N * N, *T = part + 2 * tsgram_doubles(n, N);
    rocblas_int *info = reinterpret_cast<rocblas_int *>(T + 2 * (size_t)nb * N);
    rocblas_handle h;
    if ((st = handle(m, s, h)) != FE_OK) return st;
    int Ni = (int)N, ldi = (int)ld;
    auto zw = [](double *p) { return reinterpret_cast<rocblas_double_complex *>(p); };
    for (int pass = 0; pass < 2; ++pass) {
        // D = conj(Y^H Y) = U^H U (Cholesky); with R = conj(U), Y^H Y = R^H R and
        // Y R^-1 in column-major form is Ycm <- (U^-1)^H Ycm
        if ((st = tsgram_z(h, Y, Y, n, N, ld, part, D, s)) != FE_OK) return st;
        FE_BLAS(rocsolver_zpotrf(h, rocblas_fill_upper, Ni, zw(D), Ni, info), "zpotrf");
        rocblas_int hinfo = 0;
        FE_HIPD(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s), "copy info");
        FE_HIPD(hipStreamSynchronize(s), "sync");
        if (hinfo != 0) return fail(FE_EDEVICE, "Gram matrix not positive definite (potrf info " + std::to_string(hinfo) + ")");
        FE_BLAS(rocsolver_ztrtri(h, rocblas_fill_upper, rocblas_diagonal_non_unit, Ni, zw(D), Ni, info), "ztrtri");
        FE_HIPD(launch_zero_lower_z(D, Ni, s), "zero lower");
        const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
        for (int64_t r0 = 0; r0 < n; r0 += nb) {
            int64_t rows = std::min(nb, n - r0);
            double *Yb = Y + 2 * r0 * ld;
            FE_HIPD(hipMemcpy2DAsync(T, 2 * N * sizeof(double), Yb, 2 * ld * sizeof(double), 2 * N * sizeof(double),
                                     rows, hipMemcpyDeviceToDevice, s),
                    "stage block");
            FE_BLAS(rocblas_zgemm(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, Ni, (int)rows, Ni,
                                  &one, zw(D), Ni, zw(T), Ni, &zero, zw(Yb), ldi),
                    "zgemm (Y R^-1)");
        }
    }
    return FE_OK;
}

fe_status fe_rayleigh_ritz_k(fe_mesh *m, const double *Q, double *X, double *P, int64_t N, int64_t ld, double *theta,
                             hipStream_t s) {
    if (!m || !Q || !X || !P || !theta) return fail(FE_EINVAL, "NULL argument");
    if (N < 1 || ld < N) return fail(FE_EINVAL, "need N >= 1 and ld >= N");
    if (overlap(Q, m->n, 2 * N, 2 * ld, X, m->n, 2 * N, 2 * ld) || overlap(Q, m->n, 2 * N, 2 * ld, P, m->n, 2 * N, 2 * ld) ||
        overlap(X, m->n, 2 * N, 2 * ld, P, m->n, 2 * N, 2 * ld))
        return fail(FE_EINVAL, "Q, X and P must not overlap");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    int64_t n = m->n;
    // P = H~^k Q
    fe_status st = filter_step_k(m, Q, ld, P, ld, nullptr, 0, 1.0, 0.0, 0.0, N, s);
    if (st != FE_OK) return st;
    size_t need = (1024 + 4 * (size_t)N * N + 2 * (size_t)N + 64 + 2 * tsgram_doubles(n, N)) * sizeof(double);
    if ((st = ensure_scratch_dense(m, need)) != FE_OK) return st;
    double *Hs = m->d_scratch + 1024, *Ht = Hs + 2 * (size_t)N * N, *d = Ht + 2 * (size_t)N * N, *e = d + N;
    rocblas_int *info = reinterpret_cast<rocblas_int *>(e + N);
    double *part = reinterpret_cast<double *>(info + 128);
    rocblas_handle h;
    if ((st = handle(m, s, h)) != FE_OK) return st;
    int Ni = (int)N, ni = (int)n, ldi = (int)ld;
    auto z = [](const double *p) { return reinterpret_cast<const rocblas_double_complex *>(p); };
    auto zw = [](double *p) { return reinterpret_cast<rocblas_double_complex *>(p); };
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0}, half = {0.5, 0.0};
    // Hs = conj(Q^H P); Ht = (Hs + Hs^H) / 2 = conj of the Hermitian projected matrix
    if ((st = tsgram_z(h, Q, P, n, N, ld, part, Hs, s)) != FE_OK) return st;
    FE_BLAS(rocblas_zgeam(h, rocblas_operation_none, rocblas_operation_conjugate_transpose, Ni, Ni, &half, z(Hs), Ni,
                          &half, z(Hs), Ni, zw(Ht), Ni),
            "zgeam");
    FE_BLAS(rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, Ni, zw(Ht), Ni, d, e, info), "zheevd");
    rocblas_int hinfo = 0;
    FE_HIPD(hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s), "copy info");
    FE_HIPD(hipMemcpyAsync(theta, d, N * sizeof(double), hipMemcpyDeviceToHost, s), "copy theta");
    FE_HIPD(hipStreamSynchronize(s), "sync");
    if (hinfo != 0) return fail(FE_EDEVICE, "heevd failed (info " + std::to_string(hinfo) + ")");
    // the eigenvectors W' of conj(H) are conj(W); X = Q W, i.e. Xcm = W'^H Qcm
    FE_BLAS(rocblas_zgemm(h, rocblas_operation_conjugate_transpose, rocblas_operation_none, Ni, ni, Ni, &one, z(Ht),
                          Ni, z(Q), ldi, &zero, zw(X), ldi),
            "zgemm QW");
    return FE_OK;
}

}  // extern "C"
