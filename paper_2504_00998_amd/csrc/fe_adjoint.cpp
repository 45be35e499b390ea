// Reverse-mode derivative of the Chebyshev filter.
//
// Forward:  Y_1 = alpha_0 (H~ - c) Y_0,  Y_{k+1} = alpha_k (H~ - c) Y_k - beta_k Y_{k-1}.
// For a cotangent G = dL/dY_m the adjoint runs k = m-1 .. 0:
//   Ybar_k     += alpha_k (H~ - c) Ybar_{k+1}     (H~ symmetric: the same kernel),
//   Ybar_{k-1}  = -beta_k Ybar_{k+1}               (its first contribution),
//   g_I        += alpha_k sum_j Ybar_{k+1}[I,j] Y_k[I,j],
// where g = dL/dv is the derivative with respect to the diagonal potential
// term v of H~ (the only place V_quad and E enter H~; paper Sec. 2.1 V_eff
// and Sec. 2.2.1 V_app).  dL/dX = Ybar_0; dL/dV_quad and dL/dE follow from
// v_I = sum (|J| w_q / M_I) V_quad - E (z_I - z0) by the chain rule.
//
// Memory: Y_k is either stored for every k (ckpt_stride = 1) or kept as
// pairs (Y_{js}, Y_{js+1}) every s steps and recomputed segment by segment
// in the reverse sweep; columns are processed in chunks (columns are
// independent under H~), and g is summed over chunks in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fe_internal.h"

namespace fe {

namespace {

struct VjpPlan {
    int64_t Nc = 0;     // columns per chunk
    int s = 1;          // checkpoint stride
    int J = 0;          // checkpoint pairs (s > 1)
    int64_t blocks = 0; // n x Nc blocks in the work buffer
};

VjpPlan make_plan(int64_t N, int mdeg, int s, int col_chunk) {
    VjpPlan p;
    p.Nc = col_chunk <= 0 ? N : std::min<int64_t>(col_chunk, N);
    p.s = std::max(1, s);
    if (p.s == 1) {
        p.blocks = (mdeg - 1) + 3;  // Y_1..Y_{m-1} and three adjoint blocks
    } else {
        p.J = (mdeg + p.s - 1) / p.s;
        p.blocks = 2 * (int64_t)p.J + p.s + 3;  // checkpoint pairs, one segment, adjoint
    }
    return p;
}

#define FE_HIPA(call, what)                                                                          \
    do {                                                                                             \
        hipError_t _e = (call);                                                                      \
        if (_e != hipSuccess) return fail(FE_EDEVICE, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

}  // namespace

}  // namespace fe

using namespace fe;

extern "C" {

size_t fe_cheb_filter_vjp_work_bytes(const fe_mesh *m, int64_t N, int32_t mdeg, int32_t ckpt_stride,
                                     int32_t col_chunk) {
    if (!m || N < 1 || mdeg < 1) return 0;
    VjpPlan p = make_plan(N, mdeg, ckpt_stride, col_chunk);
    return (size_t)(p.blocks * m->n * p.Nc + m->n) * sizeof(double);
}

fe_status fe_cheb_filter_vjp(fe_mesh *m, const double *X, const double *G, int64_t N, int64_t ld, int32_t mdeg,
                             double a, double b, double a0, fe_dtype prec, double *Xbar, double *Vbar,
                             double *Ebar, int32_t ckpt_stride, int32_t col_chunk, double *work, size_t work_bytes,
                             hipStream_t st) {
    fe_status rc = validate_filter_args(m, N, mdeg, a, b, a0, prec);
    if (rc != FE_OK) return rc;
    if (N == 0) return fail(FE_EINVAL, "N must be >= 1");
    if (!X || !G || !Xbar || !Vbar || !Ebar || !work) return fail(FE_EINVAL, "NULL argument");
    if (ld < N) return fail(FE_EINVAL, "ld < N");
    if (ckpt_stride < 1) return fail(FE_EINVAL, "ckpt_stride must be >= 1");
    if (col_chunk < 0) return fail(FE_EINVAL, "col_chunk must be >= 0");
    if (!m->potential_set) return fail(FE_ESTATE, "fe_set_potential has not been called");
    size_t need = fe_cheb_filter_vjp_work_bytes(m, N, mdeg, ckpt_stride, col_chunk);
    if (work_bytes < need)
        return fail(FE_ENOMEM, "work smaller than fe_cheb_filter_vjp_work_bytes (" + std::to_string(need) + " bytes)");

    const int64_t n = m->n;
    VjpPlan P = make_plan(N, mdeg, ckpt_stride, col_chunk);
    std::vector<double> al, be;
    double c;
    cheb_coefficients(mdeg, a, b, a0, al, be, c);

    double *g = work;
    auto block = [&](int64_t i) -> double * { return work + n + i * n * P.Nc; };
    FE_HIPA(launch_fill(g, n, 0.0, st), "fill");

    for (int64_t j0 = 0; j0 < N; j0 += P.Nc) {
        const int64_t Nc = std::min(P.Nc, N - j0);
        const int64_t ldb = P.Nc;  // blocks are (n x P.Nc); only Nc columns used
        const double *Xc = X + j0;
        const double *Gc = G + j0;

        // ------------------------------------------------------------ forward
        // Y_k for k >= 1: store-all slot k-1, or checkpoint slot, or rotating
        // pair inside the segment region
        double *seg = P.s == 1 ? nullptr : block(2 * (int64_t)P.J);
        double *adj = P.s == 1 ? block(mdeg - 1) : block(2 * (int64_t)P.J + P.s);
        auto fwd_buf = [&](int k) -> double * {  // k >= 1
            if (P.s == 1) return block(k - 1);
            return seg + (int64_t)(k & 1) * n * ldb;
        };
        auto ckpt_slot = [&](int k) -> double * {  // k = js or js+1, k >= 1
            int j = k / P.s, r = k % P.s;
            return block(2 * (int64_t)j + r);
        };
        if (mdeg >= 2) {
            for (int k = 0; k + 1 <= mdeg - 1; ++k) {
                const double *Yk = k == 0 ? Xc : fwd_buf(k);
                int64_t ldk = k == 0 ? ld : ldb;
                const double *Ym = nullptr;
                int64_t ldm = 0;
                if (k >= 1) {
                    Ym = k - 1 == 0 ? Xc : fwd_buf(k - 1);
                    ldm = k - 1 == 0 ? ld : ldb;
                }
                double *Yn = fwd_buf(k + 1);
                rc = filter_step(m, Yk, ldk, Yn, ldb, Ym, ldm, al[k], k >= 1 ? be[k] : 0.0, c, Nc, prec, st);
                if (rc != FE_OK) return rc;
                if (P.s > 1) {
                    int r = (k + 1) % P.s;
                    if (r == 0 || r == 1)
                        FE_HIPA(launch_axpby(ckpt_slot(k + 1), ldb, Yn, ldb, n, Nc, 1.0, 0.0, st), "copy");
                }
            }
        }

        // ------------------------------------------------------------ reverse
        auto adj_buf = [&](int k) -> double * { return adj + (int64_t)(k % 3) * n * ldb; };
        // Y_k for the reverse sweep of a segment starting at ks
        int ks_cur = -1;
        auto Y_of = [&](int k, int64_t &ldk) -> const double * {
            if (k == 0) { ldk = ld; return Xc; }
            ldk = ldb;
            if (P.s == 1) return block(k - 1);
            return seg + (int64_t)(k - ks_cur) * n * ldb;
        };
        for (int seg_j = P.s == 1 ? 0 : P.J - 1; seg_j >= 0; --seg_j) {
            int ks = P.s == 1 ? 0 : seg_j * P.s;
            int ke = P.s == 1 ? mdeg - 1 : std::min(ks + P.s, mdeg) - 1;
            if (P.s > 1) {
                // rebuild Y_ks .. Y_ke in the segment buffer
                ks_cur = ks;
                for (int k = ks; k <= ke; ++k) {
                    double *dst = seg + (int64_t)(k - ks) * n * ldb;
                    if (k == 0) continue;  // Y_0 is X itself
                    if (k == ks || k == ks + 1) {
                        FE_HIPA(launch_axpby(dst, ldb, ckpt_slot(k), ldb, n, Nc, 1.0, 0.0, st), "copy");
                        continue;
                    }
                    int64_t ldp, ldpp;
                    const double *Yp = Y_of(k - 1, ldp);
                    const double *Ypp = Y_of(k - 2, ldpp);
                    rc = filter_step(m, Yp, ldp, dst, ldb, Ypp, ldpp, al[k - 1], be[k - 1], c, Nc, prec, st);
                    if (rc != FE_OK) return rc;
                }
            }
            for (int k = ke; k >= ks; --k) {
                const double *B1 = k + 1 == mdeg ? Gc : adj_buf(k + 1);
                int64_t ld1 = k + 1 == mdeg ? ld : ldb;
                double *Bk = adj_buf(k);
                // Ybar_k += alpha_k (H~ - c) Ybar_{k+1}  (first contribution when k = m-1)
                bool first = k == mdeg - 1;
                rc = filter_step(m, B1, ld1, Bk, ldb, first ? nullptr : Bk, ldb, al[k], first ? 0.0 : -1.0, c, Nc,
                                 prec, st);
                if (rc != FE_OK) return rc;
                if (k >= 1)
                    FE_HIPA(launch_axpby(adj_buf(k - 1), ldb, B1, ld1, n, Nc, -be[k], 0.0, st), "axpby");
                int64_t ldk;
                const double *Yk = Y_of(k, ldk);
                FE_HIPA(launch_rowdot_accum(m, B1, ld1, Yk, ldk, Nc, al[k], g, st), "rowdot");
            }
        }
        FE_HIPA(launch_axpby(Xbar + j0, ld, adj_buf(0), ldb, n, Nc, 1.0, 0.0, st), "copy Xbar");
    }
    FE_HIPA(launch_potential_vjp(m, g, m->z0, Vbar, Ebar, st), "potential vjp");
    return FE_OK;
}

}  // extern "C"
