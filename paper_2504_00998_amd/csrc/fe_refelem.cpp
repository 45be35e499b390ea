// Reference element of the C0 GLL spectral-element basis (paper Sec. 2.3),
// computed on the host in FP64 when a mesh is created.
//
// Route: GLL nodes by Newton iteration on the Lobatto function
// f(x) = P_{p-1}(x) - x P_p(x) (zero at the interior GLL nodes, since
// (1-x^2) P_p'(x) = p (P_{p-1}(x) - x P_p(x))); barycentric Lagrange
// interpolation; 1-D integrals with a (p+3)-point GLL rule, exact for the
// degree-2p integrands; the 3-D cell stiffness as a Kronecker sum.
#include <cmath>
#include <vector>

#include "fe_internal.h"

namespace fe {

namespace {

// P_{n-1}(x), P_n(x) and their derivatives.
void legendre_pair(int n, double x, double &pm1, double &pn, double &dpm1, double &dpn) {
    double a = 1.0, b = x, da = 0.0, db = 1.0;  // P_0, P_1
    if (n == 0) { pm1 = 0.0; pn = 1.0; dpm1 = 0.0; dpn = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        double dnew = da + (2 * k - 1) * b;  // P'_k = P'_{k-2} + (2k-1) P_{k-1}
        a = b; b = c; da = db; db = dnew;
    }
    pm1 = a; pn = b; dpm1 = da; dpn = db;
}

}  // namespace

void gll_rule(int p, std::vector<double> &x, std::vector<double> &w) {
    x.assign(p + 1, 0.0);
    w.assign(p + 1, 0.0);
    x[0] = -1.0;
    x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double t = -std::cos(M_PI * i / p);
        for (int it = 0; it < 200; ++it) {
            double pm1, pn, dpm1, dpn;
            legendre_pair(p, t, pm1, pn, dpm1, dpn);
            double f = pm1 - t * pn;
            double df = dpm1 - pn - t * dpn;
            double step = f / df;
            t -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        x[i] = t;
    }
    for (int i = 0; i <= p; ++i) {
        double pm1, pn, dpm1, dpn;
        legendre_pair(p, x[i], pm1, pn, dpm1, dpn);
        w[i] = 2.0 / (p * (p + 1.0) * pn * pn);
    }
}

namespace {

struct Barycentric {
    std::vector<double> x, lam;
    explicit Barycentric(const std::vector<double> &nodes) : x(nodes), lam(nodes.size(), 1.0) {
        for (size_t i = 0; i < x.size(); ++i)
            for (size_t j = 0; j < x.size(); ++j)
                if (i != j) lam[i] /= (x[i] - x[j]);
    }
    // values of all basis polynomials at t
    void values(double t, std::vector<double> &out) const {
        size_t n = x.size();
        out.assign(n, 0.0);
        for (size_t j = 0; j < n; ++j)
            if (t == x[j]) { out[j] = 1.0; return; }
        double s = 0.0;
        for (size_t j = 0; j < n; ++j) { out[j] = lam[j] / (t - x[j]); s += out[j]; }
        for (size_t j = 0; j < n; ++j) out[j] /= s;
    }
    // differentiation matrix Dm[i][j] = l_j'(x_i)
    std::vector<double> diff_matrix() const {
        size_t n = x.size();
        std::vector<double> D(n * n, 0.0);
        for (size_t i = 0; i < n; ++i) {
            double diag = 0.0;
            for (size_t j = 0; j < n; ++j) {
                if (i == j) continue;
                D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
                diag -= D[i * n + j];
            }
            D[i * n + i] = diag;
        }
        return D;
    }
};

}  // namespace

// 1-D reference stiffness Khat_ij = int l_i' l_j' and mass on [-1, 1];
// rule 0: consistent mass int l_i l_j; rule 1: lumped diag(w).
void ref_matrices(int p, int rule, std::vector<double> &Khat, std::vector<double> &Mhat) {
    std::vector<double> x, w, y, wy;
    gll_rule(p, x, w);
    gll_rule(p + 2, y, wy);  // p+3 points: exact to degree 2p+1
    Barycentric B(x);
    std::vector<double> D = B.diff_matrix();
    int n = p + 1;
    Khat.assign(n * n, 0.0);
    Mhat.assign(n * n, 0.0);
    std::vector<double> lv, dv(n);
    for (size_t q = 0; q < y.size(); ++q) {
        B.values(y[q], lv);
        // l_j'(y) by interpolating the nodal derivatives (degree p-1)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += lv[i] * D[i * n + j];
            dv[j] = s;
        }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                Khat[i * n + j] += wy[q] * dv[i] * dv[j];
                if (rule == FE_RULE_EXACT) Mhat[i * n + j] += wy[q] * lv[i] * lv[j];
            }
    }
    if (rule == FE_RULE_GLL)
        for (int i = 0; i < n; ++i) Mhat[i * n + i] = w[i];
}

// A = 1/2 Kc for a cube of edge h:
//   Kc = (h/2) [Khat (x) Mhat (x) Mhat + Mhat (x) Khat (x) Mhat + Mhat (x) Mhat (x) Khat]
// with local index l = i + (p+1)(j + (p+1) k), i along x.
void cell_matrix_half(int p, int rule, double h, std::vector<double> &A) {
    std::vector<double> K, M;
    ref_matrices(p, rule, K, M);
    int n = p + 1, nc = n * n * n;
    A.assign((size_t)nc * nc, 0.0);
    double s = 0.25 * h;  // 1/2 * h/2
    for (int l = 0; l < nc; ++l) {
        int i = l % n, j = (l / n) % n, k = l / (n * n);
        for (int lp = 0; lp < nc; ++lp) {
            int ip = lp % n, jp = (lp / n) % n, kp = lp / (n * n);
            double v = K[i * n + ip] * M[j * n + jp] * M[k * n + kp] +
                       M[i * n + ip] * K[j * n + jp] * M[k * n + kp] +
                       M[i * n + ip] * M[j * n + jp] * K[k * n + kp];
            A[(size_t)l * nc + lp] = s * v;
        }
    }
}

}  // namespace fe

namespace fe {

// S = kx G_x + ky G_y with the cell advection matrices
//   G_a[l][l'] = int_c N_l dN_l'/dx_a
// of a cube of edge h (the Bloch-k term of Sec. 2.3 is -i M^-1/2 (k.G) M^-1/2
// after assembly).  Per axis the integral factors into 1-D ones: the
// derivative axis contributes Chat_ij = int l_i l_j' (degree 2p-1, so the
// (p+1)-point GLL rule is exact and Chat_ij = w_i l_j'(x_i) under either
// rule), the others (h/2) Mhat; the 2/h of the derivative cancels one h/2.
void cell_matrix_bloch(int p, int rule, double h, double kx, double ky, std::vector<double> &S) {
    std::vector<double> K, M, x, w;
    ref_matrices(p, rule, K, M);
    gll_rule(p, x, w);
    std::vector<double> D = Barycentric(x).diff_matrix();
    const int n = p + 1, nc = n * n * n;
    std::vector<double> Ch(n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ch[i * n + j] = w[i] * D[i * n + j];
    const double s = 0.25 * h * h;  // (h/2)^2
    S.assign((size_t)nc * nc, 0.0);
    for (int l = 0; l < nc; ++l) {
        const int i = l % n, j = (l / n) % n, k = l / (n * n);
        for (int lp = 0; lp < nc; ++lp) {
            const int ip = lp % n, jp = (lp / n) % n, kp = lp / (n * n);
            const double mz = M[k * n + kp];
            const double v = kx * Ch[i * n + ip] * M[j * n + jp] * mz + ky * M[i * n + ip] * Ch[j * n + jp] * mz;
            S[(size_t)l * nc + lp] = s * v;
        }
    }
}

}  // namespace fe
