// Host FP64 dense symmetric-definite eigen-decomposition for the coarsest
// level of the hierarchy (setup only; the paper allows any eigensolver for the
// small problems, Section 3).
//
// A z = lam M z  ->  M = L L^T (Cholesky), C = L^-1 A L^-T,
// C = Q T Q^T (Householder tridiagonalisation), T = W diag(lam) W^T (implicit
// symmetric QR iterations with Wilkinson shifts), Z = L^-T Q W, Z^T M Z = I.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

#include "internal.h"

namespace amgeig {

namespace {

bool cholesky(int n, std::vector<double> &L) {  // in place, lower triangle
    for (int j = 0; j < n; ++j) {
        double s = L[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) return false;
        double ljj = std::sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = L[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
        for (int i = 0; i < j; ++i) L[(size_t)i * n + j] = 0.0;
    }
    return true;
}

// X <- L^-1 X for X n x m row-major (forward substitution, column by column of X).
void lower_solve(int n, int m, const std::vector<double> &L, std::vector<double> &X) {
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < i; ++k) {
            double l = L[(size_t)i * n + k];
            if (l == 0.0) continue;
            for (int c = 0; c < m; ++c) X[(size_t)i * m + c] -= l * X[(size_t)k * m + c];
        }
        double inv = 1.0 / L[(size_t)i * n + i];
        for (int c = 0; c < m; ++c) X[(size_t)i * m + c] *= inv;
    }
}

// X <- L^-T X (backward substitution).
void upper_solve_t(int n, int m, const std::vector<double> &L, std::vector<double> &X) {
    for (int i = n - 1; i >= 0; --i) {
        for (int k = i + 1; k < n; ++k) {
            double l = L[(size_t)k * n + i];
            if (l == 0.0) continue;
            for (int c = 0; c < m; ++c) X[(size_t)i * m + c] -= l * X[(size_t)k * m + c];
        }
        double inv = 1.0 / L[(size_t)i * n + i];
        for (int c = 0; c < m; ++c) X[(size_t)i * m + c] *= inv;
    }
}

// Householder reduction of symmetric C (n x n) to tridiagonal (d, e), Q accumulated.
void tridiagonalise(int n, std::vector<double> &C, std::vector<double> &Q, std::vector<double> &d,
                    std::vector<double> &e) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n), w(n), qv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // length of the column below the diagonal
        double tail = 0.0;
        for (int i = 1; i < m; ++i) tail += C[(size_t)(k + 1 + i) * n + k] * C[(size_t)(k + 1 + i) * n + k];
        double x0 = C[(size_t)(k + 1) * n + k];
        if (tail == 0.0) continue;  // already tridiagonal in this column
        double nrm = std::sqrt(x0 * x0 + tail);
        double alpha = x0 > 0 ? -nrm : nrm;
        for (int i = 0; i < m; ++i) v[i] = C[(size_t)(k + 1 + i) * n + k];
        v[0] -= alpha;
        double vn2 = v[0] * v[0] + tail;
        double beta = 2.0 / vn2;
        // p = beta * T v on the trailing block T = C[k+1:, k+1:]
        for (int i = 0; i < m; ++i) {
            const double *row = &C[(size_t)(k + 1 + i) * n + (k + 1)];
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += row[j] * v[j];
            p[i] = beta * s;
        }
        double vp = 0.0;
        for (int i = 0; i < m; ++i) vp += v[i] * p[i];
        double K = 0.5 * beta * vp;
        for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
        for (int i = 0; i < m; ++i) {
            double *row = &C[(size_t)(k + 1 + i) * n + (k + 1)];
            for (int j = 0; j < m; ++j) row[j] -= v[i] * w[j] + w[i] * v[j];
        }
        C[(size_t)(k + 1) * n + k] = C[(size_t)k * n + (k + 1)] = alpha;
        for (int i = 1; i < m; ++i) C[(size_t)(k + 1 + i) * n + k] = C[(size_t)k * n + (k + 1 + i)] = 0.0;
        // Q <- Q (I - beta v v^T) on columns k+1..n-1
        for (int r = 0; r < n; ++r) {
            double *row = &Q[(size_t)r * n + (k + 1)];
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += row[j] * v[j];
            s *= beta;
            for (int j = 0; j < m; ++j) row[j] -= s * v[j];
        }
    }
    d.resize(n);
    e.assign(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = C[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = C[(size_t)i * n + i + 1];
}

// Implicit symmetric QR with Wilkinson shifts on the tridiagonal (d, e[i] =
// T[i][i+1]); every plane rotation G (c, s) in the plane (k, k+1) is applied as
// T <- G^T T G and Z <- Z G.  Returns false if the iteration does not settle.
bool tridiagonal_qr(int n, std::vector<double> &d, std::vector<double> &e, std::vector<double> &Z) {
    const double eps = std::numeric_limits<double>::epsilon();
    long budget = 40L * n + 100;
    for (;;) {
        for (int i = 0; i + 1 < n; ++i)
            if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
        int h = n - 1;
        while (h > 0 && e[h - 1] == 0.0) --h;
        if (h == 0) return true;
        int l = h - 1;
        while (l > 0 && e[l - 1] != 0.0) --l;
        if (--budget < 0) return false;
        // Wilkinson shift: eigenvalue of the trailing 2x2 block closer to d[h]
        double delta = 0.5 * (d[h - 1] - d[h]);
        double eh = e[h - 1];
        double den = delta + (delta >= 0 ? 1.0 : -1.0) * std::hypot(delta, eh);
        double mu = d[h] - eh * eh / den;
        double x = d[l] - mu, z = e[l];
        for (int k = l; k < h; ++k) {
            double r = std::hypot(x, z);
            double c = r == 0.0 ? 1.0 : x / r;
            double s = r == 0.0 ? 0.0 : -z / r;
            if (k > l) e[k - 1] = r;  // the bulge at (k-1, k+1) is annihilated
            double a = d[k], b = e[k], cc = d[k + 1];
            d[k] = a * c * c - 2.0 * b * c * s + cc * s * s;
            d[k + 1] = a * s * s + 2.0 * b * c * s + cc * c * c;
            e[k] = (a - cc) * c * s + b * (c * c - s * s);
            double bulge = 0.0;
            if (k + 1 < h) {
                bulge = -s * e[k + 1];
                e[k + 1] *= c;
            }
            for (int i = 0; i < n; ++i) {
                double zk = Z[(size_t)i * n + k], zk1 = Z[(size_t)i * n + k + 1];
                Z[(size_t)i * n + k] = zk * c - zk1 * s;
                Z[(size_t)i * n + k + 1] = zk * s + zk1 * c;
            }
            x = e[k];
            z = bulge;
        }
    }
}

}  // namespace

bool dense_sygv(int n, const std::vector<double> &A, const std::vector<double> &M, std::vector<double> &lam,
                std::vector<double> &Zout) {
    std::vector<double> L(M);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) L[(size_t)i * n + j] = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
    if (!cholesky(n, L)) return false;
    // C = L^-1 A L^-T
    std::vector<double> X(A);
    lower_solve(n, n, L, X);  // X = L^-1 A
    std::vector<double> Xt((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Xt[(size_t)j * n + i] = X[(size_t)i * n + j];
    lower_solve(n, n, L, Xt);  // L^-1 (L^-1 A)^T = (L^-1 A L^-T)^T
    std::vector<double> C((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) C[(size_t)i * n + j] = 0.5 * (Xt[(size_t)i * n + j] + Xt[(size_t)j * n + i]);
    std::vector<double> Q, d, e;
    tridiagonalise(n, C, Q, d, e);
    if (!tridiagonal_qr(n, d, e, Q)) return false;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
    lam.resize(n);
    std::vector<double> W((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        lam[j] = d[order[j]];
        for (int i = 0; i < n; ++i) W[(size_t)i * n + j] = Q[(size_t)i * n + order[j]];
    }
    upper_solve_t(n, n, L, W);  // Z = L^-T W
    Zout.swap(W);
    return true;
}

int guard_width(const std::vector<double> &lam, int q, double gap, int cap) {
    cap = std::min<int>(cap, (int)lam.size() - 1);
    int m = q;
    while (m < cap && lam[m] / lam[m - 1] - 1.0 < gap) ++m;
    return m;
}

}  // namespace amgeig
