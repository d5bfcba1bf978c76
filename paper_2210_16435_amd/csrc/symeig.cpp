// Dense symmetric eigensolver for the small projected matrices of the
// Rayleigh-Ritz step (order <= a few hundred), FP64 on the host.
//
// Method (Golub and Van Loan, Matrix Computations, Sections 8.3.1-8.3.3):
// Householder reduction to tridiagonal form, accumulating the orthogonal
// factor, followed by implicitly shifted QL iterations with Wilkinson-type
// shifts on the tridiagonal matrix, applying each plane rotation to the
// accumulated factor.  The factor is kept transposed (one eigenvector per
// row) so every rotation touches two contiguous rows.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "symeig.h"

namespace sfairsc {

namespace {

// Reduce symmetric A (n x n row-major, overwritten) to tridiagonal form
// Q^T A Q = tridiag(d, e) with e[i] coupling i and i+1; returns Qt = Q^T.
void tridiagonalize(int n, std::vector<double>& A, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& Qt) {
    std::vector<std::vector<double>> vs;  // Householder vectors (length n-k-1)
    std::vector<double> betas;
    std::vector<double> v(n), p(n), w(n);
    d.assign(n, 0.0);
    e.assign(n, 0.0);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // length of the column below the diagonal
        double sigma2 = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = A[(k + 1 + i) * n + k];
            sigma2 += v[i] * v[i];
        }
        double norm = std::sqrt(sigma2);
        if (norm == 0.0) {
            e[k] = 0.0;
            vs.emplace_back();
            betas.push_back(0.0);
            continue;
        }
        double alpha = v[0] >= 0 ? -norm : norm;  // reflect x onto alpha e_1
        v[0] -= alpha;
        double vtv = 0.0;
        for (int i = 0; i < m; ++i) vtv += v[i] * v[i];
        const double beta = 2.0 / vtv;
        e[k] = alpha;
        // B = A[k+1:, k+1:];  p = beta B v;  w = p - (beta/2)(p^T v) v;
        // B <- B - v w^T - w v^T
        for (int i = 0; i < m; ++i) {
            const double* row = &A[(k + 1 + i) * n + k + 1];
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += row[j] * v[j];
            p[i] = beta * s;
        }
        double ptv = 0.0;
        for (int i = 0; i < m; ++i) ptv += p[i] * v[i];
        const double kf = 0.5 * beta * ptv;
        for (int i = 0; i < m; ++i) w[i] = p[i] - kf * v[i];
        for (int i = 0; i < m; ++i) {
            double* row = &A[(k + 1 + i) * n + k + 1];
            const double vi = v[i], wi = w[i];
            for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
        }
        vs.emplace_back(v.begin(), v.begin() + m);
        betas.push_back(beta);
    }
    for (int i = 0; i < n; ++i) d[i] = A[i * n + i];
    if (n >= 2) e[n - 2] = A[(n - 1) * n + (n - 2)];
    e[n - 1] = 0.0;
    // Q = H_0 H_1 ... H_{n-3} (each H_k symmetric), so Q^T = H_{n-3} ... H_0:
    // start from I and left-multiply by H_0, H_1, ...; H_k acts on rows k+1..
    Qt.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Qt[(size_t)i * n + i] = 1.0;
    std::vector<double> tmp(n);
    for (int k = 0; k < (int)vs.size(); ++k) {
        if (betas[k] == 0.0) continue;
        const std::vector<double>& vk = vs[k];
        const int m = (int)vk.size();
        // tmp = v^T Qt[k+1:, :]
        std::fill(tmp.begin(), tmp.end(), 0.0);
        for (int i = 0; i < m; ++i) {
            const double* row = &Qt[(size_t)(k + 1 + i) * n];
            const double vi = vk[i];
            for (int j = 0; j < n; ++j) tmp[j] += vi * row[j];
        }
        for (int i = 0; i < m; ++i) {
            double* row = &Qt[(size_t)(k + 1 + i) * n];
            const double c = betas[k] * vk[i];
            for (int j = 0; j < n; ++j) row[j] -= c * tmp[j];
        }
    }
}

// Implicit QL on tridiag(d, e); rows of Zt are rotated along (Zt = Q^T on
// entry gives the eigenvectors of the original matrix as rows on exit).
void tridiag_ql(int n, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Zt) {
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) break;  // no convergence: leave as is
            // shift from the trailing 2x2 of the unreduced block at l
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                double f = s * e[i];
                const double bb = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {  // underflow: split here
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * bb;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - bb;
                // rotate eigenvector rows i and i+1
                double* zi = &Zt[(size_t)i * n];
                double* zj = &Zt[(size_t)(i + 1) * n];
                for (int t = 0; t < n; ++t) {
                    const double a = zi[t], bq = zj[t];
                    zj[t] = s * a + c * bq;
                    zi[t] = c * a - s * bq;
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
}

}  // namespace

void sym_eig(int n, const double* A, double* w, double* Z) {
    if (n <= 0) return;
    if (n == 1) {
        w[0] = A[0];
        Z[0] = 1.0;
        return;
    }
    std::vector<double> a(A, A + (size_t)n * n), d, e, Qt;
    tridiagonalize(n, a, d, e, Qt);
    tridiag_ql(n, d, e, Qt);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
    for (int j = 0; j < n; ++j) {
        const int src = order[j];
        w[j] = d[src];
        const double* row = &Qt[(size_t)src * n];
        for (int i = 0; i < n; ++i) Z[(size_t)i * n + j] = row[i];
    }
}

}  // namespace sfairsc
