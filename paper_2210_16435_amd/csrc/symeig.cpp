// Dense symmetric eigensolver for the small projected matrices of the
// Rayleigh-Ritz step (order <= a few hundred), FP64 on the host.
//
// Methods (Golub and Van Loan, Matrix Computations, Sections 8.3 and 8.2.2;
// Wilkinson, The Algebraic Eigenvalue Problem, Ch. 9):
//   * Householder reduction to tridiagonal form Q^T A Q = T (reflectors kept);
//   * all eigenvalues of T by implicitly shifted QL iterations;
//   * eigenvectors of T for the m wanted eigenvalues only, by inverse
//     iteration with a pivoted tridiagonal LU, re-orthogonalised within
//     clusters of close eigenvalues; then back-transformed, x = Q y.
// The full-vector variant (all n eigenvectors by accumulating every QL
// rotation) is kept for tests and tiny orders.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "symeig.h"

namespace sfairsc {

namespace {

constexpr double kEps = std::numeric_limits<double>::epsilon();

// sqrt(a^2 + b^2) without the overflow guards of std::hypot: the projected
// matrices here have entries bounded by the shift sigma, far from overflow.
inline double pyth(double a, double b) { return std::sqrt(a * a + b * b); }

struct Tridiag {
    int n = 0;
    std::vector<double> a;      // working matrix during the reduction
    std::vector<double> refl;   // reflector k (length n-k-1) at refl[k * n]
    std::vector<double> beta;   // reflector scalars (0: identity)
    std::vector<double> d, e;   // T = tridiag(e, d, e), e[i] couples i and i+1
};

// Householder reduction (row-major A, n x n, symmetric; only the lower
// triangle, j <= i, is read and updated).
void tridiagonalize(int n, const double* A, Tridiag& t) {
    t.n = n;
    t.a.assign(A, A + (size_t)n * n);
    t.refl.assign((size_t)n * n, 0.0);
    t.beta.assign(n, 0.0);
    t.d.assign(n, 0.0);
    t.e.assign(n, 0.0);
    std::vector<double>& a = t.a;
    std::vector<double> v(n), p(n), w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double sigma2 = 0.0;
        for (int i = 0; i < m; ++i) {
            v[i] = a[(size_t)(k + 1 + i) * n + k];
            sigma2 += v[i] * v[i];
        }
        const double norm = std::sqrt(sigma2);
        if (norm == 0.0) {
            t.e[k] = 0.0;
            continue;
        }
        const double alpha = v[0] >= 0 ? -norm : norm;
        v[0] -= alpha;
        double vtv = 0.0;
        for (int i = 0; i < m; ++i) vtv += v[i] * v[i];
        const double beta = 2.0 / vtv;
        t.e[k] = alpha;
        t.beta[k] = beta;
        // p = beta B v with B = a[k+1:, k+1:] from its lower triangle: row i
        // (entries j < i) contributes a dot product to p_i and an axpy to
        // p_j, both over contiguous memory;  then B <- B - v w^T - w v^T on
        // the lower triangle
        double* __restrict__ pp = p.data();
        const double* __restrict__ vv = v.data();
        for (int i = 0; i < m; ++i) pp[i] = 0.0;
        for (int i = 0; i < m; ++i) {
            const double* __restrict__ row = &a[(size_t)(k + 1 + i) * n + k + 1];
            const double vi = vv[i];
            double s0 = 0.0;
#pragma omp simd reduction(+ : s0)
            for (int j = 0; j < i; ++j) {
                s0 += row[j] * vv[j];
                pp[j] += vi * row[j];
            }
            pp[i] += s0 + row[i] * vi;
        }
        for (int i = 0; i < m; ++i) pp[i] *= beta;
        double ptv = 0.0;
        for (int i = 0; i < m; ++i) ptv += pp[i] * vv[i];
        const double kf = 0.5 * beta * ptv;
        double* __restrict__ ww = w.data();
        for (int i = 0; i < m; ++i) ww[i] = pp[i] - kf * vv[i];
        for (int i = 0; i < m; ++i) {
            double* __restrict__ row = &a[(size_t)(k + 1 + i) * n + k + 1];
            const double vi = vv[i], wi = ww[i];
            for (int j = 0; j <= i; ++j) row[j] -= vi * ww[j] + wi * vv[j];
        }
        // keep the reflector, contiguous
        for (int i = 0; i < m; ++i) t.refl[(size_t)k * n + i] = v[i];
    }
    for (int i = 0; i < n; ++i) t.d[i] = a[(size_t)i * n + i];
    // the last sub-diagonal entry is untouched by reflectors
    if (n >= 2) t.e[n - 2] = a[(size_t)(n - 1) * n + (n - 2)];
    t.e[n - 1] = 0.0;
}

// x <- Q x with Q = H_0 H_1 ... H_{n-3}: apply the last reflector first.
void apply_q(const Tridiag& t, double* x) {
    const int n = t.n;
    for (int k = n - 3; k >= 0; --k) {
        const double beta = t.beta[k];
        if (beta == 0.0) continue;
        const int m = n - k - 1;
        const double* v = &t.refl[(size_t)k * n];
        double* y = x + k + 1;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int i = 0;
        for (; i + 4 <= m; i += 4) {
            s0 += v[i] * y[i];
            s1 += v[i + 1] * y[i + 1];
            s2 += v[i + 2] * y[i + 2];
            s3 += v[i + 3] * y[i + 3];
        }
        for (; i < m; ++i) s0 += v[i] * y[i];
        const double s = beta * ((s0 + s1) + (s2 + s3));
        for (i = 0; i < m; ++i) y[i] -= s * v[i];
    }
}

// Implicit QL on tridiag(d, e); rotations applied to rows of Zt if given.
void tridiag_ql(int n, std::vector<double>& d, std::vector<double>& e, double* Zt) {
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= kEps * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = pyth(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i];
                const double bb = c * e[i];
                r = pyth(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = true;
                    break;
                }
                const double ir = 1.0 / r;
                s = f * ir;
                c = g * ir;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * bb;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - bb;
                if (Zt) {
                    double* zi = Zt + (size_t)i * n;
                    double* zj = Zt + (size_t)(i + 1) * n;
                    for (int t = 0; t < n; ++t) {
                        const double a = zi[t], bq = zj[t];
                        zj[t] = s * a + c * bq;
                        zi[t] = c * a - s * bq;
                    }
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
}

// LU factorisation of T - lam I with partial pivoting (tridiagonal: U has
// two super-diagonals); zero pivots replaced by +-tiny.  Stores reciprocal
// pivots so each solve is division-free.
struct TriLU {
    std::vector<double> ip, u1, u2, mult;  // 1/u0, super-diagonals, multipliers
    std::vector<char> swp;
    void factor(const std::vector<double>& d, const std::vector<double>& e, double lam, double tiny) {
        const int n = (int)d.size();
        ip.resize(n);
        u1.resize(n);
        u2.resize(n);
        mult.resize(n);
        swp.resize(n);
        double c0 = d[0] - lam, c1 = n > 1 ? e[0] : 0.0, c2 = 0.0;
        for (int i = 0; i + 1 < n; ++i) {
            const double s = e[i];
            const double n1 = d[i + 1] - lam;
            const double n2 = (i + 2 < n) ? e[i + 1] : 0.0;
            double u0, r1, r2;
            if (std::fabs(s) > std::fabs(c0)) {
                swp[i] = 1;
                u0 = s;
                u1[i] = n1;
                u2[i] = n2;
                const double mlt = c0 / s;
                mult[i] = mlt;
                r1 = c1 - mlt * n1;
                r2 = c2 - mlt * n2;
            } else {
                swp[i] = 0;
                if (std::fabs(c0) < tiny) c0 = c0 < 0 ? -tiny : tiny;
                u0 = c0;
                u1[i] = c1;
                u2[i] = c2;
                const double mlt = s / c0;
                mult[i] = mlt;
                r1 = n1 - mlt * c1;
                r2 = n2 - mlt * c2;
            }
            ip[i] = 1.0 / u0;
            c0 = r1;
            c1 = r2;
            c2 = 0.0;
        }
        if (std::fabs(c0) < tiny) c0 = c0 < 0 ? -tiny : tiny;
        ip[n - 1] = 1.0 / c0;
        u1[n - 1] = 0.0;
        u2[n - 1] = 0.0;
    }
    // b <- (T - lam I)^{-1} b
    void solve(double* b, int n) const {
        for (int i = 0; i + 1 < n; ++i) {
            if (swp[i]) std::swap(b[i], b[i + 1]);
            b[i + 1] -= mult[i] * b[i];
        }
        b[n - 1] *= ip[n - 1];
        if (n >= 2) b[n - 2] = (b[n - 2] - u1[n - 2] * b[n - 1]) * ip[n - 2];
        for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - u1[i] * b[i + 1] - u2[i] * b[i + 2]) * ip[i];
    }
};

}  // namespace

void sym_eig(int n, const double* A, double* w, double* Z) {
    if (n <= 0) return;
    if (n == 1) {
        w[0] = A[0];
        Z[0] = 1.0;
        return;
    }
    Tridiag t;
    tridiagonalize(n, A, t);
    // Zt = Q^T (row j = column j of Q), rotated along the QL iterations
    std::vector<double> Zt((size_t)n * n, 0.0);
    std::vector<double> col(n);
    for (int j = 0; j < n; ++j) {
        std::fill(col.begin(), col.end(), 0.0);
        col[j] = 1.0;
        apply_q(t, col.data());
        for (int i = 0; i < n; ++i) Zt[(size_t)j * n + i] = col[i];
    }
    std::vector<double> d = t.d, e = t.e;
    tridiag_ql(n, d, e, Zt.data());
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
    for (int j = 0; j < n; ++j) {
        const int src = order[j];
        w[j] = d[src];
        const double* row = &Zt[(size_t)src * n];
        for (int i = 0; i < n; ++i) Z[(size_t)i * n + j] = row[i];
    }
}

void SymEigSel::reduce(int n_, const double* A) {
    n = n_;
    w.assign(n > 0 ? n : 0, 0.0);
    if (n <= 0) return;
    Tridiag t;
    tridiagonalize(n, A, t);
    refl.swap(t.refl);
    beta.swap(t.beta);
    d.swap(t.d);
    e.swap(t.e);
    std::vector<double> dd = d, ee = e;
    tridiag_ql(n, dd, ee, nullptr);
    std::sort(dd.begin(), dd.end());
    w = dd;
    norm = 0.0;
    for (int i = 0; i < n; ++i)
        norm = std::max(norm, std::fabs(d[i]) + (i > 0 ? std::fabs(e[i - 1]) : 0.0) + std::fabs(e[i]));
    if (norm == 0.0) norm = 1.0;
}

void SymEigSel::vectors(int m, double* Z) {
    if (n == 1) {
        if (m >= 1) Z[0] = 1.0;
        return;
    }
    TriLU lu;
    std::vector<std::vector<double>> Y;  // eigenvectors of T
    Y.reserve(m);
    const double tiny = kEps * norm;
    const double cluster_gap = 1e-3 * norm;
    double prev_shift = -INFINITY;
    int cluster_start = 0;
    std::vector<double> x(n);
    for (int j = 0; j < m; ++j) {
        double lam = w[j];
        if (j > 0 && w[j] - w[j - 1] > cluster_gap) cluster_start = j;
        if (lam <= prev_shift + 10 * tiny) lam = prev_shift + 10 * tiny;  // separate equal shifts
        prev_shift = lam;
        lu.factor(d, e, lam, tiny);
        // start vector with no special alignment to any eigenvector
        for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.25 * (double)((i * 7 + j * 13) % 17) / 17.0;
        for (int it = 0; it < 3; ++it) {
            lu.solve(x.data(), n);
            for (int pass = 0; pass < 2; ++pass)
                for (int q = cluster_start; q < j; ++q) {
                    double dot = 0.0;
                    for (int i = 0; i < n; ++i) dot += Y[q][i] * x[i];
                    for (int i = 0; i < n; ++i) x[i] -= dot * Y[q][i];
                }
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm += x[i] * x[i];
            nrm = std::sqrt(nrm);
            if (!(nrm > 0.0) || !std::isfinite(nrm)) {
                for (int i = 0; i < n; ++i) x[i] = (i == j % n) ? 1.0 : 0.0;
                nrm = 1.0;
            }
            const double inv = 1.0 / nrm;
            for (int i = 0; i < n; ++i) x[i] *= inv;
        }
        Y.push_back(x);
    }
    // back-transform all m vectors at once: Z = Q Y with Z row-major n x m;
    // each reflector is applied as w = v^T Z[k+1:, :], Z[k+1:, :] -= beta v w^T
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) Z[(size_t)i * m + j] = Y[j][i];
    std::vector<double> wv(m);
    for (int k = n - 3; k >= 0; --k) {
        const double bk = beta[k];
        if (bk == 0.0) continue;
        const int len = n - k - 1;
        const double* v = &refl[(size_t)k * n];
        std::fill(wv.begin(), wv.end(), 0.0);
        for (int i = 0; i < len; ++i) {
            const double vi = v[i];
            const double* row = Z + (size_t)(k + 1 + i) * m;
            for (int j = 0; j < m; ++j) wv[j] += vi * row[j];
        }
        for (int j = 0; j < m; ++j) wv[j] *= bk;
        for (int i = 0; i < len; ++i) {
            const double vi = v[i];
            double* row = Z + (size_t)(k + 1 + i) * m;
            for (int j = 0; j < m; ++j) row[j] -= vi * wv[j];
        }
    }
}

}  // namespace sfairsc
