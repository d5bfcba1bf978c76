// Dense symmetric eigensolver for the small projected matrices of the
// Rayleigh-Ritz step (order <= a few hundred), FP64 on the host.
//
// Methods (Golub and Van Loan, Matrix Computations, Sections 8.3 and 8.2.2;
// Wilkinson, The Algebraic Eigenvalue Problem, Ch. 9):
//   * Householder reduction to tridiagonal form Q^T A Q = T (reflectors kept);
//   * all eigenvalues of T by implicitly shifted QL iterations (root-free
//     for the selective solver, with rotations for the full one);
//   * eigenvectors of T for the m wanted eigenvalues only, by inverse
//     iteration with a pivoted tridiagonal LU (several shifts in lockstep),
//     re-orthogonalised within clusters of close eigenvalues; then
//     back-transformed, x = Q y.
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
constexpr int kLanes = 8;  // shifts whose inverse iterations run in lockstep
constexpr int kWY = 4;     // reflectors applied together in the back-transform

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

// Eigenvalues only: root-free implicit QL (Pal, Walker and Kahan; Parlett,
// The Symmetric Eigenvalue Problem, Section 8.15).  The sweep carries the
// squares of the off-diagonal entries, E[i] = e[i]^2, and of the rotation
// cosines and sines, so no rotation takes a square root: with the shift
// sigma, gamma_i = C_i (d_i - sigma) - S_i gamma_{i+1} is the running
// diagonal remainder and P = gamma^2 / C the square of the entry the next
// rotation eliminates.  The shift is the eigenvalue of the leading 2 x 2
// closer to its first entry (one square root per sweep).
void tridiag_ql_values(int n, std::vector<double>& d, std::vector<double>& e) {
    std::vector<double> E(n, 0.0);
    for (int i = 0; i + 1 < n; ++i) E[i] = e[i] * e[i];
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (E[m] <= kEps * kEps * dd * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) break;
            const double el = std::sqrt(E[l]);
            const double g0 = (d[l + 1] - d[l]) / (2.0 * el);
            const double r0 = pyth(g0, 1.0);
            const double sigma = d[l] - el / (g0 + std::copysign(r0, g0));
            double C = 1.0, S = 0.0;
            double gamma = d[m] - sigma;
            double P = gamma * gamma;
            for (int i = m - 1; i >= l; --i) {
                const double bb = E[i];
                const double R = P + bb;
                // 1 / C = R / P: the reciprocal of P is taken beside R's, so
                // the next P needs no division after gamma
                const double ip = 1.0 / P;
                if (i != m - 1) E[i + 1] = S * R;
                const double cold = C;
                const double ir = 1.0 / R;
                C = P * ir;
                S = bb * ir;
                const double gold = gamma;
                const double alpha = d[i];
                gamma = C * (alpha - sigma) - S * gold;
                d[i + 1] = gold + (alpha - gamma);
                P = C != 0.0 ? gamma * gamma * (R * ip) : cold * bb;
            }
            E[l] = S * P;
            d[l] = sigma + gamma;
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
    tridiag_ql_values(n, dd, ee);
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
    const double tiny = kEps * norm;
    const double cluster_gap = 1e-3 * norm;
    // shifts (equal ones pulled apart) and the first index of each one's
    // cluster of close eigenvalues
    std::vector<double> shift(m);
    std::vector<int> cstart(m);
    {
        double prev = -INFINITY;
        int c0 = 0;
        for (int j = 0; j < m; ++j) {
            double lam = w[j];
            if (j > 0 && w[j] - w[j - 1] > cluster_gap) c0 = j;
            if (lam <= prev + 10 * tiny) lam = prev + 10 * tiny;
            prev = lam;
            shift[j] = lam;
            cstart[j] = c0;
        }
    }
    // Inverse iteration on kLanes shifts at once: the factorisations and
    // solves of the lanes are independent, so their division chains overlap
    // (lane-interleaved arrays, element i of lane q at [i * kLanes + q]).
    // The pivot choices differ per lane and are taken by selects.
    constexpr int L = kLanes;
    std::vector<double> Y((size_t)m * n);  // final eigenvectors of T, one per row
    std::vector<double> ip((size_t)n * L), u1((size_t)n * L), u2((size_t)n * L), mlt((size_t)n * L), x((size_t)n * L),
        xs((size_t)L * n);
    std::vector<unsigned char> swp((size_t)n * L);
    for (int j0 = 0; j0 < m; j0 += L) {
        const int na = std::min(L, m - j0);
        double lam[L];
        for (int q = 0; q < L; ++q) lam[q] = shift[j0 + std::min(q, na - 1)];
        // pivoted LU of T - lam I per lane (U has two super-diagonals)
        {
            double c0[L], c1[L];
            for (int q = 0; q < L; ++q) {
                c0[q] = d[0] - lam[q];
                c1[q] = e[0];
            }
            for (int i = 0; i + 1 < n; ++i) {
                const double sd = e[i];
                const double n2 = (i + 2 < n) ? e[i + 1] : 0.0;
#pragma omp simd
                for (int q = 0; q < L; ++q) {
                    const double n1 = d[i + 1] - lam[q];
                    const bool sw = std::fabs(sd) > std::fabs(c0[q]);
                    const double ct = std::fabs(c0[q]) < tiny ? (c0[q] < 0 ? -tiny : tiny) : c0[q];
                    const double piv = sw ? sd : ct;
                    const double inv = 1.0 / piv;
                    const double m_ = (sw ? c0[q] : sd) * inv;
                    const double v1 = sw ? n1 : c1[q];
                    const double v2 = sw ? n2 : 0.0;
                    swp[(size_t)i * L + q] = sw;
                    ip[(size_t)i * L + q] = inv;
                    mlt[(size_t)i * L + q] = m_;
                    u1[(size_t)i * L + q] = v1;
                    u2[(size_t)i * L + q] = v2;
                    c0[q] = (sw ? c1[q] : n1) - m_ * v1;
                    c1[q] = (sw ? 0.0 : n2) - m_ * v2;
                }
            }
            for (int q = 0; q < L; ++q) {
                const double ct = std::fabs(c0[q]) < tiny ? (c0[q] < 0 ? -tiny : tiny) : c0[q];
                ip[(size_t)(n - 1) * L + q] = 1.0 / ct;
                u1[(size_t)(n - 1) * L + q] = 0.0;
                u2[(size_t)(n - 1) * L + q] = 0.0;
            }
        }
        // start vectors with no special alignment to any eigenvector
        for (int i = 0; i < n; ++i)
            for (int q = 0; q < L; ++q)
                x[(size_t)i * L + q] = 1.0 + 0.25 * (double)((i * 7 + (j0 + q) * 13) % 17) / 17.0;
        for (int it = 0; it < 3; ++it) {
            // x <- (T - lam I)^{-1} x, every lane
            for (int i = 0; i + 1 < n; ++i) {
#pragma omp simd
                for (int q = 0; q < L; ++q) {
                    const double a = x[(size_t)i * L + q], bq = x[(size_t)(i + 1) * L + q];
                    const bool sw = swp[(size_t)i * L + q];
                    const double lo = sw ? bq : a, hi = sw ? a : bq;
                    x[(size_t)i * L + q] = lo;
                    x[(size_t)(i + 1) * L + q] = hi - mlt[(size_t)i * L + q] * lo;
                }
            }
            for (int q = 0; q < L; ++q) x[(size_t)(n - 1) * L + q] *= ip[(size_t)(n - 1) * L + q];
            for (int q = 0; q < L; ++q)
                x[(size_t)(n - 2) * L + q] =
                    (x[(size_t)(n - 2) * L + q] - u1[(size_t)(n - 2) * L + q] * x[(size_t)(n - 1) * L + q]) *
                    ip[(size_t)(n - 2) * L + q];
            for (int i = n - 3; i >= 0; --i) {
#pragma omp simd
                for (int q = 0; q < L; ++q)
                    x[(size_t)i * L + q] = (x[(size_t)i * L + q] - u1[(size_t)i * L + q] * x[(size_t)(i + 1) * L + q] -
                                            u2[(size_t)i * L + q] * x[(size_t)(i + 2) * L + q]) *
                                           ip[(size_t)i * L + q];
            }
            // lane by lane, on contiguous copies: orthogonalise against the
            // earlier vectors of the same cluster (finished ones, then this
            // group's earlier lanes), twice, and normalise
            for (int i = 0; i < n; ++i)
                for (int q = 0; q < L; ++q) xs[(size_t)q * n + i] = x[(size_t)i * L + q];
            for (int q = 0; q < na; ++q) {
                const int j = j0 + q;
                double* __restrict__ xq = &xs[(size_t)q * n];
                for (int pass = 0; pass < 2; ++pass) {
                    for (int r = cstart[j]; r < j; ++r) {
                        const double* __restrict__ y = r < j0 ? &Y[(size_t)r * n] : &xs[(size_t)(r - j0) * n];
                        double dot = 0.0;
#pragma omp simd reduction(+ : dot)
                        for (int i = 0; i < n; ++i) dot += y[i] * xq[i];
#pragma omp simd
                        for (int i = 0; i < n; ++i) xq[i] -= dot * y[i];
                    }
                }
                double nrm = 0.0;
#pragma omp simd reduction(+ : nrm)
                for (int i = 0; i < n; ++i) nrm += xq[i] * xq[i];
                nrm = std::sqrt(nrm);
                if (!(nrm > 0.0) || !std::isfinite(nrm)) {
                    for (int i = 0; i < n; ++i) xq[i] = (i == j % n) ? 1.0 : 0.0;
                    nrm = 1.0;
                }
                const double inv = 1.0 / nrm;
                for (int i = 0; i < n; ++i) xq[i] *= inv;
            }
            for (int i = 0; i < n; ++i)
                for (int q = 0; q < L; ++q) x[(size_t)i * L + q] = xs[(size_t)q * n + i];
        }
        for (int q = 0; q < na; ++q)
            for (int i = 0; i < n; ++i) Y[(size_t)(j0 + q) * n + i] = xs[(size_t)q * n + i];
    }
    // back-transform all m vectors at once: Z = Q Y with Z row-major n x m.
    // Q = H_0 H_1 ... H_{n-3} is applied from the last reflector down, kWY
    // reflectors at a time in compact WY form (Schreiber and Van Loan):
    // H_kb ... H_{kb+nb-1} = I - V T V^T with V the block's reflectors as
    // columns and T upper triangular, T[0:i, i] = -beta_i T[0:i, 0:i]
    // V[:, 0:i]^T v_i, T[i, i] = beta_i; then Z <- Z - V (T (V^T Z)), two
    // sweeps over Z per block instead of two per reflector.
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) Z[(size_t)i * m + j] = Y[(size_t)j * n + i];
    const int nref = n - 2;  // reflectors 0 .. n-3
    if (nref <= 0) return;
    constexpr int NB = kWY;
    std::vector<double> V((size_t)n * NB), W((size_t)NB * m), W2((size_t)NB * m);
    double T[NB][NB];
    for (int kb = ((nref - 1) / NB) * NB; kb >= 0; kb -= NB) {
        const int nb = std::min(NB, nref - kb);
        const int r0 = kb + 1;      // first row the block touches
        const int rows = n - r0;
        // V[row][r]: reflector kb + r acts on rows r0 + r .. n - 1
        for (int row = 0; row < rows; ++row)
            for (int r = 0; r < NB; ++r)
                V[(size_t)row * NB + r] =
                    (r < nb && row >= r) ? refl[(size_t)(kb + r) * n + (row - r)] : 0.0;
        for (int i = 0; i < NB; ++i)
            for (int r = 0; r < NB; ++r) T[i][r] = 0.0;
        for (int i = 0; i < nb; ++i) {
            const double tau = beta[kb + i];
            double u[NB];
            for (int r = 0; r < i; ++r) {
                double acc = 0.0;
                for (int row = i; row < rows; ++row) acc += V[(size_t)row * NB + r] * V[(size_t)row * NB + i];
                u[r] = acc;
            }
            for (int r = 0; r < i; ++r) {
                double acc = 0.0;
                for (int q = r; q < i; ++q) acc += T[r][q] * u[q];
                T[r][i] = -tau * acc;
            }
            T[i][i] = tau;
        }
        // W = V^T Z[r0:, :]
        std::fill(W.begin(), W.begin() + (size_t)nb * m, 0.0);
        for (int row = 0; row < rows; ++row) {
            const double* __restrict__ zr = Z + (size_t)(r0 + row) * m;
            const int rmax = std::min(nb, row + 1);
            for (int r = 0; r < rmax; ++r) {
                const double vr = V[(size_t)row * NB + r];
                double* __restrict__ wr = &W[(size_t)r * m];
#pragma omp simd
                for (int j = 0; j < m; ++j) wr[j] += vr * zr[j];
            }
        }
        // W2 = T W
        for (int r = 0; r < nb; ++r) {
            double* __restrict__ w2 = &W2[(size_t)r * m];
            for (int j = 0; j < m; ++j) w2[j] = 0.0;
            for (int q = r; q < nb; ++q) {
                const double tq = T[r][q];
                const double* __restrict__ wq = &W[(size_t)q * m];
#pragma omp simd
                for (int j = 0; j < m; ++j) w2[j] += tq * wq[j];
            }
        }
        // Z[r0:, :] -= V W2
        for (int row = 0; row < rows; ++row) {
            double* __restrict__ zr = Z + (size_t)(r0 + row) * m;
            const int rmax = std::min(nb, row + 1);
            for (int r = 0; r < rmax; ++r) {
                const double vr = V[(size_t)row * NB + r];
                const double* __restrict__ w2 = &W2[(size_t)r * m];
#pragma omp simd
                for (int j = 0; j < m; ++j) zr[j] -= vr * w2[j];
            }
        }
    }
}

}  // namespace sfairsc
