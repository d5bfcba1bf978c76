// Checks the library's small dense symmetric eigensolvers (host code):
// A z_j = w_j z_j, Z^T Z = I and ascending w, for random and clustered
// spectra.  Prints one line per case: n, kind, residual, orthogonality,
// ordering violation, for both the full and the selective solver.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "symeig.h"

static void check(int n, const std::vector<double>& A, const std::vector<double>& w, const std::vector<double>& Z,
                  int m, double* res, double* orth, double* order) {
    double r = 0.0, o = 0.0, od = 0.0, an = 0.0;
    for (double v : A) an = std::fmax(an, std::fabs(v));
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += A[(size_t)i * n + q] * Z[(size_t)q * m + j];
            r = std::fmax(r, std::fabs(s - w[j] * Z[(size_t)i * m + j]));
        }
    for (int a = 0; a < m; ++a)
        for (int c = 0; c < m; ++c) {
            double s = 0.0;
            for (int q = 0; q < n; ++q) s += Z[(size_t)q * m + a] * Z[(size_t)q * m + c];
            o = std::fmax(o, std::fabs(s - (a == c ? 1.0 : 0.0)));
        }
    for (int j = 1; j < (int)w.size(); ++j) od = std::fmax(od, w[j - 1] - w[j]);
    *res = r / (an > 0 ? an : 1.0);
    *orth = o;
    *order = od;
}

int main() {
    std::mt19937_64 rng(20230419);
    std::normal_distribution<double> nd;
    for (int n : {1, 2, 3, 4, 7, 8, 16, 33, 64, 100}) {
        for (int kind = 0; kind < 2; ++kind) {
            // kind 0: random symmetric; kind 1: Q diag(clustered) Q^T
            std::vector<double> A((size_t)n * n, 0.0);
            if (kind == 0) {
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = nd(rng);
            } else {
                std::vector<double> d(n), Q((size_t)n * n);
                for (int i = 0; i < n; ++i) d[i] = (i % 3 == 0) ? 1.0 : (i % 3 == 1 ? 1.0 + 1e-9 * i : 5.0);
                for (double& v : Q) v = nd(rng);
                for (int j = 0; j < n; ++j) {  // Gram-Schmidt columns
                    for (int p = 0; p < j; ++p) {
                        double s = 0.0;
                        for (int i = 0; i < n; ++i) s += Q[(size_t)i * n + p] * Q[(size_t)i * n + j];
                        for (int i = 0; i < n; ++i) Q[(size_t)i * n + j] -= s * Q[(size_t)i * n + p];
                    }
                    double s = 0.0;
                    for (int i = 0; i < n; ++i) s += Q[(size_t)i * n + j] * Q[(size_t)i * n + j];
                    s = std::sqrt(s);
                    for (int i = 0; i < n; ++i) Q[(size_t)i * n + j] /= s;
                }
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        double s = 0.0;
                        for (int q = 0; q < n; ++q) s += Q[(size_t)i * n + q] * d[q] * Q[(size_t)j * n + q];
                        A[(size_t)i * n + j] = s;
                    }
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i];
            }
            std::vector<double> w(n), Z((size_t)n * n);
            sfairsc::sym_eig(n, A.data(), w.data(), Z.data());
            double r, o, od;
            check(n, A, w, Z, n, &r, &o, &od);
            std::printf("full %d %d %.3e %.3e %.3e\n", n, kind, r, o, od);
            sfairsc::SymEigSel sel;
            sel.reduce(n, A.data());
            const int m = (n + 1) / 2;
            std::vector<double> Zs((size_t)n * m);
            sel.vectors(m, Zs.data());
            check(n, A, sel.w, Zs, m, &r, &o, &od);
            double dw = 0.0;
            for (int j = 0; j < n; ++j) dw = std::fmax(dw, std::fabs(sel.w[j] - w[j]));
            std::printf("sel %d %d %.3e %.3e %.3e %.3e\n", n, kind, r, o, od, dw);
        }
    }
    return 0;
}
