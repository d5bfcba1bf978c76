// Small dense symmetric eigensolvers (host, FP64).
#pragma once

#include <vector>

namespace sfairsc {

// All eigenpairs.  A: n x n symmetric, row-major.  w: eigenvalues ascending.
// Z: row-major n x n with the eigenvector of w[j] in column j.
void sym_eig(int n, const double* A, double* w, double* Z);

// Eigenvalues, then eigenvectors of the m smallest only.
struct SymEigSel {
    int n = 0;
    double norm = 1.0;
    std::vector<double> w;  // all eigenvalues, ascending (after reduce)
    // Householder reduction to tridiagonal form and every eigenvalue.
    void reduce(int n, const double* A);
    // Eigenvectors of w[0..m-1] as the columns of Z (row-major n x m).
    void vectors(int m, double* Z);

   private:
    std::vector<double> refl, beta, d, e;
};

}  // namespace sfairsc
