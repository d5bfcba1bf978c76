// Small dense symmetric eigensolver (host, FP64).
#pragma once

namespace sfairsc {

// A: n x n symmetric, row-major.  w: eigenvalues ascending.  Z: row-major
// n x n with the eigenvector of w[j] in column j.
void sym_eig(int n, const double* A, double* w, double* Z);

}  // namespace sfairsc
