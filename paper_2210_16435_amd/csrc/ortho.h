// Block orthogonalisation of one Krylov expansion on the matrix cores.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sfairsc {

struct OrthoArgs {
    double* V;          // basis, row-major n x ld
    int ld;
    int64_t n;
    int cv;             // columns [0, cv) to orthogonalise against (incl. V_next)
    int b;              // block width; the new block lands in V[:, cv : cv + b]
    const void* t;      // sparse-product output (compact n x BW)
    bool t_is_float;
    int BW;
    const int32_t* grp;
    const double* cs;   // d^{-1/2} or nullptr
    const double* rtab; // deflation table [h][32]; nullptr: t already holds Y
    const double* lc = nullptr;    // L C (n x lcw): Y_i also loses LC_i utab
    int lcw = 0, m = 0;            // its row stride (>= 4) and columns
    const double* utab = nullptr;  // [m][32]
    double* T;          // projected matrix (device, ldt x ldt)
    int ldt;
    double thresh;      // Cholesky pivot threshold (rank deficiency)
    double* part;       // partial sums, ortho_part_doubles(n)
    double* small;      // ortho_small_doubles()
    double* gsave;      // b x b Gram of the failed block (repair path)
    double* rc;         // coupling R (b x b) on success
    int* flag;          // flag[0] = failure, flag[1] = its column,
                        // flag[2] = 1 (first Cholesky) or 2 (second)
    hipStream_t stream;
    // optional (block widths 4 and 8): the new block as the operator's next
    // input, written by the last pass: its compact copy (n x b, float when
    // xp_float) and per-block sums of c_i x_i per group (h groups, output-
    // major by XCD slot over ortho_nblk(n) blocks)
    void* xp = nullptr;
    bool xp_float = false;
    double* xsum = nullptr;
    int h = 0;
};

// Workgroups of the expansion's last pass when it writes the operator's
// input (the blocks of xsum).
int ortho_nblk(int64_t n);

size_t ortho_part_doubles(int64_t n);
size_t ortho_small_doubles();

// R1 (b x b, the first Cholesky factor of the last expansion) inside `small`.
double* ortho_r1(double* small);

// Passes A-D of the expansion (see ortho.hip).  Asynchronous.
int ortho_expand(const OrthoArgs& a);

// Cholesky-QR twice of the start block V[:, 0:b] on the matrix cores.
int ortho_start(double* V, int ld, int64_t n, int b, const double* ident, double thresh, double* part, double* small,
                double* gsave, double* rc, int* flag, hipStream_t s);

// Out[i, 0:b] = rscale_i (V[i, 0:kin] M) on the matrix cores (M kin x b
// row-major, b <= 32, kin a multiple of 4; Out row-major with leading
// dimension ldo; rscale optional).
int ortho_product(double* V, int ld, int64_t n, int kin, const double* M, int b, double* Out, int ldo,
                  const double* rscale, hipStream_t s);

// Layout of the thick-restart rotation's factor, which the Rayleigh-Ritz
// kernel writes and ortho_rotate reads (c basis columns, p kept, block b):
//  * rot_whole(c, b): M = [Z[:, 0:p] 0; 0 I_b] ((c + b) x (p + b)) in slices
//    of 48 columns (slice t: (c + b) x wt row-major), one update per slice
//    (while a slice fits 64 KB of LDS);
//  * otherwise Z[:, 0:p] in slices of 32 columns (slice t: c x wt), then the
//    b x b identity, which moves the next block in an update of its own
//    (reading b columns rather than c + b for every slice).
__host__ __device__ inline bool rot_whole(int c, int b) { return (c + b) * 48 * 8 <= 64 * 1024; }

// Thick-restart rotation into a second basis buffer (see ortho.hip); every
// launch returns at once while *skip is nonzero.
int ortho_rotate(double* V, double* Vout, int ld, int64_t n, int c, int p, int b, const double* Qchunks,
                 hipStream_t s, const int* skip = nullptr);

}  // namespace sfairsc
