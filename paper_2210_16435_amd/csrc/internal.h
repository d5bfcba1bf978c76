// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sfairsc.h"
#include "ortho.h"
#include "rr.h"

namespace sfairsc {

// Library limits.
constexpr int kMaxBlock = 32;     // widest block of vectors (columns)
constexpr int kMaxGroups = 32;    // h
constexpr int kMaxBasis = 192;    // Krylov basis columns before a restart
constexpr int kMaxK = 64;         // wanted eigenpairs / k-means dimension
constexpr int kLdMax = kMaxBasis + kMaxBlock;  // basis leading dimension
// A relative gap (theta_{k+1} - theta_k) / sigma at most this multiple of the
// tolerance marks the k-dimensional eigenspace as not determined.
constexpr double kDegenerateGap = 100.0;

// Output-major partial sums by XCD: consecutive workgroups run on different
// XCDs (round robin over 8), so block blk's slot is (blk mod 8) per + blk / 8
// with per = ceil(nblk / 8): each XCD's blocks fill whole lines of a row
// (its L2 writes them back whole) and a row of 8 per slots is read
// contiguously.  Slots past nblk are never written and never read.
__host__ __device__ inline int xcd_row(int nblk) { return 8 * ((nblk + 7) >> 3); }
__host__ __device__ inline int xcd_slot(int blk, int nblk) { return (blk & 7) * ((nblk + 7) >> 3) + (blk >> 3); }
__device__ inline bool xcd_valid(int slot, int nblk) {
    const int per = (nblk + 7) >> 3;
    const int x = slot / per;
    return (slot - x * per) * 8 + x < nblk;
}

int set_error(int code, const char* fmt, ...);

#define SF_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            return ::sfairsc::set_error(SFAIRSC_E_HIP, "%s failed: %s", #call, \
                                        hipGetErrorString(e_));               \
    } while (0)

#define SF_TRY(expr)              \
    do {                          \
        int r_ = (expr);          \
        if (r_ != SFAIRSC_OK)     \
            return r_;            \
    } while (0)

// A device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need);
    void release();
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Workspace of the operator L^sigma for blocks up to kMaxBlock columns.
struct OpWork {
    int nblk_spmm = 0;  // partial-sum slots of the SpMM epilogue
    int nblk_proj = 0;  // partial-sum slots of the input projection
    DevBuf part_in;     // [nblk_proj][h][b] double (b <= 32)
    DevBuf part_out;    // [nblk_spmm][h][b] double (b <= 32)
    DevBuf small;       // R_in, S, R_out tables: 3 x [h][32] double
    DevBuf xp;          // projected input, n x BW (float or double)
    DevBuf t;           // sparse product output, n x BW (float or double)
    DevBuf xpad, ypad;  // padding copies for b not in {4, 8, 16, 32}
    DevBuf lc;          // L C (n x lcw, row-major, double): the constraint's image
    DevBuf ctlc;        // C^T L C ([h-1][32], double)
    int lcw = 0;        // row stride of lc; 0 until formed
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// Workspace of the Krylov-Schur solver.
struct EigWork {
    DevBuf V;       // n x ld basis (row-major), double
    DevBuf V2;      // second basis buffer (restart rotation target)
    DevBuf T;       // ld x ld projected matrix, double
    DevBuf part;    // tall-skinny partial sums
    DevBuf small;   // H1, H2, Gram, R, Rinv, coupling, flags ...
    DevBuf Q;       // ld x ld restart / rotation matrix
    DevBuf X;       // n x kMaxK output staging
    DevBuf opart;   // partial sums of the matrix-core passes
    DevBuf osmall;  // their reduced sums and coefficient matrices
    DevBuf rr;      // Rayleigh-Ritz kernel: scratch, eigenvalues, Ritz vectors, record
    // second stream: the Rayleigh-Ritz kernel runs beside the look-ahead
    // operator application of the solve's stream
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_wait = nullptr;
    // Pinned host staging for host-to-device uploads: a pageable source may
    // be read by the DMA engine after hipMemcpyAsync returns, so every
    // upload is first copied here and the region is only reused after the
    // stream has been synchronised.
    double* pin = nullptr;
    size_t pin_cap = 0, pin_off = 0;
};

struct KmWork {
    DevBuf d2, cs, cent, lab, best, part, misc;
};

struct GradWork {
    DevBuf hrow;  // H staged row-major for the backward kernel
};

// Workspace of a general constraint matrix (basis Q of range(C)).
struct ConWork {
    DevBuf part;   // per-block partial sums, kConMaxBlocks x 32 x 32 doubles
    DevBuf small;  // reduced sums and small coefficient matrices
    DevBuf cbuf;   // C during set-up, n x qld
};
constexpr int kConMaxBlocks = 256;

// A sparse 0/1 membership matrix G (n x m) whose projection is computed by
// LSQR (C = D^{-1/2} (G - 1 z^T) or G - 1 z^T).
constexpr int kMaxMembers = 1 << 20;
struct Memb {
    int m = 0, nseg = 0;
    double inner_tol = 1e-12;
    int max_inner = 200;
    int32_t* grow = nullptr;       // [n+1] memberships of each vertex
    int32_t* gcol = nullptr;       // [nnz_G]
    int32_t* tcol = nullptr;       // [nnz_G] members of each group, by group
    int32_t* seg_start = nullptr;  // [nseg+1] segments of tcol (<= 1024 members)
    int32_t* seg_group = nullptr;  // [nseg]
    int32_t* gseg = nullptr;       // [m+1] segments of each group
    double* z = nullptr;           // [m] column means (0 without centring)
    long long* stats = nullptr;    // solves, steps, max steps, unconverged columns
    DevBuf work;                   // u, v, d, x, x1, sums, partials
};

}  // namespace sfairsc

struct sfairsc_graph {
    int64_t n = 0, nnz = 0;
    int h = 1, normalized = 0, value_dtype = SFAIRSC_F64;
    int device = 0;
    double sigma = 0.0, dmin = 0.0, dmax = 0.0;
    int32_t* rowptr = nullptr;  // [n+1]
    int32_t* col = nullptr;     // [nnz]
    int32_t* grp = nullptr;     // [n]
    void* wval = nullptr;       // [nnz] original weights (value dtype)
    double* val64 = nullptr;    // [nnz] off-diagonal magnitudes: w or w-hat
    float* val32 = nullptr;     // [nnz] the same rounded to float
    double* diag64 = nullptr;   // [n] d (unnormalized) or 1 (normalized)
    float* diag32 = nullptr;    // [n]
    double* cs = nullptr;       // [n] d^{-1/2} (normalized); nullptr otherwise
    double* deg = nullptr;      // [n] degrees
    double* gpar = nullptr;     // device: p[h], Ginv[(h-1)^2]
    std::vector<int64_t> count; // group sizes
    std::vector<double> p;      // group fractions |V_s| / n
    std::vector<double> ginv;   // (C^T C)^{-1}, (h-1) x (h-1)
    // General constraint (replaces the group form when set): Q, row-major
    // n x qld with qld in {4, 8, 16, 32}, orthonormal columns spanning
    // range(C), columns qrank..qld-1 zero.
    double* qbas = nullptr;
    int qrank = 0, qld = 0;
    // Sparse membership constraint projected by LSQR (replaces both forms).
    sfairsc::Memb* memb = nullptr;
    sfairsc::OpWork op;
    sfairsc::EigWork eig;
    sfairsc::KmWork km;
    sfairsc::GradWork gw;
    sfairsc::ConWork cw;
};

namespace sfairsc {

// Dimension of the constrained subspace: n minus the number of independent
// constraints (h - 1 groups, or the rank of a general F).
// (a membership matrix counts m, an upper bound of its rank).
inline int64_t free_dim(const sfairsc_graph* g) {
    return g->memb ? g->n - g->memb->m : g->qbas ? g->n - g->qrank : g->n - g->h + 1;
}

// Apply Y = L^sigma X for X, Y in row-major blocks with leading dimensions.
// b <= 32.  mixed = float sparse product.  If timing events are given, the
// SpMM launch is bracketed by them (ev_begin recorded before, ev_end after).
int op_apply(sfairsc_graph* g, const double* X, int ldx, double* Y, int ldy,
             int b, int mixed, double sigma, hipStream_t s,
             hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr,
             const int* skip_flag = nullptr);

// X <- P X = X - C (C^T C)^{-1} C^T X in place (X double, ldx, b <= 32).
int op_project(sfairsc_graph* g, double* X, int ldx, int b, hipStream_t s);

// General constraint (g->qbas set): the projection steps of the operator
// with P = I - Q Q^T.
//   gen_project_in:  S = Q^T X (kept in the handle's workspace) and
//                    X' = X - Q S written compact (stride BW) as float or double.
//   gen_correct:     Y = T - Q (Q^T T - sigma S), T compact stride BW (float
//                    or double), Y double with leading dimension ldy.
//   gen_project:     X <- X - Q Q^T X in place.
int gen_project_in(sfairsc_graph* g, const double* X, int ldx, int b, int BW, bool to_float, void* Xp,
                   hipStream_t s, const int* skip);
int gen_correct(sfairsc_graph* g, const void* T, bool t_float, int BW, int b, double sigma, double* Y, int ldy,
                hipStream_t s, const int* skip);
int gen_project(sfairsc_graph* g, double* X, int ldx, int b, hipStream_t s);

// The same three steps for a membership constraint, each one LSQR solve
// (one cooperative launch).  lsqr_correct uses the solution of the last
// lsqr_project_in: Y = T - C (x_T - sigma x_X).
int lsqr_project_in(sfairsc_graph* g, const double* X, int ldx, int b, int BW, bool to_float, void* Xp,
                    hipStream_t s, const int* skip);
int lsqr_correct(sfairsc_graph* g, const void* T, bool t_float, int BW, int b, double sigma, double* Y, int ldy,
                 hipStream_t s, const int* skip);
int lsqr_project(sfairsc_graph* g, double* X, int ldx, int b, hipStream_t s);
void free_memb(sfairsc_graph* g);

// Layout of EigWork::rr (doubles): kernel scratch, then the eigenvalues,
// the first k Ritz vectors (c x k), the host record and a c x c block for
// the eigenvectors of the small-matrix calls.
struct RrBufs {
    double* work;
    double* theta;
    double* zk;
    double* rec;
    double* zout;
};
int rr_buffers(sfairsc_graph* g, RrBufs* out);

// All eigenpairs of a small symmetric device matrix (order c <= kMaxBasis,
// row-major, leading dimension ldt), copied to the host: w ascending, Z
// row-major c x c with the eigenvector of w[j] in column j.  Runs the
// Rayleigh-Ritz kernel on `s` and synchronises it (set-up and repair paths).
int small_eig_host(sfairsc_graph* g, const double* dT, int c, int ldt, double* w, double* Z, hipStream_t s);

// Free the per-device workspaces of batched launches (device buffers, pinned
// host buffer, events).  Called when the last graph handle is destroyed.
void batched_release_workspaces();

// The operator up to (not including) the output deflation: SpMM with its
// C^T epilogue sums and the deflation tables.  The caller forms
// Y_i = T_i - c_i rtab[g_i] - sum_{s < m} lc[i][s] utab[s] (fused into its
// next pass); with lc == nullptr the last term is absent.
struct OpOut {
    const void* t;       // n x BW compact, float if is_float else double
    bool is_float;
    int BW;
    const double* rtab;  // [h][32]; nullptr: t already holds Y (general constraint)
    const double* lc = nullptr;    // L C, n x lcw (double); nullptr: T = L P X already
    int lcw = 0, m = 0;            // its row stride and columns (h - 1)
    const double* utab = nullptr;  // U_in = G^{-1} C^T X, [m][32]
};
// L C and C^T L C for the operator's reassociated form (group constraint,
// h >= 2); a no-op otherwise or when already formed.
int op_prepare_lc(sfairsc_graph* g, hipStream_t s);
// prepared_nblk > 0: the compact input (op.xp) and its per-block group sums
// (op.part_in, that many blocks) were already written, by the
// orthogonalisation pass that produced X (see op_input_target).
int op_apply_t(sfairsc_graph* g, const double* X, int ldx, int b, int mixed, double sigma, hipStream_t s,
               hipEvent_t ev_begin, hipEvent_t ev_end, const int* skip, OpOut* out, int prepared_nblk = 0);
// Where a producer of the operator's next input writes it (compact copy,
// group-sum partials), when op_apply_t takes a prepared input for block
// width b: both null otherwise.
struct OpInput {
    void* xp;
    double* xsum;
};
int op_input_target(sfairsc_graph* g, int b, OpInput* in);

// Raw sparse product T = L X (no projection), X/T compact row-major n x b.
int op_spmm_raw(sfairsc_graph* g, const void* X, void* T, int b, int mixed,
                hipStream_t s);


}  // namespace sfairsc
