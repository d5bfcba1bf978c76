// A general constraint matrix F (n x m, any m <= 32 columns, any rank).
//
// The method needs F only through the projector P = I - C (C^T C)^{-1} C^T
// with C = D^{-1/2} F (normalized) or C = F (eq. mv-Pw, Section 3.2); the
// group structure of Lemma 2.1 is what makes the default path cheap, not
// what makes it correct.  The random-Laplacian workload of Section 5 uses a
// random placeholder F, and overlapping groups (Section 6) give an F that
// may lose rank, for which a rank-revealing factorization comes first.
//
// Set-up (once per constraint): C is formed row-major (optionally after
// centring the columns of F, which turns overlapping 0/1 memberships into
// F_0 = G - 1 z^T), its Gram matrix C^T C is reduced on the GPU and
// diagonalised on the host.  Directions whose singular value is below
// rank_tol times the largest are dropped (the rank-revealing step); the
// kept ones give Q1 = C U_r diag(w_r)^{-1/2}, which has orthonormal columns
// up to about eps kappa^2, and Cholesky-QR passes on Q1 (at most three,
// until Q^T Q = I to 1e-12) give Q, orthonormal, with range(Q) = range(C)
// to rounding.  Then P = I - Q Q^T.
//
// The operator's projection steps become tall-skinny products with Q:
// S = Q^T X (per-block partials, reduced in a fixed order), X' = X - Q S,
// and after the sparse product Y = T - Q (Q^T T - sigma S).  Each is one
// pass over n rows reading a row of Q (qld doubles) beside the row of X:
// HBM-bound, so vector FMAs, not matrix cores.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "reduce.h"

namespace sfairsc {

constexpr int kConThreads = 256;

static int con_width(int m) { return m <= 4 ? 4 : m <= 8 ? 8 : m <= 16 ? 16 : 32; }

static int pow2_at_least(int b) {
    int p = 1;
    while (p < b) p <<= 1;
    return p;
}

static int con_blocks(int64_t rows, int rows_per_block) {
    int64_t g = (rows + rows_per_block - 1) / rows_per_block;
    if (g < 1) g = 1;
    if (g > kConMaxBlocks) g = kConMaxBlocks;
    return (int)g;
}

// part[block][t * b + j] = sum over the block's rows i of Q[i][t] X[i][j]
// for t < r, j < b.  BW threads per row (BW a power of two >= b), rows
// strided by the grid; the row slots of a wavefront are combined with
// shuffles, the four wavefronts through LDS.
template <int RP, class TT>
__global__ __launch_bounds__(kConThreads) void k_qt_partial(const TT* __restrict__ X, int ldx, int b, int BW,
                                                             int64_t n, const double* __restrict__ Q, int r,
                                                             double* __restrict__ part, const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[kConThreads / 64][RP][32];
    const int tid = threadIdx.x;
    const int j = tid & (BW - 1);
    const int rs = tid / BW;
    const int rb = kConThreads / BW;
    double acc[RP];
#pragma unroll
    for (int t = 0; t < RP; ++t) acc[t] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * rb + rs; i < n; i += (int64_t)gridDim.x * rb) {
        const double x = j < b ? (double)X[i * ldx + j] : 0.0;
        const double2* q = reinterpret_cast<const double2*>(Q + i * RP);
#pragma unroll
        for (int t = 0; t < RP / 2; ++t) {
            const double2 v = q[t];
            acc[2 * t] += v.x * x;
            acc[2 * t + 1] += v.y * x;
        }
    }
    for (int off = BW; off < 64; off <<= 1) {
#pragma unroll
        for (int t = 0; t < RP; ++t) acc[t] += __shfl_xor(acc[t], off);
    }
    const int lane = tid & 63, w = tid >> 6;
    if (lane < BW) {
#pragma unroll
        for (int t = 0; t < RP; ++t) red[w][t][lane] = acc[t];
    }
    __syncthreads();
    const int O = r * b;
    for (int e = tid; e < O; e += kConThreads) {
        const int t = e / b, jj = e - t * b;
        double s = red[0][t][jj];
        for (int q = 1; q < kConThreads / 64; ++q) s += red[q][t][jj];
        part[(size_t)blockIdx.x * O + e] = s;
    }
}

// Xp[i][j] = X[i][j] - sum_t Q[i][t] S[t][j] (j < b), 0 for b <= j < BW;
// compact stride BW in type OT.
template <class OT>
__global__ __launch_bounds__(kConThreads) void k_qs_apply(const double* __restrict__ X, int ldx, int b, int BW,
                                                           int64_t n, const double* __restrict__ Q, int RP, int r,
                                                           const double* __restrict__ S, OT* __restrict__ Xp,
                                                           const int* skip) {
    if (skip && *skip) return;
    __shared__ double Ss[32 * 32];
    for (int e = threadIdx.x; e < r * b; e += kConThreads) Ss[e] = S[e];
    __syncthreads();
    const int64_t total = n * BW;
    for (int64_t idx = blockIdx.x * (int64_t)kConThreads + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kConThreads) {
        const int64_t i = idx / BW;
        const int j = (int)(idx - i * BW);
        double v = 0.0;
        if (j < b) {
            v = X[i * ldx + j];
            const double* q = Q + i * RP;
            for (int t = 0; t < r; ++t) v -= q[t] * Ss[t * b + j];
        }
        Xp[idx] = (OT)v;
    }
}

// Y[i][j] = T[i][j] - sum_t Q[i][t] U[t][j], U = A - sigma B (r x b), j < b.
// T may be Y itself (in-place projection with A = S, sigma = 0): each
// element is read and written by the same thread.
template <class TT>
__global__ __launch_bounds__(kConThreads) void k_qu_correct(const TT* T, int ldt, int b, int64_t n,
                                                             const double* __restrict__ Q, int RP, int r,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ B, double sigma, double* Y,
                                                             int ldy, const int* skip) {
    if (skip && *skip) return;
    __shared__ double Us[32 * 32];
    for (int e = threadIdx.x; e < r * b; e += kConThreads) Us[e] = sigma != 0.0 ? A[e] - sigma * B[e] : A[e];
    __syncthreads();
    const int64_t total = n * b;
    for (int64_t idx = blockIdx.x * (int64_t)kConThreads + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kConThreads) {
        const int64_t i = idx / b;
        const int j = (int)(idx - i * b);
        double v = (double)T[i * ldt + j];
        const double* q = Q + i * RP;
        for (int t = 0; t < r; ++t) v -= q[t] * Us[t * b + j];
        Y[i * ldy + j] = v;
    }
}

// ---- set-up kernels ---------------------------------------------------------

// Column sums of F (column-major, leading dimension ldf): block t sums
// column t; fixed per-thread strides and a fixed tree, so reproducible.
__global__ __launch_bounds__(1024) void k_col_sums(const double* __restrict__ F, int64_t ldf, int64_t n,
                                                    double* __restrict__ sums) {
    __shared__ double red[1024];
    const double* f = F + (int64_t)blockIdx.x * ldf;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += f[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// C[i][t] = c_i (F[i][t] - mu_t) for t < m, 0 for m <= t < RP.
__global__ __launch_bounds__(kConThreads) void k_form_c(const double* __restrict__ F, int64_t ldf, int m,
                                                         int64_t n, const double* __restrict__ colsum,
                                                         const double* __restrict__ cs, int RP,
                                                         double* __restrict__ C) {
    const int64_t total = n * RP;
    for (int64_t idx = blockIdx.x * (int64_t)kConThreads + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kConThreads) {
        const int64_t i = idx / RP;
        const int t = (int)(idx - i * RP);
        double v = 0.0;
        if (t < m) {
            v = F[(int64_t)t * ldf + i];
            if (colsum) v -= colsum[t] / (double)n;
            if (cs) v *= cs[i];
        }
        C[idx] = v;
    }
}

// Out[i][c] = sum_{t < kin} In[i][t] M[t][c] for c < kout, 0 for
// kout <= c < RP (row-major, stride RP; M row-major kin x kout).  One thread
// per row reads its whole input row before writing, so Out may be In.
template <int RP>
__global__ __launch_bounds__(kConThreads) void k_row_mul(const double* In, int kin, int64_t n,
                                                          const double* __restrict__ M, int kout, double* Out) {
    __shared__ double Ms[32 * 32];
    for (int e = threadIdx.x; e < kin * kout; e += kConThreads) Ms[e] = M[e];
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)kConThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kConThreads) {
        double a[RP];
#pragma unroll
        for (int t = 0; t < RP; ++t) a[t] = t < kin ? In[i * RP + t] : 0.0;
#pragma unroll
        for (int c = 0; c < RP; ++c) {
            double v = 0.0;
            if (c < kout)
                for (int t = 0; t < kin; ++t) v += a[t] * Ms[t * kout + c];
            Out[i * RP + c] = v;
        }
    }
}

// ---- host helpers -----------------------------------------------------------

// sums[t * b + j] = sum_i Q[i][t] X[i][j]  (t < r, j < b), deterministic.
template <class TT>
static int qt_sums(sfairsc_graph* g, const TT* X, int ldx, int b, int BW, const double* Q, int RP, int r,
                   double* sums, hipStream_t s, const int* skip) {
    const int nblk = con_blocks(g->n, kConThreads / BW);
    double* part = g->cw.part.as<double>();
    switch (RP) {
        case 4:
            k_qt_partial<4, TT><<<nblk, kConThreads, 0, s>>>(X, ldx, b, BW, g->n, Q, r, part, skip);
            break;
        case 8:
            k_qt_partial<8, TT><<<nblk, kConThreads, 0, s>>>(X, ldx, b, BW, g->n, Q, r, part, skip);
            break;
        case 16:
            k_qt_partial<16, TT><<<nblk, kConThreads, 0, s>>>(X, ldx, b, BW, g->n, Q, r, part, skip);
            break;
        default:
            k_qt_partial<32, TT><<<nblk, kConThreads, 0, s>>>(X, ldx, b, BW, g->n, Q, r, part, skip);
            break;
    }
    const int O = r * b;
    k_reduce_partials<<<reduce_grid(O), kRedElems * kRedSlices, 0, s>>>(part, nblk, O, sums, skip);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

static int row_mul(int RP, const double* In, int kin, int64_t n, const double* M, int kout, double* Out,
                   hipStream_t s) {
    const int grid = (int)std::min<int64_t>((n + kConThreads - 1) / kConThreads, 4096);
    switch (RP) {
        case 4:
            k_row_mul<4><<<grid, kConThreads, 0, s>>>(In, kin, n, M, kout, Out);
            break;
        case 8:
            k_row_mul<8><<<grid, kConThreads, 0, s>>>(In, kin, n, M, kout, Out);
            break;
        case 16:
            k_row_mul<16><<<grid, kConThreads, 0, s>>>(In, kin, n, M, kout, Out);
            break;
        default:
            k_row_mul<32><<<grid, kConThreads, 0, s>>>(In, kin, n, M, kout, Out);
            break;
    }
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

// Small-matrix slots inside cw.small (doubles).
constexpr int kSlotS = 0;          // S = Q^T X of the current operator call
constexpr int kSlotT = 1024;       // Q^T T
constexpr int kSlotM = 2048;       // coefficient matrix for k_row_mul
constexpr int kSlotSum = 3072;     // set-up sums
constexpr int kSmallDoubles = 4096;

static int ensure_con(sfairsc_graph* g) {
    SF_TRY(g->cw.part.ensure((size_t)kConMaxBlocks * 32 * 32 * sizeof(double)));
    SF_TRY(g->cw.small.ensure((size_t)kSmallDoubles * sizeof(double)));
    return SFAIRSC_OK;
}

static int wait_download(double* dst, const double* src, size_t count, hipStream_t s) {
    SF_HIP(hipStreamSynchronize(s));
    SF_HIP(hipMemcpy(dst, src, count * sizeof(double), hipMemcpyDeviceToHost));
    return SFAIRSC_OK;
}

static int upload_now(double* dst, const double* src, size_t count, hipStream_t s) {
    SF_HIP(hipStreamSynchronize(s));
    SF_HIP(hipMemcpy(dst, src, count * sizeof(double), hipMemcpyHostToDevice));
    return SFAIRSC_OK;
}

// Upper Cholesky factor G = R^T R of an r x r symmetric matrix and R^{-1}
// (row-major).  False if a pivot is not positive.
static bool chol_inverse(int r, const std::vector<double>& G, std::vector<double>& Rinv) {
    std::vector<double> R(r * r, 0.0);
    for (int i = 0; i < r; ++i) {
        for (int j = i; j < r; ++j) {
            double v = G[i * r + j];
            for (int t = 0; t < i; ++t) v -= R[t * r + i] * R[t * r + j];
            if (i == j) {
                if (!(v > 0.0)) return false;
                R[i * r + i] = std::sqrt(v);
            } else {
                R[i * r + j] = v / R[i * r + i];
            }
        }
    }
    Rinv.assign(r * r, 0.0);
    for (int c = 0; c < r; ++c) {
        for (int i = c; i >= 0; --i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int t = i + 1; t <= c; ++t) v -= R[i * r + t] * Rinv[t * r + c];
            Rinv[i * r + c] = v / R[i * r + i];
        }
    }
    return true;
}

static int set_constraint_impl(sfairsc_graph* g, const double* F, int64_t ldf, int m, int center, double rank_tol,
                               int* rank_out, hipStream_t s) {
    const int64_t n = g->n;
    const int RP = con_width(m);
    SF_TRY(ensure_con(g));
    SF_TRY(g->cw.cbuf.ensure((size_t)n * RP * sizeof(double)));
    double* C = g->cw.cbuf.as<double>();
    double* small = g->cw.small.as<double>();
    double* sums = small + kSlotSum;
    double* Mdev = small + kSlotM;

    // C (row-major n x RP), centred and scaled
    if (center) k_col_sums<<<m, 1024, 0, s>>>(F, ldf, n, sums);
    const int gf = (int)std::min<int64_t>((n * RP + kConThreads - 1) / kConThreads, 8192);
    k_form_c<<<gf, kConThreads, 0, s>>>(F, ldf, m, n, center ? sums : nullptr, g->normalized ? g->cs : nullptr, RP,
                                        C);
    SF_HIP(hipGetLastError());

    // Gram C^T C
    SF_TRY(qt_sums<double>(g, C, RP, m, RP, C, RP, m, sums, s, nullptr));
    std::vector<double> G(m * m), w(m), Z(m * m);
    SF_TRY(wait_download(G.data(), sums, (size_t)m * m, s));
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < i; ++j) G[i * m + j] = G[j * m + i] = 0.5 * (G[i * m + j] + G[j * m + i]);
    for (double v : G)
        if (!std::isfinite(v)) return set_error(SFAIRSC_E_ARG, "F has a non-finite entry");
    // eigenpairs of the Gram matrix (still in `sums`) on the device
    SF_TRY(small_eig_host(g, sums, m, m, w.data(), Z.data(), s));
    const double wmax = w[m - 1];
    if (!(wmax > 0.0)) return set_error(SFAIRSC_E_ARG, "the constraint matrix is zero");
    const double cut = rank_tol * rank_tol * wmax;
    std::vector<int> keep;
    for (int i = m - 1; i >= 0; --i)
        if (w[i] > cut) keep.push_back(i);
    const int r = (int)keep.size();
    if (r >= n) return set_error(SFAIRSC_E_ARG, "rank %d leaves no free direction (n=%lld)", r, (long long)n);

    // Q1 = C U_r diag(w_r)^{-1/2}
    std::vector<double> M1(m * r);
    for (int t = 0; t < m; ++t)
        for (int c = 0; c < r; ++c) M1[t * r + c] = Z[t * m + keep[c]] / std::sqrt(w[keep[c]]);
    if (!g->qbas || g->qld != RP) {
        if (g->qbas) (void)hipFree(g->qbas);
        g->qbas = nullptr;
        hipError_t e = hipMalloc((void**)&g->qbas, (size_t)n * RP * sizeof(double) + 16);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            g->qbas = nullptr;
            return set_error(SFAIRSC_E_NOMEM, "hipMalloc of the constraint basis failed");
        }
    }
    double* Q = g->qbas;
    SF_TRY(upload_now(Mdev, M1.data(), M1.size(), s));
    SF_TRY(row_mul(RP, C, m, n, Mdev, r, Q, s));

    // Cholesky-QR passes until Q^T Q = I to 1e-12 (1e-10 after two passes:
    // the Gram sums over n rows carry their own rounding)
    std::vector<double> G2(r * r), Rinv;
    for (int pass = 0;; ++pass) {
        SF_TRY(qt_sums<double>(g, Q, RP, r, RP, Q, RP, r, sums, s, nullptr));
        SF_TRY(wait_download(G2.data(), sums, (size_t)r * r, s));
        double dev = 0.0;
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) dev = std::max(dev, std::fabs(G2[i * r + j] - (i == j ? 1.0 : 0.0)));
        if (dev <= 1e-12 || (pass >= 2 && dev <= 1e-10)) break;
        if (pass == 3) return set_error(SFAIRSC_E_ARG, "constraint basis not orthonormal (%.2e) after 3 passes", dev);
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < i; ++j) G2[i * r + j] = G2[j * r + i] = 0.5 * (G2[i * r + j] + G2[j * r + i]);
        if (!chol_inverse(r, G2, Rinv)) return set_error(SFAIRSC_E_ARG, "constraint basis lost rank");
        SF_TRY(upload_now(Mdev, Rinv.data(), Rinv.size(), s));
        SF_TRY(row_mul(RP, Q, r, n, Mdev, r, Q, s));
    }
    SF_HIP(hipStreamSynchronize(s));
    g->qrank = r;
    g->qld = RP;
    g->cw.cbuf.release();
    if (rank_out) *rank_out = r;
    return SFAIRSC_OK;
}

// ---- operator steps ---------------------------------------------------------

int gen_project_in(sfairsc_graph* g, const double* X, int ldx, int b, int BW, bool to_float, void* Xp,
                   hipStream_t s, const int* skip) {
    SF_TRY(ensure_con(g));
    double* S = g->cw.small.as<double>() + kSlotS;
    SF_TRY(qt_sums<double>(g, X, ldx, b, pow2_at_least(b), g->qbas, g->qld, g->qrank, S, s, skip));
    const int grid = (int)std::min<int64_t>((g->n * BW + kConThreads - 1) / kConThreads, 8192);
    if (to_float)
        k_qs_apply<float><<<grid, kConThreads, 0, s>>>(X, ldx, b, BW, g->n, g->qbas, g->qld, g->qrank, S, (float*)Xp,
                                                       skip);
    else
        k_qs_apply<double><<<grid, kConThreads, 0, s>>>(X, ldx, b, BW, g->n, g->qbas, g->qld, g->qrank, S,
                                                        (double*)Xp, skip);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

int gen_correct(sfairsc_graph* g, const void* T, bool t_float, int BW, int b, double sigma, double* Y, int ldy,
                hipStream_t s, const int* skip) {
    double* S = g->cw.small.as<double>() + kSlotS;
    double* QT = g->cw.small.as<double>() + kSlotT;
    const int grid = (int)std::min<int64_t>((g->n * b + kConThreads - 1) / kConThreads, 8192);
    if (t_float) {
        SF_TRY(qt_sums<float>(g, (const float*)T, BW, b, BW, g->qbas, g->qld, g->qrank, QT, s, skip));
        k_qu_correct<float><<<grid, kConThreads, 0, s>>>((const float*)T, BW, b, g->n, g->qbas, g->qld, g->qrank, QT,
                                                         S, sigma, Y, ldy, skip);
    } else {
        SF_TRY(qt_sums<double>(g, (const double*)T, BW, b, BW, g->qbas, g->qld, g->qrank, QT, s, skip));
        k_qu_correct<double><<<grid, kConThreads, 0, s>>>((const double*)T, BW, b, g->n, g->qbas, g->qld, g->qrank,
                                                          QT, S, sigma, Y, ldy, skip);
    }
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

int gen_project(sfairsc_graph* g, double* X, int ldx, int b, hipStream_t s) {
    SF_TRY(ensure_con(g));
    double* S = g->cw.small.as<double>() + kSlotS;
    SF_TRY(qt_sums<double>(g, X, ldx, b, pow2_at_least(b), g->qbas, g->qld, g->qrank, S, s, nullptr));
    const int grid = (int)std::min<int64_t>((g->n * b + kConThreads - 1) / kConThreads, 8192);
    k_qu_correct<double><<<grid, kConThreads, 0, s>>>(X, ldx, b, g->n, g->qbas, g->qld, g->qrank, S, S, 0.0, X, ldx,
                                                      nullptr);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" int sfairsc_graph_set_constraint(sfairsc_graph_t g, const double* F, int64_t ldf, int32_t m,
                                            int32_t center, double rank_tol, int32_t* rank, hipStream_t stream) {
    if (!g || !F) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (m < 1 || m > kMaxGroups) return set_error(SFAIRSC_E_ARG, "m=%d outside [1, %d]", m, kMaxGroups);
    if (ldf < g->n) return set_error(SFAIRSC_E_ARG, "ldf=%lld < n=%lld", (long long)ldf, (long long)g->n);
    if (center != 0 && center != 1) return set_error(SFAIRSC_E_ARG, "center must be 0 or 1");
    if (rank_tol == 0.0) rank_tol = 1e-6;
    if (!(rank_tol >= 1e-7 && rank_tol < 1.0))
        return set_error(SFAIRSC_E_ARG, "rank_tol=%g outside [1e-7, 1)", rank_tol);
    int r = 0;
    (void)hipStreamSynchronize(stream);
    free_memb(g);
    const int st = set_constraint_impl(g, F, ldf, m, center, rank_tol, &r, stream);
    if (st != SFAIRSC_OK) {
        (void)hipStreamSynchronize(stream);
        if (g->qbas) (void)hipFree(g->qbas);
        g->qbas = nullptr;
        g->qrank = g->qld = 0;
        g->cw.cbuf.release();
        return st;
    }
    if (rank) *rank = r;
    return SFAIRSC_OK;
}
