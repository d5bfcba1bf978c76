// Gradient of the sum of the k smallest fair eigenvalues with respect to the
// stored edge weights.  With X the fair eigenvectors,
// sum_{i<=k} lambda_i = tr(X^T L X) (Theorem 2.1) and, F not depending on W,
// the envelope theorem gives d/dw_ij = ||X_i - X_j||^2 for an undirected edge
// (unnormalized variant).  In the normalized variant the lambda_l are
// eigenvalues of the pencil (L, D) on null(F^T) with h_l^T D h_l = 1, and the
// weight also moves d_i and d_j, which adds -lambda_l (h_il^2 + h_jl^2).
// Each of the two stored copies carries half.
//
// H arrives column-major (n x k).  It is first staged row-major with the row
// stride kp rounded up to 16 doubles, so that the row of a neighbour is one
// aligned 128-byte line (k <= 16) instead of k lines scattered n apart; the
// staging reads 64 rows of every column coalesced into LDS and writes the
// rows out contiguously.  For the normalized variant q_i = sum_l lambda_l
// H_il^2 is formed per vertex beside it.  Then one to four CSR rows per
// wavefront, one lane per stored entry (i, j): row i of H is read once per
// row, row j (and q_j) once per entry.
#include "internal.h"

namespace sfairsc {

constexpr int kStageRows = 64;

// Hr[i][l] = H[l][i] for l < k, 0 for k <= l < kp; one block per 64 rows.
__global__ __launch_bounds__(256) void k_stage_rows(const double* __restrict__ H, int64_t n, int k, int kp,
                                                     double* __restrict__ Hr) {
    extern __shared__ double tile[];  // [kStageRows][kp + 1]
    const int ld = kp + 1;
    for (int64_t i0 = (int64_t)blockIdx.x * kStageRows; i0 < n; i0 += (int64_t)gridDim.x * kStageRows) {
        const int rows = (int)min<int64_t>(kStageRows, n - i0);
        for (int idx = threadIdx.x; idx < kStageRows * kp; idx += blockDim.x) {
            const int l = idx / kStageRows, r = idx - l * kStageRows;
            tile[r * ld + l] = (l < k && r < rows) ? H[(int64_t)l * n + i0 + r] : 0.0;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < rows * kp; idx += blockDim.x) {
            const int r = idx / kp, l = idx - r * kp;
            Hr[i0 * kp + idx] = tile[r * ld + l];
        }
        __syncthreads();
    }
}

// Eigenvalues by value: at most kMaxK doubles in the kernel arguments.
struct EigvalArg {
    double v[kMaxK];
};

__global__ __launch_bounds__(256) void k_row_quad(const double* __restrict__ H, int64_t n, int k, EigvalArg lam,
                                                  double* __restrict__ q) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int l = 0; l < k; ++l) {
            const double x = H[(int64_t)l * n + i];
            s += lam.v[l] * (x * x);
        }
        q[i] = s;
    }
}

// NORM: subtract 0.5 (q_i + q_j) (normalized variant); q is unused otherwise.
// RPW rows per wavefront (64 / RPW lanes each, one lane per stored entry):
// short rows share a wavefront, so that more gathers are in flight.  Row i
// of H is read once per row into registers (up to 16 values; wider rows are
// read per entry), row j once per entry.
template <class GT, bool NORM, int RPW>
__global__ __launch_bounds__(256) void k_eigsum_grad(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ Hr,
                                                      const double* __restrict__ q, int64_t n, int k, int kp,
                                                      GT* __restrict__ grad) {
    constexpr int G = 64 / RPW;
    constexpr int KR = 8;  // pairs held in registers
    const int lane = threadIdx.x & 63;
    const int sub = lane / G, sl = lane - sub * G;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int h2 = (k + 1) >> 1;  // pairs holding the k values (the padding is zero)
    for (int64_t i0 = wave * RPW; i0 < n; i0 += nwaves * RPW) {
        const int64_t i = i0 + sub;
        const bool rv = i < n;
        const int32_t e0 = rv ? rowptr[i] : 0, e1 = rv ? rowptr[i + 1] : 0;
        const double2* a = reinterpret_cast<const double2*>(Hr + (rv ? i : 0) * kp);
        double2 ar[KR];
#pragma unroll
        for (int c = 0; c < KR; ++c) ar[c] = c < h2 ? a[c] : make_double2(0.0, 0.0);
        const double qi = (NORM && rv) ? q[i] : 0.0;
        for (int32_t e = e0 + sl; e < e1; e += G) {
            const int64_t j = col[e];
            const double2* b = reinterpret_cast<const double2*>(Hr + j * kp);
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int c = 0; c < KR; ++c) {
                if (c < h2) {
                    const double2 y = b[c];
                    const double d0 = ar[c].x - y.x, d1 = ar[c].y - y.y;
                    s0 += d0 * d0;
                    s1 += d1 * d1;
                }
            }
            for (int c = KR; c < h2; ++c) {
                const double2 x = a[c], y = b[c];
                const double d0 = x.x - y.x, d1 = x.y - y.y;
                s0 += d0 * d0;
                s1 += d1 * d1;
            }
            double r = s0 + s1;
            if (NORM) r -= qi + q[j];
            grad[e] = (GT)(0.5 * r);
        }
    }
}

}  // namespace sfairsc

using namespace sfairsc;

template <class GT, int RPW>
static void launch_grad_r(bool norm, int blocks, hipStream_t stream, const int32_t* rowptr, const int32_t* col,
                          const double* Hr, const double* q, int64_t n, int k, int kp, void* grad) {
    if (norm)
        k_eigsum_grad<GT, true, RPW><<<blocks, 256, 0, stream>>>(rowptr, col, Hr, q, n, k, kp, (GT*)grad);
    else
        k_eigsum_grad<GT, false, RPW><<<blocks, 256, 0, stream>>>(rowptr, col, Hr, q, n, k, kp, (GT*)grad);
}

// Rows per wavefront from the average row length (as the sparse product).
template <class GT>
static void launch_grad(bool norm, double avg, hipStream_t stream, const int32_t* rowptr, const int32_t* col,
                        const double* Hr, const double* q, int64_t n, int k, int kp, void* grad) {
    const int rpw = avg <= 12.0 ? 4 : (avg <= 48.0 ? 2 : 1);
    int64_t blocks = (n * 64 / rpw + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 16384) blocks = 16384;
    if (rpw == 4)
        launch_grad_r<GT, 4>(norm, (int)blocks, stream, rowptr, col, Hr, q, n, k, kp, grad);
    else if (rpw == 2)
        launch_grad_r<GT, 2>(norm, (int)blocks, stream, rowptr, col, Hr, q, n, k, kp, grad);
    else
        launch_grad_r<GT, 1>(norm, (int)blocks, stream, rowptr, col, Hr, q, n, k, kp, grad);
}

extern "C" int sfairsc_eigsum_backward(sfairsc_graph_t g, const double* H, int32_t k, const double* eigenvalues,
                                       void* grad, hipStream_t stream) {
    if (!g || !H || !grad) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (k < 1 || k > kMaxK) return set_error(SFAIRSC_E_ARG, "k=%d out of range", k);
    const bool norm = g->normalized != 0;
    if (norm && !eigenvalues)
        return set_error(SFAIRSC_E_ARG, "the normalized variant needs the k eigenvalues");
    EigvalArg lam{};
    if (norm)
        for (int l = 0; l < k; ++l) lam.v[l] = eigenvalues[l];
    if (g->nnz == 0) return SFAIRSC_OK;
    const int kp = (k + 15) & ~15;  // rows of whole, aligned 128-byte lines
    const size_t hr_doubles = (size_t)g->n * kp;
    SF_TRY(g->gw.hrow.ensure((hr_doubles + (norm ? (size_t)g->n : 0)) * sizeof(double)));
    double* Hr = g->gw.hrow.as<double>();
    double* q = norm ? Hr + hr_doubles : nullptr;
    int64_t sb = (g->n + kStageRows - 1) / kStageRows;
    if (sb > 8192) sb = 8192;
    k_stage_rows<<<(int)sb, 256, (size_t)kStageRows * (kp + 1) * sizeof(double), stream>>>(H, g->n, k, kp, Hr);
    if (norm) {
        int64_t qb = (g->n + 255) / 256;
        if (qb > 4096) qb = 4096;
        k_row_quad<<<(int)qb, 256, 0, stream>>>(H, g->n, k, lam, q);
    }
    const double avg = (double)g->nnz / (double)g->n;
    if (g->value_dtype == SFAIRSC_F32)
        launch_grad<float>(norm, avg, stream, g->rowptr, g->col, Hr, q, g->n, k, kp, grad);
    else
        launch_grad<double>(norm, avg, stream, g->rowptr, g->col, Hr, q, g->n, k, kp, grad);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}
