// Gradient of the sum of the k smallest fair eigenvalues with respect to the
// stored edge weights.  With X the fair eigenvectors,
// sum_{i<=k} lambda_i = tr(X^T L X) (Theorem 2.1) and, F not depending on W,
// the envelope theorem gives d/dw_ij = ||X_i - X_j||^2 for an undirected edge
// (unnormalized variant).  In the normalized variant the lambda_l are
// eigenvalues of the pencil (L, D) on null(F^T) with h_l^T D h_l = 1, and the
// weight also moves d_i and d_j, which adds -lambda_l (h_il^2 + h_jl^2).
// Each of the two stored copies carries half.
//
// H arrives column-major (n x k).  It is first staged row-major with rows
// padded to an even length kp, so that the row of a neighbour is one
// contiguous run of kp doubles (one or two cache lines) instead of k lines
// scattered n apart; for the normalized variant q_i = sum_l lambda_l H_il^2
// is formed per vertex beside it.  Then one wavefront per CSR row i, one lane
// per stored entry (i, j): row i of H is read once per wavefront (a
// broadcast), row j (and q_j) once per entry.
#include "internal.h"

namespace sfairsc {

__global__ __launch_bounds__(256) void k_stage_rows(const double* __restrict__ H, int64_t n, int k, int kp,
                                                     double* __restrict__ Hr) {
    const int64_t total = n * kp;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / kp;
        const int l = (int)(idx - i * kp);
        Hr[idx] = l < k ? H[(int64_t)l * n + i] : 0.0;
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
template <class GT, bool NORM>
__global__ __launch_bounds__(256) void k_eigsum_grad(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ Hr,
                                                      const double* __restrict__ q, int64_t n, int kp,
                                                      GT* __restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int h2 = kp >> 1;
    for (int64_t i = wave; i < n; i += nwaves) {
        const int32_t e0 = rowptr[i], e1 = rowptr[i + 1];
        const double2* a = reinterpret_cast<const double2*>(Hr + i * kp);
        const double qi = NORM ? q[i] : 0.0;
        for (int32_t e = e0 + lane; e < e1; e += 64) {
            const int64_t j = col[e];
            const double2* b = reinterpret_cast<const double2*>(Hr + j * kp);
            double s0 = 0.0, s1 = 0.0;
            for (int c = 0; c < h2; ++c) {
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

template <class GT>
static void launch_grad(bool norm, int blocks, hipStream_t stream, const int32_t* rowptr, const int32_t* col,
                        const double* Hr, const double* q, int64_t n, int kp, void* grad) {
    if (norm)
        k_eigsum_grad<GT, true><<<blocks, 256, 0, stream>>>(rowptr, col, Hr, q, n, kp, (GT*)grad);
    else
        k_eigsum_grad<GT, false><<<blocks, 256, 0, stream>>>(rowptr, col, Hr, q, n, kp, (GT*)grad);
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
    const int kp = (k + 1) & ~1;
    const size_t hr_doubles = (size_t)g->n * kp;
    SF_TRY(g->gw.hrow.ensure((hr_doubles + (norm ? (size_t)g->n : 0)) * sizeof(double)));
    double* Hr = g->gw.hrow.as<double>();
    double* q = norm ? Hr + hr_doubles : nullptr;
    int64_t sb = (g->n * kp + 255) / 256;
    if (sb > 4096) sb = 4096;
    k_stage_rows<<<(int)sb, 256, 0, stream>>>(H, g->n, k, kp, Hr);
    if (norm) {
        int64_t qb = (g->n + 255) / 256;
        if (qb > 4096) qb = 4096;
        k_row_quad<<<(int)qb, 256, 0, stream>>>(H, g->n, k, lam, q);
    }
    int64_t blocks = (g->n * 64 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (g->value_dtype == SFAIRSC_F32)
        launch_grad<float>(norm, (int)blocks, stream, g->rowptr, g->col, Hr, q, g->n, kp, grad);
    else
        launch_grad<double>(norm, (int)blocks, stream, g->rowptr, g->col, Hr, q, g->n, kp, grad);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}
