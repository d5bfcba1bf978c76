// Gradient of the sum of the k smallest fair eigenvalues with respect to the
// stored edge weights (unnormalized variant).  With X the fair eigenvectors,
// sum_{i<=k} lambda_i = tr(X^T L X) (Theorem 2.1) and, F not depending on W,
// the envelope theorem gives d/dw_ij = ||X_i - X_j||^2 for an undirected edge;
// each of the two stored copies carries half.
//
// H arrives column-major (n x k).  It is first staged row-major with rows
// padded to an even length kp, so that the row of a neighbour is one
// contiguous run of kp doubles (one or two cache lines) instead of k lines
// scattered n apart.  Then one wavefront per CSR row i, one lane per stored
// entry (i, j): row i of H is read once per wavefront (a broadcast), row j
// once per entry.
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

template <class GT>
__global__ __launch_bounds__(256) void k_eigsum_grad(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ Hr,
                                                      int64_t n, int kp, GT* __restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int h2 = kp >> 1;
    for (int64_t i = wave; i < n; i += nwaves) {
        const int32_t e0 = rowptr[i], e1 = rowptr[i + 1];
        const double2* a = reinterpret_cast<const double2*>(Hr + i * kp);
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
            grad[e] = (GT)(0.5 * (s0 + s1));
        }
    }
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" int sfairsc_eigsum_backward(sfairsc_graph_t g, const double* H, int32_t k, void* grad,
                                       hipStream_t stream) {
    if (!g || !H || !grad) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (g->normalized)
        return set_error(SFAIRSC_E_ARG, "eigenvalue-sum gradient is implemented for the unnormalized variant only");
    if (k < 1 || k > kMaxK) return set_error(SFAIRSC_E_ARG, "k=%d out of range", k);
    if (g->nnz == 0) return SFAIRSC_OK;
    const int kp = (k + 1) & ~1;
    SF_TRY(g->gw.hrow.ensure((size_t)g->n * kp * sizeof(double)));
    double* Hr = g->gw.hrow.as<double>();
    int64_t sb = (g->n * kp + 255) / 256;
    if (sb > 4096) sb = 4096;
    k_stage_rows<<<(int)sb, 256, 0, stream>>>(H, g->n, k, kp, Hr);
    int64_t blocks = (g->n * 64 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (g->value_dtype == SFAIRSC_F32)
        k_eigsum_grad<float><<<(int)blocks, 256, 0, stream>>>(g->rowptr, g->col, Hr, g->n, kp, (float*)grad);
    else
        k_eigsum_grad<double><<<(int)blocks, 256, 0, stream>>>(g->rowptr, g->col, Hr, g->n, kp, (double*)grad);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}
