// Gradient of the sum of the k smallest fair eigenvalues with respect to the
// stored edge weights (unnormalized variant).  With X the fair eigenvectors,
// sum_{i<=k} lambda_i = tr(X^T L X) (Theorem 2.1) and, F not depending on W,
// the envelope theorem gives d/dw_ij = ||X_i - X_j||^2 for an undirected edge;
// each of the two stored copies carries half.  One wavefront per row: the row
// of H is loaded once and every stored neighbour j reads H_j (k values).
#include "internal.h"

namespace sfairsc {

template <class GT>
__global__ __launch_bounds__(256) void k_eigsum_grad(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ H,
                                                      int64_t n, int k, GT* __restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < n; i += nwaves) {
        const int32_t a = rowptr[i], e_end = rowptr[i + 1];
        for (int32_t e = a + lane; e < e_end; e += 64) {
            const int64_t j = col[e];
            double s = 0.0;
            for (int l = 0; l < k; ++l) {
                const double d = H[(int64_t)l * n + i] - H[(int64_t)l * n + j];
                s += d * d;
            }
            grad[e] = (GT)(0.5 * s);
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
    int64_t waves = g->n;
    int64_t blocks = (waves * 64 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (g->value_dtype == SFAIRSC_F32)
        k_eigsum_grad<float><<<(int)blocks, 256, 0, stream>>>(g->rowptr, g->col, H, g->n, k, (float*)grad);
    else
        k_eigsum_grad<double><<<(int)blocks, 256, 0, stream>>>(g->rowptr, g->col, H, g->n, k, (double*)grad);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}
