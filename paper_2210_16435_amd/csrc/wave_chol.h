// Cholesky factor and inverse of a small SPD matrix held by one wavefront.
#pragma once

#include <hip/hip_runtime.h>

namespace sfairsc {

// Lane l's value of v, in every lane (l uniform across the wavefront; a
// constant in the unrolled loops below): two scalar reads of the lane, no
// trip through the LDS crossbar as a shuffle would take.
__device__ __forceinline__ double wave_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// One wavefront factors a B x B SPD matrix in registers.  Lane j (< B)
// holds column j of G in g[0..B); on return g holds column j of R
// (G = R^T R, R upper triangular) and ri column j of R^{-1}.  Returns false
// (uniformly across the wavefront) if a pivot is <= thresh.  Every lane of
// the wavefront must be active.
template <int B>
__device__ bool wave_chol_inv(double (&g)[B], double (&ri)[B], double thresh) {
    const int j = threadIdx.x & 63;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        double piv = wave_lane(g[k], k);
        if (!(piv > thresh)) {
            ok = false;
            piv = 1.0;
        }
        const double rkk = sqrt(piv);
        const double inv = 1.0 / rkk;
        const double rkj = (j > k) ? g[k] * inv : (j == k ? rkk : 0.0);
        g[k] = rkj;
#pragma unroll
        for (int i = k + 1; i < B; ++i) g[i] -= wave_lane(rkj, i) * rkj;
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int t = i + 1; t < B; ++t) acc -= wave_lane(g[i], t) * ri[t];
        const double rinv = 1.0 / wave_lane(g[i], i);
        ri[i] = (i <= j) ? acc * rinv : 0.0;
    }
    return ok;
}

}  // namespace sfairsc
