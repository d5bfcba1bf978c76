// Deterministic reduction of per-block partial sums: out[e] = sum over
// blocks b (in increasing b, 16 interleaved slices combined in slice order)
// of part[b][e].  Each workgroup covers 64 elements with 16 slices, so the
// partials are read by ceil(O / 64) workgroups in parallel.
#pragma once

#include <hip/hip_runtime.h>

namespace sfairsc {

constexpr int kRedElems = 64;
constexpr int kRedSlices = 16;

template <int UNUSED = 0>
__global__ __launch_bounds__(kRedElems * kRedSlices) void k_reduce_partials(const double* __restrict__ part,
                                                                              int nblk, int O,
                                                                              double* __restrict__ out,
                                                                              const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[kRedElems * kRedSlices];
    const int el = threadIdx.x % kRedElems, sl = threadIdx.x / kRedElems;
    const int e = blockIdx.x * kRedElems + el;
    double s = 0.0;
    if (e < O)
        for (int blk = sl; blk < nblk; blk += kRedSlices) s += part[(size_t)blk * O + e];
    red[threadIdx.x] = s;
    __syncthreads();
    if (sl == 0 && e < O) {
        double t = 0.0;
        for (int q = 0; q < kRedSlices; ++q) t += red[q * kRedElems + el];
        out[e] = t;
    }
}

inline int reduce_grid(int O) { return (O + kRedElems - 1) / kRedElems; }

}  // namespace sfairsc
