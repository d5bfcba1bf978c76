// Deterministic reduction of per-block partial sums: out[e] = sum over
// blocks b of part[b][e], in a fixed order (64 interleaved slices, each
// split over four accumulators, combined in slice order).  Each workgroup
// covers 16 elements with 64 slices, so the partials are read by
// ceil(O / 16) workgroups in parallel and, with at most 256 partials, every
// thread issues all of its loads at once: the kernel is one load latency
// deep rather than four.
#pragma once

#include <hip/hip_runtime.h>

namespace sfairsc {

constexpr int kRedElems = 16;
constexpr int kRedSlices = 64;

template <int UNUSED = 0>
__global__ __launch_bounds__(kRedElems * kRedSlices) void k_reduce_partials(const double* __restrict__ part,
                                                                              int nblk, int O,
                                                                              double* __restrict__ out,
                                                                              const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[kRedElems * kRedSlices];
    const int el = threadIdx.x % kRedElems, sl = threadIdx.x / kRedElems;
    const int e = blockIdx.x * kRedElems + el;
    // four independent accumulators keep several loads in flight
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < O) {
        int blk = sl;
        for (; blk + 3 * kRedSlices < nblk; blk += 4 * kRedSlices) {
            s0 += part[(size_t)blk * O + e];
            s1 += part[(size_t)(blk + kRedSlices) * O + e];
            s2 += part[(size_t)(blk + 2 * kRedSlices) * O + e];
            s3 += part[(size_t)(blk + 3 * kRedSlices) * O + e];
        }
        for (; blk < nblk; blk += kRedSlices) s0 += part[(size_t)blk * O + e];
    }
    red[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (sl == 0 && e < O) {
        // the slices in order, read sixteen at a time so that the reads
        // are in flight together
        double t = 0.0;
        for (int q0 = 0; q0 < kRedSlices; q0 += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = red[(q0 + u) * kRedElems + el];
#pragma unroll
            for (int u = 0; u < 16; ++u) t += v[u];
        }
        out[e] = t;
    }
}

inline int reduce_grid(int O) { return (O + kRedElems - 1) / kRedElems; }

}  // namespace sfairsc
