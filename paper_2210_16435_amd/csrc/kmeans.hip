// k-means on the rows of H (Alg. 3 step 4: "apply k-means clustering to the
// rows of H").  The paper does not specify the variant; this one is:
//   * k-means++ seeding (Arthur and Vassilvitskii 2007): first centre row
//     floor(u n); centre t >= 1 is the first row whose inclusive prefix sum
//     of D^2 (squared distance to the nearest chosen centre) exceeds u * total
//     (row floor(u n) when total = 0);
//   * uniforms u from SplitMix64 (Steele, Lea and Flood 2014): restart r,
//     draw t uses output number r * 2^32 + t + 1 of the stream seeded with
//     `seed`, top 53 bits scaled to [0, 1);
//   * Lloyd: nearest centroid by squared distance (ties: lowest index); stop
//     when no label changes or after max_iter assignments, else move each
//     centroid to its rows' mean; an empty cluster takes the row farthest
//     from its own centroid (ties: lowest row), each row used once;
//   * best inertia over restarts (ties: earliest), labels renumbered by
//     first appearance.
// H is read column-major (n x kdim) so consecutive threads read consecutive
// rows.  Sums use fixed per-block partials combined in block order.
#include <algorithm>
#include <climits>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace sfairsc {

namespace {

constexpr int kKmThreads = 256;
constexpr int kKmMaxBlocks = 1024;
constexpr int kChunk = 1024;  // rows per prefix-sum chunk in the seeding

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ inline double sm_uniform(uint64_t seed, uint64_t restart, uint64_t draw) {
    const uint64_t idx = (restart << 32) + draw + 1;
    const uint64_t z = sm_mix(seed + idx * 0x9E3779B97F4A7C15ull);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

// cent[t] = H[idx]; d2 = (t == 0) ? dist : min(d2, dist) to that centre.
// All restarts at once: restart r = blockIdx.y works on its own slices
// (idxp[r], cent + r K kdim, d2 + r n); the same holds for every kernel
// below that takes a restart index.
__global__ __launch_bounds__(kKmThreads) void k_pp_update(const double* __restrict__ H, int64_t n, int kdim, int K,
                                                          const int64_t* __restrict__ idxp, int t,
                                                          double* __restrict__ cent, double* __restrict__ d2) {
    __shared__ double c[kMaxK];
    const int r = blockIdx.y;
    cent += (size_t)r * K * kdim;
    d2 += (size_t)r * n;
    const int64_t idx = idxp[r];
    if (threadIdx.x < kdim) c[threadIdx.x] = H[(int64_t)threadIdx.x * n + idx];
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < kdim) cent[t * kdim + threadIdx.x] = c[threadIdx.x];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int l = 0; l < kdim; ++l) {
            const double d = H[(int64_t)l * n + i] - c[l];
            s += d * d;
        }
        d2[i] = (t == 0) ? s : fmin(d2[i], s);
    }
}

// Chunk sums of d2 (chunk = kChunk rows, one block per chunk, fixed tree).
__global__ __launch_bounds__(kKmThreads) void k_chunk_sums(const double* __restrict__ d2, int64_t n,
                                                           double* __restrict__ csum, int cst) {
    __shared__ double red[kKmThreads];
    d2 += (size_t)blockIdx.y * n;
    csum += (size_t)blockIdx.y * cst;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    double s = 0.0;
    for (int q = threadIdx.x; q < kChunk; q += kKmThreads) {
        const int64_t i = base + q;
        if (i < n) s += d2[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kKmThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) csum[blockIdx.x] = red[0];
}

// D^2 sampling: index of the first row whose inclusive prefix sum exceeds
// u * total.  One wavefront: lane l sums a contiguous segment of the chunk
// sums (total = the lanes' inclusive scan), the ballot of "prefix > target"
// names the segment, a short scan the chunk; inside the chunk every lane
// sums 16 consecutive rows and the same steps name the row.  Every order is
// fixed, so the pick is reproducible; where rounding leaves no prefix above
// the target, the last row of the range is taken.
__global__ __launch_bounds__(64) void k_pp_pick(const double* __restrict__ d2, const double* __restrict__ csum,
                                                int cst, int nchunks, int64_t n, uint64_t seed, int t,
                                                int64_t* __restrict__ idxp) {
    const int lane = threadIdx.x, r = blockIdx.y;
    d2 += (size_t)r * n;
    csum += (size_t)r * cst;
    idxp += r;
    const double u = sm_uniform(seed, (uint64_t)r, (uint64_t)t);
    const int S = (nchunks + 63) / 64;
    const int c0 = min(nchunks, lane * S), c1 = min(nchunks, c0 + S);
    double seg = 0.0;
    for (int c = c0; c < c1; ++c) seg += csum[c];
    double incl = seg;
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    const double total = __shfl(incl, 63);
    int64_t pick = (int64_t)(u * (double)n);
    if (pick >= n) pick = n - 1;
    if (total > 0.0) {
        const double target = u * total;
        const unsigned long long mseg = __ballot(incl > target);
        if (mseg == 0) {
            pick = n - 1;
        } else {
            const int L = __builtin_ctzll(mseg);
            double acc = __shfl(incl - seg, L);
            const int s0 = min(nchunks, L * S), s1 = min(nchunks, s0 + S);
            int c = s0;
            for (; c + 1 < s1; ++c) {
                const double v = csum[c];
                if (acc + v > target) break;
                acc += v;
            }
            // chunk c: rows [base, end), 16 per lane
            const int64_t base = (int64_t)c * kChunk;
            const int64_t end = min(n, base + kChunk);
            const int64_t e0 = min(end, base + 16 * lane), e1 = min(end, e0 + 16);
            double part = 0.0;
            for (int64_t i = e0; i < e1; ++i) part += d2[i];
            double in2 = part;
            for (int off = 1; off < 64; off <<= 1) {
                const double t = __shfl_up(in2, off);
                if (lane >= off) in2 += t;
            }
            const unsigned long long mrow = __ballot(acc + in2 > target);
            if (mrow == 0) {
                pick = end - 1;
            } else {
                const int L2 = __builtin_ctzll(mrow);
                double a2 = acc + __shfl(in2 - part, L2);
                const int64_t r0 = min(end, base + 16 * L2), r1 = min(end, r0 + 16);
                int64_t i = r0;
                for (; i < r1; ++i) {
                    a2 += d2[i];
                    if (a2 > target) break;
                }
                pick = i < r1 ? i : r1 - 1;
            }
        }
    }
    if (lane == 0) *idxp = pick;
}

// Assignment: label_i = argmin_j ||H_i - c_j||^2; per-block changed count.
// KD bounds kdim (8, 16, 32 or 64) so that the row stays in registers.
template <int KD>
__global__ __launch_bounds__(kKmThreads) void k_assign(const double* __restrict__ H, int64_t n, int kdim, int K,
                                                       const double* __restrict__ cent, int32_t* __restrict__ lab,
                                                       double* __restrict__ mind, int* __restrict__ changed_part,
                                                       const int* __restrict__ done) {
    {
        const int r = blockIdx.y;
        cent += (size_t)r * K * kdim;
        lab += (size_t)r * n;
        mind += (size_t)r * n;
        changed_part += (size_t)r * gridDim.x;
        done += 2 * r;
    }
    if (*done) return;
    __shared__ double c[kMaxK * kMaxK];
    __shared__ int cnt[kKmThreads];
    for (int o = threadIdx.x; o < K * kdim; o += blockDim.x) c[o] = cent[o];
    __syncthreads();
    int changed = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double x[KD];
#pragma unroll
        for (int l = 0; l < KD; ++l) x[l] = l < kdim ? H[(int64_t)l * n + i] : 0.0;
        double best = INFINITY;
        int bj = 0;
        for (int j = 0; j < K; ++j) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < KD; ++l) {
                if (l < kdim) {
                    const double d = x[l] - c[j * kdim + l];
                    s += d * d;
                }
            }
            if (s < best) {
                best = s;
                bj = j;
            }
        }
        if (lab[i] != bj) ++changed;
        lab[i] = bj;
        mind[i] = best;
    }
    cnt[threadIdx.x] = changed;
    __syncthreads();
    for (int w = kKmThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) changed_part[blockIdx.x] = cnt[0];
}

// Per-block cluster sums: each wave walks its rows in order; lane l < kdim
// owns dimension l.  part: [blk][K][kdim], cpart: [blk][K].
__global__ __launch_bounds__(kKmThreads) void k_cluster_sums(const double* __restrict__ H, int64_t n, int kdim,
                                                             int K, const int32_t* __restrict__ lab,
                                                             double* __restrict__ part, int* __restrict__ cpart,
                                                             const int* __restrict__ done) {
    {
        const int r = blockIdx.y;
        lab += (size_t)r * n;
        part += (size_t)r * gridDim.x * K * kdim;
        cpart += (size_t)r * gridDim.x * K;
        done += 2 * r;
    }
    if (*done) return;
    constexpr int kWaves = kKmThreads / 64;
    extern __shared__ double sh[];  // [kWaves][K][kdim] sums, then [kWaves][K] counts (as double)
    double* sums = sh;
    double* cnts = sh + kWaves * K * kdim;
    for (int o = threadIdx.x; o < kWaves * K * (kdim + 1); o += blockDim.x) sh[o] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t rows_per_block = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    const int64_t per_wave = (r1 - r0 + kWaves - 1) / kWaves;
    const int64_t w0 = r0 + wave * per_wave, w1 = min(r1, w0 + per_wave);
    double* ws = sums + wave * K * kdim;
    // rows in order, eight at a time with their loads issued first
    int64_t i = w0;
    for (; i + 8 <= w1; i += 8) {
        int jj[8];
        double hv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            jj[u] = lab[i + u];
            hv[u] = lane < kdim ? H[(int64_t)lane * n + i + u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (lane < kdim) ws[jj[u] * kdim + lane] += hv[u];
            if (lane == 0) cnts[wave * K + jj[u]] += 1.0;
        }
    }
    for (; i < w1; ++i) {
        const int j = lab[i];
        if (lane < kdim) ws[j * kdim + lane] += H[(int64_t)lane * n + i];
        if (lane == 0) cnts[wave * K + j] += 1.0;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < K * kdim; o += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += sums[w * K * kdim + o];
        part[(size_t)blockIdx.x * K * kdim + o] = s;
    }
    for (int o = threadIdx.x; o < K; o += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += cnts[w * K + o];
        cpart[(size_t)blockIdx.x * K + o] = (int)s;
    }
}

// Combine: stop test, centroid means, empty-cluster refill.
// state[0] = done, state[1] = assignments so far.
__global__ __launch_bounds__(1024) void k_update(const double* __restrict__ H, int64_t n, int kdim, int K,
                                                 const int* __restrict__ changed_part, int nb_assign,
                                                 const double* __restrict__ part, const int* __restrict__ cpart,
                                                 int nb_sum, const double* __restrict__ mind,
                                                 double* __restrict__ cent, int* __restrict__ state, int max_iter) {
    __shared__ int changed, iters;
    __shared__ int cnt[kMaxK];
    __shared__ double bestv[1024];
    __shared__ int64_t besti[1024];
    __shared__ int64_t used[kMaxK];
    {
        const int r = blockIdx.y;
        changed_part += (size_t)r * nb_assign;
        part += (size_t)r * nb_sum * K * kdim;
        cpart += (size_t)r * nb_sum * K;
        mind += (size_t)r * n;
        cent += (size_t)r * K * kdim;
        state += 2 * r;
    }
    if (state[0]) return;
    // the counts are integers: shared atomics give the exact sums
    if (threadIdx.x == 0) changed = 0;
    if (threadIdx.x < K) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < nb_assign; b += blockDim.x) atomicAdd(&changed, changed_part[b]);
    for (int o = threadIdx.x; o < nb_sum * K; o += blockDim.x) atomicAdd(&cnt[o % K], cpart[o]);
    // the assignment count, read and advanced by one thread, shared with all
    if (threadIdx.x == 0) {
        iters = state[1] + 1;
        state[1] = iters;
    }
    __syncthreads();
    if (changed == 0 || iters >= max_iter) {
        if (threadIdx.x == 0) state[0] = 1;
        return;
    }
    // centroid sums in a fixed order: P interleaved slices of the blocks per
    // output (bestv as scratch), then the slices in order
    const int O = K * kdim;
    if (O <= (int)blockDim.x) {
        const int P = blockDim.x / O;
        const int t = threadIdx.x;
        if (t < P * O) {
            const int o = t % O, sl = t / O;
            double s0 = 0.0;
            int b = sl;
            // blocks sl, sl + P, ... in order, eight loads in flight
            for (; b + 7 * P < nb_sum; b += 8 * P) {
                double x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = part[(size_t)(b + u * P) * O + o];
#pragma unroll
                for (int u = 0; u < 8; ++u) s0 += x[u];
            }
            for (; b < nb_sum; b += P) s0 += part[(size_t)b * O + o];
            bestv[t] = s0;
        }
        __syncthreads();
        if (t < O) {
            const int j = t / kdim;
            if (cnt[j] > 0) {
                double s0 = 0.0;
                for (int sl = 0; sl < P; ++sl) s0 += bestv[sl * O + t];
                cent[t] = s0 / (double)cnt[j];
            }
        }
    } else {
        for (int o = threadIdx.x; o < O; o += blockDim.x) {
            const int j = o / kdim;
            if (cnt[j] > 0) {
                double s0 = 0.0;
                for (int b = 0; b < nb_sum; ++b) s0 += part[(size_t)b * O + o];
                cent[o] = s0 / (double)cnt[j];
            }
        }
    }
    __syncthreads();
    int nused = 0;
    for (int j = 0; j < K; ++j) {
        if (cnt[j] > 0) continue;
        // farthest row from its own centroid among rows not yet used
        double bv = -1.0;
        int64_t bi = INT64_MAX;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            bool u = false;
            for (int q = 0; q < nused; ++q) u = u || used[q] == i;
            if (u) continue;
            const double v = mind[i];
            if (v > bv) {
                bv = v;
                bi = i;
            }
        }
        bestv[threadIdx.x] = bv;
        besti[threadIdx.x] = bi;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                const double v2 = bestv[threadIdx.x + w];
                const int64_t i2 = besti[threadIdx.x + w];
                if (v2 > bestv[threadIdx.x] || (v2 == bestv[threadIdx.x] && i2 < besti[threadIdx.x])) {
                    bestv[threadIdx.x] = v2;
                    besti[threadIdx.x] = i2;
                }
            }
            __syncthreads();
        }
        const int64_t pick = besti[0];
        if (threadIdx.x < kdim && pick < n) cent[j * kdim + threadIdx.x] = H[(int64_t)threadIdx.x * n + pick];
        if (threadIdx.x == 0) used[nused] = pick;
        ++nused;
        __syncthreads();
    }
}

// Per-block sums of mind (inertia), fixed tree.
__global__ __launch_bounds__(kKmThreads) void k_sum(const double* __restrict__ v, int64_t n,
                                                    double* __restrict__ part, int cst) {
    __shared__ double red[kKmThreads];
    v += (size_t)blockIdx.y * n;
    part += (size_t)blockIdx.y * cst;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kKmThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// first[j] = smallest row with label j (labels < K <= 64; atomicMin: order
// independent).  A thread's rows increase, so only the first row of each
// label it meets can be its minimum: one shared atomic per thread and label,
// then one global atomic per block and label.
__global__ __launch_bounds__(kKmThreads) void k_first(const int32_t* __restrict__ lab, int64_t n, int K,
                                                       long long* __restrict__ first) {
    __shared__ long long smin[kMaxK];
    for (int j = threadIdx.x; j < K; j += kKmThreads) smin[j] = LLONG_MAX;
    __syncthreads();
    uint64_t seen = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int l = lab[i];
        if (!((seen >> l) & 1)) {
            seen |= 1ull << l;
            atomicMin(&smin[l], (long long)i);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < K; j += kKmThreads)
        if (smin[j] != LLONG_MAX) atomicMin(&first[j], smin[j]);
}

__global__ void k_relabel(const int32_t* __restrict__ lab, int64_t n, const int32_t* __restrict__ map,
                          int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = map[lab[i]];
}

// The first k-means++ pick of every restart: row floor(u n) of its first draw.
__global__ void k_first_pick(int R, int64_t n, uint64_t seed, int64_t* __restrict__ idxp) {
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        int64_t i0 = (int64_t)(sm_uniform(seed, (uint64_t)r, 0) * (double)n);
        if (i0 >= n) i0 = n - 1;
        idxp[r] = i0;
    }
}

// The best restart: each restart's inertia is its per-block partial sums of
// k_sum added in block order (one thread per restart); the smallest wins,
// ties to the earliest restart, and a restart whose inertia is not below
// infinity (or NaN) never does (restart 0 if none is).  kst[0] = its
// inertia, kst[1] = its index.
__global__ __launch_bounds__(kKmThreads) void k_best_restart(const double* __restrict__ part, int nb, int cst, int R,
                                                              double* __restrict__ kst) {
    __shared__ double sb[kKmThreads];
    __shared__ int si[kKmThreads];
    const int none = 0x7fffffff;
    double best = INFINITY;
    int bi = none;
    for (int r = threadIdx.x; r < R; r += kKmThreads) {
        const double* p = part + (size_t)r * cst;
        double s = 0.0;
        int b = 0;
        for (; b + 16 <= nb; b += 16) {
            double x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) x[u] = p[b + u];
#pragma unroll
            for (int u = 0; u < 16; ++u) s += x[u];
        }
        for (; b < nb; ++b) s += p[b];
        if (s < best) {
            best = s;
            bi = r;
        }
    }
    sb[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = kKmThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double ob = sb[threadIdx.x + w];
            const int oi = si[threadIdx.x + w];
            if (ob < sb[threadIdx.x] || (ob == sb[threadIdx.x] && oi < si[threadIdx.x])) {
                sb[threadIdx.x] = ob;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        kst[0] = sb[0];
        kst[1] = (double)(si[0] == none ? 0 : si[0]);
    }
}

// The best restart's labels.
__global__ void k_copy_best(const double* __restrict__ kst, const int32_t* __restrict__ lab, int64_t n,
                            int32_t* __restrict__ dst) {
    const int64_t off = (int64_t)kst[1] * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = lab[off + i];
}

static int grid_n(int64_t n, int cap) {
    int64_t g = (n + kKmThreads - 1) / kKmThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

static int labels_impl(sfairsc_graph* g, const double* H, int kdim, int K, int R, uint64_t seed, int max_iter,
                       int32_t* labels, double* inertia_out, hipStream_t s) {
    const int64_t n = g->n;
    KmWork& w = g->km;
    const int nchunks = (int)((n + kChunk - 1) / kChunk);
    const int nb = grid_n(n, kKmMaxBlocks);
    const int nbs = std::max(1, std::min<int>(nb, 256));
    const int cst = std::max(std::max(nchunks, nb), K);  // per-restart stride of csum
    // every restart has its own slices: the restarts run side by side, each
    // kernel launch covering all of them (restart = blockIdx.y), each
    // restart's arithmetic exactly that of a restart run alone
    SF_TRY(w.d2.ensure((size_t)R * n * sizeof(double)));
    SF_TRY(w.cs.ensure((size_t)R * cst * sizeof(double)));
    SF_TRY(w.cent.ensure((size_t)R * K * kdim * sizeof(double)));
    SF_TRY(w.lab.ensure((size_t)R * n * sizeof(int32_t)));
    SF_TRY(w.best.ensure((size_t)n * sizeof(int32_t)));
    SF_TRY(w.part.ensure((size_t)R * nbs * std::max(K * kdim, 2 * K) * sizeof(double)));
    SF_TRY(w.misc.ensure((size_t)R * (nb + nbs * K + 2) * sizeof(int) + ((size_t)R + 16) * sizeof(int64_t)));
    double* d2 = w.d2.as<double>();  // D^2 during seeding, then min distances
    double* csum = w.cs.as<double>();
    double* cent = w.cent.as<double>();
    int32_t* lab = w.lab.as<int32_t>();
    int32_t* best = w.best.as<int32_t>();
    double* part = w.part.as<double>();
    int64_t* idxp = reinterpret_cast<int64_t*>(w.misc.p);                        // [R]
    double* kst = reinterpret_cast<double*>(idxp + R);                            // best inertia, restart
    int* state = reinterpret_cast<int*>(kst + 8);                                 // [R][2]
    int* changed_part = state + 2 * (size_t)R;                                    // [R][nb]
    int* cpart = changed_part + (size_t)R * nb;                                   // [R][nbs][K]
    const size_t sum_lds = (size_t)(kKmThreads / 64) * K * (kdim + 1) * sizeof(double);

    // k-means++ seeding, all restarts at once
    k_first_pick<<<1, 256, 0, s>>>(R, n, seed, idxp);
    for (int t = 0; t < K; ++t) {
        if (t > 0) {
            k_chunk_sums<<<dim3(nchunks, R), kKmThreads, 0, s>>>(d2, n, csum, cst);
            k_pp_pick<<<dim3(1, R), 64, 0, s>>>(d2, csum, cst, nchunks, n, seed, t, idxp);
        }
        k_pp_update<<<dim3(grid_n(n, 2048), R), kKmThreads, 0, s>>>(H, n, kdim, K, idxp, t, cent, d2);
    }
    SF_HIP(hipGetLastError());
    // Lloyd, all restarts at once; a finished restart's launches return at
    // once, and every eighth round the host checks whether all have finished
    k_fill_i32<<<grid_n((int64_t)R * n, 4096), kKmThreads, 0, s>>>(lab, (int64_t)R * n, -1);
    SF_HIP(hipMemsetAsync(state, 0, 2 * (size_t)R * sizeof(int), s));
    std::vector<int> hstate(2 * (size_t)R, 0);
    while (true) {
        for (int it = 0; it < 8; ++it) {
            if (kdim <= 8)
                k_assign<8><<<dim3(nb, R), kKmThreads, 0, s>>>(H, n, kdim, K, cent, lab, d2, changed_part, state);
            else if (kdim <= 16)
                k_assign<16><<<dim3(nb, R), kKmThreads, 0, s>>>(H, n, kdim, K, cent, lab, d2, changed_part, state);
            else if (kdim <= 32)
                k_assign<32><<<dim3(nb, R), kKmThreads, 0, s>>>(H, n, kdim, K, cent, lab, d2, changed_part, state);
            else
                k_assign<64><<<dim3(nb, R), kKmThreads, 0, s>>>(H, n, kdim, K, cent, lab, d2, changed_part, state);
            k_cluster_sums<<<dim3(nbs, R), kKmThreads, sum_lds, s>>>(H, n, kdim, K, lab, part, cpart, state);
            k_update<<<dim3(1, R), 1024, 0, s>>>(H, n, kdim, K, changed_part, nb, part, cpart, nbs, d2, cent, state,
                                                 max_iter);
        }
        SF_HIP(hipGetLastError());
        SF_HIP(hipMemcpyAsync(hstate.data(), state, 2 * (size_t)R * sizeof(int), hipMemcpyDeviceToHost, s));
        SF_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (int r = 0; r < R; ++r) all = all && hstate[2 * (size_t)r] != 0;
        if (all) break;
    }
    // inertias and the best restart on the device
    k_sum<<<dim3(nb, R), kKmThreads, 0, s>>>(d2, n, csum, cst);
    k_best_restart<<<1, kKmThreads, 0, s>>>(csum, nb, cst, R, kst);
    k_copy_best<<<grid_n(n, 2048), kKmThreads, 0, s>>>(kst, lab, n, best);
    SF_HIP(hipGetLastError());
    double best_inertia = INFINITY;
    SF_HIP(hipMemcpyAsync(&best_inertia, kst, sizeof(double), hipMemcpyDeviceToHost, s));
    // renumber by first appearance
    long long* first = reinterpret_cast<long long*>(part);
    std::vector<long long> hfirst(K, (long long)INT64_MAX);
    SF_HIP(hipMemcpyAsync(first, hfirst.data(), K * sizeof(long long), hipMemcpyHostToDevice, s));
    k_first<<<grid_n(n, 2048), kKmThreads, 0, s>>>(best, n, K, first);
    SF_HIP(hipMemcpyAsync(hfirst.data(), first, K * sizeof(long long), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    std::vector<int> order(K);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hfirst[a] < hfirst[b]; });
    std::vector<int32_t> map(K);
    for (int q = 0; q < K; ++q) map[order[q]] = q;
    int32_t* dmap = reinterpret_cast<int32_t*>(csum);
    SF_HIP(hipMemcpyAsync(dmap, map.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
    k_relabel<<<grid_n(n, 2048), kKmThreads, 0, s>>>(best, n, dmap, labels);
    SF_HIP(hipGetLastError());
    SF_HIP(hipStreamSynchronize(s));
    if (inertia_out) *inertia_out = best_inertia;
    return SFAIRSC_OK;
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" int sfairsc_labels(sfairsc_graph_t g, const double* H, int32_t kdim, int32_t n_clusters,
                              int32_t n_restarts, uint64_t seed, int32_t max_iter, int32_t* labels, double* inertia,
                              hipStream_t stream) {
    if (!g || !H || !labels) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (kdim < 1 || kdim > kMaxK) return set_error(SFAIRSC_E_ARG, "kdim=%d outside [1, %d]", kdim, kMaxK);
    if (n_clusters < 2 || n_clusters > kMaxK || n_clusters > g->n)
        return set_error(SFAIRSC_E_ARG, "n_clusters=%d out of range", n_clusters);
    if (n_restarts < 1) return set_error(SFAIRSC_E_ARG, "n_restarts must be >= 1");
    if ((size_t)(256 / 64) * n_clusters * (kdim + 1) * sizeof(double) > 65536)
        return set_error(SFAIRSC_E_ARG, "n_clusters * (kdim + 1) must not exceed 2048");
    if (max_iter <= 0) max_iter = 300;
    return labels_impl(g, H, kdim, n_clusters, n_restarts, seed, max_iter, labels, inertia, stream);
}
