// The deflated operator L^sigma = P (L_n - sigma I) P + sigma I (eq. asigma),
// applied to a block of b <= 32 vectors as the matvec formula of Section 3.4:
//   S  = C^T X                              (group-segmented reduction)
//   X' = P X = X - C G^{-1} S               (eq. mv-Pw, G = C^T C)
//   T  = L_n X'                             (CSR SpMM; epilogue sums C^T T)
//   Y  = P T - sigma X' + sigma X = T - C G^{-1} (C^T T - sigma S)
// C is never formed.  With F from Lemma 2.1 (first h-1 groups kept),
//   (C^T Z)_s   = A_s - p_s sum_t A_t,  A_t = sum_{i in V_t} c_i Z_i,
//   (C U)_i     = c_i R_{g_i},  R_s = U_s - q (s < h-1),  R_{h-1} = -q,
//   q           = sum_{s<h-1} p_s U_s,
// with c_i = d_i^{-1/2} (normalized) or 1, p_s = |V_s| / n.
//
// The solver applies the same operator reassociated (op_apply_t):
//   T = L_n P X = T0 - (L_n C) U_in,  T0 = L_n X,  U_in = G^{-1} C^T X,
//   C^T T = C^T T0 - (C^T L_n C) U_in,
// with L_n C and C^T L_n C formed once per graph.  The block's compaction
// then also sums C^T X, the sparse product reads the block itself and sums
// C^T T0, and one kernel turns both into the tables of both corrections:
// three launches instead of five, and no pass between the two reductions.
//
// Every reduction has a fixed order (per-block partials combined in block
// order), so results are bitwise reproducible run to run.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"
#include "reduce.h"

namespace sfairsc {

constexpr int kSpmmThreads = 512;            // 8 waves
constexpr int kSpmmWaves = kSpmmThreads / 64;
#ifndef SF_SPMM_MAX_BLOCKS
#define SF_SPMM_MAX_BLOCKS 1024
#endif
constexpr int kSpmmMaxBlocks = SF_SPMM_MAX_BLOCKS;
constexpr int kProjThreads = 256;
constexpr int kProjMaxBlocks = 256;
constexpr int kFinThreads = 1024;

// 16-byte vector of 4 floats or 2 doubles.
template <class VT>
struct Vec16;
template <>
struct Vec16<float> {
    static constexpr int N = 4;
    float v[4];
    __device__ static Vec16 load(const float* p) {
        float4 t = *reinterpret_cast<const float4*>(p);
        return Vec16{{t.x, t.y, t.z, t.w}};
    }
    __device__ void store(float* p) const { *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]); }
};
template <>
struct Vec16<double> {
    static constexpr int N = 2;
    double v[2];
    __device__ static Vec16 load(const double* p) {
        double2 t = *reinterpret_cast<const double2*>(p);
        return Vec16{{t.x, t.y}};
    }
    __device__ void store(double* p) const { *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]); }
};

// ---------------------------------------------------------------------------
// A_s partial sums of c_i X_i per group.  part: [gridDim.x][h][b].
__global__ __launch_bounds__(kProjThreads) void k_proj_partial(const double* __restrict__ X, int ldx, int b,
                                                                int64_t n, const int32_t* __restrict__ grp,
                                                                const double* __restrict__ cs, int h,
                                                                double* __restrict__ part, const int* skip) {
    if (skip && *skip) return;
    extern __shared__ double acc[];  // [kProjThreads / 32][h][32]
    const int col = threadIdx.x & 31;
    const int rsub = threadIdx.x >> 5;
    constexpr int R = kProjThreads / 32;
    for (int o = threadIdx.x; o < R * h * 32; o += kProjThreads) acc[o] = 0.0;
    __syncthreads();
    if (col < b) {
        double* mine = acc + rsub * h * 32 + col;
        for (int64_t i = (int64_t)blockIdx.x * R + rsub; i < n; i += (int64_t)gridDim.x * R) {
            double c = cs ? cs[i] : 1.0;
            mine[grp[i] * 32] += c * X[i * ldx + col];
        }
    }
    __syncthreads();
    for (int o = threadIdx.x; o < h * b; o += kProjThreads) {
        const int g = o / b, j = o - g * b;
        double s = 0.0;
        for (int r = 0; r < R; ++r) s += acc[r * h * 32 + g * 32 + j];
        part[(size_t)blockIdx.x * h * b + o] = s;
    }
}

// The same partial sums for a power-of-two width b (4..32), with every lane
// busy: a wavefront covers 64 / b rows per load, each lane keeps eight
// groups' sums in registers (all h groups in ceil(h / 8) passes over its
// rows), and four rows per lane are loaded together.  The block handles a
// contiguous run of rows; its wavefronts' sums are combined in wavefront
// order.  part: [gridDim.x][h][b], as k_proj_partial.
__global__ __launch_bounds__(kProjThreads) void k_proj_partial_p2(const double* __restrict__ X, int ldx, int b,
                                                                   int64_t n, const int32_t* __restrict__ grp,
                                                                   const double* __restrict__ cs, int h,
                                                                   double* __restrict__ part, const int* skip) {
    if (skip && *skip) return;
    constexpr int NWV = kProjThreads / 64;
    __shared__ double wsum[NWV][kMaxGroups * 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lb = 31 - __clz(b);
    const int col = lane & (b - 1), rl = lane >> lb, rpw = 64 >> lb;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
    const int64_t step = (int64_t)NWV * rpw;
    for (int g0 = 0; g0 < h; g0 += 8) {
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        int64_t i = r0 + (int64_t)wave * rpw + rl;
        for (; i + 3 * step < r1; i += 4 * step) {
            int gi[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t r = i + u * step;
                gi[u] = grp[r] - g0;
                v[u] = (cs ? cs[r] : 1.0) * X[r * ldx + col];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[q] += (gi[u] == q) ? v[u] : 0.0;
        }
        for (; i < r1; i += step) {
            const int gi = grp[i] - g0;
            const double v = (cs ? cs[i] : 1.0) * X[i * ldx + col];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += (gi == q) ? v : 0.0;
        }
        for (int off = b; off < 64; off <<= 1)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += __shfl_xor(acc[q], off);
        if (rl == 0)
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (g0 + q < h) wsum[wave][(g0 + q) * b + col] = acc[q];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < h * b; o += kProjThreads) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) sum += wsum[w][o];
        part[(size_t)blockIdx.x * h * b + o] = sum;
    }
}

// X compacted (row stride b) in type OT and the per-block sums of c_i X~_i
// per group, X~ the compacted value (so that they are the sums of what the
// sparse product reads), output-major by XCD slot.  Power-of-two b (4..32),
// laid out as k_proj_partial_p2.
template <class OT>
__global__ __launch_bounds__(kProjThreads) void k_compact_sums(const double* __restrict__ X, int ldx, int b,
                                                               int64_t n, const int32_t* __restrict__ grp,
                                                               const double* __restrict__ cs, int h,
                                                               OT* __restrict__ Xp, double* __restrict__ part,
                                                               const int* skip) {
    if (skip && *skip) return;
    constexpr int NWV = kProjThreads / 64;
    __shared__ double wsum[NWV][kMaxGroups * 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lb = 31 - __clz(b);
    const int col = lane & (b - 1), rl = lane >> lb, rpw = 64 >> lb;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(n, r0 + per);
    const int64_t step = (int64_t)NWV * rpw;
    for (int g0 = 0; g0 < h; g0 += 8) {
        const bool wr = g0 == 0;  // the compacted block is written on the first pass
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        int64_t i = r0 + (int64_t)wave * rpw + rl;
        for (; i + 3 * step < r1; i += 4 * step) {
            int gi[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t r = i + u * step;
                gi[u] = grp[r] - g0;
                const OT xv = (OT)X[r * ldx + col];
                if (wr) Xp[r * b + col] = xv;
                v[u] = (cs ? cs[r] : 1.0) * (double)xv;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[q] += (gi[u] == q) ? v[u] : 0.0;
        }
        for (; i < r1; i += step) {
            const int gi = grp[i] - g0;
            const OT xv = (OT)X[i * ldx + col];
            if (wr) Xp[i * b + col] = xv;
            const double v = (cs ? cs[i] : 1.0) * (double)xv;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += (gi == q) ? v : 0.0;
        }
        for (int off = b; off < 64; off <<= 1)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += __shfl_xor(acc[q], off);
        if (rl == 0)
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (g0 + q < h) wsum[wave][(g0 + q) * b + col] = acc[q];
    }
    __syncthreads();
    const int rowlen = xcd_row(gridDim.x), sl = xcd_slot(blockIdx.x, gridDim.x);
    for (int o = threadIdx.x; o < h * b; o += kProjThreads) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) sum += wsum[w][o];
        part[(size_t)o * rowlen + sl] = sum;
    }
}

static void launch_proj_partial(const double* X, int ldx, int b, int64_t n, const int32_t* grp, const double* cs,
                                int h, double* part, int nblk, const int* skip, hipStream_t s) {
    if (b >= 4 && b <= 32 && (b & (b - 1)) == 0)
        k_proj_partial_p2<<<nblk, kProjThreads, 0, s>>>(X, ldx, b, n, grp, cs, h, part, skip);
    else
        k_proj_partial<<<nblk, kProjThreads, (size_t)(kProjThreads / 32) * h * 32 * sizeof(double), s>>>(
            X, ldx, b, n, grp, cs, h, part, skip);
}

// Combine per-block partial group sums and solve with G^{-1}.
//   A = sum over blocks;  Z_s = A_s - p_s sum_t A_t  (s < h-1)
//   if S_sub: Z -= sigma * S_sub   (output side: C^T T - sigma C^T X)
//   U = Ginv Z; R table as in the file header.  Optionally store Z in S_out.
__global__ __launch_bounds__(kFinThreads) void k_group_finalize(const double* __restrict__ part, int nblk, int h,
                                                                 int b, const double* __restrict__ gpar,
                                                                 const double* __restrict__ S_sub, double sigma,
                                                                 double* __restrict__ S_out,
                                                                 double* __restrict__ Rtab, const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[kFinThreads];
    __shared__ double A[kMaxGroups * 32];
    __shared__ double U[kMaxGroups * 32];
    const int O = h * b;              // <= kFinThreads since h, b <= 32
    const int P = kFinThreads / O;    // threads per output
    const int t = threadIdx.x;
    {
        // eight independent accumulators keep several partial loads in flight
        const int o = t % O, sub = t / O;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, s5 = 0.0, s6 = 0.0, s7 = 0.0;
        if (sub < P) {
            int blk = sub;
            for (; blk + 7 * P < nblk; blk += 8 * P) {
                s0 += part[(size_t)blk * O + o];
                s1 += part[(size_t)(blk + P) * O + o];
                s2 += part[(size_t)(blk + 2 * P) * O + o];
                s3 += part[(size_t)(blk + 3 * P) * O + o];
                s4 += part[(size_t)(blk + 4 * P) * O + o];
                s5 += part[(size_t)(blk + 5 * P) * O + o];
                s6 += part[(size_t)(blk + 6 * P) * O + o];
                s7 += part[(size_t)(blk + 7 * P) * O + o];
            }
            for (; blk < nblk; blk += P) s0 += part[(size_t)blk * O + o];
        }
        red[t] = ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7));
    }
    __syncthreads();
    if (t < O) {
        double tot = 0.0;
        for (int q = 0; q < P; ++q) tot += red[q * O + t];
        A[(t / b) * 32 + t % b] = tot;
    }
    __syncthreads();
    const int m = h - 1;
    const double* p = gpar;
    const double* Ginv = gpar + h;
    const int j = t;
    if (j < b) {
        double tot = 0.0;
        for (int s = 0; s < h; ++s) tot += A[s * 32 + j];
        // Z_s = (C^T Z)_s, reusing red[] as scratch: red[s * 32 + j]
        for (int s = 0; s < m; ++s) {
            double z = A[s * 32 + j] - p[s] * tot;
            if (S_out) S_out[s * 32 + j] = z;
            if (S_sub) z -= sigma * S_sub[s * 32 + j];
            red[s * 32 + j] = z;
        }
        double q = 0.0;
        for (int s = 0; s < m; ++s) {
            double u = 0.0;
            for (int r = 0; r < m; ++r) u += Ginv[s * m + r] * red[r * 32 + j];
            U[s * 32 + j] = u;
            q += p[s] * u;
        }
        for (int s = 0; s < m; ++s) Rtab[s * 32 + j] = U[s * 32 + j] - q;
        Rtab[m * 32 + j] = -q;
    } else if (j < 32) {
        for (int s = 0; s < h; ++s) Rtab[s * 32 + j] = 0.0;
        if (S_out)
            for (int s = 0; s < m; ++s) S_out[s * 32 + j] = 0.0;
    }
}

// Both tables of the reassociated operator from the per-block sums of c_i X_i
// (partx, nbx blocks: the compaction) and of c_i T0_i (partt, nbt blocks: the
// sparse product's epilogue), T0 = L_n X, both output-major by XCD slot (sum
// s of column j in row s b + j):
//   S = C^T X,  U_in = G^{-1} S                         -> Utab [h-1][32]
//   C^T T = C^T T0 - (C^T L_n C) U_in                   (ctlc [h-1][32])
//   U_out = G^{-1} (C^T T - sigma S), R table of U_out  -> Rtab [h][32]
// (C^T Z as in the file header).  Nothing here mixes the block's columns:
// one workgroup per column j (32 of them, those past b write zeros), one
// wavefront per sum with its lanes over the blocks.
constexpr int kFin2Threads = 1024;
__global__ __launch_bounds__(kFin2Threads) void k_group_finalize2(const double* __restrict__ partx, int nbx,
                                                                   const double* __restrict__ partt, int nbt, int h,
                                                                   int b, const double* __restrict__ gpar,
                                                                   const double* __restrict__ ctlc, double sigma,
                                                                   double* __restrict__ Rtab,
                                                                   double* __restrict__ Utab, const int* skip) {
    if (skip && *skip) return;
    __shared__ double A[2][kMaxGroups];
    __shared__ double gp[kMaxGroups + kMaxGroups * kMaxGroups];
    __shared__ double cl[kMaxGroups * kMaxGroups];
    __shared__ double Z[kMaxGroups], U[kMaxGroups], W[kMaxGroups];
    const int j = blockIdx.x, m = h - 1;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (j >= b) {
        for (int s = t; s < h; s += kFin2Threads) Rtab[s * 32 + j] = 0.0;
        for (int s = t; s < m; s += kFin2Threads) Utab[s * 32 + j] = 0.0;
        return;
    }
    for (int e = t; e < h + m * m; e += kFin2Threads) gp[e] = gpar[e];
    for (int e = t; e < m * m; e += kFin2Threads) cl[e] = ctlc[(e / m) * 32 + e % m];
    for (int r = w; r < 2 * h; r += kFin2Threads / 64) {
        const int nb = r < h ? nbx : nbt, rowlen = xcd_row(nb);
        const double* src = r < h ? partx + ((size_t)r * b + j) * rowlen : partt + ((size_t)(r - h) * b + j) * rowlen;
        // eight loads per lane in flight at once
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int sl = lane;
        if (rowlen == nb) {  // every slot written
            for (; sl + 7 * 64 < rowlen; sl += 8 * 64)
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] += src[sl + u * 64];
        }
#pragma unroll 4
        for (; sl < rowlen; sl += 64) {
            const double v = src[sl];
            if (xcd_valid(sl, nb)) a[0] += v;
        }
        double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) A[r < h ? 0 : 1][r < h ? r : r - h] = v;
    }
    __syncthreads();
    const double* p = gp;
    const double* Ginv = gp + h;
    double tx = 0.0, tt = 0.0;
    for (int s = 0; s < h; ++s) {
        tx += A[0][s];
        tt += A[1][s];
    }
    if (t < m) Z[t] = A[0][t] - p[t] * tx;  // S
    __syncthreads();
    if (t < m) {
        double u = 0.0;
        for (int r = 0; r < m; ++r) u += Ginv[t * m + r] * Z[r];
        U[t] = u;
        Utab[t * 32 + j] = u;
    }
    __syncthreads();
    if (t < m) {  // C^T T - sigma S
        double z = A[1][t] - p[t] * tt;
        for (int r = 0; r < m; ++r) z -= cl[t * m + r] * U[r];
        W[t] = z - sigma * Z[t];
    }
    __syncthreads();
    if (t < m) {  // U_out
        double u = 0.0;
        for (int r = 0; r < m; ++r) u += Ginv[t * m + r] * W[r];
        Z[t] = u;
    }
    __syncthreads();
    if (t < h) {
        double q = 0.0;
        for (int s = 0; s < m; ++s) q += p[s] * Z[s];
        Rtab[t * 32 + j] = (t < m ? Z[t] : 0.0) - q;
    }
}

// C compact (n x lcw, double): C[i][s] = c_i (1[g_i = s] - p_s) for s < h-1,
// zero in the padding columns.
__global__ __launch_bounds__(256) void k_build_c(int64_t n, int m, int lcw, const int32_t* __restrict__ grp,
                                                  const double* __restrict__ cs, const double* __restrict__ gpar,
                                                  double* __restrict__ Cm) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n * lcw;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / lcw;
        const int s = (int)(idx - i * lcw);
        double v = 0.0;
        if (s < m) v = (cs ? cs[i] : 1.0) * ((grp[i] == s ? 1.0 : 0.0) - gpar[s]);
        Cm[idx] = v;
    }
}

// X'_i = X_i - c_i R_{g_i}, written compact (stride BW) in type OT; without
// a table (Rtab == nullptr) X itself.
template <class OT>
__global__ __launch_bounds__(256) void k_proj_apply(const double* __restrict__ X, int ldx, int b, int BW, int64_t n,
                                                     const int32_t* __restrict__ grp, const double* __restrict__ cs,
                                                     const double* __restrict__ Rtab, OT* __restrict__ Xp,
                                                     const int* skip) {
    if (skip && *skip) return;
    const int64_t total = n * BW;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / BW;
        int j = (int)(idx - i * BW);
        double v = 0.0;
        if (j < b) {
            v = X[i * ldx + j];
            if (Rtab) v -= (cs ? cs[i] : 1.0) * Rtab[grp[i] * 32 + j];
        }
        Xp[idx] = (OT)v;
    }
}

// T = diag * X' - W X' (CSR), epilogue: per-group sums of c_i T_i into
// part[block][h][b], or (om) output-major by XCD slot (xcd_slot) for the
// column-parallel finalisation.  X', T compact n x BW in type VT; the
// products accumulate in VT (float in mixed precision).
//
// A wavefront takes RPW rows at once, G = 64 / RPW lanes each.  A row's
// nonzeros go in chunks of G: one coalesced load of their columns and
// values, then every gather of the chunk issued back to back (G / NS per
// lane, NS = G / LPR nonzeros per instruction, LPR lanes per 16-byte row
// vector).  Every row of the wavefront runs the wavefront's largest chunk
// count, so the cross-lane shuffles stay uniform.  Several rows per
// wavefront shorten the chain of dependent loads each wavefront walks
// through when rows are short.
template <class VT, int BW, int RPW>
__global__ __launch_bounds__(kSpmmThreads) void k_spmm(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const VT* __restrict__ val, const VT* __restrict__ diag,
                                                        const VT* __restrict__ X, VT* __restrict__ T, int64_t n,
                                                        const int32_t* __restrict__ grp,
                                                        const double* __restrict__ cs, int h, int b,
                                                        double* __restrict__ part, int om, const int* skip) {
    if (skip && *skip) return;
    using V = Vec16<VT>;
    constexpr int VEC = V::N;
    constexpr int LPR = BW / VEC;   // lanes per row vector
    constexpr int G = 64 / RPW;     // lanes per row
    constexpr int NS = G / LPR;     // nonzeros per gather instruction
    constexpr int IT = G / NS;      // gathers per lane per chunk (= LPR)
    static_assert(NS >= 1, "row group narrower than a row vector");
    extern __shared__ double gacc[];  // [kSpmmWaves][h][BW]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int sub = lane / G, sl = lane - sub * G;
    const int slot = sl / LPR;
    const int cl = sl - slot * LPR;
    const bool epi = part != nullptr;
    if (epi) {
        for (int o = threadIdx.x; o < kSpmmWaves * h * BW; o += kSpmmThreads) gacc[o] = 0.0;
        __syncthreads();
    }
    double* wacc = gacc + wave * h * BW;
    const int64_t rstride = (int64_t)gridDim.x * kSpmmWaves * RPW;
    for (int64_t row0 = ((int64_t)blockIdx.x * kSpmmWaves + wave) * RPW; row0 < n; row0 += rstride) {
        const int64_t row = row0 + sub;
        const bool rv = row < n;
        const int32_t a = rv ? rowptr[row] : 0;
        const int32_t e_end = rv ? rowptr[row + 1] : 0;
        // the wavefront's largest chunk count
        int nch = (e_end - a + G - 1) / G;
#pragma unroll
        for (int off = G; off < 64; off <<= 1) nch = max(nch, __shfl_xor(nch, off));
        VT acc[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = VT(0);
        int32_t base = a;
        for (int ch = 0; ch < nch; ++ch, base += G) {
            const int cnt = max(0, min(G, e_end - base));
            const int32_t my_col = sl < cnt ? col[base + sl] : 0;
            const VT my_val = sl < cnt ? val[base + sl] : VT(0);
            V x[IT];
            VT w[IT];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int src = it * NS + slot;
                const int32_t j = __shfl(my_col, sub * G + src);
                w[it] = __shfl(my_val, sub * G + src);
                if (src < cnt)
                    x[it] = V::load(X + (int64_t)j * BW + cl * VEC);
                else
                    x[it] = V{};
            }
#pragma unroll
            for (int it = 0; it < IT; ++it)
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += w[it] * x[it].v[v];
        }
#pragma unroll
        for (int off = LPR; off < G; off <<= 1)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += __shfl_xor(acc[v], off);
        V t;
        if (rv && slot == 0) {
            V xi = V::load(X + row * BW + cl * VEC);
            const VT dg = diag[row];
#pragma unroll
            for (int v = 0; v < VEC; ++v) t.v[v] = dg * xi.v[v] - acc[v];
            t.store(T + row * BW + cl * VEC);
        }
        if (epi) {
            // rows of one wavefront may share a group: add one row at a time
            const double c = (rv && cs) ? cs[row] : 1.0;
            const int gi = rv ? grp[row] : 0;
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                if (sub == r && rv && slot == 0) {
                    double* dst = wacc + gi * BW + cl * VEC;
#pragma unroll
                    for (int v = 0; v < VEC; ++v) dst[v] += c * (double)t.v[v];
                }
            }
        }
    }
    if (epi) {
        __syncthreads();
        for (int o = threadIdx.x; o < h * b; o += kSpmmThreads) {
            const int s = o / b, jj = o - s * b;
            double tot = 0.0;
            for (int w = 0; w < kSpmmWaves; ++w) tot += gacc[w * h * BW + s * BW + jj];
            if (om)
                part[(size_t)o * xcd_row(gridDim.x) + xcd_slot(blockIdx.x, gridDim.x)] = tot;
            else
                part[(size_t)blockIdx.x * h * b + o] = tot;
        }
    }
}

// Y_i = T_i - c_i R_{g_i} (T compact stride BW, type TT) into Y (double, ldy).
template <class TT>
__global__ __launch_bounds__(256) void k_defl_apply(const TT* __restrict__ T, int BW, int b, int64_t n,
                                                     const int32_t* __restrict__ grp, const double* __restrict__ cs,
                                                     const double* __restrict__ Rtab, double* __restrict__ Y, int ldy,
                                                     const int* skip) {
    if (skip && *skip) return;
    const int64_t total = n * b;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / b;
        int j = (int)(idx - i * b);
        double c = cs ? cs[i] : 1.0;
        Y[i * ldy + j] = (double)T[i * BW + j] - c * Rtab[grp[i] * 32 + j];
    }
}

// ---------------------------------------------------------------------------
static int pad_width(int b) { return b <= 4 ? 4 : b <= 8 ? 8 : b <= 16 ? 16 : 32; }

static int grid_rows(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

static int ensure_op(sfairsc_graph* g) {
    OpWork& w = g->op;
    const int64_t n = g->n;
    w.nblk_spmm = grid_rows(n, kSpmmWaves, kSpmmMaxBlocks);
    w.nblk_proj = grid_rows(n, kProjThreads / 32, kProjMaxBlocks);
    // (rows of the output-major layouts round the block count up to 8)
    // (the input sums may also come from the orthogonalisation's last pass,
    // over up to 256 blocks)
    SF_TRY(w.part_in.ensure((size_t)xcd_row(std::max(w.nblk_proj, 256)) * g->h * 32 * sizeof(double)));
    SF_TRY(w.part_out.ensure((size_t)xcd_row(w.nblk_spmm) * g->h * 32 * sizeof(double)));
    SF_TRY(w.small.ensure((size_t)5 * kMaxGroups * 32 * sizeof(double)));
    SF_TRY(w.xp.ensure((size_t)n * 32 * sizeof(double)));
    SF_TRY(w.t.ensure((size_t)n * 32 * sizeof(double)));
    return SFAIRSC_OK;
}

template <class VT>
static void launch_spmm(sfairsc_graph* g, int BW, const VT* X, VT* T, const VT* val, const VT* diag, int b,
                        double* part, int nblk, hipStream_t s, const int* skip, int om = 0) {
    size_t lds = part ? (size_t)kSpmmWaves * g->h * BW * sizeof(double) : 0;
    // rows per wavefront: short rows share a wavefront (at most 4)
    const double avg = g->n > 0 ? (double)g->nnz / (double)g->n : 0.0;
    const int rpw = avg <= 24.0 ? 4 : (avg <= 96.0 ? 2 : 1);
#define SF_SPMM_CASE(W, R)                                                                                     \
    k_spmm<VT, W, R><<<nblk, kSpmmThreads, lds, s>>>(g->rowptr, g->col, val, diag, X, T, g->n, g->grp, g->cs, \
                                                     g->h, b, part, om, skip)
#define SF_SPMM_RPW(W)                 \
    case W:                            \
        if (rpw == 4)                  \
            SF_SPMM_CASE(W, 4);        \
        else if (rpw == 2)             \
            SF_SPMM_CASE(W, 2);        \
        else                           \
            SF_SPMM_CASE(W, 1);        \
        break;
    switch (BW) {
        SF_SPMM_RPW(4)
        SF_SPMM_RPW(8)
        SF_SPMM_RPW(16)
        SF_SPMM_RPW(32)
    }
#undef SF_SPMM_RPW
#undef SF_SPMM_CASE
}

// The operator with a general constraint (g->qbas: X' = X - Q Q^T X, or
// g->memb: the same projections by LSQR).  For g->qbas: X' = X - Q Q^T X
// compact, the sparse product without the group epilogue, then
// Y = T - Q (Q^T T - sigma Q^T X) into Y (double, leading dimension ldy).
static int gen_apply(sfairsc_graph* g, const double* X, int ldx, int b, int mixed, double sigma, hipStream_t s,
                     hipEvent_t ev_begin, hipEvent_t ev_end, const int* skip, double* Y, int ldy) {
    OpWork& w = g->op;
    const int BW = pad_width(b);
    if (g->memb) {
        SF_TRY(lsqr_project_in(g, X, ldx, b, BW, mixed != 0, w.xp.p, s, skip));
    } else {
        SF_TRY(gen_project_in(g, X, ldx, b, BW, mixed != 0, w.xp.p, s, skip));
    }
    if (ev_begin) SF_HIP(hipEventRecord(ev_begin, s));
    if (mixed)
        launch_spmm<float>(g, BW, w.xp.as<float>(), w.t.as<float>(), g->val32, g->diag32, b, nullptr, w.nblk_spmm,
                           s, skip);
    else
        launch_spmm<double>(g, BW, w.xp.as<double>(), w.t.as<double>(), g->val64, g->diag64, b, nullptr,
                            w.nblk_spmm, s, skip);
    if (ev_end) SF_HIP(hipEventRecord(ev_end, s));
    SF_HIP(hipGetLastError());
    if (g->memb) return lsqr_correct(g, w.t.p, mixed != 0, BW, b, sigma, Y, ldy, s, skip);
    return gen_correct(g, w.t.p, mixed != 0, BW, b, sigma, Y, ldy, s, skip);
}

// Device buffers of one operator application with the group constraint.
struct OpBufs {
    double* part_in;  // [nblk_proj][h][b]
    int nblk_proj;
    double* part_out;  // [nblk_spmm][h][b]
    int nblk_spmm;
    double* small;  // R_in, S, R_out tables: 3 x [kMaxGroups][32]
    void* xp;       // projected input, n x BW (float or double)
    void* t;        // sparse product output, n x BW (float or double)
};

// S = C^T X, X' = P X, T = L_n X' (with C^T T), R_out table: everything up
// to the deflation of the output, in the buffers B.
static int op_apply_core(sfairsc_graph* g, const double* X, int ldx, int b, int mixed, double sigma, hipStream_t s,
                         hipEvent_t ev_begin, hipEvent_t ev_end, const int* skip, const OpBufs& B, OpOut* out) {
    const int BW = pad_width(b);
    const int64_t n = g->n;
    double* Rin = B.small;
    double* Sx = Rin + kMaxGroups * 32;
    double* Rout = Sx + kMaxGroups * 32;
    const int h = g->h;

    // S = C^T X, R_in table
    launch_proj_partial(X, ldx, b, n, g->grp, g->cs, h, B.part_in, B.nblk_proj, skip, s);
    k_group_finalize<<<1, kFinThreads, 0, s>>>(B.part_in, B.nblk_proj, h, b, g->gpar, nullptr, 0.0, Sx, Rin, skip);
    const int ga = grid_rows(n * BW, 256, 8192);
    if (mixed) {
        float* xp = static_cast<float*>(B.xp);
        float* t = static_cast<float*>(B.t);
        k_proj_apply<float><<<ga, 256, 0, s>>>(X, ldx, b, BW, n, g->grp, g->cs, Rin, xp, skip);
        if (ev_begin) SF_HIP(hipEventRecord(ev_begin, s));
        launch_spmm<float>(g, BW, xp, t, g->val32, g->diag32, b, B.part_out, B.nblk_spmm, s, skip);
        if (ev_end) SF_HIP(hipEventRecord(ev_end, s));
    } else {
        double* xp = static_cast<double*>(B.xp);
        double* t = static_cast<double*>(B.t);
        k_proj_apply<double><<<ga, 256, 0, s>>>(X, ldx, b, BW, n, g->grp, g->cs, Rin, xp, skip);
        if (ev_begin) SF_HIP(hipEventRecord(ev_begin, s));
        launch_spmm<double>(g, BW, xp, t, g->val64, g->diag64, b, B.part_out, B.nblk_spmm, s, skip);
        if (ev_end) SF_HIP(hipEventRecord(ev_end, s));
    }
    // U = G^{-1} (C^T T - sigma S), R_out table
    k_group_finalize<<<1, kFinThreads, 0, s>>>(B.part_out, B.nblk_spmm, h, b, g->gpar, Sx, sigma, nullptr, Rout,
                                               skip);
    SF_HIP(hipGetLastError());
    out->t = B.t;
    out->is_float = mixed != 0;
    out->BW = BW;
    out->rtab = Rout;
    return SFAIRSC_OK;
}

// Y = T - C R_out (the deflation of the output) into Y (double, ldy).
static int op_deflate(sfairsc_graph* g, const OpOut& o, int b, double* Y, int ldy, hipStream_t s, const int* skip) {
    const int64_t n = g->n;
    if (o.is_float)
        k_defl_apply<float><<<grid_rows(n * b, 256, 8192), 256, 0, s>>>((const float*)o.t, o.BW, b, n, g->grp, g->cs,
                                                                         o.rtab, Y, ldy, skip);
    else
        k_defl_apply<double><<<grid_rows(n * b, 256, 8192), 256, 0, s>>>((const double*)o.t, o.BW, b, n, g->grp,
                                                                          g->cs, o.rtab, Y, ldy, skip);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

// The reassociated form: group constraint, L C formed, and a power-of-two
// block width from 4 to 16 (the compaction's layout).  At 32 the launches it
// saves are a rounding error against millisecond kernels, and the L C term
// would land in the first orthogonalisation pass's widest variant, whose
// registers are already short.
static bool fused_fits(const sfairsc_graph* g, int b) {
    return g->h >= 2 && g->op.lcw > 0 && b >= 4 && b <= 16 && (b & (b - 1)) == 0;
}

int op_prepare_lc(sfairsc_graph* g, hipStream_t s) {
    const int h = g->h, m = h - 1;
    if (m < 1 || g->qbas || g->memb || g->op.lcw > 0) return SFAIRSC_OK;
    SF_TRY(ensure_op(g));
    OpWork& w = g->op;
    const int64_t n = g->n;
    const int lcw = pad_width(m);
    SF_TRY(w.lc.ensure((size_t)n * lcw * sizeof(double)));
    SF_TRY(w.ctlc.ensure((size_t)kMaxGroups * 32 * sizeof(double)));
    // C in the operator's input buffer, then L_n C by the FP64 sparse product
    double* Cm = w.xp.as<double>();
    k_build_c<<<grid_rows(n * lcw, 256, 8192), 256, 0, s>>>(n, m, lcw, g->grp, g->cs, g->gpar, Cm);
    launch_spmm<double>(g, lcw, Cm, w.lc.as<double>(), g->val64, g->diag64, m, nullptr, w.nblk_spmm, s, nullptr);
    // C^T (L_n C): the group sums of its columns combined as C^T Z (S_out);
    // the R table it also writes goes to a spare slot
    launch_proj_partial(w.lc.as<double>(), lcw, m, n, g->grp, g->cs, h, w.part_in.as<double>(), w.nblk_proj,
                        nullptr, s);
    double* spare = w.small.as<double>() + 4 * kMaxGroups * 32;
    k_group_finalize<<<1, kFinThreads, 0, s>>>(w.part_in.as<double>(), w.nblk_proj, h, m, g->gpar, nullptr, 0.0,
                                               w.ctlc.as<double>(), spare, nullptr);
    SF_HIP(hipGetLastError());
    w.lcw = lcw;
    return SFAIRSC_OK;
}

// The reassociated operator: X compacted (no projection), T0 = L_n X with
// both epilogue sums, then the two tables (R_out for C, U_in for L_n C).
static int op_apply_fused(sfairsc_graph* g, const double* X, int ldx, int b, int mixed, double sigma,
                          hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end, const int* skip, OpOut* out,
                          int prepared_nblk) {
    OpWork& w = g->op;
    const int BW = pad_width(b);
    const int64_t n = g->n;
    const int h = g->h;
    double* Rout = w.small.as<double>() + 2 * kMaxGroups * 32;
    double* Uin = w.small.as<double>() + 3 * kMaxGroups * 32;
    // the compact input and its group sums: already written by the last
    // orthogonalisation pass (prepared_nblk > 0 blocks of sums), or here
    const bool prep = prepared_nblk > 0;
    const int nblk_x = prep ? prepared_nblk : w.nblk_proj;
    if (mixed) {
        if (!prep)
            k_compact_sums<float><<<w.nblk_proj, kProjThreads, 0, s>>>(X, ldx, b, n, g->grp, g->cs, h,
                                                                     w.xp.as<float>(), w.part_in.as<double>(), skip);
        if (ev_begin) SF_HIP(hipEventRecord(ev_begin, s));
        launch_spmm<float>(g, BW, w.xp.as<float>(), w.t.as<float>(), g->val32, g->diag32, b,
                           w.part_out.as<double>(), w.nblk_spmm, s, skip, 1);
        if (ev_end) SF_HIP(hipEventRecord(ev_end, s));
    } else {
        if (!prep)
            k_compact_sums<double><<<w.nblk_proj, kProjThreads, 0, s>>>(X, ldx, b, n, g->grp, g->cs, h,
                                                                      w.xp.as<double>(), w.part_in.as<double>(), skip);
        if (ev_begin) SF_HIP(hipEventRecord(ev_begin, s));
        launch_spmm<double>(g, BW, w.xp.as<double>(), w.t.as<double>(), g->val64, g->diag64, b,
                            w.part_out.as<double>(), w.nblk_spmm, s, skip, 1);
        if (ev_end) SF_HIP(hipEventRecord(ev_end, s));
    }
    k_group_finalize2<<<32, kFin2Threads, 0, s>>>(w.part_in.as<double>(), nblk_x, w.part_out.as<double>(),
                                                  w.nblk_spmm, h, b, g->gpar, w.ctlc.as<double>(), sigma, Rout, Uin,
                                                  skip);
    SF_HIP(hipGetLastError());
    out->t = w.t.p;
    out->is_float = mixed != 0;
    out->BW = BW;
    out->rtab = Rout;
    out->lc = w.lc.as<double>();
    out->lcw = w.lcw;
    out->m = h - 1;
    out->utab = Uin;
    return SFAIRSC_OK;
}

int op_input_target(sfairsc_graph* g, int b, OpInput* in) {
    in->xp = nullptr;
    in->xsum = nullptr;
    if (g->qbas || g->memb || !fused_fits(g, b)) return SFAIRSC_OK;
    SF_TRY(ensure_op(g));
    in->xp = g->op.xp.p;
    in->xsum = g->op.part_in.as<double>();
    return SFAIRSC_OK;
}

int op_apply_t(sfairsc_graph* g, const double* X, int ldx, int b, int mixed, double sigma, hipStream_t s,
               hipEvent_t ev_begin, hipEvent_t ev_end, const int* skip, OpOut* out, int prepared_nblk) {
    if (b < 1 || b > kMaxBlock) return set_error(SFAIRSC_E_ARG, "block width %d outside [1, 32]", b);
    SF_TRY(ensure_op(g));
    if (g->qbas || g->memb) {
        // Y lands in the (no longer needed) projected-input buffer, in double
        const int BW = pad_width(b);
        SF_TRY(gen_apply(g, X, ldx, b, mixed, sigma, s, ev_begin, ev_end, skip, g->op.xp.as<double>(), BW));
        out->t = g->op.xp.p;
        out->is_float = false;
        out->BW = BW;
        out->rtab = nullptr;
        return SFAIRSC_OK;
    }
    if (fused_fits(g, b))
        return op_apply_fused(g, X, ldx, b, mixed, sigma, s, ev_begin, ev_end, skip, out, prepared_nblk);
    if (prepared_nblk > 0) return set_error(SFAIRSC_E_ARG, "internal: prepared operator input on the general path");
    OpWork& w = g->op;
    const OpBufs B{w.part_in.as<double>(), w.nblk_proj, w.part_out.as<double>(), w.nblk_spmm, w.small.as<double>(),
                   w.xp.p, w.t.p};
    return op_apply_core(g, X, ldx, b, mixed, sigma, s, ev_begin, ev_end, skip, B, out);
}

// The public operator keeps the paper's order: X' = P X first.
int op_apply(sfairsc_graph* g, const double* X, int ldx, double* Y, int ldy, int b, int mixed, double sigma,
             hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end, const int* skip) {
    if (b < 1 || b > kMaxBlock) return set_error(SFAIRSC_E_ARG, "block width %d outside [1, 32]", b);
    SF_TRY(ensure_op(g));
    if (g->qbas || g->memb) return gen_apply(g, X, ldx, b, mixed, sigma, s, ev_begin, ev_end, skip, Y, ldy);
    OpWork& w = g->op;
    const OpBufs B{w.part_in.as<double>(), w.nblk_proj, w.part_out.as<double>(), w.nblk_spmm, w.small.as<double>(),
                   w.xp.p, w.t.p};
    OpOut o;
    SF_TRY(op_apply_core(g, X, ldx, b, mixed, sigma, s, ev_begin, ev_end, skip, B, &o));
    return op_deflate(g, o, b, Y, ldy, s, skip);
}

// ---------------------------------------------------------------------------
// The operator without allocation: its scratch is a file-scope device array
// (one copy per GPU, held until the process ends), reached through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

// Device address of `scratch` on device dev, looked up once per device with
// that device current.
static int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kScratchDevices) return set_error(SFAIRSC_E_ARG, "device %d outside [0, %d)", dev, kScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        SF_HIP(hipGetDevice(&cur));
        if (cur != dev) SF_HIP(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return set_error(SFAIRSC_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SFAIRSC_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int op_apply_noalloc(sfairsc_graph* g, const double* X, double* Y, int b, int mixed, double sigma,
                            hipStream_t s) {
    if (g->qbas || g->memb)
        return set_error(SFAIRSC_E_ARG, "the no-allocation operator takes the group constraint only");
    const int64_t n = g->n;
    const int h = g->h;
    const int BW = pad_width(b);
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    const int nblk_spmm = grid_rows(n, kSpmmWaves, kSpmmMaxBlocks);
    const int nblk_proj = grid_rows(n, kProjThreads / 32, kProjMaxBlocks);
    const size_t o_in = 0;
    const size_t o_out = o_in + align256((size_t)nblk_proj * h * b * sizeof(double));
    const size_t o_small = o_out + align256((size_t)nblk_spmm * h * b * sizeof(double));
    const size_t o_xp = o_small + align256((size_t)5 * kMaxGroups * 32 * sizeof(double));
    const size_t o_t = o_xp + align256((size_t)n * BW * es);
    const size_t need = o_t + align256((size_t)n * BW * es);
    if (need > kNoAllocScratchBytes)
        return set_error(SFAIRSC_E_ARG,
                         "n = %lld with block width %d needs %zu bytes of scratch, more than the %zu of the "
                         "no-allocation operator",
                         (long long)n, b, need, kNoAllocScratchBytes);
    void* base = nullptr;
    SF_TRY(scratch_address(g->device, &base));
    char* p = static_cast<char*>(base);
    const OpBufs B{reinterpret_cast<double*>(p + o_in),  nblk_proj, reinterpret_cast<double*>(p + o_out), nblk_spmm,
                   reinterpret_cast<double*>(p + o_small), p + o_xp, p + o_t};
    OpOut o;
    SF_TRY(op_apply_core(g, X, b, b, mixed, sigma, s, nullptr, nullptr, nullptr, B, &o));
    return op_deflate(g, o, b, Y, b, s, nullptr);
}

// X_i -= c_i R_{g_i} in place (X double, leading dimension ldx, b columns).
__global__ __launch_bounds__(256) void k_proj_inplace(double* __restrict__ X, int ldx, int b, int64_t n,
                                                       const int32_t* __restrict__ grp, const double* __restrict__ cs,
                                                       const double* __restrict__ Rtab) {
    const int64_t total = n * b;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / b;
        int j = (int)(idx - i * b);
        double c = cs ? cs[i] : 1.0;
        X[i * ldx + j] -= c * Rtab[grp[i] * 32 + j];
    }
}

int op_project(sfairsc_graph* g, double* X, int ldx, int b, hipStream_t s) {
    if (b < 1 || b > kMaxBlock) return set_error(SFAIRSC_E_ARG, "block width %d outside [1, 32]", b);
    if (g->memb) return lsqr_project(g, X, ldx, b, s);
    if (g->qbas) return gen_project(g, X, ldx, b, s);
    SF_TRY(ensure_op(g));
    OpWork& w = g->op;
    double* Rin = w.small.as<double>();
    double* Sx = Rin + kMaxGroups * 32;
    const int h = g->h;
    launch_proj_partial(X, ldx, b, g->n, g->grp, g->cs, h, w.part_in.as<double>(), w.nblk_proj, nullptr, s);
    double* sums = Rin + 4 * kMaxGroups * 32;
    k_reduce_partials<<<reduce_grid(h * b), kRedElems * kRedSlices, 0, s>>>(w.part_in.as<double>(), w.nblk_proj,
                                                                            h * b, sums, nullptr);
    k_group_finalize<<<1, kFinThreads, 0, s>>>(sums, 1, h, b, g->gpar, nullptr, 0.0, Sx, Rin, nullptr);
    k_proj_inplace<<<grid_rows(g->n * b, 256, 8192), 256, 0, s>>>(X, ldx, b, g->n, g->grp, g->cs, Rin);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

// Pad / unpad copies between a user block of width b and the stride-BW layout.
template <class T>
__global__ void k_repack(const T* __restrict__ src, int lds_, T* __restrict__ dst, int ldd, int64_t n, int bcopy,
                         int bfill) {
    const int64_t total = n * bfill;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / bfill;
        int j = (int)(idx - i * bfill);
        dst[i * ldd + j] = j < bcopy ? src[i * lds_ + j] : T(0);
    }
}

int op_spmm_raw(sfairsc_graph* g, const void* X, void* T, int b, int mixed, hipStream_t s) {
    if (b < 1 || b > kMaxBlock) return set_error(SFAIRSC_E_ARG, "block width %d outside [1, 32]", b);
    SF_TRY(ensure_op(g));
    OpWork& w = g->op;
    const int BW = pad_width(b);
    const int64_t n = g->n;
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    const void* xin = X;
    void* tout = T;
    const bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)T % 16 == 0);
    if (BW != b || !aligned) {
        SF_TRY(w.xpad.ensure((size_t)n * BW * es));
        SF_TRY(w.ypad.ensure((size_t)n * BW * es));
        int gr = grid_rows(n * BW, 256, 8192);
        if (mixed)
            k_repack<float><<<gr, 256, 0, s>>>((const float*)X, b, w.xpad.as<float>(), BW, n, b, BW);
        else
            k_repack<double><<<gr, 256, 0, s>>>((const double*)X, b, w.xpad.as<double>(), BW, n, b, BW);
        xin = w.xpad.p;
        tout = w.ypad.p;
    }
    if (mixed)
        launch_spmm<float>(g, BW, (const float*)xin, (float*)tout, g->val32, g->diag32, b, nullptr, w.nblk_spmm, s,
                           nullptr);
    else
        launch_spmm<double>(g, BW, (const double*)xin, (double*)tout, g->val64, g->diag64, b, nullptr, w.nblk_spmm,
                            s, nullptr);
    if (BW != b || !aligned) {
        int gr = grid_rows(n * b, 256, 8192);
        if (mixed)
            k_repack<float><<<gr, 256, 0, s>>>(w.ypad.as<float>(), BW, (float*)T, b, n, b, b);
        else
            k_repack<double><<<gr, 256, 0, s>>>(w.ypad.as<double>(), BW, (double*)T, b, n, b, b);
    }
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" int sfairsc_apply_operator(sfairsc_graph_t g, const double* X, double* Y, int32_t b, int precision,
                                      double sigma, hipStream_t stream) {
    if (!g || !X || !Y) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (precision != SFAIRSC_PREC_FP64 && precision != SFAIRSC_PREC_MIXED)
        return set_error(SFAIRSC_E_ARG, "unknown precision %d", precision);
    if (b < 1 || b > kMaxBlock) return set_error(SFAIRSC_E_ARG, "block width %d outside [1, 32]", b);
    if (sigma <= 0.0) sigma = g->sigma;
    return op_apply(g, X, b, Y, b, b, precision == SFAIRSC_PREC_MIXED, sigma, stream);
}

extern "C" int sfairsc_apply_operator_noalloc(sfairsc_graph_t g, const double* X, double* Y, int32_t b,
                                              int precision, double sigma, hipStream_t stream) {
    if (!g || !X || !Y) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (precision != SFAIRSC_PREC_FP64 && precision != SFAIRSC_PREC_MIXED)
        return set_error(SFAIRSC_E_ARG, "unknown precision %d", precision);
    if (b < 1 || b > kMaxBlock) return set_error(SFAIRSC_E_ARG, "block width %d outside [1, 32]", b);
    if (sigma <= 0.0) sigma = g->sigma;
    return op_apply_noalloc(g, X, Y, b, precision == SFAIRSC_PREC_MIXED, sigma, stream);
}

extern "C" int sfairsc_spmm(sfairsc_graph_t g, const void* X, void* T, int32_t b, int precision,
                            hipStream_t stream) {
    if (!g || !X || !T) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (precision != SFAIRSC_PREC_FP64 && precision != SFAIRSC_PREC_MIXED)
        return set_error(SFAIRSC_E_ARG, "unknown precision %d", precision);
    return op_spmm_raw(g, X, T, b, precision == SFAIRSC_PREC_MIXED, stream);
}
