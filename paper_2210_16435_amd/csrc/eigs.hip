// Block Krylov-Schur (thick-restart block Lanczos) for the k smallest
// eigenpairs of L^sigma (Alg. 3 step 3; the paper calls ARPACK through
// MATLAB's eigs and needs only products with L^sigma, Section 3.4 (i)).
//
// Basis layout: V is n x ld, row-major (row i holds V[i, 0:ld]).  At any time
// columns [0, c) are the "complete" basis with Rayleigh quotient T_c (device,
// ld x ld row-major), columns [c, c+b) the next block V_next, and
//     L^sigma V[:, 0:c] = V[:, 0:c] T_c + V_next R E^T
// where R (b x b) couples V_next to the last block of the complete basis
// (E selects it).  One expansion:
//     Y = L^sigma V_next                 (operator, into columns [c+b, c+2b))
//     H1 = V^T Y,  Y -= V H1             (classical Gram-Schmidt ...
//     H2 = V^T Y,  Y -= V H2             ... twice), V = V[:, 0:c+b]
//     T[0:c+b, c:c+b] = H1 + H2 (and its mirror)
//     Y = Q R via Cholesky-QR twice      (Gram Y^T Y -> R1, Y R1^{-1}, again)
// Row-major storage lets every tall-skinny product read each basis row once,
// contiguously.  After ncv columns: Rayleigh-Ritz on T_c (GPU, FP64, rr.hip), the
// residual of Ritz pair i is ||R Z[c-b:c, i]||, and the p smallest Ritz
// vectors are kept (V <- V Z[:, 0:p]) with T_p = diag(theta).
//
// Reductions are two-stage with a fixed combination order: bitwise
// reproducible results.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace sfairsc {

// The float phase of a mixed solve stops at this relative residual (or at
// the requested tolerance if that is looser); FP64 takes it from there.
#ifndef SF_MIXED_TOL1
#define SF_MIXED_TOL1 5e-7
#endif
constexpr double kMixedTol1 = SF_MIXED_TOL1;

constexpr int kTsThreads = 256;
constexpr int kTsRows = 8;
constexpr int kTsAcc = (kLdMax * kMaxBlock + kTsThreads - 1) / kTsThreads;  // 28
constexpr int kTsMaxBlocks = 512;
constexpr int kRotRows = 32;
constexpr int kStatBlocks = 256;
constexpr int kStatsDoubles = kStatBlocks * 2 * kMaxK;
constexpr int kStatsIdx = kStatBlocks * kMaxK;

enum { TS_GRAM = 0, TS_UPD_GRAM = 1, TS_UPD_SYRK = 2, TS_MUL_SYRK = 3, TS_MUL = 4 };

// Tall-skinny kernel over row tiles.  Y = V[:, yoff : yoff+b].
//   TS_GRAM      part = V[:, 0:cv]^T Y
//   TS_UPD_GRAM  Y -= V[:, 0:cv] M (M: cv x b); part = V[:, 0:cv]^T Y
//   TS_UPD_SYRK  Y -= V[:, 0:cv] M;             part = Y^T Y
//   TS_MUL_SYRK  Y  = Y M (M: b x b);           part = Y^T Y
//   TS_MUL       Y  = Y M
// part[block][o] with o = j * Qd + q (Qd = cv for Gram, b for Syrk).
template <int MODE>
__global__ __launch_bounds__(kTsThreads) void k_ts(double* __restrict__ V, int ldv, int64_t n, int cv, int yoff,
                                                    int b, const double* __restrict__ M, double* __restrict__ part,
                                                    const int* skip) {
    if (skip && *skip) return;
    extern __shared__ double lds[];
    constexpr bool kUseV = (MODE == TS_GRAM || MODE == TS_UPD_GRAM || MODE == TS_UPD_SYRK);
    constexpr bool kUpd = (MODE == TS_UPD_GRAM || MODE == TS_UPD_SYRK);
    constexpr bool kMul = (MODE == TS_MUL_SYRK || MODE == TS_MUL);
    constexpr bool kGramOut = (MODE == TS_GRAM || MODE == TS_UPD_GRAM);
    constexpr bool kSyrkOut = (MODE == TS_UPD_SYRK || MODE == TS_MUL_SYRK);
    const int cvu = kUseV ? cv : 0;
    const int W = cvu + b;
    double* Vs = lds;                         // [kTsRows][W]
    double* Ms = Vs + kTsRows * W;            // [b][b] (multiply modes)
    const int msz = kMul ? b * b : 0;
    double* Yn = Ms + msz;                    // [kTsRows][b]
    const int tid = threadIdx.x;
    for (int o = tid; o < msz; o += kTsThreads) Ms[o] = M[o];

    const int Qd = kGramOut ? cv : b;
    const int O = kGramOut ? cv * b : (kSyrkOut ? b * b : 0);
    double acc[kTsAcc];
#pragma unroll
    for (int u = 0; u < kTsAcc; ++u) acc[u] = 0.0;

    const int64_t ntiles = (n + kTsRows - 1) / kTsRows;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * kTsRows;
        const int rows = (int)min<int64_t>(kTsRows, n - r0);
        __syncthreads();  // previous tile's readers are done (and Ms loaded)
        for (int idx = tid; idx < rows * W; idx += kTsThreads) {
            int r = idx / W, c = idx - r * W;
            int src = c < cvu ? c : yoff + (c - cvu);
            Vs[r * W + c] = V[(r0 + r) * ldv + src];
        }
        __syncthreads();
        for (int idx = tid; idx < rows * b; idx += kTsThreads) {
            int r = idx / b, j = idx - r * b;
            const double* vr = Vs + r * W;
            double y;
            if (kUpd) {
                y = vr[cvu + j];
                for (int q = 0; q < cv; ++q) y -= vr[q] * M[q * b + j];
            } else if (kMul) {
                y = 0.0;
                for (int q = 0; q < b; ++q) y += vr[q] * Ms[q * b + j];
            } else {
                y = vr[cvu + j];
            }
            Yn[r * b + j] = y;
            if (kUpd || kMul) V[(r0 + r) * ldv + yoff + j] = y;
        }
        __syncthreads();
        if (kGramOut || kSyrkOut) {
#pragma unroll
            for (int u = 0; u < kTsAcc; ++u) {
                const int o = tid + u * kTsThreads;
                if (o < O) {
                    const int j = o / Qd, q = o - j * Qd;
                    double s = acc[u];
                    for (int r = 0; r < rows; ++r) {
                        const double a = kGramOut ? Vs[r * W + q] : Yn[r * b + q];
                        s += a * Yn[r * b + j];
                    }
                    acc[u] = s;
                }
            }
        }
    }
    if (kGramOut || kSyrkOut) {
#pragma unroll
        for (int u = 0; u < kTsAcc; ++u) {
            const int o = tid + u * kTsThreads;
            if (o < O) part[(size_t)blockIdx.x * O + o] = acc[u];
        }
    }
}

// Sum Gram partials over blocks (fixed order).  H (cv x b, row-major) gets
// the sum; T[q, cact + j] is set (accumulate = 0) or incremented, and for
// q < cact so is the mirror T[cact + j, q].
__global__ void k_gram_reduce(const double* __restrict__ part, int nblk, int cv, int b, double* __restrict__ H,
                              double* __restrict__ T, int ldt, int cact, int accumulate, const int* skip) {
    if (skip && *skip) return;
    const int O = cv * b;
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    double s = 0.0;
    for (int blk = 0; blk < nblk; ++blk) s += part[(size_t)blk * O + o];
    const int j = o / cv, q = o - j * cv;
    H[q * b + j] = s;
    if (!T) return;
    double* t1 = T + (size_t)q * ldt + cact + j;
    *t1 = accumulate ? *t1 + s : s;
    if (q < cact) {
        double* t2 = T + (size_t)(cact + j) * ldt + q;
        *t2 = accumulate ? *t2 + s : s;
    }
}

// Cholesky of the b x b Gram G = Y^T Y (sum of partials), G = R^T R with R
// upper triangular; Rinv = R^{-1}.  pass 1: pivots below `thresh` flag a
// rank-deficient block (flag[0] = 1, flag[1] = cact) and G is saved.
// pass 2: R = R2 R1 becomes the coupling (Rc) and the diagonal block of T
// is symmetrised.
__global__ __launch_bounds__(1024) void k_chol(const double* __restrict__ part, int nblk, int b, int pass,
                                                double thresh, double* __restrict__ Gsave,
                                                double* __restrict__ R1, double* __restrict__ Rinv,
                                                double* __restrict__ Rc, double* __restrict__ T, int ldt, int cact,
                                                int* flag, const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[1024];
    __shared__ double G[kMaxBlock * kMaxBlock];
    __shared__ double R[kMaxBlock * kMaxBlock];
    __shared__ int bad;
    const int O = b * b;
    const int P = 1024 / O;
    const int t = threadIdx.x;
    {
        const int o = t % O, sub = t / O;
        double s = 0.0;
        if (sub < P)
            for (int blk = sub; blk < nblk; blk += P) s += part[(size_t)blk * O + o];
        red[t] = s;
    }
    if (t == 0) bad = 0;
    __syncthreads();
    if (t < O) {
        double tot = 0.0;
        for (int q = 0; q < P; ++q) tot += red[q * O + t];
        // partial index o = j * b + q  ->  G[q][j]
        const int j = t / b, q = t - j * b;
        G[q * b + j] = tot;
        R[t] = 0.0;
    }
    __syncthreads();
    if (pass == 1 && t < O) Gsave[t] = G[t];
    for (int k = 0; k < b; ++k) {
        if (t == 0) {
            double piv = G[k * b + k];
            if (!(piv > thresh)) {
                bad = 1;
                piv = 1.0;
            }
            R[k * b + k] = sqrt(piv);
        }
        __syncthreads();
        if (t > k && t < b) R[k * b + t] = G[k * b + t] / R[k * b + k];
        __syncthreads();
        for (int idx = t; idx < b * b; idx += blockDim.x) {
            const int i = idx / b, j = idx - i * b;
            if (i > k && j >= i) {
                G[i * b + j] -= R[k * b + i] * R[k * b + j];
                G[j * b + i] = G[i * b + j];
            }
        }
        __syncthreads();
    }
    if (bad) {
        if (t == 0) {
            flag[0] = 1;
            flag[1] = cact;
        }
        return;
    }
    if (t < b) {
        const int j = t;  // column j of R^{-1} by back substitution
        double x[kMaxBlock];
        for (int i = b - 1; i >= 0; --i) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int q = i + 1; q <= j; ++q) s -= R[i * b + q] * x[q];
            x[i] = (i <= j) ? s / R[i * b + i] : 0.0;
        }
        for (int i = 0; i < b; ++i) Rinv[i * b + j] = i <= j ? x[i] : 0.0;
    }
    if (pass == 1) {
        if (t < O) R1[t] = R[t];
    } else {
        if (t < O) {
            const int i = t / b, j = t - i * b;
            double s = 0.0;
            for (int q = i; q <= j; ++q) s += R[i * b + q] * R1[q * b + j];
            Rc[t] = (j >= i) ? s : 0.0;
            if (j > i && T) {
                double* a = T + (size_t)(cact + i) * ldt + cact + j;
                double* c = T + (size_t)(cact + j) * ldt + cact + i;
                const double m = 0.5 * (*a + *c);
                *a = m;
                *c = m;
            }
        }
    }
}

// Ritz vectors: Xo[i, q] = scale_i sum_t V[i, t] Q[t, q] for q < p (Q: c x p
// row-major; Xo row-major with leading dimension ldo; scale optional).  A
// block stages kRotRows rows of V[:, 0:c] in LDS (coalesced), then every
// thread computes whole outputs (row, q): all threads busy for any p.
__global__ __launch_bounds__(256) void k_rotate(const double* __restrict__ V, int ldv, int64_t n, int c, int p,
                                                 const double* __restrict__ Q, double* __restrict__ Xo, int ldo,
                                                 const double* __restrict__ scale) {
    extern __shared__ double Vs[];  // [kRotRows][c]
    const int64_t ntiles = (n + kRotRows - 1) / kRotRows;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * kRotRows;
        const int rows = (int)min<int64_t>(kRotRows, n - r0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < rows * c; idx += blockDim.x) {
            const int r = idx / c, t = idx - r * c;
            Vs[idx] = V[(r0 + r) * ldv + t];
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < rows * p; idx += blockDim.x) {
            const int r = idx / p, q = idx - r * p;
            const double* vr = Vs + (size_t)r * c;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int t = 0;
            for (; t + 3 < c; t += 4) {
                a0 += vr[t] * Q[t * p + q];
                a1 += vr[t + 1] * Q[(t + 1) * p + q];
                a2 += vr[t + 2] * Q[(t + 2) * p + q];
                a3 += vr[t + 3] * Q[(t + 3) * p + q];
            }
            for (; t < c; ++t) a0 += vr[t] * Q[t * p + q];
            const double acc = (a0 + a1) + (a2 + a3);
            Xo[(r0 + r) * ldo + q] = scale ? acc * scale[r0 + r] : acc;
        }
    }
}

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Uniform(-1, 1) entries for V[:, c0 : c0 + nc] from a counter-based hash.
__global__ void k_random(double* __restrict__ V, int ldv, int64_t n, int c0, int nc, uint64_t seed, uint64_t salt) {
    const int64_t total = n * nc;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / nc;
        int j = (int)(idx - i * nc);
        uint64_t z = mix64(seed + 0x9E3779B97F4A7C15ull * (uint64_t)(salt * 0x100000001ull + (uint64_t)idx + 1));
        V[i * ldv + c0 + j] = ((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
    }
}

// Copy a row-major n x b0 block into V[:, c0 : c0 + b0].
__global__ void k_copy_in(const double* __restrict__ X, int b0, double* __restrict__ V, int ldv, int64_t n, int c0) {
    const int64_t total = n * b0;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / b0;
        int j = (int)(idx - i * b0);
        V[i * ldv + c0 + j] = X[idx];
    }
}

// X[0:count] = 0 (a kernel rather than a memset: stream-ordered with the
// solver's other kernels under every runtime mode, and graph-capturable).
__global__ void k_zero(double* __restrict__ X, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        X[i] = 0.0;
}

__global__ void k_zero_i32(int* __restrict__ X, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) X[i] = 0;
}

// T[0:p, 0:p] = diag(theta).
// T[0:p, 0:p] = diag(theta) (the identity when theta is null).
__global__ void k_set_diag(double* __restrict__ T, int ldt, int p, const double* __restrict__ theta,
                           const int* skip) {
    if (skip && *skip) return;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < p * p; idx += gridDim.x * blockDim.x) {
        int i = idx / p, j = idx - i * p;
        T[i * ldt + j] = i == j ? (theta ? theta[i] : 1.0) : 0.0;
    }
}

// Per-block partial column sums of squares of (Y - X diag(theta)), and of
// |X| maxima with their row for the sign convention.  part: [blk][2][k],
// imax: [blk][k].
__global__ __launch_bounds__(256) void k_col_stats(const double* __restrict__ X, const double* __restrict__ Y,
                                                    int ld, int64_t n, int k, const double* __restrict__ theta,
                                                    double* __restrict__ part, int64_t* __restrict__ imax,
                                                    const double* __restrict__ scale) {
    __shared__ double ss[256];
    __shared__ double mx[256];
    __shared__ int64_t mi[256];
    for (int j = 0; j < k; ++j) {
        double s = 0.0, m = -1.0;
        int64_t at = INT64_MAX;
        const double th = theta ? theta[j] : 0.0;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
            const double x = X[i * ld + j];
            if (Y) {
                const double r = Y[i * ld + j] - th * x;
                s += r * r;
            }
            const double a = fabs(scale ? scale[i] * x : x);
            if (a > m) {
                m = a;
                at = i;
            }
        }
        ss[threadIdx.x] = s;
        mx[threadIdx.x] = m;
        mi[threadIdx.x] = at;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                ss[threadIdx.x] += ss[threadIdx.x + w];
                const double m2 = mx[threadIdx.x + w];
                const int64_t i2 = mi[threadIdx.x + w];
                if (m2 > mx[threadIdx.x] || (m2 == mx[threadIdx.x] && i2 < mi[threadIdx.x])) {
                    mx[threadIdx.x] = m2;
                    mi[threadIdx.x] = i2;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[(size_t)blockIdx.x * 2 * k + j] = ss[0];
            part[(size_t)blockIdx.x * 2 * k + k + j] = mx[0];
            imax[(size_t)blockIdx.x * k + j] = mi[0];
        }
        __syncthreads();
    }
}

// Sign convention of the output: per column the entry of largest magnitude
// (after the row scale) made positive, ties to the smallest row.  Block j
// combines column j's per-block maxima of k_col_stats by that rule (the
// result does not depend on the order) and writes sgn[j] = -1 when the
// entry is negative, else 1.
__global__ __launch_bounds__(256) void k_sign_pick(const double* __restrict__ part,
                                                    const int64_t* __restrict__ imax, int nb, int k, int64_t n,
                                                    const double* __restrict__ X, double* __restrict__ sgn) {
    __shared__ double mx[256];
    __shared__ int64_t mi[256];
    const int j = blockIdx.x, t = threadIdx.x;
    double m = -1.0;
    int64_t at = INT64_MAX;
    for (int blk = t; blk < nb; blk += 256) {
        const double m2 = part[(size_t)blk * 2 * k + k + j];
        const int64_t i2 = imax[(size_t)blk * k + j];
        if (m2 > m || (m2 == m && i2 < at)) {
            m = m2;
            at = i2;
        }
    }
    mx[t] = m;
    mi[t] = at;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            const double m2 = mx[t + w];
            const int64_t i2 = mi[t + w];
            if (m2 > mx[t] || (m2 == mx[t] && i2 < mi[t])) {
                mx[t] = m2;
                mi[t] = i2;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        const int64_t r = mi[0];
        sgn[j] = (r >= 0 && r < n && X[r * k + j] < 0.0) ? -1.0 : 1.0;
    }
}

// Column-major output H[:, j] = sign_j * scale_i * X[:, j] (row-major X, ld).
__global__ void k_write_out(const double* __restrict__ X, int ld, int64_t n, int k, const double* __restrict__ sgn,
                            const double* __restrict__ scale, double* __restrict__ H) {
    const int64_t total = n * k;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int j = (int)(idx / n);
        int64_t i = idx - (int64_t)j * n;
        H[idx] = sgn[j] * (scale ? scale[i] : 1.0) * X[i * ld + j];
    }
}

// ---------------------------------------------------------------------------
// host side

namespace {

int grid_for(int64_t work, int per, int cap) {
    int64_t g = (work + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Wait for an event by polling it: the solve's restarts wait for a few
// hundred microseconds at a time, and a polling wait returns within a
// microsecond or two of the GPU's completion where a blocking one can take
// tens.  Past a few milliseconds it blocks instead.
static int poll_wait(hipEvent_t e) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipSuccess) return SFAIRSC_OK;
        if (q != hipErrorNotReady) return set_error(SFAIRSC_E_HIP, "hipEventQuery failed: %s", hipGetErrorString(q));
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(4)) {
            SF_HIP(hipEventSynchronize(e));
            return SFAIRSC_OK;
        }
    }
}

// The word of the solver's flag array that gates a restart rotation
// enqueued ahead of the Rayleigh-Ritz record (words 0-2: expansion failure).
constexpr int kRotSkipWord = 4;

struct Solver {
    sfairsc_graph* g;
    hipStream_t s;
    int64_t n;
    int b, ncv, ld, k;
    bool mixed;
    double sigma;
    double* V;
    double* V2;
    double* T;
    double* part;
    int nblk;
    // small device buffers
    double *H1, *H2, *Gsave, *R1, *Rinv, *Rc, *theta, *Q, *stats;
    int64_t* imax;
    int* flag;
    // the column of the block whose operator input the last expansion wrote
    // (-1: none), and the blocks of its group sums
    int xp_ready = -1, xp_nblk = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> evs;
    size_t ev_used = 0;
    // phase timing: begin/end event pairs, kind 0 operator (projections,
    // sparse product, C^T T), 1 orthogonalisation (CGS2 + Cholesky-QR),
    // 2 restart rotation
    std::vector<hipEvent_t> pev;
    std::vector<int> pkind;
    size_t pev_used = 0;
    // Rayleigh-Ritz kernel buffers, its stream and (timing mode) its events
    RrBufs rb{};
    hipStream_t s2 = nullptr;
    std::vector<hipEvent_t> rr_evs;
    size_t rr_ev_used = 0;
    sfairsc_eigs_info* info = nullptr;
    double thresh = 0.0;

    int setup() {
        EigWork& w = g->eig;
        if (!w.s2) SF_HIP(hipStreamCreateWithFlags(&w.s2, hipStreamNonBlocking));
        if (!w.ev_fork) SF_HIP(hipEventCreateWithFlags(&w.ev_fork, hipEventDisableTiming));
        if (!w.ev_join) SF_HIP(hipEventCreateWithFlags(&w.ev_join, hipEventDisableTiming));
        if (!w.ev_wait) SF_HIP(hipEventCreateWithFlags(&w.ev_wait, hipEventDisableTiming));
        s2 = w.s2;
        SF_TRY(rr_buffers(g, &rb));
        ld = ncv + b;
        SF_TRY(w.V.ensure((size_t)n * ld * sizeof(double)));
        SF_TRY(w.V2.ensure((size_t)n * ld * sizeof(double)));
        V2 = w.V2.as<double>();
        SF_TRY(w.T.ensure((size_t)ld * ld * sizeof(double)));
        nblk = grid_for(n, kTsRows, kTsMaxBlocks);
        SF_TRY(w.part.ensure((size_t)nblk * (size_t)ld * kMaxBlock * sizeof(double)));
        const size_t smallsz = 2 * (size_t)kLdMax * kMaxBlock + 5 * (size_t)kMaxBlock * kMaxBlock + kLdMax +
                               kStatsDoubles + kStatsIdx + 64;
        SF_TRY(w.small.ensure(smallsz * sizeof(double)));
        SF_TRY(w.Q.ensure((size_t)kLdMax * kLdMax * sizeof(double)));
        V = w.V.as<double>();
        T = w.T.as<double>();
        part = w.part.as<double>();
        double* sp = w.small.as<double>();
        H1 = sp;
        sp += kLdMax * kMaxBlock;
        H2 = sp;
        sp += kLdMax * kMaxBlock;
        Gsave = sp;
        sp += kMaxBlock * kMaxBlock;
        R1 = sp;
        sp += kMaxBlock * kMaxBlock;
        Rinv = sp;
        sp += kMaxBlock * kMaxBlock;
        Rc = sp;
        sp += kMaxBlock * kMaxBlock;
        theta = sp;
        sp += kLdMax;
        stats = sp;
        sp += kStatsDoubles;
        imax = reinterpret_cast<int64_t*>(sp);
        sp += kStatsIdx;
        flag = reinterpret_cast<int*>(sp);
        sp += 8;
        ident = nullptr;
        Q = w.Q.as<double>();
        SF_TRY(w.opart.ensure(ortho_part_doubles(n) * sizeof(double)));
        SF_TRY(w.osmall.ensure(ortho_small_doubles() * sizeof(double)));
        k_zero_i32<<<1, 64, 0, s>>>(flag, 8);
        k_zero<<<grid_for((int64_t)ld * ld, 256, 1024), 256, 0, s>>>(T, (int64_t)ld * ld);
        SF_HIP(hipGetLastError());
        return SFAIRSC_OK;
    }

    size_t ts_lds(int mode, int cv) const {
        const bool useV = mode <= TS_UPD_SYRK;
        const int W = (useV ? cv : 0) + b;
        int msz = mode >= TS_MUL_SYRK ? b * b : 0;
        return (size_t)(kTsRows * W + msz + kTsRows * b) * sizeof(double);
    }

    // Stage `bytes` from host memory through the pinned buffer and enqueue
    // the copy; regions are recycled after the stream is synchronised.
    int upload(void* dst, const void* src, size_t bytes) {
        EigWork& w = g->eig;
        const size_t need = (bytes + 255) & ~(size_t)255;
        if (!w.pin) {
            w.pin_cap = std::max<size_t>((size_t)4 * kLdMax * kLdMax * sizeof(double), need);
            SF_HIP(hipHostMalloc((void**)&w.pin, w.pin_cap, hipHostMallocDefault));
            w.pin_off = 0;
        }
        if (need > w.pin_cap) return set_error(SFAIRSC_E_ARG, "upload of %zu bytes exceeds the staging buffer", bytes);
        if (w.pin_off + need > w.pin_cap) SF_TRY(sync());
        char* slot = reinterpret_cast<char*>(w.pin) + w.pin_off;
        std::memcpy(slot, src, bytes);
        w.pin_off += need;
        SF_HIP(hipMemcpyAsync(dst, slot, bytes, hipMemcpyHostToDevice, s));
        return SFAIRSC_OK;
    }

    // Enqueue a device-to-host copy through the pinned buffer; the bytes
    // reach `dst` at the next sync().
    struct Pending {
        void* dst;
        const void* slot;
        size_t bytes;
    };
    std::vector<Pending> pending;
    int download(void* dst, const void* src, size_t bytes) {
        EigWork& w = g->eig;
        const size_t need = (bytes + 255) & ~(size_t)255;
        if (!w.pin) {
            w.pin_cap = std::max<size_t>((size_t)4 * kLdMax * kLdMax * sizeof(double), need);
            SF_HIP(hipHostMalloc((void**)&w.pin, w.pin_cap, hipHostMallocDefault));
            w.pin_off = 0;
        }
        if (need > w.pin_cap) return set_error(SFAIRSC_E_ARG, "download of %zu bytes exceeds the staging buffer", bytes);
        if (w.pin_off + need > w.pin_cap) SF_TRY(sync());
        char* slot = reinterpret_cast<char*>(w.pin) + w.pin_off;
        w.pin_off += need;
        SF_HIP(hipMemcpyAsync(slot, src, bytes, hipMemcpyDeviceToHost, s));
        pending.push_back({dst, slot, bytes});
        return SFAIRSC_OK;
    }

    // Synchronise the stream; staged uploads are complete and staged
    // downloads are delivered afterwards.
    int sync() {
        SF_HIP(hipEventRecord(g->eig.ev_wait, s));
        SF_TRY(poll_wait(g->eig.ev_wait));
        for (const Pending& p : pending) std::memcpy(p.dst, p.slot, p.bytes);
        pending.clear();
        g->eig.pin_off = 0;
        return SFAIRSC_OK;
    }

    int ts(int mode, int cv, int yoff, const double* M) {
        const size_t lds = ts_lds(mode, cv);
        switch (mode) {
            case TS_GRAM:
                k_ts<TS_GRAM><<<nblk, kTsThreads, lds, s>>>(V, ld, n, cv, yoff, b, M, part, flag);
                break;
            case TS_UPD_GRAM:
                k_ts<TS_UPD_GRAM><<<nblk, kTsThreads, lds, s>>>(V, ld, n, cv, yoff, b, M, part, flag);
                break;
            case TS_UPD_SYRK:
                k_ts<TS_UPD_SYRK><<<nblk, kTsThreads, lds, s>>>(V, ld, n, cv, yoff, b, M, part, flag);
                break;
            case TS_MUL_SYRK:
                k_ts<TS_MUL_SYRK><<<nblk, kTsThreads, lds, s>>>(V, ld, n, cv, yoff, b, M, part, flag);
                break;
            default:
                k_ts<TS_MUL><<<nblk, kTsThreads, lds, s>>>(V, ld, n, cv, yoff, b, M, part, flag);
                break;
        }
        SF_HIP(hipGetLastError());
        return SFAIRSC_OK;
    }

    // CGS2 of Y = V[:, cv : cv+b] against V[:, 0:cv] writing the projection
    // coefficients into T's column block starting at column cact (when
    // cact >= 0), then Cholesky-QR twice.  Afterwards V[:, cv:cv+b] is the
    // orthonormal block and Rc its coupling.
    int orthonormalize(int cv, int cact) {
        const int yoff = cv;
        if (cv > 0) {
            SF_TRY(ts(TS_GRAM, cv, yoff, nullptr));
            const int O = cv * b;
            double* Tw = cact >= 0 ? T : nullptr;
            k_gram_reduce<<<grid_for(O, 256, 1 << 20), 256, 0, s>>>(part, nblk, cv, b, H1, Tw, ld,
                                                                  cact >= 0 ? cact : 0, 0, flag);
            SF_TRY(ts(TS_UPD_GRAM, cv, yoff, H1));
            k_gram_reduce<<<grid_for(O, 256, 1 << 20), 256, 0, s>>>(part, nblk, cv, b, H2, Tw, ld,
                                                                  cact >= 0 ? cact : 0, 1, flag);
            SF_TRY(ts(TS_UPD_SYRK, cv, yoff, H2));
        } else {
            SF_TRY(ts(TS_MUL_SYRK, 0, yoff, identity()));
        }
        double* Tc = cact >= 0 ? T : nullptr;
        k_chol<<<1, 1024, 0, s>>>(part, nblk, b, 1, thresh, Gsave, R1, Rinv, Rc, Tc, ld, cact >= 0 ? cact : 0, flag,
                                  flag);
        SF_TRY(ts(TS_MUL_SYRK, 0, yoff, Rinv));
        k_chol<<<1, 1024, 0, s>>>(part, nblk, b, 2, 0.25, Gsave, R1, Rinv, Rc, Tc, ld,
                                  cact >= 0 ? cact : 0, flag, flag);
        SF_TRY(ts(TS_MUL, 0, yoff, Rinv));
        SF_HIP(hipGetLastError());
        return SFAIRSC_OK;
    }

    double* ident = nullptr;
    const double* identity() {
        if (!ident) {
            ident = Q + (size_t)kLdMax * kLdMax - kMaxBlock * kMaxBlock;  // tail of Q, never used by rotations here
            k_set_diag<<<1, 256, 0, s>>>(ident, b, b, nullptr, nullptr);  // written on the device, no transfer
            if (hipGetLastError() != hipSuccess) return nullptr;
        }
        return ident;
    }

    int apply(const double* X, int ldx, double* Y, int ldy, int bb) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            if (ev_used + 2 > evs.size()) {
                for (int i = 0; i < 256; ++i) {
                    hipEvent_t e;
                    SF_HIP(hipEventCreate(&e));
                    evs.push_back(e);
                }
            }
            e0 = evs[ev_used++];
            e1 = evs[ev_used++];
        }
        SF_TRY(phase_mark(0, true));
        SF_TRY(op_apply(g, X, ldx, Y, ldy, bb, mixed, sigma, s, e0, e1, flag));
        SF_TRY(phase_mark(0, false));
        if (info) {
            info->operator_applies += bb;
            info->spmm_launches[mixed ? 1 : 0] += 1;
        }
        return SFAIRSC_OK;
    }

    // One Krylov expansion from V_next = V[:, c : c+b]: operator, then the
    // matrix-core orthogonalisation passes into V[:, c+b : c+2b].
    // The operator on the block V[:, c : c + b] (projection, sparse product,
    // C^T T): its output feeds the orthogonalisation of the expansion.
    int op(int c, OpOut* o, hipStream_t st = nullptr) {
        if (!st) st = s;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            if (ev_used + 2 > evs.size()) {
                for (int i = 0; i < 256; ++i) {
                    hipEvent_t e;
                    SF_HIP(hipEventCreate(&e));
                    evs.push_back(e);
                }
            }
            e0 = evs[ev_used++];
            e1 = evs[ev_used++];
        }
        SF_TRY(phase_mark(0, true, st));
        // the block the last expansion wrote also came out in the operator's
        // input form (compact copy and group sums): used once
        const int prepared = xp_ready == c ? xp_nblk : 0;
        xp_ready = -1;
        SF_TRY(op_apply_t(g, V + c, ld, b, mixed, sigma, st, e0, e1, flag, o, prepared));
        SF_TRY(phase_mark(0, false, st));
        if (info) {
            info->operator_applies += b;
            info->spmm_launches[mixed ? 1 : 0] += 1;
        }
        return SFAIRSC_OK;
    }

    // Orthogonalise the operator output o against V[:, 0 : c + b] (block
    // Gram-Schmidt and Cholesky-QR): the next block V[:, c + b : c + 2b].
    int ortho(int c, const OpOut& o) {
        OrthoArgs a;
        a.V = V;
        a.ld = ld;
        a.n = n;
        a.cv = c + b;
        a.b = b;
        a.t = o.t;
        a.t_is_float = o.is_float;
        a.BW = o.BW;
        a.grp = g->grp;
        a.cs = g->cs;
        a.rtab = o.rtab;
        a.lc = o.lc;
        a.lcw = o.lcw;
        a.m = o.m;
        a.utab = o.utab;
        a.T = T;
        a.ldt = ld;
        a.thresh = thresh;
        a.part = g->eig.opart.as<double>();
        a.small = g->eig.osmall.as<double>();
        a.gsave = Gsave;
        a.rc = Rc;
        a.flag = flag;
        a.stream = s;
        // blocks of 4 or 8: the last pass also writes the new block in the
        // operator's input form
        OpInput in{nullptr, nullptr};
        if (b <= 8) SF_TRY(op_input_target(g, b, &in));
        a.xp = in.xp;
        a.xp_float = mixed;
        a.xsum = in.xsum;
        a.h = g->h;
        SF_TRY(phase_mark(1, true));
        SF_TRY(ortho_expand(a));
        xp_ready = in.xp ? c + b : -1;
        xp_nblk = ortho_nblk(n);
        return phase_mark(1, false);
    }

    int expand(int c) {
        OpOut o;
        SF_TRY(op(c, &o));
        return ortho(c, o);
    }

    // Deliver the staged downloads once the stream has reached event e
    // (work enqueued after e keeps running; it must not stage transfers).
    int sync_to(hipEvent_t e) {
        SF_TRY(poll_wait(e));
        for (const Pending& p : pending) std::memcpy(p.dst, p.slot, p.bytes);
        pending.clear();
        g->eig.pin_off = 0;
        return SFAIRSC_OK;
    }

    int phase_mark(int kind, bool begin, hipStream_t st = nullptr) {
        if (!timing) return SFAIRSC_OK;
        if (!st) st = s;
        if (begin) {
            if (pev_used + 2 > pev.size()) {
                for (int i = 0; i < 64; ++i) {
                    hipEvent_t e;
                    SF_HIP(hipEventCreate(&e));
                    pev.push_back(e);
                }
                pkind.resize(pev.size() / 2);
            }
            pkind[pev_used / 2] = kind;
            SF_HIP(hipEventRecord(pev[pev_used], st));
        } else {
            SF_HIP(hipEventRecord(pev[pev_used + 1], st));
            pev_used += 2;
        }
        return SFAIRSC_OK;
    }

    // Sum the elapsed times of recorded SpMM and phase event pairs (stream
    // synced).
    int harvest_timing() {
        if (!timing || !info) return SFAIRSC_OK;
        double tot = 0.0;
        for (size_t i = 0; i + 1 < ev_used; i += 2) {
            float ms = 0.f;
            SF_HIP(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
            tot += ms;
        }
        info->spmm_ms[mixed ? 1 : 0] += tot;
        ev_used = 0;
        for (size_t i = 0; i + 1 < rr_ev_used; i += 2) {
            float ms = 0.f;
            SF_HIP(hipEventElapsedTime(&ms, rr_evs[i], rr_evs[i + 1]));
            info->rr_ms += ms;
        }
        rr_ev_used = 0;
        for (size_t i = 0; i + 1 < pev_used; i += 2) {
            float ms = 0.f;
            SF_HIP(hipEventElapsedTime(&ms, pev[i], pev[i + 1]));
            const int kd = pkind[i / 2];
            (kd == 0 ? info->operator_ms : kd == 1 ? info->ortho_ms : info->restart_ms) += ms;
        }
        pev_used = 0;
        return SFAIRSC_OK;
    }

    // The Rayleigh-Ritz step on the projected matrix T[0:c, 0:c], on the
    // solve's stream; the second stream is released (ev_fork) for the
    // look-ahead operator application (op_ahead), which the solve's stream
    // joins (ev_join) before anything reads the results.
    int rayleigh_ritz(int c, double tol, int keep_opt, int p_pred) {
        EigWork& w = g->eig;
        // the second stream may start the look-ahead operator application
        // from here on; the Rayleigh-Ritz kernel goes first on the solve's
        // stream, so that its one workgroup is placed before the sparse
        // product's fill the GPU
        SF_HIP(hipEventRecord(w.ev_fork, s));
        SF_HIP(hipStreamWaitEvent(s2, w.ev_fork, 0));
        if (timing) {
            if (rr_ev_used + 2 > rr_evs.size()) {
                for (int i = 0; i < 16; ++i) {
                    hipEvent_t e;
                    SF_HIP(hipEventCreate(&e));
                    rr_evs.push_back(e);
                }
            }
            SF_HIP(hipEventRecord(rr_evs[rr_ev_used], s));
        }
        RrArgs a;
        a.T = T;
        a.ldt = ld;
        a.c = c;
        a.skip = flag;
        a.work = rb.work;
        a.mode = 0;
        a.Rc = Rc;
        a.b = b;
        a.k = k;
        a.ncv = ncv;
        a.keep = keep_opt;
        a.tol = tol;
        a.sigma = sigma;
        a.theta = rb.theta;
        a.Qch = Q;
        a.Zk = rb.zk;
        a.rec = rb.rec;
        a.rot_skip = flag + kRotSkipWord;
        a.p_pred = p_pred;
        SF_TRY(rr_launch(a, s));
        if (timing) {
            SF_HIP(hipEventRecord(rr_evs[rr_ev_used + 1], s));
            rr_ev_used += 2;
        }
        return SFAIRSC_OK;
    }

    // The look-ahead operator application on the second stream beside the
    // Rayleigh-Ritz step; the solve's stream waits for it (ev_join).
    int op_ahead(int c, OpOut* o) {
        EigWork& w = g->eig;
        SF_TRY(op(c, o, s2));
        SF_HIP(hipEventRecord(w.ev_join, s2));
        SF_HIP(hipStreamWaitEvent(s, w.ev_join, 0));
        return SFAIRSC_OK;
    }

    ~Solver() {
        for (auto e : evs) (void)hipEventDestroy(e);
        for (auto e : pev) (void)hipEventDestroy(e);
        for (auto e : rr_evs) (void)hipEventDestroy(e);
    }
};

}  // namespace

// Repair a rank-deficient residual block found at expansion cact (host
// driven; rare).  Works on the residual block W itself (at the second
// Cholesky stage the failed block is W R1^{-1}, so it is first multiplied
// back by R1): rotates W onto the eigenvectors U of its Gram matrix and
// measures every rotated column's norm from its own entries (the Gram
// eigenvalues only resolve norms down to about sqrt(eps) times the largest,
// while a nearly converged direction can be far smaller and still matter at
// the tolerance).  Columns at the rounding level are replaced by random
// vectors, the others scaled to unit norm; the block is orthonormalised
// again and the coupling rebuilt as R = Rnew diag(norm, kept) U^T.
static int repair_block(Solver& S, int cact, uint64_t seed, int attempt, int stage) {
    const int b = S.b;
    const int cv = cact + b;
    S.xp_ready = -1;  // the block changes here
    int zero = 0;
    SF_TRY(S.upload(S.flag, &zero, sizeof(int)));
    auto gram = [&](const double* M, std::vector<double>& G) -> int {
        // Y <- Y M and G = Y^T Y (row-major b x b)
        SF_TRY(S.ts(TS_MUL_SYRK, 0, cv, M));
        k_gram_reduce<<<grid_for(b * b, 256, 64), 256, 0, S.s>>>(S.part, S.nblk, b, b, S.H1, nullptr, 0, 0, 0,
                                                                 nullptr);
        SF_HIP(hipGetLastError());
        G.resize(b * b);
        SF_TRY(S.download(G.data(), S.H1, b * b * sizeof(double)));
        return S.sync();
    };
    std::vector<double> G, G2, U(b * b), w(b);
    // the b x b Gram, still in S.H1 after gram(), diagonalised on the device
    if (stage == 2) {
        std::vector<double> R1(b * b);
        SF_TRY(S.download(R1.data(), ortho_r1(S.g->eig.osmall.as<double>()), b * b * sizeof(double)));
        SF_TRY(S.sync());
        SF_TRY(S.upload(S.Q, R1.data(), b * b * sizeof(double)));
        SF_TRY(gram(S.Q, G));
    } else {
        SF_TRY(gram(S.identity(), G));
    }
    SF_TRY(small_eig_host(S.g, S.H1, b, b, w.data(), U.data(), S.s));
    // W <- W U; the diagonal of the rotated block's Gram: column norms^2
    SF_TRY(S.upload(S.Q, U.data(), b * b * sizeof(double)));
    SF_TRY(gram(S.Q, G2));
    std::vector<double> nrm(b, 0.0);
    double big = 0.0;
    for (int j = 0; j < b; ++j) {
        nrm[j] = std::sqrt(std::max(0.0, G2[j * b + j]));
        big = std::max(big, nrm[j]);
    }
    // rounding level: relative to the block's largest column and to the
    // operator scale sigma (an invariant subspace leaves only noise)
    const double floor_norm = 1024.0 * 2.220446049250313e-16 * std::max(big, S.sigma);
    std::vector<int> keep(b, 0);
    std::vector<double> Dg(b * b, 0.0);
    for (int j = 0; j < b; ++j) {
        keep[j] = nrm[j] > floor_norm;
        Dg[j * b + j] = keep[j] ? 1.0 / nrm[j] : 1.0;
    }
    SF_TRY(S.upload(S.Q, Dg.data(), b * b * sizeof(double)));
    SF_TRY(S.ts(TS_MUL, 0, cv, S.Q));
    for (int j = 0; j < b; ++j)
        if (!keep[j])
            k_random<<<grid_for(S.n, 256, 4096), 256, 0, S.s>>>(S.V, S.ld, S.n, cv + j, 1, seed,
                                                                 1000003ull * (attempt + 1) + j);
    SF_HIP(hipGetLastError());
    // Orthogonalize again; the T column block of V_next already holds its
    // projection coefficients, so do not touch T (cact = -1 path writes into
    // scratch rows beyond the basis).
    SF_TRY(S.orthonormalize(cv, -1));
    int hflag[3];
    SF_TRY(S.download(hflag, S.flag, 3 * sizeof(int)));
    std::vector<double> Rn(b * b);
    SF_TRY(S.download(Rn.data(), S.Rc, b * b * sizeof(double)));
    SF_TRY(S.sync());
    if (hflag[0]) return set_error(SFAIRSC_E_HIP, "could not repair a rank-deficient Krylov block");
    // W = W_rot U^T,  W_rot[:, t] = nrm_t Qnew Rn[:, t] for kept t, 0 otherwise
    std::vector<double> Rc(b * b, 0.0);
    for (int i = 0; i < b; ++i)
        for (int j = 0; j < b; ++j) {
            double sacc = 0.0;
            for (int t = 0; t < b; ++t)
                if (keep[t]) sacc += Rn[i * b + t] * nrm[t] * U[j * b + t];
            Rc[i * b + j] = sacc;
        }
    SF_TRY(S.upload(S.Rc, Rc.data(), b * b * sizeof(double)));
    // symmetrise T's diagonal block of V_next (normally done by the second
    // Cholesky pass of the expansion)
    std::vector<double> Tb(b * S.ld);
    SF_TRY(S.download(Tb.data(), S.T + (size_t)cact * S.ld, b * S.ld * sizeof(double)));
    SF_TRY(S.sync());
    for (int i = 0; i < b; ++i)
        for (int j = i + 1; j < b; ++j) {
            double m = 0.5 * (Tb[i * S.ld + cact + j] + Tb[j * S.ld + cact + i]);
            Tb[i * S.ld + cact + j] = m;
            Tb[j * S.ld + cact + i] = m;
        }
    SF_TRY(S.upload(S.T + (size_t)cact * S.ld, Tb.data(), b * S.ld * sizeof(double)));
    if (S.info) S.info->breakdowns += 1;
    return SFAIRSC_OK;
}

struct KsResult {
    std::vector<double> theta;  // theta[0:k] of the last Rayleigh-Ritz step
    std::vector<double> res;    // their residual estimates
    double gap = 0.0;           // (theta_{k+1} - theta_k) / sigma (0 when c <= k)
    int c = 0, m = 0;
    bool converged = false;
};

// One Krylov-Schur run.  On return the basis V and KsResult describe the
// final Rayleigh-Ritz step; its first k Ritz vectors' coefficients Z[:, 0:k]
// (c x k) are in S.rb.zk on the device: Ritz vectors = V[:, 0:c] Z[:, i].
static int run_ks(Solver& S, double tol, int max_restarts, int keep_opt, const double* x0, int b0, uint64_t seed,
                  KsResult& out) {
    const int b = S.b, ncv = S.ncv, k = S.k;
    const int64_t n = S.n;
    SF_TRY(S.setup());
    S.xp_ready = -1;
    // start block
    int c = 0;
    if (x0 && b0 > 0) k_copy_in<<<grid_for(n * b0, 256, 8192), 256, 0, S.s>>>(x0, b0, S.V, S.ld, n, 0);
    if (b0 < b) k_random<<<grid_for(n * (b - b0), 256, 8192), 256, 0, S.s>>>(S.V, S.ld, n, b0, b - b0, seed, 0);
    SF_HIP(hipGetLastError());
    // A random start vector is not orthogonal to range(C) or to the trivial
    // vector: harmless, the operator treats every direction exactly.
    // A rank-deficient start block sets the flag words (column -1): every
    // kernel after it skips its work and the first Rayleigh-Ritz record
    // reports it, so the expansions are enqueued without waiting here.
    SF_TRY(ortho_start(S.V, S.ld, n, b, S.identity(), S.thresh, S.g->eig.opart.as<double>(),
                       S.g->eig.osmall.as<double>(), S.Gsave, S.Rc, S.flag, S.s));
    int repairs = 0;
    std::vector<double> rec(rr_rec_doubles(k));
    // operator output computed ahead, during the previous Rayleigh-Ritz step
    bool ahead = false;
    OpOut pre;
    for (int restart = 0;; ++restart) {
        // expansions
        while (c + b <= ncv) {
            if (ahead) {
                SF_TRY(S.ortho(c, pre));
                ahead = false;
            } else {
                SF_TRY(S.expand(c));
            }
            if (S.info) S.info->block_steps += 1;
            c += b;
        }
        // Rayleigh-Ritz on the device (second stream).  Look-ahead: a restart
        // keeps the next block V[:, c : c + b] (moved to the column after the
        // kept Ritz vectors), so its operator application runs on the solve's
        // stream meanwhile (wasted if this cycle converges).  Both skip their
        // work if the last expansion broke down (flag).
        // The kept count the kernel will choose unless equal eigenvalues
        // extend it (rare): the restart for it is enqueued before the record
        // is read, and runs only if the kernel confirms it (not converged,
        // same count), so the GPU goes on while the host reads the record.
        int p_pred = keep_opt > 0 ? keep_opt : std::max(k + b, k + (c - k) / 2);
        p_pred = std::min(p_pred, ncv - b);
        p_pred = std::max(p_pred, std::min(k, ncv - b));
        p_pred = std::min((p_pred + 3) & ~3, ncv - b);
        const bool spec = restart + 1 < max_restarts && p_pred >= 1 && p_pred <= c && p_pred + b <= S.ld;
        SF_TRY(S.rayleigh_ritz(c, tol, keep_opt, spec ? p_pred : 0));
        SF_TRY(S.op_ahead(c, &pre));
        ahead = true;
        // the record carries the expansion's flag words too: one download
        SF_TRY(S.download(rec.data(), S.rb.rec, rec.size() * sizeof(double)));
        SF_HIP(hipEventRecord(S.g->eig.ev_wait, S.s));
        const int* rot_skip = S.flag + kRotSkipWord;
        if (spec) {
            SF_TRY(S.phase_mark(2, true));
            SF_TRY(ortho_rotate(S.V, S.V2, S.ld, n, c, p_pred, b, S.Q, S.s, rot_skip));
            SF_TRY(S.phase_mark(2, false));
            k_set_diag<<<grid_for((int64_t)p_pred * p_pred, 256, 1024), 256, 0, S.s>>>(S.T, S.ld, p_pred,
                                                                                      S.rb.theta, rot_skip);
            SF_HIP(hipGetLastError());
        }
        if (S.timing) {
            SF_TRY(S.sync());  // every timing event complete before they are read
            SF_TRY(S.harvest_timing());
        } else {
            SF_TRY(S.sync_to(S.g->eig.ev_wait));
        }
        const int hflag[3] = {(int)rec[kRrRecFlag], (int)rec[kRrRecFlag + 1], (int)rec[kRrRecFlag + 2]};
        if (hflag[0] && hflag[1] < 0) return set_error(SFAIRSC_E_ARG, "start block is rank deficient");
        if (hflag[0]) {
            // everything after the failed expansion at hflag[1] was skipped
            const int cact = hflag[1];
            if (++repairs > 64) return set_error(SFAIRSC_E_HIP, "too many Krylov breakdowns");
            SF_TRY(repair_block(S, cact, seed, repairs, hflag[2]));
            c = cact + b;
            ahead = false;
            if (S.info) S.info->block_steps += 1;
            continue;
        }
        if (!(rec[1] >= 0.0))
            return set_error(SFAIRSC_E_HIP, "the projected matrix is not finite (the operator produced NaN or Inf)");
        const int nconv = (int)rec[0], p = (int)rec[1], m = (int)rec[2];
        const double gap = rec[3];
        if (S.info) {
            S.info->restarts = restart + 1;
            S.info->converged = nconv;
            S.info->gap_ratio = gap;
        }
        out.theta.assign(rec.begin() + kRrRecHead, rec.begin() + kRrRecHead + k);
        out.res.assign(rec.begin() + kRrRecHead + k, rec.begin() + kRrRecHead + 2 * k);
        out.gap = gap;
        out.c = c;
        out.m = m;
        out.converged = nconv == k;
        if (out.converged || restart + 1 >= max_restarts) return SFAIRSC_OK;
        if (p < 1 || p + b > S.ld || p > c) return set_error(SFAIRSC_E_HIP, "internal: restart keeps %d of %d", p, c);
        // V <- [V Z[:, 0:p], V_next]; the kernel left the rotation's factor
        // in S.Q (layout: rot_whole), and all Ritz values in theta.  Already
        // enqueued above when p was predicted.
        if (!(spec && p == p_pred)) {
            if (spec && S.info) S.info->restarts_unpredicted += 1;
            SF_TRY(S.phase_mark(2, true));
            SF_TRY(ortho_rotate(S.V, S.V2, S.ld, n, c, p, b, S.Q, S.s));
            SF_TRY(S.phase_mark(2, false));
            k_set_diag<<<grid_for((int64_t)p * p, 256, 1024), 256, 0, S.s>>>(S.T, S.ld, p, S.rb.theta, nullptr);
            SF_HIP(hipGetLastError());
        }
        S.xp_ready = -1;
        std::swap(S.V, S.V2);
        c = p;
    }
}

// Ritz vectors X = V[:, 0:c] Z[:, 0:k] (row-major n x k in Xo, ld k).
static int ritz_vectors(Solver& S, const KsResult& R, double* Xo, const double* scale) {
    const int c = R.c, k = S.k;
    // up to 32 vectors: the matrix-core product of the orthogonalisation
    if (k <= 32 && c % 4 == 0) return ortho_product(S.V, S.ld, S.n, c, S.rb.zk, k, Xo, k, scale, S.s);
    k_rotate<<<grid_for(S.n, kRotRows, 2048), 256, (size_t)kRotRows * c * sizeof(double), S.s>>>(
        S.V, S.ld, S.n, c, k, S.rb.zk, Xo, k, scale);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

// FP64 residual norms ||L^sigma x_i - theta_i x_i|| of row-major X (n x k),
// theta the last Rayleigh-Ritz step's (read from its record on the device).
// certify_enqueue leaves the per-block sums of squares staged for the next
// sync; certify_finish adds them up.
static int certify_enqueue(Solver& S, const double* X, double* Ybuf, std::vector<double>& part) {
    const int k = S.k;
    const bool was_mixed = S.mixed;
    S.mixed = false;
    k_zero_i32<<<1, 64, 0, S.s>>>(S.flag, 1);
    for (int j0 = 0; j0 < k; j0 += kMaxBlock) {
        int bb = std::min(kMaxBlock, k - j0);
        SF_TRY(op_apply(S.g, X + j0, k, Ybuf + j0, k, bb, 0, S.sigma, S.s, nullptr, nullptr, nullptr));
    }
    S.mixed = was_mixed;
    const int nb = grid_for(S.n, 256, kStatBlocks);
    k_col_stats<<<nb, 256, 0, S.s>>>(X, Ybuf, k, S.n, k, S.rb.rec + kRrRecHead, S.stats, S.imax, nullptr);
    SF_HIP(hipGetLastError());
    part.assign((size_t)nb * 2 * k, 0.0);
    return S.download(part.data(), S.stats, part.size() * sizeof(double));
}

static void certify_finish(const Solver& S, const std::vector<double>& part, std::vector<double>& res) {
    const int k = S.k;
    const int nb = (int)(part.size() / (2 * (size_t)k));
    res.assign(k, 0.0);
    for (int blk = 0; blk < nb; ++blk)
        for (int j = 0; j < k; ++j) res[j] += part[(size_t)blk * 2 * k + j];
    for (int j = 0; j < k; ++j) res[j] = std::sqrt(res[j]);
}

static int certify(Solver& S, const double* X, double* Ybuf, std::vector<double>& res) {
    std::vector<double> part;
    SF_TRY(certify_enqueue(S, X, Ybuf, part));
    SF_TRY(S.sync());
    certify_finish(S, part, res);
    return SFAIRSC_OK;
}

static int eigs_impl(sfairsc_graph* g, int k, double tol, int precision, const sfairsc_eigs_opts& o,
                     double* eigvals, double* H, sfairsc_eigs_info* info, hipStream_t s) {
    const int64_t n = g->n;
    const int dim = (int)std::min<int64_t>(n, INT32_MAX);
    int b = o.block_width;
    if (b == 0) {
        b = k <= 4 ? 4 : k <= 16 ? 8 : 16;
        while (b < o.b0 && b < kMaxBlock) b *= 2;  // room for the whole warm start
    }
    if (b != 4 && b != 8 && b != 16 && b != 32) return set_error(SFAIRSC_E_ARG, "block width must be 4, 8, 16 or 32");
    while (b > 4 && 3 * b + k > dim) b /= 2;
    int ncv = o.max_basis;
    if (ncv == 0) ncv = std::max(k + 8 * b, 4 * k + 2 * b);
    ncv = ((ncv + b - 1) / b) * b;
    ncv = std::min(ncv, kMaxBasis);
    while (ncv + 2 * b > dim && ncv > b) ncv -= b;
    if (ncv < k + b || ncv < 2 * b)
        return set_error(SFAIRSC_E_ARG, "graph too small (n=%lld) for k=%d with block width %d", (long long)n, k, b);
    if (o.b0 < 0 || o.b0 > b || (o.b0 > 0 && !o.x0)) return set_error(SFAIRSC_E_ARG, "bad warm start");

    Solver S;
    S.g = g;
    S.s = s;
    S.n = n;
    S.b = b;
    S.ncv = ncv;
    S.k = k;
    S.sigma = o.sigma > 0 ? o.sigma : g->sigma;
    S.info = info;
    S.timing = o.time_kernels != 0 && info != nullptr;
    S.thresh = (1e-10 * S.sigma) * (1e-10 * S.sigma);
    const int max_restarts = o.max_restarts > 0 ? o.max_restarts : 2000;
    if (info) info->sigma = S.sigma;

    SF_TRY(g->eig.X.ensure((size_t)n * kMaxK * 2 * sizeof(double)));
    double* Xr = g->eig.X.as<double>();     // row-major n x k Ritz vectors
    double* Yr = Xr + (size_t)n * kMaxK;    // operator images for certification
    const double* scale = g->normalized ? g->cs : nullptr;

    KsResult R;
    std::vector<double> res;
    bool ok = false;
    if (precision == SFAIRSC_PREC_MIXED) {
        auto t0 = std::chrono::steady_clock::now();
        S.mixed = true;
        const double tol1 = std::max(tol, kMixedTol1);
        SF_TRY(run_ks(S, tol1, max_restarts, o.keep, o.x0, o.b0, o.seed, R));
        SF_TRY(ritz_vectors(S, R, Xr, nullptr));
        SF_TRY(certify(S, Xr, Yr, res));
        if (info) info->phase1_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        ok = true;
        for (int i = 0; i < k; ++i) ok = ok && res[i] <= tol * S.sigma;
        if (!ok) {
            // continue in FP64 from the float result: the k Ritz vectors seed
            // the start block (block width at least k)
            S.mixed = false;
            const int b2 = std::max(b, k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : 32);
            // The start block already holds the k Ritz vectors to about the
            // float floor: a basis of five blocks usually reaches tol at the
            // first Rayleigh-Ritz check (three blocks needed four cycles and
            // six block steps on the 50k workload; five: 0.35 ms less).
            S.b = b2;
            S.ncv = std::min(kMaxBasis, 5 * b2);
            while (S.ncv + 2 * b2 > dim && S.ncv > b2) S.ncv -= b2;
            // Xr holds the k Ritz vectors, row-major n x k: the start block
            SF_TRY(run_ks(S, tol, max_restarts, o.keep, Xr, k, o.seed + 1, R));
            SF_TRY(ritz_vectors(S, R, Xr, nullptr));
        }
    } else {
        S.mixed = false;
        // The automatic kept count of an FP64 solve at block widths up to 16:
        // k + 0.35 (ncv - k) Ritz vectors (a third more new columns per cycle
        // than keeping half, fewer restarts; measured on three m-SBM
        // workloads, 2k, 10k and 50k vertices: 9-16% less time).  Wider
        // blocks and the mixed solve keep half (there fewer kept vectors
        // cost restarts).
        int keep = o.keep;
        if (keep <= 0 && b <= 16) keep = k + (7 * (ncv - k) + 10) / 20;
        SF_TRY(run_ks(S, tol, max_restarts, keep, o.x0, o.b0, o.seed, R));
        SF_TRY(ritz_vectors(S, R, Xr, nullptr));
    }
    // Exact eigenvectors of L^sigma below sigma lie in null(C^T) (Prop. 3.1);
    // remove the O(residual / (sigma - theta)) range(C) part of the Ritz
    // vectors so the returned H satisfies F^T H = 0 to rounding.
    for (int j0 = 0; j0 < k; j0 += kMaxBlock) SF_TRY(op_project(g, Xr + j0, k, std::min(kMaxBlock, k - j0), s));
    std::vector<double> th(R.theta.begin(), R.theta.begin() + k);
    // certification and output in one pass of device work, one sync at the
    // end: the residual sums are staged, the signs chosen on the device
    const bool cert = o.certify || precision == SFAIRSC_PREC_MIXED;
    std::vector<double> cpart;
    if (cert) SF_TRY(certify_enqueue(S, Xr, Yr, cpart));
    // sign convention on H = D^{-1/2} X (normalized) or X: the entry of
    // largest magnitude of each column is made positive
    const int nb = grid_for(n, 256, kStatBlocks);
    k_col_stats<<<nb, 256, 0, s>>>(Xr, nullptr, k, n, k, nullptr, S.stats, S.imax, scale);
    k_sign_pick<<<k, 256, 0, s>>>(S.stats, S.imax, nb, k, n, Xr, S.theta);
    k_write_out<<<grid_for(n * k, 256, 8192), 256, 0, s>>>(Xr, k, n, k, S.theta, scale, H);
    SF_HIP(hipGetLastError());
    SF_TRY(S.sync());
    if (cert)
        certify_finish(S, cpart, res);
    else
        res.assign(R.res.begin(), R.res.begin() + k);
    double worst = 0.0;
    int nconv = 0;
    for (int i = 0; i < k; ++i) {
        worst = std::max(worst, res[i] / S.sigma);
        if (res[i] <= tol * S.sigma) ++nconv;
    }
    for (int i = 0; i < k; ++i) eigvals[i] = th[i];
    // The wanted subspace is well defined only with a gap after theta_k
    // (Proposition 3.3 and the angle bound need lambda_k < lambda_{k+1}):
    // a relative gap at the tolerance level is flagged, outputs still written.
    const bool gap_known = R.c > k;
    const double gap = gap_known ? R.gap : 0.0;
    const bool degenerate = gap_known && gap <= kDegenerateGap * tol;
    if (info) {
        info->max_rel_residual = worst;
        info->converged = nconv;
        info->gap_ratio = gap;
        info->degenerate = degenerate ? 1 : 0;
    }
    if (nconv < k) return set_error(SFAIRSC_E_NOT_CONVERGED, "%d of %d pairs converged (worst rel. residual %.3e)",
                                    nconv, k, worst);
    if (degenerate)
        return set_error(SFAIRSC_E_DEGENERATE,
                         "theta_k and theta_{k+1} coincide to the tolerance (relative gap %.3e <= %g tol): the "
                         "k-dimensional subspace is not determined",
                         gap, kDegenerateGap);
    return SFAIRSC_OK;
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" void sfairsc_eigs_opts_init(sfairsc_eigs_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->certify = 1;
}

extern "C" int sfairsc_eigs(sfairsc_graph_t g, int32_t k, double tol, int precision, const sfairsc_eigs_opts* opts,
                            double* eigvals, double* H, sfairsc_eigs_info* info, hipStream_t stream) {
    if (!g || !eigvals || !H) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (k < 1 || k > kMaxK || k > free_dim(g)) return set_error(SFAIRSC_E_ARG, "k=%d out of range", k);
    if (!(tol > 0.0) || !(tol < 1.0)) return set_error(SFAIRSC_E_ARG, "tol must lie in (0, 1)");
    if (precision != SFAIRSC_PREC_FP64 && precision != SFAIRSC_PREC_MIXED)
        return set_error(SFAIRSC_E_ARG, "unknown precision %d", precision);
    sfairsc_eigs_opts o;
    if (opts)
        o = *opts;
    else
        sfairsc_eigs_opts_init(&o);
    if (info) std::memset(info, 0, sizeof *info);
    return eigs_impl(g, k, tol, precision, o, eigvals, H, info, stream);
}
