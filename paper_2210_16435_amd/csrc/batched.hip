// Batched fair eigensolves: many independent graphs in one persistent launch.
//
// Every graph of a batch gets the whole method of the single-graph solver:
// the deflated operator L^sigma = P (L_n - sigma I) P + sigma I (eq. asigma)
// applied through the group-sum form of P (eq. mv-Pw, Section 3.4), a block
// Krylov-Schur (thick-restart Lanczos) iteration, classical Gram-Schmidt
// twice and Cholesky-QR twice on the FP64 matrix cores, a Rayleigh-Ritz
// step and the fair output H (Alg. 3 step 3, Proposition 3.3).
//
// Design: one cooperative launch, bulk-synchronous.  The block steps of all
// graphs still iterating advance together, as a fixed sequence of phases
// separated by grid barriers.
//   * Row phases (group sums, projection, the CSR product, the four
//     matrix-core passes, the restart rotation) run over items: 1024
//     consecutive rows of one graph, one item per workgroup at a time, 64
//     rows per wavefront.  All graphs' items are spread over all compute
//     units, so a large graph no longer runs on one compute unit.  An item
//     reduces its wavefronts' partial sums in LDS and leaves one partial per
//     item in HBM.
//   * Graph phases (summing a graph's item partials in item order, the
//     group-sum tables, the small Cholesky factors, the projected matrix T_m
//     and the Rayleigh-Ritz step) run on the graph's owner workgroup.  The
//     small symmetric eigenproblem is solved in LDS by cyclic Jacobi with a
//     round-robin ordering: each round applies all m/2 disjoint rotations at
//     once as a two-sided update of 2 x 2 blocks, so a round costs two
//     workgroup barriers.
// Every reduction has a fixed order: results are bitwise reproducible for a
// given device.  A graph leaves the block steps once converged (or out of
// restarts); the output phases (projection onto null(C^T), FP64
// certification, signs, H) run once for all graphs at the end.  The last few
// graphs of a large batch cannot fill the GPU: the launch can stop early and
// leave them, with their current Ritz vectors, to the single-graph solver.
// The launch requires all workgroups to be resident at once (a cooperative
// launch, which fails cleanly otherwise).
//
// The block width b, the basis size and the CSR rows handled together by a
// wavefront are chosen per graph, by default from a tuning table filled by
// timed trials (sfairsc_autotune).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "wave_chol.h"

namespace cg = cooperative_groups;

namespace sfairsc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// A load through a global-address-space pointer.  The kernel reaches its
// buffers through pointers stored in memory, so the compiler cannot prove
// they are global and emits flat loads; a flat load counts against the LDS
// counter too, and waiting for one then waits for every outstanding one.
// All buffers here are device memory.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
    return *((const __attribute__((address_space(1))) T*)p);
}

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

#ifndef SF_BATCH_THREADS
#define SF_BATCH_THREADS 1024
#endif
#ifndef SF_ITEM_FN
#define SF_ITEM_FN __forceinline__
#endif
constexpr int NT = SF_BATCH_THREADS;            // threads of a workgroup
constexpr int NW = NT / 64;                     // wavefronts
constexpr int BMAX = 16;                        // widest block
constexpr int NCVMAX = 80;                      // basis columns before a restart
constexpr int LDT = NCVMAX + 1;                 // LDS row stride of the Jacobi matrices
constexpr int RTMAX = (NCVMAX + 15) / 16;       // row tiles of a Gram product
constexpr int KCH = (NCVMAX + BMAX + 15) / 16;  // 16-column chunks of an update input
constexpr int HMAX = kMaxGroups;                // groups
constexpr int KMAXB = 48;                       // wanted pairs
#ifndef SF_BATCH_ITEM_ROWS
#define SF_BATCH_ITEM_ROWS 1024
#endif
constexpr int IROWS = SF_BATCH_ITEM_ROWS;       // rows of an item
constexpr int WROWS = IROWS / NW;               // rows of a wavefront in an item
static_assert(WROWS % 16 == 0, "a wavefront takes whole 16-row tiles");
constexpr int WRED = 512;                       // LDS doubles per wavefront partial
constexpr int PSTRIDE = (RTMAX + 1) * 256;      // doubles of an item's partial slot
static_assert(HMAX * 16 <= WRED && 2 * 256 <= WRED, "wavefront partial too small");

// Per-graph small buffers (doubles), one block per graph.
constexpr int OFF_T = 0;                          // T_m, NCVMAX x NCVMAX
constexpr int OFF_Z = OFF_T + NCVMAX * NCVMAX;    // rotation, NCVMAX x NCVMAX
constexpr int OFF_M = OFF_Z + NCVMAX * NCVMAX;    // update coefficients, (NCVMAX + BMAX) x 16
constexpr int OFF_TAB = OFF_M + (NCVMAX + BMAX) * 16;  // tables: input R, C^T X, output R
constexpr int OFF_R = OFF_TAB + 3 * HMAX * 16;   // R1, Rc (16 x 16 each)
constexpr int OFF_AUX = OFF_R + 2 * 256;          // theta [NCVMAX], signs [16]
constexpr int SMALL_DOUBLES = OFF_AUX + NCVMAX + 16;

struct Graph {
    const int32_t* rowptr;
    const int32_t* col;
    const float* val32;
    const double* val64;
    const float* diag32;
    const double* diag64;
    const int32_t* grp;
    const double* cs;    // d^{-1/2} (normalized) or nullptr
    const double* gpar;  // p[h], Ginv[(h-1)^2]
    double* V;           // n x ld basis, row-major
    void* xp;            // n x 16 (8-byte slots): projected block
    void* tt;            // n x 16 (8-byte slots): sparse product
    double* H;           // output, column-major n x k
    double* theta;       // output eigenvalues [KMAXB]
    double* sm;          // small buffers (SMALL_DOUBLES)
    int64_t n;
    int32_t h, k, b, ncv, ld, rows, max_restarts, certify;
    int32_t item0, nitems;
    double sigma, tol;
    double tol_conv;  // Ritz residual target (below tol with float products)
    uint64_t seed;
};

struct GState {
    int32_t active;  // block steps continue
    int32_t status;  // 0 converged, 1 not converged, 2 breakdown, 3 certification failed, 4 bad shape,
                     // 5 handed off with its current Ritz vectors in V[:, 0:k]
    int32_t out;     // the output phases apply (Ritz vectors of the last Rayleigh-Ritz step)
    int32_t m, restarts, steps, nconv;
    int32_t rot_m, rot_p, rot_nb;  // pending rotation (rot_p > 0)

    double est, gap, maxres;
    uint64_t t_done;
    uint64_t ph[8];  // compute-unit clock ticks spent on the graph, by phase
};

struct Item {
    int32_t g, pad;
    int64_t row0;  // rows [row0, min(n, row0 + IROWS))
};

struct Launch {
    const Graph* graphs;
    GState* st;
    const Item* items;
    double* part;  // nitems x PSTRIDE
    int* active;   // graphs still in their block steps
    int* alist;    // items of the selected graphs (see build_list)
    int* nalist;   // their number
    uint64_t* t_start;
    uint64_t* steplog;  // optional: per block step, wall clock and active graphs / items
    int ng, nitems, max_steps;
    int handoff;  // leave the block steps once at most this many graphs remain
};

struct Shared {
    union {
        struct {
            double A[NCVMAX * LDT];
            double Z[NCVMAX * LDT];
        } j;                    // Jacobi (graph phases)
        double wred[NW * WRED];  // wavefront partials (row phases)
    } u;
    double red[PSTRIDE];
    double gZ[HMAX * 16];
    double R1[256], Ri[256], R2[256];
    double theta[NCVMAX], res[NCVMAX];
    double wsum[NW * 2];
    double2 jcs[NCVMAX / 2];  // Jacobi rotations of a round: (cos, sin)
    int2 jpq[NCVMAX / 2];     // and their index pairs
    int perm[NCVMAX];
    int iscan[NT];
    int iflag[4];
};
static_assert(sizeof(Shared) <= 150 * 1024, "LDS budget");

template <class VT>
struct Vec16;
template <>
struct Vec16<float> {
    static constexpr int N = 4;
    float v[4];
    __device__ static Vec16 load(const float* p) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        return Vec16{{t.x, t.y, t.z, t.w}};
    }
    __device__ void store(float* p) const { *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]); }
};
template <>
struct Vec16<double> {
    static constexpr int N = 2;
    double v[2];
    __device__ static Vec16 load(const double* p) {
        const double2 t = *reinterpret_cast<const double2*>(p);
        return Vec16{{t.x, t.y}};
    }
    __device__ void store(double* p) const { *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]); }
};

template <class VT>
__device__ __forceinline__ const VT* pick(const float* f, const double* d);
template <>
__device__ __forceinline__ const float* pick<float>(const float* f, const double*) {
    return f;
}
template <>
__device__ __forceinline__ const double* pick<double>(const float*, const double* d) {
    return d;
}

__device__ __forceinline__ int ilog2(int b) { return b == 4 ? 2 : b == 8 ? 3 : 4; }

// Uniform in [-1, 1) from the SplitMix64 output function of (seed, index).
__device__ __forceinline__ double rnd_pm1(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (idx + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// ===========================================================================
// Workgroup reductions of wavefront partials (fixed order).

// Rows of 16 in the wavefronts' partials (wred[w * WRED + 16 r + j], r <
// rows) summed over the wavefronts, compacted to out[r * cols + j], j < cols.
__device__ __forceinline__ void wg_combine(const double* wred, int rows, int cols, double* __restrict__ out) {
    __syncthreads();
    for (int e = threadIdx.x; e < rows * 16; e += NT) {
        if ((e & 15) >= cols) continue;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += wred[w * WRED + e];
        out[(e >> 4) * cols + (e & 15)] = s;
    }
    __syncthreads();
}

// The wavefronts' Gram tiles summed over the workgroup and compacted:
// tiles t < ng (from acc[t]) hold rows 16 t ... of a (rows x b) product,
// stored at out[i * b + j]; with SYRK, acc[NTL - 1] holds a b x b product,
// stored after it at out[rows * b + i * b + j].  MFMA D layout: lane l,
// register r hold row 4 r + l / 16, column l % 16 of a tile.
template <int NTL, bool SYRK>
__device__ __forceinline__ void wg_tiles(const d4 (&acc)[NTL], int ng, int rows, int b, double* wred, double* __restrict__ out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nt = ng + (SYRK ? 1 : 0);
    for (int t0 = 0; t0 < nt; t0 += 2) {
#pragma unroll
        for (int r = 0; r < NTL; ++r) {
            const bool is_syrk = SYRK && r == NTL - 1;
            const int t = is_syrk ? ng : r;
            if ((is_syrk || r < ng) && (t == t0 || t == t0 + 1)) {
                double* p = wred + w * WRED + (t - t0) * 256 + lane * 4;
                p[0] = acc[r][0];
                p[1] = acc[r][1];
                p[2] = acc[r][2];
                p[3] = acc[r][3];
            }
        }
        __syncthreads();
        const int cnt = min(2, nt - t0) * 256;
        for (int e = threadIdx.x; e < cnt; e += NT) {
            const int t = t0 + (e >> 8), l = (e & 255) >> 2, il = 4 * (e & 3) + (l >> 4), j = l & 15;
            if (j >= b) continue;
            int dst;
            if (t < ng) {
                const int i = 16 * t + il;
                if (i >= rows) continue;
                dst = i * b + j;
            } else {
                if (il >= b) continue;
                dst = rows * b + il * b + j;
            }
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < NW; ++v) s += wred[v * WRED + e];
            out[dst] = s;
        }
        __syncthreads();
    }
}

// Sum of v over the workgroup (fixed order); two values at once.
__device__ __forceinline__ void wg_sum2(double& a, double& b, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < NW; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
    __syncthreads();
}

// ===========================================================================
// Row work of one wavefront: rows [r0, r1) (at most WROWS, a multiple of 16
// apart from the graph's last rows), no barriers.

// out[s * 16 + j] = sum over rows r in [r0, r1) of group s of c_r X[r][j],
// j < bw (bw in {4, 8, 16}), s < h.
template <class XT>
__device__ SF_ITEM_FN void w_gsum(const XT* X, int64_t ldx, int64_t r0, int64_t r1, int bw, int h,
                                    const int32_t* __restrict__ grp, const double* __restrict__ cs,
                                    double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int col = lane & (bw - 1), rl = lane >> ilog2(bw), rpw = 64 / bw;
    for (int g0 = 0; g0 < h; g0 += 8) {
        double acc[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[s] = 0.0;
        int64_t i = r0 + rl;
        for (; i + 3 * rpw < r1; i += 4 * rpw) {
            int gi[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t r = i + u * rpw;
                gi[u] = grp[r] - g0;
                v[u] = (cs ? cs[r] : 1.0) * (double)X[r * ldx + col];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int s = 0; s < 8; ++s) acc[s] += (gi[u] == s) ? v[u] : 0.0;
        }
        for (; i < r1; i += rpw) {
            const int gi = grp[i] - g0;
            const double v = (cs ? cs[i] : 1.0) * (double)X[i * ldx + col];
#pragma unroll
            for (int s = 0; s < 8; ++s) acc[s] += (gi == s) ? v : 0.0;
        }
        for (int off = bw; off < 64; off <<= 1)
#pragma unroll
            for (int s = 0; s < 8; ++s) acc[s] += __shfl_xor(acc[s], off);
        if (rl == 0)
#pragma unroll
            for (int s = 0; s < 8; ++s)
                if (g0 + s < h) out[(g0 + s) * 16 + col] = acc[s];
    }
}

// out_r = X_r - c_r R_{g_r} for rows [r0, r1), columns j < bw.
template <class OT>
__device__ SF_ITEM_FN void w_proj(const double* X, int64_t ldx, int64_t r0, int64_t r1, int bw,
                                    const int32_t* __restrict__ grp, const double* __restrict__ cs,
                                    const double* __restrict__ R, OT* out, int64_t ldo) {
    const int lane = threadIdx.x & 63;
    const int lb = ilog2(bw);
    const int64_t tot = (r1 - r0) * bw;
    for (int64_t idx = lane; idx < tot; idx += 64) {
        const int64_t i = r0 + (idx >> lb);
        const int j = (int)(idx & (bw - 1));
        const double c = cs ? cs[i] : 1.0;
        out[i * ldo + j] = (OT)(X[i * ldx + j] - c * R[grp[i] * 16 + j]);
    }
}

// T_r = diag_r X_r - sum_e val_e X_{col_e} for rows [r0, r1) (X, T compact
// n x b).  `rows` rows share the wavefront, 64 / rows lanes each; within a
// row, lanes split into nonzero slots of b / VEC lanes.
template <class VT>
__device__ SF_ITEM_FN void w_spmm(const Graph& t, const VT* __restrict__ X, VT* __restrict__ T, int64_t r0,
                                    int64_t r1, int b, int rows) {
    using V = Vec16<VT>;
    constexpr int VEC = V::N;
    const VT* __restrict__ val = pick<VT>(t.val32, t.val64);
    const VT* __restrict__ diag = pick<VT>(t.diag32, t.diag64);
    const int lane = threadIdx.x & 63;
    const int LPR = b / VEC;
    rows = min(rows, 64 / LPR);
    const int G = 64 / rows;
    const int sub = lane / G, sl = lane - sub * G;
    const int NS = G / LPR;
    const int slot = sl / LPR, cl = sl - slot * LPR;
    for (int64_t base = r0; base < r1; base += rows) {
        const int64_t row = base + sub;
        VT acc[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = VT(0);
        if (row < r1) {
            const int e0 = t.rowptr[row], e1 = t.rowptr[row + 1];
            int e = e0 + slot;
            for (; e + 3 * NS < e1; e += 4 * NS) {
                int j[4];
                VT w[4];
                V x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    j[u] = t.col[e + u * NS];
                    w[u] = val[e + u * NS];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = V::load(X + (int64_t)j[u] * b + cl * VEC);
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[v] += w[u] * x[u].v[v];
            }
            for (; e < e1; e += NS) {
                const int j0 = t.col[e];
                const VT w0 = val[e];
                const V x0 = V::load(X + (int64_t)j0 * b + cl * VEC);
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += w0 * x0.v[v];
            }
        }
        for (int off = LPR; off < G; off <<= 1)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += __shfl_xor(acc[v], off);
        if (row < r1 && slot == 0) {
            const V xi = V::load(X + row * b + cl * VEC);
            const VT dg = diag[row];
            V o;
#pragma unroll
            for (int v = 0; v < VEC; ++v) o.v[v] = dg * xi.v[v] - acc[v];
            o.store(T + row * b + cl * VEC);
        }
    }
}

// Pass A over 16-row tiles [tile0, tile1): Y0 = T - C U2 into
// V[:, cv : cv + b]; V[:, 0:cv]^T Y0 summed over the workgroup into out
// (cv x b, row-major; every wavefront of the workgroup calls it).
template <class SpT>
__device__ SF_ITEM_FN void w_pass_a(const Graph& t, double* V, int ld, int cv, int b, const SpT* __restrict__ T,
                                      const double* __restrict__ R2, int64_t tile0, int64_t tile1, double* wred,
                                      double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nrt = (cv + 15) >> 4;
    d4 acc[RTMAX];
#pragma unroll
    for (int r = 0; r < RTMAX; ++r) acc[r] = d4{0, 0, 0, 0};
    const int64_t n = t.n;
    for (int64_t tile = tile0; tile < tile1; ++tile) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = tile * 16 + 4 * q + lk;
            const bool rv = row < n;
            double y = 0.0;
            if (rv && li < b) {
                const double c = t.cs ? gload(t.cs + row) : 1.0;
                y = (double)gload(T + row * b + li) - c * gload(R2 + gload(t.grp + row) * 16 + li);
                V[row * ld + cv + li] = y;
            }
            // every basis load of the step first, unconditionally (row 0 /
            // column 0 stand in past n or cv), zeroed only at the use: a
            // select right after a load would wait for it
            const int64_t rs = rv ? row : 0;
            double araw[RTMAX];
#pragma unroll
            for (int rt = 0; rt < RTMAX; ++rt) {
                const int col = rt * 16 + li;
                araw[rt] = gload(V + rs * ld + (rt < nrt && col < cv ? col : 0));
            }
#pragma unroll
            for (int rt = 0; rt < RTMAX; ++rt) {
                if (rt < nrt) {
                    const double a = (rv && rt * 16 + li < cv) ? araw[rt] : 0.0;
                    acc[rt] = mfma16(a, y, acc[rt]);
                }
            }
        }
    }
    wg_tiles<RTMAX, false>(acc, nrt, cv, b, wred, out);
}

// Ynew = V[:, coff : coff + kin] M (M: kin x 16, columns >= b zero) into
// V[:, yoff : yoff + b] over tiles [tile0, tile1), in place (all inputs of
// a tile are in registers before its first store).  GRAM: V[:, 0:cv]^T Ynew
// (cv x b); SYRK: Ynew^T Ynew (b x b) after it; both row-major, summed over
// the workgroup into out (every wavefront of the workgroup calls it).
template <bool GRAM, bool SYRK>
__device__ SF_ITEM_FN void w_upd(int64_t n, double* V, int ld, int coff, int kin, int yoff, int b, int cv,
                                   const double* __restrict__ M, int64_t tile0, int64_t tile1, double* wred,
                                   double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nrt = GRAM ? (cv + 15) >> 4 : 0;
    constexpr int NG = (GRAM ? RTMAX : 0) + 1;
    d4 acc[NG];
#pragma unroll
    for (int r = 0; r < NG; ++r) acc[r] = d4{0, 0, 0, 0};
    for (int64_t tile = tile0; tile < tile1; ++tile) {
        const int64_t row0 = tile * 16;
        d4 D = d4{0, 0, 0, 0};
        {
            const int64_t row = row0 + li;
            const bool rv = row < n;
            const double* src = V + row * ld + coff + 4 * lk;
            // the row chunk in two halves (fewer live registers); every
            // input of the tile is read before its first store
            constexpr int KH = (KCH + 1) / 2;
#pragma unroll
            for (int hb = 0; hb < 2; ++hb) {
                double4 x[KH];
#pragma unroll
                for (int cc = 0; cc < KH; ++cc) {
                    const int c = hb * KH + cc;
                    x[cc] = make_double4(0, 0, 0, 0);
                    if (c < KCH && rv && c * 16 + 4 * lk < kin) {
                        const d4 v = gload(reinterpret_cast<const d4*>(src + c * 16));
                        x[cc] = make_double4(v[0], v[1], v[2], v[3]);
                    }
                }
#pragma unroll
                for (int cc = 0; cc < KH; ++cc) {
                    const int c = hb * KH + cc;
                    if (c < KCH && c * 16 < kin) {
                        const double xs[4] = {x[cc].x, x[cc].y, x[cc].z, x[cc].w};
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const int kr = c * 16 + 4 * lk + s;
                            const double bm = kr < kin ? gload(M + kr * 16 + li) : 0.0;
                            D = mfma16(xs[s], bm, D);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = row0 + 4 * q + lk;
            if (row < n && li < b) V[row * ld + yoff + li] = D[q];
        }
        if (GRAM) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // the step's basis loads first (as in w_pass_a)
                const int64_t row = row0 + 4 * q + lk;
                const bool rv = row < n;
                const int64_t rs = rv ? row : 0;
                double araw[RTMAX];
#pragma unroll
                for (int rt = 0; rt < RTMAX; ++rt) {
                    const int col = rt * 16 + li;
                    araw[rt] = gload(V + rs * ld + (rt < nrt && col < cv ? col : 0));
                }
#pragma unroll
                for (int rt = 0; rt < RTMAX; ++rt) {
                    if (rt < nrt) {
                        const double a = (rv && rt * 16 + li < cv) ? araw[rt] : 0.0;
                        acc[rt] = mfma16(a, D[q], acc[rt]);
                    }
                }
            }
        }
        if (GRAM || SYRK)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[NG - 1] = mfma16(D[q], D[q], acc[NG - 1]);
    }
    if constexpr (GRAM || SYRK) wg_tiles<NG, true>(acc, nrt, GRAM ? cv : 0, b, wred, out);
}

// V[:, 0:p] = V[:, 0:m] Z (Z: m x p, row stride zs) and, if nb > 0,
// V[:, p : p + nb] = V[:, m : m + nb], over tiles [tile0, tile1), in place
// (every input of a tile is in registers before its first store).
__device__ SF_ITEM_FN void w_rotate(int64_t n, double* V, int ld, int m, const double* __restrict__ Z, int zs,
                                      int p, int nb, int64_t tile0, int64_t tile1) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nct = (p + 15) >> 4;
    for (int64_t tile = tile0; tile < tile1; ++tile) {
        const int64_t row0 = tile * 16;
        double4 x[RTMAX];
        {
            const int64_t row = row0 + li;
            const bool rv = row < n;
            const double* s = V + row * ld + 4 * lk;
#pragma unroll
            for (int c = 0; c < RTMAX; ++c) {
                x[c] = make_double4(0, 0, 0, 0);
                if (rv && c * 16 + 4 * lk < m) x[c] = *reinterpret_cast<const double4*>(s + c * 16);
            }
        }
        double nx[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = row0 + 4 * q + lk;
            nx[q] = (row < n && li < nb) ? V[row * ld + m + li] : 0.0;
        }
        for (int c = 0; c < nct; ++c) {
            const int col = c * 16 + li;
            d4 D = d4{0, 0, 0, 0};
#pragma unroll
            for (int ch = 0; ch < RTMAX; ++ch) {
                if (ch * 16 < m) {
                    const double xs[4] = {x[ch].x, x[ch].y, x[ch].z, x[ch].w};
#pragma unroll
                    for (int st = 0; st < 4; ++st) {
                        const int kr = ch * 16 + 4 * lk + st;
                        const double bm = (kr < m && col < p) ? Z[kr * zs + col] : 0.0;
                        D = mfma16(xs[st], bm, D);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = row0 + 4 * q + lk;
                if (row < n && col < p) V[row * ld + col] = D[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = row0 + 4 * q + lk;
            if (row < n && li < nb) V[row * ld + p + li] = nx[q];
        }
    }
}

// Residual partials of the certification, 16 columns:
// out[j] = sum over rows of (T_r[j] - c_r R2[g_r][j] - theta_j X[r][j])^2.
__device__ SF_ITEM_FN void w_resid(const Graph& t, const double* X, int ld, const double* __restrict__ T,
                                     const double* __restrict__ R2, const double* __restrict__ th, int kc,
                                     int64_t r0, int64_t r1, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, rl = lane >> 4;
    const double thj = col < kc ? th[col] : 0.0;
    double acc = 0.0;
    for (int64_t i = r0 + rl; i < r1; i += 4) {
        const double c = t.cs ? t.cs[i] : 1.0;
        const double y = T[i * 16 + col] - c * R2[t.grp[i] * 16 + col];
        const double r = y - thj * X[i * ld + col];
        acc += r * r;
    }
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    if (rl == 0) out[col] = acc;
}

// Sign partials, 16 columns: the largest |c_r X[r][j]| over the rows (lowest
// row on ties): out[j] = magnitude, out[16 + j] = row, out[32 + j] = value.
__device__ SF_ITEM_FN void w_signs(const Graph& t, const double* X, int ld, int64_t r0, int64_t r1,
                                     double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, rl = lane >> 4;
    double best = -1.0, bv = 0.0;
    int64_t bi = 0;
    for (int64_t i = r0 + rl; i < r1; i += 4) {
        const double v = (t.cs ? t.cs[i] : 1.0) * X[i * ld + col];
        const double a = fabs(v);
        if (a > best) {
            best = a;
            bi = i;
            bv = v;
        }
    }
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
        const double ob = __shfl_xor(best, off);
        const int64_t oi = __shfl_xor(bi, off);
        const double ov = __shfl_xor(bv, off);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
            bv = ov;
        }
    }
    if (rl == 0) {
        out[col] = best;
        out[16 + col] = (double)bi;
        out[32 + col] = bv;
    }
}

// The signs' maximum over a set of partials (lowest row on ties), 16 columns.
__device__ __forceinline__ void sign_merge(const double* p, double& b0, double& i0, double& v0) {
    const int j = threadIdx.x & 15;
    const double ob = p[j], oi = p[16 + j];
    if (ob > b0 || (ob == b0 && oi < i0)) {
        b0 = ob;
        i0 = oi;
        v0 = p[32 + j];
    }
}

// ===========================================================================
// Graph phases: the graph's owner workgroup.

// dst[e] = sum over the graph's items of part[item][e], e < cnt, in a fixed
// order (item residues modulo 8, then a fixed tree).
__device__ __forceinline__ void g_reduce(const double* __restrict__ part, int item0, int nitems, int cnt, double* dst) {
    for (int e = threadIdx.x; e < cnt; e += NT) {
        const double* p = part + (size_t)item0 * PSTRIDE + e;
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = 0.0;
        for (int it = 0; it < nitems; it += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (it + u < nitems) a[u] += p[(size_t)(it + u) * PSTRIDE];
        }
        dst[e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    __syncthreads();
}

// From the group sums A ([h][bw]) of a block Z: S = C^T Z (A_s - p_s sum_t
// A_t, s < h-1), optionally stored in Sout; then S -= sigma * Ssub;
// U = Ginv S; R_s = U_s - q (s < h-1), R_{h-1} = -q, q = sum_s p_s U_s, so
// that (C U)_i = c_i R_{g_i}.  R and Sout may be global.
__device__ __forceinline__ void g_finalize(const double* A, int h, int bw, const double* __restrict__ gpar, double* Sout,
                           const double* Ssub, double sigma, double* zs, double* R) {
    const int j = threadIdx.x;
    if (j < bw) {
        const int m = h - 1;
        const double* p = gpar;
        const double* Ginv = gpar + h;
        double tot = 0.0;
        for (int s = 0; s < h; ++s) tot += A[s * bw + j];
        for (int s = 0; s < m; ++s) {
            double z = A[s * bw + j] - p[s] * tot;
            if (Sout) Sout[s * 16 + j] = z;
            if (Ssub) z -= sigma * Ssub[s * 16 + j];
            zs[s * 16 + j] = z;
        }
        double q = 0.0;
        for (int s = 0; s < m; ++s) {
            double u = 0.0;
            for (int r = 0; r < m; ++r) u += Ginv[s * m + r] * zs[r * 16 + j];
            R[s * 16 + j] = u;
            q += p[s] * u;
        }
        for (int s = 0; s < m; ++s) R[s * 16 + j] -= q;
        R[m * 16 + j] = -q;
    }
    __syncthreads();
}

template <int B>
__device__ __forceinline__ bool chol_wave(const double* G, int b, double thresh, double* R, double* Rinv) {
    const int j = threadIdx.x;
    double g[B], ri[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        double v = 0.0;
        if (j < B) v = (i < b && j < b) ? G[i * b + j] : (i == j ? 1.0 : 0.0);
        g[i] = v;
        ri[i] = 0.0;
    }
    const bool ok = wave_chol_inv<B>(g, ri, thresh);
    if (j < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            R[i * 16 + j] = (i < B && j < B) ? g[i < B ? i : 0] : (i == j ? 1.0 : 0.0);
            Rinv[i * 16 + j] = (i < B && j < B) ? ri[i < B ? i : 0] : (i == j ? 1.0 : 0.0);
        }
    }
    return ok;
}

// Cholesky factor R (row-major 16 x 16, identity beyond b) and R^{-1} of the
// b x b matrix G (row-major), by wavefront 0.  Returns false on every thread
// of the workgroup if a pivot is <= thresh.
__device__ __forceinline__ bool g_chol(const double* G, int b, double thresh, double* R, double* Rinv, Shared& S) {
    if (threadIdx.x < 64) {
        const bool ok = b <= 4   ? chol_wave<4>(G, b, thresh, R, Rinv)
                        : b <= 8 ? chol_wave<8>(G, b, thresh, R, Rinv)
                                 : chol_wave<16>(G, b, thresh, R, Rinv);
        if (threadIdx.x == 0) S.iflag[0] = ok ? 1 : 0;
    }
    __syncthreads();
    const bool ok = S.iflag[0] != 0;
    __syncthreads();
    return ok;
}

// Eigen-decomposition of the symmetric m x m matrix A (LDS, stride LDT) by
// cyclic Jacobi, round-robin ordering, rotations accumulated into Z (LDS,
// stride LDT, the identity on entry).  A round's m/2 rotations are disjoint
// and applied at once: a thread takes a 2 x 2 block of entries (rows of pair
// a, columns of pair c, a <= c) and writes J_a^T A_ac J_c and its mirror
// from the old values, so a round needs one barrier after the rotation
// angles and one after the update.  The blocks and the (row, pair) updates
// of Z are spread evenly over the threads once per call.  Rotations whose
// off-diagonal entry is at most 1e-16 ||A||_F (the rounding level of the
// rotations themselves) are skipped and blocks of two skipped pairs are not
// touched; the sweeps stop after one without rotations (at most 40).  On
// return diag(A) holds the eigenvalues and Z the eigenvectors as columns.
__device__ __forceinline__ void g_jacobi(double* A, int m, double* Z, Shared& S) {
    const int t = threadIdx.x;
    const int mm = m + (m & 1), np = mm / 2, rr = mm - 1;
    // this thread's block (pair ba, pair bc), if any
    static_assert((NCVMAX / 2) * (NCVMAX / 2 + 1) / 2 <= NT, "one Jacobi block per thread");
    int ba = -1, bc = -1;
    {
        int idx = t, a = 0;
        if (idx < np * (np + 1) / 2) {
            while (idx >= np - a) {
                idx -= np - a;
                ++a;
            }
            ba = a;
            bc = a + idx;
        }
    }
    // this thread's (row, pair) updates of Z
    constexpr int ZMAX = (NCVMAX * (NCVMAX / 2) + NT - 1) / NT;
    int zi[ZMAX], zp[ZMAX];
#pragma unroll
    for (int u = 0; u < ZMAX; ++u) {
        const int idx = t + u * NT;
        zi[u] = -1;
        zp[u] = 0;
        if (idx < m * np) {
            zi[u] = idx / np;
            zp[u] = idx - zi[u] * np;
        }
    }
    double off = 0.0, dg = 0.0;
    for (int idx = t; idx < m * m; idx += NT) {
        const int i = idx / m, j = idx - i * m;
        const double v = A[i * LDT + j];
        if (i != j)
            off += v * v;
        else
            dg += v * v;
    }
    wg_sum2(off, dg, S.wsum);
    const double tiny = 1e-16 * sqrt(dg + off);
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (t == 0) S.iflag[2] = 0;
        __syncthreads();
        for (int r = 0; r < rr; ++r) {
            if (t < np) {
                int p, q;
                if (t == 0) {
                    p = r;
                    q = rr;
                } else {
                    p = r + t;
                    if (p >= rr) p -= rr;
                    q = r - t;
                    if (q < 0) q += rr;
                }
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, sn = 0.0;
                if (q < m) {
                    const double apq = A[p * LDT + q];
                    if (fabs(apq) > tiny) {
                        const double th = (A[q * LDT + q] - A[p * LDT + p]) / (2.0 * apq);
                        const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        sn = tt * c;
                        S.iflag[2] = 1;
                    }
                }
                S.jcs[t] = make_double2(c, sn);
                S.jpq[t] = make_int2(p, q);
            }
            __syncthreads();
            // A <- J^T A J on this thread's 2 x 2 block (mirrored); entries
            // with an index >= m (the padding index of odd m) are neither
            // read nor written
            if (ba >= 0) {
                const double2 cs1 = S.jcs[ba], cs2 = S.jcs[bc];
                if (cs1.y != 0.0 || cs2.y != 0.0) {
                    const int2 pq1 = S.jpq[ba], pq2 = S.jpq[bc];
                    const int p1 = pq1.x, q1 = pq1.y, p2 = pq2.x, q2 = pq2.y;
                    const bool vq1 = q1 < m, vq2 = q2 < m;
                    const double c1 = cs1.x, s1 = cs1.y, c2 = cs2.x, s2 = cs2.y;
                    const double x00 = A[p1 * LDT + p2];
                    const double x01 = vq2 ? A[p1 * LDT + q2] : 0.0;
                    const double x10 = vq1 ? A[q1 * LDT + p2] : 0.0;
                    const double x11 = (vq1 && vq2) ? A[q1 * LDT + q2] : 0.0;
                    // columns: Y = X J2
                    const double y00 = c2 * x00 - s2 * x01, y01 = s2 * x00 + c2 * x01;
                    const double y10 = c2 * x10 - s2 * x11, y11 = s2 * x10 + c2 * x11;
                    // rows: J1^T Y
                    const double z00 = c1 * y00 - s1 * y10, z01 = c1 * y01 - s1 * y11;
                    const double z10 = s1 * y00 + c1 * y10, z11 = s1 * y01 + c1 * y11;
                    A[p1 * LDT + p2] = z00;
                    if (vq2) A[p1 * LDT + q2] = z01;
                    if (vq1) A[q1 * LDT + p2] = z10;
                    if (vq1 && vq2) A[q1 * LDT + q2] = z11;
                    if (bc != ba) {
                        A[p2 * LDT + p1] = z00;
                        if (vq2) A[q2 * LDT + p1] = z01;
                        if (vq1) A[p2 * LDT + q1] = z10;
                        if (vq1 && vq2) A[q2 * LDT + q1] = z11;
                    }
                }
            }
            // Z <- Z J
#pragma unroll
            for (int u = 0; u < ZMAX; ++u) {
                if (zi[u] < 0) continue;
                const double2 cs = S.jcs[zp[u]];
                if (cs.y == 0.0) continue;
                const int2 pq = S.jpq[zp[u]];
                double* z = Z + zi[u] * LDT;
                const double a0 = z[pq.x], a1 = z[pq.y];
                z[pq.x] = cs.x * a0 - cs.y * a1;
                z[pq.y] = cs.y * a0 + cs.x * a1;
            }
            __syncthreads();
        }
        if (S.iflag[2] == 0) break;
        __syncthreads();
    }
}

__device__ __forceinline__ void stop(GState& s, int status, int* active) {
    s.active = 0;
    s.status = status;
    s.t_done = wall_clock64();
    atomicSub(active, 1);
}

// ===========================================================================
// The launch.

enum Ph { PH_OP = 0, PH_A, PH_B, PH_C, PH_D, PH_RR, PH_ROT, PH_IO };

// The Rayleigh-Ritz step of a graph whose basis is full (m columns), by its
// owner workgroup: T_m diagonalized by Jacobi in LDS, the Ritz pairs in
// ascending order, the residual estimates ||Rc z_last||, the convergence
// test and the restart (or final) rotation, applied by the next row phase.
__device__ __forceinline__ void rayleigh_ritz(const Graph& g, GState& s, int m, int* active, Shared& S) {
    const int tid = threadIdx.x;
    const uint64_t t0 = wall_clock64();
    const int b = g.b, k = g.k;
    const int restarts = s.restarts;
    double* Ag = g.sm + OFF_T;
    double* Zg = g.sm + OFF_Z;
    for (int e = tid; e < m * m; e += NT) {
        const int i = e / m, j = e - i * m;
        S.u.j.A[i * LDT + j] = Ag[i * NCVMAX + j];
        S.u.j.Z[i * LDT + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    g_jacobi(S.u.j.A, m, S.u.j.Z, S);
    for (int e = tid; e < 256; e += NT) S.R2[e] = g.sm[OFF_R + 256 + e];  // coupling Rc
    if (tid < m) {
        const double w = S.u.j.A[tid * LDT + tid];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double o = S.u.j.A[j * LDT + j];
            rank += (o < w || (o == w && j < tid)) ? 1 : 0;
        }
        S.perm[rank] = tid;
        S.theta[rank] = w;
    }
    __syncthreads();
    // residual estimates ||Rc z_last|| of the Ritz pairs
    if (tid < m) {
        const int c = S.perm[tid];
        double s2 = 0.0;
        for (int i = 0; i < b; ++i) {
            double v = 0.0;
            for (int j = i; j < b; ++j) v += S.R2[i * 16 + j] * S.u.j.Z[(m - b + j) * LDT + c];
            s2 += v * v;
        }
        S.res[tid] = sqrt(s2);
    }
    if (tid == 0) {
        bool finite = true;
        for (int r = 0; r < m; ++r) finite &= isfinite(S.theta[r]);
        S.iflag[1] = finite ? 1 : 0;
    }
    __syncthreads();
    const bool finite = S.iflag[1] != 0;
    int nconv = 0;
    double est = 0.0;
    const double tolabs = g.tol_conv * g.sigma;
    for (int r = 0; r < k; ++r) {
        nconv += S.res[r] <= tolabs ? 1 : 0;
        est = fmax(est, S.res[r]);
    }
    const bool fin = nconv == k || restarts >= g.max_restarts;
    // rotation: the k Ritz vectors when finished, else the p kept ones
    // (k < p <= m - b, p a multiple of b)
    const int ptarget = max(k + 1, (m + k) / 2);
    const int nd = max(1, (m - ptarget) / b);
    const int p = fin ? k : m - nd * b;
    for (int e = tid; e < m * p; e += NT) {
        const int q = e / p, r = e - q * p;
        Zg[q * NCVMAX + r] = S.u.j.Z[q * LDT + S.perm[r]];
    }
    for (int r = tid; r < m; r += NT) g.sm[OFF_AUX + r] = S.theta[r];
    if (!fin) {
        for (int e = tid; e < p * p; e += NT) {
            const int i = e / p, j = e - i * p;
            Ag[i * NCVMAX + j] = (i == j) ? S.theta[i] : 0.0;
        }
    }
    __syncthreads();
    if (tid == 0) {
        s.nconv = nconv;
        s.est = est / g.sigma;
        s.gap = m > k ? (S.theta[k] - S.theta[k - 1]) / g.sigma : 0.0;
        if (!finite) {
            stop(s, 2, active);
        } else {
            s.rot_m = m;
            s.rot_p = p;
            s.rot_nb = fin ? 0 : b;
            if (fin) {
                s.out = 1;
                stop(s, nconv == k ? 0 : 1, active);
            } else {
                s.m = p;
                s.restarts = restarts + 1;
            }
        }
    }
    __syncthreads();
    if (tid == 0)
        __hip_atomic_fetch_add(&s.ph[PH_RR], (uint64_t)(wall_clock64() - t0), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// The items of the graphs still in their block steps (out: of the graphs
// with output), in graph order, into alist / nalist.  Workgroup 0 only.
__device__ __forceinline__ void build_list(const Launch& L, bool out, Shared& S) {
    int base = 0;
    for (int g0 = 0; g0 < L.ng; g0 += NT) {
        const int gi = g0 + threadIdx.x;
        int cnt = 0;
        if (gi < L.ng) {
            const GState& s = L.st[gi];
            cnt = (out ? s.out : s.active) ? L.graphs[gi].nitems : 0;
        }
        S.iscan[threadIdx.x] = cnt;
        __syncthreads();
        for (int off = 1; off < NT; off <<= 1) {
            const int v = threadIdx.x >= off ? S.iscan[threadIdx.x - off] : 0;
            __syncthreads();
            S.iscan[threadIdx.x] += v;
            __syncthreads();
        }
        const int excl = base + S.iscan[threadIdx.x] - cnt;
        if (cnt) {
            const int i0 = L.graphs[gi].item0;
            for (int j = 0; j < cnt; ++j) L.alist[excl + j] = i0 + j;
        }
        base += S.iscan[NT - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *L.nalist = base;
}

__device__ __forceinline__ void add_ticks(GState& s, int ph, uint64_t t0) {
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(&s.ph[ph], (uint64_t)(wall_clock64() - t0), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// Row phase: every workgroup takes the listed items blockIdx.x,
// + gridDim.x, ... and runs f on each: f(g (graph), s (state), it (item),
// wr0 / wr1 (this wavefront's rows), wt0 / wt1 (its 16-row tiles), slot (the
// item's partial slot), wp (this wavefront's LDS partial), tid, wave, S,
// t0_ (the item's start clock)) returns false, before any work, when the
// graph does not take part (uniform for the graph).  One non-inlined
// instance per phase, the row work inlined into it.  (Every helper of the
// kernel is inlined: the kernel makes no calls.)
template <class F>
__device__ __forceinline__ void items_phase(Launch L, Shared& S, int ph, F f) {
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int j_ = blockIdx.x, n_ = *L.nalist; j_ < n_; j_ += gridDim.x) {
        const int it = L.alist[j_];
        const Item itm = L.items[it];
        const Graph& g = L.graphs[itm.g];
        GState& s = L.st[itm.g];
        const uint64_t t0_ = wall_clock64();
        const int64_t wr0 = min(g.n, itm.row0 + (int64_t)wave * WROWS);
        const int64_t wr1 = min(g.n, wr0 + WROWS);
        const int64_t wt0 = wr0 >> 4, wt1 = wr1 > wr0 ? (wr1 + 15) >> 4 : wt0;
        double* slot = L.part + (size_t)it * PSTRIDE;
        double* wp = S.u.wred + wave * WRED;
        if (f(g, s, it, wr0, wr1, wt0, wt1, slot, wp, tid, wave, S, t0_)) add_ticks(s, ph, t0_);
    }
}

#define SF_ITEMS(PH, COND, ...)                                                                          \
    items_phase(L, S, PH,                                                                                \
                [=](const Graph& g, GState& s, int it, int64_t wr0, int64_t wr1, int64_t wt0, int64_t wt1, \
                    double* slot, double* wp, int tid, int wave, Shared& S, uint64_t t0_) -> bool {      \
                    (void)it;                                                                            \
                    (void)wr0;                                                                           \
                    (void)wr1;                                                                           \
                    (void)wt0;                                                                           \
                    (void)wt1;                                                                           \
                    (void)slot;                                                                          \
                    (void)wp;                                                                            \
                    (void)wave;                                                                          \
                    (void)t0_;                                                                           \
                    if (!(COND)) return false;                                                           \
                    __VA_ARGS__;                                                                         \
                    return true;                                                                         \
                })

// Graph phase: workgroup blockIdx.x owns graphs blockIdx.x, + gridDim.x, ...
// Every thread reads COND before the body may change the state.
#define SF_GRAPHS(PH, COND, ...)                                \
    for (int gi = blockIdx.x; gi < L.ng; gi += gridDim.x) {     \
        const Graph& g = L.graphs[gi];                          \
        GState& s = L.st[gi];                                   \
        const bool on_ = (COND);                                \
        __syncthreads();                                        \
        if (!on_) continue;                                     \
        const uint64_t t0_ = wall_clock64();                    \
        __VA_ARGS__;                                            \
        add_ticks(s, PH, t0_);                                  \
    }

template <class SpT>
__global__ __launch_bounds__(NT) void k_batched(Launch L) {
    __shared__ Shared S;
    cg::grid_group grid = cg::this_grid();
    const int tid = threadIdx.x;
    const int wave = tid >> 6;

    // ---- set-up and the random start block ----------------------------------
    if (blockIdx.x == 0 && tid == 0) *L.t_start = wall_clock64();
    SF_GRAPHS(PH_IO, true, {
        const bool ok = (g.b == 4 || g.b == 8 || g.b == 16) && g.ncv <= NCVMAX && g.ncv % 4 == 0 &&
                        g.ld >= g.ncv + g.b && g.ld % 4 == 0 && g.k >= 1 && g.k <= KMAXB && g.k + g.b < g.ncv &&
                        g.ld >= ((g.k + 15) / 16) * 16 && g.h >= 1 && g.h <= HMAX && g.rows >= 1 && g.rows <= 64 &&
                        (g.rows & (g.rows - 1)) == 0 && g.n >= 2 * (int64_t)g.ld;
        if (tid == 0) {
            s.active = 1;
            s.status = 0;
            s.out = 0;
            s.m = 0;
            s.restarts = 0;
            s.steps = 0;
            s.nconv = 0;
            s.rot_p = 0;
            s.est = 0.0;
            s.gap = 0.0;
            s.maxres = 0.0;
            s.t_done = 0;
            for (int q = 0; q < 8; ++q) s.ph[q] = 0;
            if (!ok) stop(s, 4, L.active);
        }
        for (int e = tid; e < 256; e += NT) g.sm[OFF_M + e] = ((e >> 4) == (e & 15)) ? 1.0 : 0.0;
    });
    grid.sync();
    if (blockIdx.x == 0) build_list(L, false, S);
    grid.sync();
    // random start block and its group sums
    SF_ITEMS(PH_IO, s.active, {
        const int b = g.b;
        for (int64_t idx = (tid & 63); idx < (wr1 - wr0) * b; idx += 64) {
            const int64_t i = wr0 + idx / b;
            const int j = (int)(idx % b);
            g.V[i * g.ld + j] = rnd_pm1(g.seed, (uint64_t)(i * b + j));
        }
        __syncthreads();
        w_gsum(g.V, g.ld, wr0, wr1, b, g.h, g.grp, g.cs, wp);
        wg_combine(S.u.wred, g.h * 16, b, slot);
    });
    grid.sync();
    SF_GRAPHS(PH_IO, s.active, {
        g_reduce(L.part, g.item0, g.nitems, g.h * g.b, S.red);
        g_finalize(S.red, g.h, g.b, g.gpar, nullptr, nullptr, 0.0, S.gZ, g.sm + OFF_TAB);
    });
    grid.sync();
    // projection onto null(C^T), then the Gram matrix (first Cholesky-QR pass, M = I)
    SF_ITEMS(PH_IO, s.active, {
        w_proj<double>(g.V, g.ld, wr0, wr1, g.b, g.grp, g.cs, g.sm + OFF_TAB, g.V, g.ld);
        __syncthreads();
        w_upd<false, true>(g.n, g.V, g.ld, 0, g.b, 0, g.b, 0, g.sm + OFF_M, wt0, wt1, S.u.wred, slot);
    });
    grid.sync();
    SF_GRAPHS(PH_IO, s.active, {
        g_reduce(L.part, g.item0, g.nitems, g.b * g.b, S.red);
        if (!g_chol(S.red, g.b, 0.0, S.R1, S.Ri, S)) {
            if (tid == 0) stop(s, 2, L.active);
        } else {
            for (int e = tid; e < 256; e += NT) g.sm[OFF_M + e] = S.Ri[e];
        }
    });
    grid.sync();
    SF_ITEMS(PH_IO, s.active,
             w_upd<false, true>(g.n, g.V, g.ld, 0, g.b, 0, g.b, 0, g.sm + OFF_M, wt0, wt1, S.u.wred, slot));
    grid.sync();
    SF_GRAPHS(PH_IO, s.active, {
        g_reduce(L.part, g.item0, g.nitems, g.b * g.b, S.red);
        if (!g_chol(S.red, g.b, 0.25, S.R2, S.Ri, S)) {
            if (tid == 0) stop(s, 2, L.active);
        } else {
            for (int e = tid; e < 256; e += NT) g.sm[OFF_M + e] = S.Ri[e];
        }
    });
    grid.sync();
    // the orthonormal start block, and its group sums for the first operator
    SF_ITEMS(PH_IO, s.active, {
        w_upd<false, false>(g.n, g.V, g.ld, 0, g.b, 0, g.b, 0, g.sm + OFF_M, wt0, wt1, S.u.wred, slot);
        __syncthreads();
        w_gsum(g.V, g.ld, wr0, wr1, g.b, g.h, g.grp, g.cs, wp);
        wg_combine(S.u.wred, g.h, g.b, slot);
    });
    grid.sync();
    SF_GRAPHS(PH_IO, s.active, {
        g_reduce(L.part, g.item0, g.nitems, g.h * g.b, S.red);
        g_finalize(S.red, g.h, g.b, g.gpar, g.sm + OFF_TAB + HMAX * 16, nullptr, 0.0, S.gZ, g.sm + OFF_TAB);
    });
    grid.sync();

    // ---- block steps: basis V[:, 0:m], current block V[:, m : m + b] ----------
    int listed = -1;       // active count when the item list was built
    int listed_items = 0;  // items in that list
    for (int step = 0; step < L.max_steps; ++step) {
        const int act = __hip_atomic_load(L.active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (act <= L.handoff) break;
        if (act != listed) {
            if (blockIdx.x == 0) build_list(L, false, S);
            grid.sync();
            listed = act;
            listed_items = *L.nalist;
        }
#ifdef SF_BATCH_STEPLOG
        if (blockIdx.x == 0 && tid == 0 && L.steplog) {
            L.steplog[2 * step] = wall_clock64();
            L.steplog[2 * step + 1] = (uint64_t)act | ((uint64_t)listed_items << 32);
        }
#endif
        // restart rotation (if pending), then X' = P X (the tables of X are current)
        SF_ITEMS(PH_OP, s.active, {
            if (s.rot_p > 0) {
                w_rotate(g.n, g.V, g.ld, s.rot_m, g.sm + OFF_Z, NCVMAX, s.rot_p, s.rot_nb, wt0, wt1);
                add_ticks(s, PH_ROT, t0_);
                if (tid == 0)
                    __hip_atomic_fetch_add(&s.ph[PH_OP], (uint64_t)0 - (wall_clock64() - t0_), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            w_proj<SpT>(g.V + s.m, g.ld, wr0, wr1, g.b, g.grp, g.cs, g.sm + OFF_TAB, static_cast<SpT*>(g.xp), g.b);
        });
        grid.sync();
        // sparse product and its group sums
        SF_ITEMS(PH_OP, s.active, {
            w_spmm<SpT>(g, static_cast<const SpT*>(g.xp), static_cast<SpT*>(g.tt), wr0, wr1, g.b, g.rows);
            __syncthreads();
            w_gsum(static_cast<const SpT*>(g.tt), g.b, wr0, wr1, g.b, g.h, g.grp, g.cs, wp);
            wg_combine(S.u.wred, g.h, g.b, slot);
        });
        grid.sync();
        SF_GRAPHS(PH_OP, s.active, {
            if (tid == 0) s.rot_p = 0;
            g_reduce(L.part, g.item0, g.nitems, g.h * g.b, S.red);
            g_finalize(S.red, g.h, g.b, g.gpar, nullptr, g.sm + OFF_TAB + HMAX * 16, g.sigma, S.gZ,
                       g.sm + OFF_TAB + 2 * HMAX * 16);
        });
        grid.sync();
        // pass A: output deflation Y0 = T - C U and H1 = V^T Y0
        SF_ITEMS(PH_A, s.active,
                 w_pass_a<SpT>(g, g.V, g.ld, s.m + g.b, g.b, static_cast<const SpT*>(g.tt),
                               g.sm + OFF_TAB + 2 * HMAX * 16, wt0, wt1, S.u.wred, slot));
        grid.sync();
        SF_GRAPHS(PH_A, s.active, {
            const int m = s.m, b = g.b, cv = m + b;
            double* T = g.sm + OFF_T;
            double* M = g.sm + OFF_M;
            g_reduce(L.part, g.item0, g.nitems, cv * b, S.red);
            // H1 into T's column block; M1 = [-H1; I]
            for (int e = tid; e < (cv + b) * 16; e += NT) {
                const int q = e >> 4, j = e & 15;
                if (q < cv) {
                    const double hv = j < b ? S.red[q * b + j] : 0.0;
                    M[e] = -hv;
                    if (j < b) {
                        T[q * NCVMAX + m + j] = hv;
                        if (q < m) T[(m + j) * NCVMAX + q] = hv;
                    }
                } else {
                    M[e] = (q - cv == j) ? 1.0 : 0.0;
                }
            }
        });
        grid.sync();
        // pass B: Y' = Y0 - V H1; H2 = V^T Y', G1 = Y'^T Y'
        SF_ITEMS(PH_B, s.active,
                 w_upd<true, true>(g.n, g.V, g.ld, 0, s.m + 2 * g.b, s.m + g.b, g.b, s.m + g.b, g.sm + OFF_M, wt0,
                                   wt1, S.u.wred, slot));
        grid.sync();
        SF_GRAPHS(PH_B, s.active, {
            const int m = s.m, b = g.b, cv = m + b;
            const double thresh = (1e-10 * g.sigma) * (1e-10 * g.sigma);
            double* T = g.sm + OFF_T;
            double* M = g.sm + OFF_M;
            g_reduce(L.part, g.item0, g.nitems, (cv + b) * b, S.red);
            for (int e = tid; e < cv * b; e += NT) {
                const int q = e / b, j = e - q * b;
                const double hv = S.red[q * b + j];
                T[q * NCVMAX + m + j] += hv;
                if (q < m) T[(m + j) * NCVMAX + q] += hv;
            }
            __syncthreads();
            for (int e = tid; e < b * b; e += NT) {
                const int i = e / b, j = e - i * b;
                if (j > i) {
                    const double a = T[(m + i) * NCVMAX + m + j], c = T[(m + j) * NCVMAX + m + i];
                    const double mv = 0.5 * (a + c);
                    T[(m + i) * NCVMAX + m + j] = mv;
                    T[(m + j) * NCVMAX + m + i] = mv;
                }
            }
            if (!g_chol(S.red + cv * b, b, thresh, S.R1, S.Ri, S)) {
                if (tid == 0) stop(s, 2, L.active);
            } else {
                for (int e = tid; e < 256; e += NT) g.sm[OFF_R + e] = S.R1[e];
                // M2 = [-H2 R1^{-1}; R1^{-1}]
                for (int e = tid; e < (cv + b) * 16; e += NT) {
                    const int q = e >> 4, j = e & 15;
                    double acc = 0.0;
                    if (j < b) {
                        if (q < cv) {
                            for (int u = 0; u <= j; ++u) acc -= S.red[q * b + u] * S.Ri[u * 16 + j];
                        } else {
                            acc = S.Ri[(q - cv) * 16 + j];
                        }
                    }
                    M[e] = acc;
                }
            }
        });
        grid.sync();
        // pass C: Y1 = (Y' - V H2) R1^{-1}, G2 = Y1^T Y1
        SF_ITEMS(PH_C, s.active,
                 w_upd<false, true>(g.n, g.V, g.ld, 0, s.m + 2 * g.b, s.m + g.b, g.b, s.m + g.b, g.sm + OFF_M,
                                    wt0, wt1, S.u.wred, slot));
        grid.sync();
        SF_GRAPHS(PH_C, s.active, {
            g_reduce(L.part, g.item0, g.nitems, g.b * g.b, S.red);
            for (int e = tid; e < 256; e += NT) S.R1[e] = g.sm[OFF_R + e];
            __syncthreads();
            if (!g_chol(S.red, g.b, 0.25, S.R2, S.Ri, S)) {
                if (tid == 0) stop(s, 2, L.active);
            } else {
                // coupling Rc = R2 R1; M3 = R2^{-1}
                for (int e = tid; e < 256; e += NT) {
                    const int i = e >> 4, j = e & 15;
                    double acc = 0.0;
                    for (int u = i; u <= j; ++u) acc += S.R2[i * 16 + u] * S.R1[u * 16 + j];
                    g.sm[OFF_R + 256 + e] = acc;
                    g.sm[OFF_M + e] = S.Ri[e];
                }
            }
        });
        grid.sync();
        // pass D: the next block, and its group sums
        SF_ITEMS(PH_D, s.active, {
            const int cv = s.m + g.b;
            w_upd<false, false>(g.n, g.V, g.ld, cv, g.b, cv, g.b, 0, g.sm + OFF_M, wt0, wt1, S.u.wred, slot);
            __syncthreads();
            w_gsum(g.V + cv, g.ld, wr0, wr1, g.b, g.h, g.grp, g.cs, wp);
            wg_combine(S.u.wred, g.h, g.b, slot);
        });
        grid.sync();
        // tables of the next block; Rayleigh-Ritz and the restart when the basis is full
        SF_GRAPHS(PH_D, s.active, {
            const int b = g.b;
            const int m = s.m + b;
            const int steps = s.steps + 1;
            g_reduce(L.part, g.item0, g.nitems, g.h * b, S.red);
            g_finalize(S.red, g.h, b, g.gpar, g.sm + OFF_TAB + HMAX * 16, nullptr, 0.0, S.gZ, g.sm + OFF_TAB);
            if (tid == 0) s.steps = steps;
            if (m + b <= g.ncv) {
                if (tid == 0) s.m = m;
            } else {
                const uint64_t t1 = wall_clock64();
                rayleigh_ritz(g, s, m, L.active, S);
                // counted as Rayleigh-Ritz time by rayleigh_ritz
                if (tid == 0)
                    __hip_atomic_fetch_add(&s.ph[PH_D], (uint64_t)0 - (wall_clock64() - t1), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
            }
        });
        grid.sync();
    }
    // graphs still iterating (step limit or hand-off): no output here; after a
    // restart, V[:, 0:k] holds the current Ritz vectors (the expansions since
    // only append columns)
    SF_GRAPHS(PH_IO, s.active, {
        if (tid == 0) stop(s, s.restarts > 0 ? 5 : 1, L.active);
    });
    grid.sync();

    // ---- output: Ritz vectors, projection, certification, signs, H -------------
    if (blockIdx.x == 0) build_list(L, true, S);
    grid.sync();
    SF_ITEMS(PH_IO, s.out && s.rot_p > 0,
             w_rotate(g.n, g.V, g.ld, s.rot_m, g.sm + OFF_Z, NCVMAX, s.rot_p, 0, wt0, wt1));
    grid.sync();
    for (int c0 = 0; c0 < KMAXB; c0 += 16) {
        SF_ITEMS(PH_IO, s.out && g.k > c0, {
            w_gsum(g.V + c0, g.ld, wr0, wr1, 16, g.h, g.grp, g.cs, wp);
            wg_combine(S.u.wred, g.h, 16, slot);
        });
        grid.sync();
        SF_GRAPHS(PH_IO, s.out && g.k > c0, {
            g_reduce(L.part, g.item0, g.nitems, g.h * 16, S.red);
            g_finalize(S.red, g.h, 16, g.gpar, nullptr, nullptr, 0.0, S.gZ, g.sm + OFF_TAB);
        });
        grid.sync();
        // projection in place; with certification, the group sums of the result
        SF_ITEMS(PH_IO, s.out && g.k > c0, {
            w_proj<double>(g.V + c0, g.ld, wr0, wr1, 16, g.grp, g.cs, g.sm + OFF_TAB, g.V + c0, g.ld);
            if (g.certify) {
                __syncthreads();
                w_gsum(g.V + c0, g.ld, wr0, wr1, 16, g.h, g.grp, g.cs, wp);
                wg_combine(S.u.wred, g.h, 16, slot);
            }
        });
        grid.sync();
        // certification: one FP64 application of the operator to the 16 columns
        SF_GRAPHS(PH_IO, s.out && g.k > c0 && g.certify, {
            g_reduce(L.part, g.item0, g.nitems, g.h * 16, S.red);
            g_finalize(S.red, g.h, 16, g.gpar, g.sm + OFF_TAB + HMAX * 16, nullptr, 0.0, S.gZ, g.sm + OFF_TAB);
        });
        grid.sync();
        SF_ITEMS(PH_IO, s.out && g.k > c0 && g.certify,
                 w_proj<double>(g.V + c0, g.ld, wr0, wr1, 16, g.grp, g.cs, g.sm + OFF_TAB,
                                static_cast<double*>(g.xp), 16));
        grid.sync();
        SF_ITEMS(PH_IO, s.out && g.k > c0 && g.certify, {
            w_spmm<double>(g, static_cast<const double*>(g.xp), static_cast<double*>(g.tt), wr0, wr1, 16, 8);
            __syncthreads();
            w_gsum(static_cast<const double*>(g.tt), 16, wr0, wr1, 16, g.h, g.grp, g.cs, wp);
            wg_combine(S.u.wred, g.h, 16, slot);
        });
        grid.sync();
        SF_GRAPHS(PH_IO, s.out && g.k > c0 && g.certify, {
            g_reduce(L.part, g.item0, g.nitems, g.h * 16, S.red);
            g_finalize(S.red, g.h, 16, g.gpar, nullptr, g.sm + OFF_TAB + HMAX * 16, g.sigma, S.gZ,
                       g.sm + OFF_TAB + 2 * HMAX * 16);
        });
        grid.sync();
        // residual and sign partials
        SF_ITEMS(PH_IO, s.out && g.k > c0, {
            if (g.certify) {
                w_resid(g, g.V + c0, g.ld, static_cast<const double*>(g.tt), g.sm + OFF_TAB + 2 * HMAX * 16,
                        g.sm + OFF_AUX + c0, min(16, g.k - c0), wr0, wr1, wp);
            } else if ((tid & 63) < 16) {
                wp[tid & 63] = 0.0;
            }
            w_signs(g, g.V + c0, g.ld, wr0, wr1, wp + 16);
            __syncthreads();
            if (tid < 16) {
                double r2 = 0.0, b0 = -1.0, i0 = 0.0, v0 = 0.0;
                for (int w = 0; w < NW; ++w) {
                    r2 += S.u.wred[w * WRED + tid];
                    sign_merge(S.u.wred + w * WRED + 16, b0, i0, v0);
                }
                slot[tid] = r2;
                slot[16 + tid] = b0;
                slot[32 + tid] = i0;
                slot[48 + tid] = v0;
            }
            __syncthreads();
        });
        grid.sync();
        SF_GRAPHS(PH_IO, s.out && g.k > c0, {
            if (tid < 16) {
                double r2 = 0.0, b0 = -1.0, i0 = 0.0, v0 = 0.0;
                for (int it = 0; it < g.nitems; ++it) {
                    const double* p = L.part + (size_t)(g.item0 + it) * PSTRIDE;
                    r2 += p[tid];
                    sign_merge(p + 16, b0, i0, v0);
                }
                S.res[tid] = sqrt(r2) / g.sigma;
                g.sm[OFF_AUX + NCVMAX + tid] = v0 < 0.0 ? -1.0 : 1.0;
            }
            __syncthreads();
            if (tid == 0 && g.certify) {
                double mr = s.maxres;
                for (int j = 0; j < 16 && c0 + j < g.k; ++j) mr = fmax(mr, S.res[j]);
                s.maxres = mr;
            }
        });
        grid.sync();
        // H = sign * C-scaled columns (D^{-1/2} X when normalized), column-major
        SF_ITEMS(PH_IO, s.out && g.k > c0, {
            const int kc = min(16, g.k - c0);
            const int64_t nr = wr1 - wr0;
            for (int64_t idx = (tid & 63); idx < nr * kc; idx += 64) {
                const int j = (int)(idx / nr);
                const int64_t i = wr0 + (idx - (int64_t)j * nr);
                const double c = g.cs ? g.cs[i] : 1.0;
                g.H[(int64_t)(c0 + j) * g.n + i] = g.sm[OFF_AUX + NCVMAX + j] * c * g.V[i * g.ld + c0 + j];
            }
        });
        grid.sync();
    }
    SF_GRAPHS(PH_IO, s.out, {
        for (int r = tid; r < g.k; r += NT) g.theta[r] = g.sm[OFF_AUX + r];
        if (tid == 0) {
            if (!g.certify) s.maxres = s.est;
            if (s.status == 0 && g.certify && s.maxres > g.tol) s.status = 3;
        }
    });
}

#undef SF_ITEMS
#undef SF_GRAPHS

__global__ void k_set_i32(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}
// host side

constexpr double kFloatTolFloor = 5e-7;  // tolerances below: double products
// Once at most kHandoffGraphs graphs of a batch of at least kHandoffMinBatch
// remain, they leave the launch (a few graphs cannot fill the grid) and are
// finished by sfairsc_eigs from their current Ritz vectors.
constexpr int kHandoffGraphs = 3;
constexpr int kHandoffMinBatch = 32;

struct Cfg {
    int b = 8, ncv = 48, rows = 1;
};

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Default basis size for k wanted pairs at block width b: room for about six
// blocks beyond k (and four times k), capped at the LDS limit.
int default_ncv(int k, int b) {
    return std::min(NCVMAX / b * b, round_up(std::max(k + 6 * b, 4 * k + 2 * b), b));
}

bool cfg_valid(const Cfg& c, int k) {
    return (c.b == 4 || c.b == 8 || c.b == 16) && c.ncv % c.b == 0 && c.ncv <= NCVMAX && c.ncv >= k + 1 + c.b &&
           c.rows >= 1 && c.rows <= 64 && (c.rows & (c.rows - 1)) == 0;
}

int max_rows(int b, bool dbl) {
    const int vec = dbl ? 2 : 4;
    return 64 / std::max(1, b / vec);
}

// Built-in configuration.  Block width 8 up to k = 16: with 16 a k = 9..16
// graph needs an 80-column basis, whose Rayleigh-Ritz step (1.3 ms on one
// workgroup) holds up the grid; on the 256-graph workload b = 8 took the
// launch from 0.75 to 0.60 s.
Cfg default_cfg(int64_t n, int64_t nnz, int k, bool dbl) {
    Cfg c;
    c.b = k <= 4 ? 4 : (k <= 16 ? 8 : 16);
    c.ncv = default_ncv(k, c.b);
    const double deg = n > 0 ? (double)nnz / (double)n : 1.0;
    const int vec = dbl ? 2 : 4;
    const int lpr = std::max(1, c.b / vec);
    int slots = 1;
    while (slots * 2 <= std::max(1.0, deg / 2)) slots *= 2;
    const int G = std::min(64, std::max(lpr, lpr * slots));
    c.rows = std::max(1, 64 / G);
    return c;
}

struct Key {
    int nlog, deg, kb, prec, norm;
    bool operator<(const Key& o) const {
        if (nlog != o.nlog) return nlog < o.nlog;
        if (deg != o.deg) return deg < o.deg;
        if (kb != o.kb) return kb < o.kb;
        if (prec != o.prec) return prec < o.prec;
        return norm < o.norm;
    }
};

Key key_of(int64_t n, int64_t nnz, int k, bool dbl, int normalized) {
    Key key;
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= n) ++l;
    key.nlog = l;
    const double d = (double)nnz / (double)std::max<int64_t>(1, n);
    key.deg = d < 16 ? 0 : d < 32 ? 1 : d < 64 ? 2 : 3;
    key.kb = k <= 4 ? 0 : k <= 8 ? 1 : k <= 16 ? 2 : 3;
    key.prec = dbl ? 0 : 1;
    key.norm = normalized ? 1 : 0;
    return key;
}

struct Entry {
    Cfg cfg;
    double ms = 0.0;
};

std::mutex g_tab_mu;
std::map<Key, Entry> g_table;
bool g_env_loaded = false;

int load_table_file(const char* path, bool replace);

void maybe_load_env() {
    // caller holds g_tab_mu
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char* p = std::getenv("SFAIRSC_TUNING_FILE");
    if (p && *p) {
        // errors leave the table empty (lookups fall back to the defaults)
        FILE* f = std::fopen(p, "r");
        if (f) {
            std::fclose(f);
            load_table_file(p, false);
        }
    }
}

// Per-device workspace of batched launches (grow-only).
struct BatchWork {
    DevBuf big, meta;
    DevBuf x0;  // warm start of a handed-off graph
    void* pin = nullptr;
    size_t pin_bytes = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int cus = 0;
    int grid_f = 0, grid_d = 0;  // resident workgroups of the float / double launch
    int wall_khz = 0;
};
std::mutex g_bw_mu;
BatchWork g_bw[64];

}  // namespace

void batched_release_workspaces() {
    std::lock_guard<std::mutex> lk(g_bw_mu);
    for (BatchWork& w : g_bw) {
        w.big.release();
        w.meta.release();
        w.x0.release();
        if (w.pin) (void)hipHostFree(w.pin);
        w.pin = nullptr;
        w.pin_bytes = 0;
        if (w.e0) (void)hipEventDestroy(w.e0);
        if (w.e1) (void)hipEventDestroy(w.e1);
        w.e0 = w.e1 = nullptr;
        w.cus = 0;  // the next launch re-creates the events
    }
}

namespace {

struct RunItem {
    sfairsc_graph* g;
    int k;
    Cfg cfg;
    double* H;  // device output (nullptr: workspace scratch)
};

struct RunOut {
    std::vector<GState> st;
    std::vector<double> theta;  // [count][KMAXB]
    std::vector<const double*> V;  // each graph's basis (valid until the next launch)
    std::vector<int> ld;
    uint64_t t_start = 0;
    double kernel_ms = 0.0;
    double tick_ms = 0.0;  // ms per wall-clock tick
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// One cooperative launch over the items (every workgroup resident at once).
// Synchronises `stream`.
int run_items(const std::vector<RunItem>& items, double tol, bool dbl, double sigma_override, int max_restarts,
              int certify, uint64_t seed, int handoff, hipStream_t stream, RunOut* ro) {
    int dev = 0;
    SF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(SFAIRSC_E_ARG, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_bw_mu);
    BatchWork& w = g_bw[dev];
    if (!w.cus) {
        hipDeviceProp_t prop;
        SF_HIP(hipGetDeviceProperties(&prop, dev));
        int coop = 0;
        SF_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        if (!coop) return set_error(SFAIRSC_E_HIP, "device %d has no cooperative launches", dev);
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        int occ_f = 0, occ_d = 0;
        SF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_f, reinterpret_cast<const void*>(&k_batched<float>),
                                                           NT, 0));
        SF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_d, reinterpret_cast<const void*>(&k_batched<double>),
                                                           NT, 0));
        if (occ_f < 1 || occ_d < 1) return set_error(SFAIRSC_E_HIP, "batched kernel cannot be resident on device %d", dev);
        w.grid_f = prop.multiProcessorCount * occ_f;
        w.grid_d = prop.multiProcessorCount * occ_d;
        w.wall_khz = khz;
        SF_HIP(hipEventCreate(&w.e0));
        SF_HIP(hipEventCreate(&w.e1));
        w.cus = prop.multiProcessorCount;
    }
    const int count = (int)items.size();
    // launch order: estimated cost per row, largest first, so that the
    // costliest items lead the item lists
    std::vector<double> cost(count);
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) {
        const sfairsc_graph* g = items[i].g;
        cost[i] = (double)items[i].cfg.b * ((double)g->nnz / (double)std::max<int64_t>(1, g->n) + 3.0 * items[i].cfg.ncv);
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    // workspace layout (by launch position)
    std::vector<size_t> offV(count), offX(count), offT(count), offH(count), offS(count);
    std::vector<int> item0(count), nit(count);
    size_t tot = 0;
    int nitems = 0;
    for (int i = 0; i < count; ++i) {
        const RunItem& it = items[order[i]];
        const int64_t n = it.g->n;
        const int ld = std::max(it.cfg.ncv + it.cfg.b, round_up(it.k, 16));
        offV[i] = tot;
        tot += align256((size_t)n * ld * 8);
        offX[i] = tot;
        tot += align256((size_t)n * 16 * 8);
        offT[i] = tot;
        tot += align256((size_t)n * 16 * 8);
        offH[i] = tot;
        if (!it.H) tot += align256((size_t)n * it.k * 8);
        offS[i] = tot;
        tot += align256((size_t)SMALL_DOUBLES * 8);
        item0[i] = nitems;
        nit[i] = (int)((n + IROWS - 1) / IROWS);
        nitems += nit[i];
    }
    const size_t offPart = tot;
    tot += align256((size_t)nitems * PSTRIDE * 8);
    SF_TRY(w.big.ensure(std::max<size_t>(tot, 256)));
    const size_t b_graphs = align256(sizeof(Graph) * count), b_items = align256(sizeof(Item) * nitems);
    const size_t b_st = align256(sizeof(GState) * count), b_theta = align256(sizeof(double) * KMAXB * count);
    const size_t b_list = align256(sizeof(int) * nitems);
    const size_t meta_bytes = b_graphs + b_items + b_st + b_theta + b_list + 256 + 256;
    SF_TRY(w.meta.ensure(meta_bytes));
    const size_t pin_need = std::max(b_graphs + b_items, b_st + b_theta + 256);
    if (w.pin_bytes < pin_need) {
        if (w.pin) (void)hipHostFree(w.pin);
        w.pin = nullptr;
        w.pin_bytes = 0;
        SF_HIP(hipHostMalloc(&w.pin, pin_need, 0));
        w.pin_bytes = pin_need;
    }
    char* base = w.big.as<char>();
    char* mb = w.meta.as<char>();
    Graph* d_graphs = reinterpret_cast<Graph*>(mb);
    Item* d_items = reinterpret_cast<Item*>(mb + b_graphs);
    GState* d_st = reinterpret_cast<GState*>(mb + b_graphs + b_items);
    double* d_theta = reinterpret_cast<double*>(mb + b_graphs + b_items + b_st);
    int* d_active = reinterpret_cast<int*>(mb + b_graphs + b_items + b_st + b_theta);
    uint64_t* d_tstart = reinterpret_cast<uint64_t*>(mb + b_graphs + b_items + b_st + b_theta + 256);
    int* d_alist = reinterpret_cast<int*>(mb + b_graphs + b_items + b_st + b_theta + 512);
    int* d_nalist = d_active + 1;

    // the upload goes through the pinned buffer (stream-ordered with the previous launch's download)
    SF_HIP(hipStreamSynchronize(stream));
    char* hp = static_cast<char*>(w.pin);
    Graph* h_graphs = reinterpret_cast<Graph*>(hp);
    Item* h_items = reinterpret_cast<Item*>(hp + b_graphs);
    std::vector<const double*> h_graphs_v(count);
    std::vector<int> h_graphs_ld(count);
    for (int i = 0; i < count; ++i) {
        const RunItem& it = items[order[i]];
        sfairsc_graph* g = it.g;
        Graph t{};
        t.rowptr = g->rowptr;
        t.col = g->col;
        t.val32 = g->val32;
        t.val64 = g->val64;
        t.diag32 = g->diag32;
        t.diag64 = g->diag64;
        t.grp = g->grp;
        t.cs = g->cs;
        t.gpar = g->gpar;
        t.V = reinterpret_cast<double*>(base + offV[i]);
        t.xp = base + offX[i];
        t.tt = base + offT[i];
        t.H = it.H ? it.H : reinterpret_cast<double*>(base + offH[i]);
        t.theta = d_theta + (size_t)i * KMAXB;
        t.sm = reinterpret_cast<double*>(base + offS[i]);
        t.n = g->n;
        t.h = g->h;
        t.k = it.k;
        t.b = it.cfg.b;
        t.ncv = it.cfg.ncv;
        t.ld = std::max(it.cfg.ncv + it.cfg.b, round_up(it.k, 16));
        t.rows = std::min(it.cfg.rows, max_rows(it.cfg.b, dbl));
        t.max_restarts = max_restarts;
        t.certify = certify;
        t.item0 = item0[i];
        t.nitems = nit[i];
        t.sigma = sigma_override > 0 ? sigma_override : g->sigma;
        t.tol = tol;
        // float products: converge the Ritz residuals to half the tolerance
        // so that the FP64 certification (which sees the float rounding of
        // the operator) meets tol
        t.tol_conv = dbl ? tol : std::max(0.5 * tol, kFloatTolFloor);
        t.seed = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(order[i] + 1));
        h_graphs[i] = t;
        h_graphs_v[i] = t.V;
        h_graphs_ld[i] = t.ld;
        for (int j = 0; j < nit[i]; ++j) {
            Item itm{};
            itm.g = i;
            itm.row0 = (int64_t)j * IROWS;
            h_items[item0[i] + j] = itm;
        }
    }
    SF_HIP(hipMemcpyAsync(d_graphs, h_graphs, b_graphs + b_items, hipMemcpyHostToDevice, stream));
    k_set_i32<<<1, 64, 0, stream>>>(d_active, count);
    SF_HIP(hipGetLastError());
    Launch L{};
    L.graphs = d_graphs;
    L.st = d_st;
    L.items = d_items;
    L.part = reinterpret_cast<double*>(base + offPart);
    L.active = d_active;
    L.alist = d_alist;
    L.nalist = d_nalist;
    L.t_start = d_tstart;
#ifdef SF_BATCH_STEPLOG
    DevBuf slog;
    const char* slog_path = std::getenv("SFAIRSC_BATCH_STEPLOG");
    if (slog_path) {
        SF_TRY(slog.ensure(sizeof(uint64_t) * 2 * (size_t)((max_restarts + 2) * (NCVMAX / 4) + 4)));
        SF_HIP(hipMemsetAsync(slog.p, 0, slog.bytes, stream));
        L.steplog = slog.as<uint64_t>();
    }
#endif
    L.ng = count;
    L.nitems = nitems;
    L.max_steps = (max_restarts + 2) * (NCVMAX / 4) + 4;
    L.handoff = handoff;
    void* args[] = {&L};
    SF_HIP(hipEventRecord(w.e0, stream));
    if (dbl)
        SF_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batched<double>), dim3(w.grid_d), dim3(NT),
                                          args, 0, stream));
    else
        SF_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batched<float>), dim3(w.grid_f), dim3(NT),
                                          args, 0, stream));
    SF_HIP(hipEventRecord(w.e1, stream));
    // results back through the pinned buffer
    GState* h_st = reinterpret_cast<GState*>(hp);
    double* h_theta = reinterpret_cast<double*>(hp + b_st);
    uint64_t* h_t0 = reinterpret_cast<uint64_t*>(hp + b_st + b_theta);
    SF_HIP(hipMemcpyAsync(h_st, d_st, b_st + b_theta, hipMemcpyDeviceToHost, stream));
    SF_HIP(hipMemcpyAsync(h_t0, d_tstart, sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    SF_HIP(hipStreamSynchronize(stream));
    float ms = 0.0f;
    SF_HIP(hipEventElapsedTime(&ms, w.e0, w.e1));
    ro->kernel_ms = ms;
    ro->tick_ms = 1.0 / (double)w.wall_khz;
    ro->t_start = *h_t0;
#ifdef SF_BATCH_STEPLOG
    if (L.steplog) {
        std::vector<uint64_t> h(slog.bytes / 8);
        SF_HIP(hipMemcpy(h.data(), slog.p, slog.bytes, hipMemcpyDeviceToHost));
        FILE* f = std::fopen(slog_path, "w");
        if (f) {
            for (size_t i = 0; i + 1 < h.size() && h[i]; i += 2)
                std::fprintf(f, "%llu %llu %llu\n", (unsigned long long)(h[i] - *h_t0),
                             (unsigned long long)(h[i + 1] & 0xffffffffull), (unsigned long long)(h[i + 1] >> 32));
            std::fclose(f);
        }
        slog.release();
    }
#endif
    ro->st.resize(count);
    ro->theta.resize((size_t)KMAXB * count);
    ro->V.resize(count);
    ro->ld.resize(count);
    for (int i = 0; i < count; ++i) {
        ro->st[order[i]] = h_st[i];
        ro->V[order[i]] = h_graphs_v[i];
        ro->ld[order[i]] = h_graphs_ld[i];
        std::memcpy(ro->theta.data() + (size_t)order[i] * KMAXB, h_theta + (size_t)i * KMAXB, sizeof(double) * KMAXB);
    }
    return SFAIRSC_OK;
}

bool lookup_cfg(int64_t n, int64_t nnz, int k, bool dbl, int normalized, Cfg* out) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    maybe_load_env();
    auto it = g_table.find(key_of(n, nnz, k, dbl, normalized));
    if (it == g_table.end() || !cfg_valid(it->second.cfg, k)) return false;
    *out = it->second.cfg;
    return true;
}

// Minimal reader for the table format written by sfairsc_tuning_save: a
// JSON object with an "entries" array of flat objects of integer / real
// fields.
int load_table_file(const char* path, bool replace) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(SFAIRSC_E_ARG, "cannot open tuning file %s", path);
    std::string s;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
    std::fclose(f);
    const size_t ent = s.find("\"entries\"");
    if (ent == std::string::npos) return set_error(SFAIRSC_E_ARG, "tuning file %s has no entries", path);
    std::map<Key, Entry> tab;
    size_t pos = s.find('[', ent);
    if (pos == std::string::npos) return set_error(SFAIRSC_E_ARG, "tuning file %s: malformed entries", path);
    for (;;) {
        const size_t ob = s.find('{', pos);
        const size_t close = s.find(']', pos);
        if (ob == std::string::npos || (close != std::string::npos && close < ob)) break;
        const size_t cb = s.find('}', ob);
        if (cb == std::string::npos) return set_error(SFAIRSC_E_ARG, "tuning file %s: unterminated entry", path);
        const std::string obj = s.substr(ob + 1, cb - ob - 1);
        auto field = [&](const char* name, double* v) -> bool {
            const std::string pat = std::string("\"") + name + "\"";
            const size_t p = obj.find(pat);
            if (p == std::string::npos) return false;
            const size_t c = obj.find(':', p + pat.size());
            if (c == std::string::npos) return false;
            char* end = nullptr;
            const double x = std::strtod(obj.c_str() + c + 1, &end);
            if (end == obj.c_str() + c + 1) return false;
            *v = x;
            return true;
        };
        double nlog, deg, kb, prec, norm, bw, ncv, rows, ms = 0.0;
        if (!field("n_log2", &nlog) || !field("degree_bucket", &deg) || !field("k_bucket", &kb) ||
            !field("double_spmm", &prec) || !field("normalized", &norm) || !field("block_width", &bw) ||
            !field("max_basis", &ncv) || !field("spmm_rows", &rows))
            return set_error(SFAIRSC_E_ARG, "tuning file %s: entry missing a field", path);
        field("ms", &ms);
        // "double_spmm": 1 is the key's precision class 0
        const Key key{(int)nlog, (int)deg, (int)kb, (int)prec ? 0 : 1, (int)norm};
        Entry e;
        e.cfg.b = (int)bw;
        e.cfg.ncv = (int)ncv;
        e.cfg.rows = (int)rows;
        e.ms = ms;
        tab[key] = e;
        pos = cb + 1;
    }
    if (replace) g_table.clear();
    for (auto& kv : tab) g_table[kv.first] = kv.second;
    return SFAIRSC_OK;
}

std::vector<Cfg> stage1_candidates(int k, int64_t n, int64_t nnz, bool dbl) {
    std::vector<Cfg> out;
    const Cfg d = default_cfg(n, nnz, k, dbl);
    for (int b : {4, 8, 16}) {
        for (int extra : {0, 3, 5}) {
            Cfg c;
            c.b = b;
            c.ncv = extra ? std::min(NCVMAX / b * b, round_up(round_up(k, 4) + extra * b, b)) : default_ncv(k, b);
            // rows by the same degree rule as the default, for this b
            const double deg = (double)nnz / (double)std::max<int64_t>(1, n);
            const int lpr = std::max(1, b / (dbl ? 2 : 4));
            int slots = 1;
            while (slots * 2 <= std::max(1.0, deg / 2)) slots *= 2;
            c.rows = std::max(1, 64 / std::min(64, std::max(lpr, lpr * slots)));
            if (!cfg_valid(c, k)) continue;
            bool dup = false;
            for (auto& o : out) dup |= (o.b == c.b && o.ncv == c.ncv);
            if (!dup) out.push_back(c);
        }
    }
    if (out.empty() && cfg_valid(d, k)) out.push_back(d);
    return out;
}

}  // namespace
}  // namespace sfairsc

using namespace sfairsc;

static int check_batch_args(const sfairsc_graph_t* graphs, int32_t count, const int32_t* k, double tol,
                            int precision) {
    if (!graphs || !k) return set_error(SFAIRSC_E_ARG, "graphs and k must not be NULL");
    if (count < 1 || count > (1 << 20)) return set_error(SFAIRSC_E_ARG, "count %d outside [1, 2^20]", count);
    if (!(tol > 0.0) || !std::isfinite(tol)) return set_error(SFAIRSC_E_ARG, "tolerance must be positive and finite");
    if (precision != SFAIRSC_PREC_FP64 && precision != SFAIRSC_PREC_MIXED)
        return set_error(SFAIRSC_E_ARG, "unknown precision %d", precision);
    int dev = 0;
    SF_HIP(hipGetDevice(&dev));
    for (int i = 0; i < count; ++i) {
        if (!graphs[i]) return set_error(SFAIRSC_E_ARG, "graph %d is NULL", i);
        if (graphs[i]->device != dev)
            return set_error(SFAIRSC_E_ARG, "graph %d lives on device %d, current device is %d", i, graphs[i]->device,
                             dev);
        const int64_t kmax = std::min<int64_t>(kMaxK, free_dim(graphs[i]));
        if (k[i] < 1 || k[i] > kmax) return set_error(SFAIRSC_E_ARG, "k[%d] = %d outside [1, %lld]", i, k[i], (long long)kmax);
    }
    return SFAIRSC_OK;
}

extern "C" int sfairsc_eigs_batched(const sfairsc_graph_t* graphs, int32_t count, const int32_t* k, double tol,
                                    int precision, const sfairsc_eigs_opts* opts, double* const* eigvals,
                                    double* const* H, sfairsc_batch_info* infos, hipStream_t stream) {
    SF_TRY(check_batch_args(graphs, count, k, tol, precision));
    if (!eigvals || !H) return set_error(SFAIRSC_E_ARG, "eigvals and H must not be NULL");
    for (int i = 0; i < count; ++i)
        if (!eigvals[i] || !H[i]) return set_error(SFAIRSC_E_ARG, "eigvals[%d] or H[%d] is NULL", i, i);
    sfairsc_eigs_opts o;
    sfairsc_eigs_opts_init(&o);
    if (opts) o = *opts;
    if (o.block_width != 0 && o.block_width != 4 && o.block_width != 8 && o.block_width != 16)
        return set_error(SFAIRSC_E_ARG, "batched block width must be 0, 4, 8 or 16 (got %d)", o.block_width);
    if (o.max_basis < 0 || o.max_basis > NCVMAX)
        return set_error(SFAIRSC_E_ARG, "batched max_basis must be in [0, %d] (got %d)", NCVMAX, o.max_basis);
    if (o.x0) return set_error(SFAIRSC_E_ARG, "batched solves take no warm start");
    const bool dbl = precision == SFAIRSC_PREC_FP64 || tol < kFloatTolFloor;
    const int max_restarts = o.max_restarts > 0 ? o.max_restarts : 500;

    // per-graph configuration; graphs the launch cannot take go to sfairsc_eigs
    std::vector<RunItem> items;
    std::vector<int> item_of(count, -1);
    std::vector<Cfg> cfgs(count);
    std::vector<int> from_table(count, 0);
    for (int i = 0; i < count; ++i) {
        sfairsc_graph* g = graphs[i];
        Cfg c = default_cfg(g->n, g->nnz, k[i], dbl);
        if (o.block_width == 0 && o.max_basis == 0) {
            Cfg tc;
            if (lookup_cfg(g->n, g->nnz, k[i], dbl, g->normalized, &tc)) {
                c = tc;
                from_table[i] = 1;
            }
        } else {
            if (o.block_width) c.b = o.block_width;
            c.ncv = o.max_basis ? o.max_basis
                                : default_ncv(k[i], c.b);
            const Cfg d = default_cfg(g->n, g->nnz, k[i], dbl);
            c.rows = std::min(d.rows, max_rows(c.b, dbl));
        }
        c.rows = std::min(c.rows, max_rows(c.b, dbl));
        cfgs[i] = c;
        const int ld = std::max(c.ncv + c.b, round_up(k[i], 16));
        // a general constraint matrix has no group form: single-graph solver
        const bool ok = cfg_valid(c, k[i]) && k[i] <= KMAXB && g->n >= 2 * (int64_t)ld && !g->qbas && !g->memb;
        if (!ok) {
            if (o.block_width || o.max_basis) {
                if (!cfg_valid(c, k[i]) || k[i] > KMAXB)
                    return set_error(SFAIRSC_E_ARG,
                                     "graph %d: block width %d / basis %d cannot hold k = %d (need a multiple of the "
                                     "block width, <= %d, >= k + 1 + b)",
                                     i, c.b, c.ncv, k[i], NCVMAX);
            }
            continue;
        }
        item_of[i] = (int)items.size();
        items.push_back(RunItem{g, k[i], c, H[i]});
    }
    RunOut ro;
    if (!items.empty())
        SF_TRY(run_items(items, tol, dbl, o.sigma, max_restarts, o.certify ? 1 : 0, o.seed,
                         (int)items.size() >= kHandoffMinBatch ? kHandoffGraphs : 0, stream, &ro));

    int ret = SFAIRSC_OK;
    for (int i = 0; i < count; ++i) {
        sfairsc_batch_info inf{};
        inf.block_width = cfgs[i].b;
        inf.max_basis = cfgs[i].ncv;
        inf.spmm_rows = std::min(cfgs[i].rows, max_rows(cfgs[i].b, dbl));
        inf.from_table = from_table[i];
        inf.double_spmm = dbl ? 1 : 0;
        inf.batch_ms = ro.kernel_ms;
        const int it = item_of[i];
        bool need_single = it < 0;
        const double* warm = nullptr;  // hand-off: the launch's current Ritz vectors
        int warm_ld = 0;
        if (it >= 0) {
            const GState& s = ro.st[it];
            inf.batch_status = s.status;
            inf.restarts = s.restarts;
            inf.block_steps = s.steps;
            inf.converged = s.nconv;
            inf.max_rel_residual = s.maxres;
            inf.gap_ratio = s.gap;
            inf.sigma = o.sigma > 0 ? o.sigma : graphs[i]->sigma;
            inf.graph_ms = s.t_done >= ro.t_start ? (double)(s.t_done - ro.t_start) * ro.tick_ms : 0.0;
            for (int p = 0; p < 8; ++p) inf.phase_ms[p] = (double)s.ph[p] * ro.tick_ms;
            if (s.status == 0) {
                std::memcpy(eigvals[i], ro.theta.data() + (size_t)it * KMAXB, sizeof(double) * k[i]);
            } else {
                need_single = true;
                if (s.status == 5) {
                    warm = ro.V[it];
                    warm_ld = ro.ld[it];
                }
            }
        } else {
            inf.batch_status = -1;
        }
        if (need_single) {
            // solved by the single-graph GPU solver instead
            sfairsc_eigs_opts so;
            sfairsc_eigs_opts_init(&so);
            so.seed = o.seed;
            so.sigma = o.sigma;
            so.certify = o.certify;
            so.max_restarts = o.max_restarts;
            if (warm) {
                // the first min(k, 16) Ritz vectors, compacted to n x b0 row-major
                const int b0 = std::min(k[i], 16);
                const int64_t n = graphs[i]->n;
                int dev = 0;
                SF_HIP(hipGetDevice(&dev));
                DevBuf& xb = g_bw[dev].x0;
                SF_TRY(xb.ensure(sizeof(double) * (size_t)n * b0));
                SF_HIP(hipMemcpy2DAsync(xb.p, sizeof(double) * b0, warm, sizeof(double) * warm_ld, sizeof(double) * b0,
                                        n, hipMemcpyDeviceToDevice, stream));
                so.x0 = xb.as<double>();
                so.b0 = b0;
            }
            sfairsc_eigs_info si{};
            const int r = sfairsc_eigs(graphs[i], k[i], tol, precision, &so, eigvals[i], H[i], &si, stream);
            inf.path = 1;
            inf.restarts = si.restarts;
            inf.block_steps = si.block_steps;
            inf.converged = si.converged;
            inf.max_rel_residual = si.max_rel_residual;
            inf.gap_ratio = si.gap_ratio;
            inf.sigma = si.sigma;
            inf.status = r;
            if (r != SFAIRSC_OK && r != SFAIRSC_E_NOT_CONVERGED && r != SFAIRSC_E_DEGENERATE) {
                if (infos) infos[i] = inf;
                return r;
            }
            if (r == SFAIRSC_E_NOT_CONVERGED) ret = SFAIRSC_E_NOT_CONVERGED;
        }
        // a graph converged in the launch whose theta_k and theta_{k+1}
        // coincide to the tolerance: the k-dimensional subspace is not
        // determined (the single-graph solver sets this status itself)
        if (!need_single && inf.status == SFAIRSC_OK && inf.gap_ratio <= kDegenerateGap * tol)
            inf.status = SFAIRSC_E_DEGENERATE;
        if (inf.status == SFAIRSC_E_DEGENERATE && ret == SFAIRSC_OK) ret = SFAIRSC_E_DEGENERATE;
        if (infos) infos[i] = inf;
    }
    if (ret == SFAIRSC_E_NOT_CONVERGED) set_error(ret, "some graphs did not converge (see their status)");
    if (ret == SFAIRSC_E_DEGENERATE)
        set_error(ret, "some graphs have theta_k ~ theta_{k+1} to the tolerance (see their status)");
    return ret;
}

extern "C" int sfairsc_autotune(const sfairsc_graph_t* graphs, int32_t count, const int32_t* k, double tol,
                                int precision, int32_t per_bucket, hipStream_t stream) {
    SF_TRY(check_batch_args(graphs, count, k, tol, precision));
    if (per_bucket < 1 || per_bucket > 16) return set_error(SFAIRSC_E_ARG, "per_bucket %d outside [1, 16]", per_bucket);
    const bool dbl = precision == SFAIRSC_PREC_FP64 || tol < kFloatTolFloor;
    // representatives per bucket
    std::map<Key, std::vector<int>> reps;
    for (int i = 0; i < count; ++i) {
        sfairsc_graph* g = graphs[i];
        if (k[i] > KMAXB || g->qbas || g->memb) continue;
        auto& v = reps[key_of(g->n, g->nnz, k[i], dbl, g->normalized)];
        if ((int)v.size() < per_bucket) v.push_back(i);
    }
    struct Trial {
        Key key;
        Cfg cfg;
        std::vector<int> item_idx;
    };
    auto run_trials = [&](std::vector<Trial>& trials, std::vector<double>* score) -> int {
        std::vector<RunItem> items;
        for (auto& tr : trials) {
            for (int gi : reps[tr.key]) {
                const int ld = std::max(tr.cfg.ncv + tr.cfg.b, round_up(k[gi], 16));
                if (graphs[gi]->n < 2 * (int64_t)ld) continue;
                tr.item_idx.push_back((int)items.size());
                items.push_back(RunItem{graphs[gi], k[gi], tr.cfg, nullptr});
            }
        }
        score->assign(trials.size(), 1e300);
        if (items.empty()) return SFAIRSC_OK;
        RunOut ro;
        SF_TRY(run_items(items, tol, dbl, 0.0, 500, 1, 0, 0, stream, &ro));
        for (size_t t = 0; t < trials.size(); ++t) {
            double s = 0.0;
            bool ok = !trials[t].item_idx.empty();
            for (int ii : trials[t].item_idx) {
                const GState& st = ro.st[ii];
                if (st.status != 0) ok = false;
                // the graph's compute-unit time over all phases
                for (int p = 0; p < 8; ++p) s += (double)st.ph[p] * ro.tick_ms;
            }
            (*score)[t] = ok ? s : 1e300;
        }
        return SFAIRSC_OK;
    };
    // stage 1: block width and basis size
    std::vector<Trial> t1;
    for (auto& kv : reps) {
        const int gi = kv.second[0];
        const int kk = k[gi];
        for (const Cfg& c : stage1_candidates(kk, graphs[gi]->n, graphs[gi]->nnz, dbl)) {
            bool fits = true;
            for (int r : kv.second) fits &= cfg_valid(c, k[r]);
            if (fits) t1.push_back(Trial{kv.first, c, {}});
        }
    }
    std::vector<double> s1;
    SF_TRY(run_trials(t1, &s1));
    std::map<Key, std::pair<Cfg, double>> best;
    for (size_t t = 0; t < t1.size(); ++t) {
        auto it = best.find(t1[t].key);
        if (s1[t] < 1e299 && (it == best.end() || s1[t] < it->second.second)) best[t1[t].key] = {t1[t].cfg, s1[t]};
    }
    // stage 2: rows per wavefront in the sparse product
    std::vector<Trial> t2;
    for (auto& kv : best) {
        const Cfg c0 = kv.second.first;
        for (int rows = 1; rows <= max_rows(c0.b, dbl); rows *= 2) {
            if (rows == c0.rows) continue;
            Cfg c = c0;
            c.rows = rows;
            t2.push_back(Trial{kv.first, c, {}});
        }
    }
    std::vector<double> s2;
    SF_TRY(run_trials(t2, &s2));
    for (size_t t = 0; t < t2.size(); ++t) {
        auto& bsf = best[t2[t].key];
        if (s2[t] < bsf.second) bsf = {t2[t].cfg, s2[t]};
    }
    std::lock_guard<std::mutex> lk(g_tab_mu);
    maybe_load_env();
    for (auto& kv : best) {
        Entry e;
        e.cfg = kv.second.first;
        e.ms = kv.second.second / std::max<size_t>(1, reps[kv.first].size());
        g_table[kv.first] = e;
    }
    return SFAIRSC_OK;
}

extern "C" int sfairsc_tuning_save(const char* path) {
    if (!path) return set_error(SFAIRSC_E_ARG, "path must not be NULL");
    std::lock_guard<std::mutex> lk(g_tab_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(SFAIRSC_E_ARG, "cannot write %s", path);
    std::fprintf(f, "{\n  \"format\": \"sfairsc-tuning-1\",\n  \"entries\": [\n");
    size_t i = 0;
    for (auto& kv : g_table) {
        const Key& key = kv.first;
        const Entry& e = kv.second;
        std::fprintf(f,
                     "    {\"n_log2\": %d, \"degree_bucket\": %d, \"k_bucket\": %d, \"double_spmm\": %d, "
                     "\"normalized\": %d, \"block_width\": %d, \"max_basis\": %d, \"spmm_rows\": %d, \"ms\": %.6g}%s\n",
                     key.nlog, key.deg, key.kb, key.prec == 0 ? 1 : 0, key.norm, e.cfg.b, e.cfg.ncv, e.cfg.rows, e.ms,
                     ++i < g_table.size() ? "," : "");
    }
    std::fprintf(f, "  ]\n}\n");
    const bool bad = std::ferror(f) != 0;
    std::fclose(f);
    if (bad) return set_error(SFAIRSC_E_ARG, "error writing %s", path);
    return SFAIRSC_OK;
}

extern "C" int sfairsc_tuning_load(const char* path) {
    if (!path) return set_error(SFAIRSC_E_ARG, "path must not be NULL");
    std::lock_guard<std::mutex> lk(g_tab_mu);
    g_env_loaded = true;
    return load_table_file(path, true);
}

extern "C" int sfairsc_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    g_env_loaded = true;
    g_table.clear();
    return SFAIRSC_OK;
}

extern "C" int sfairsc_tuning_size(void) {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    maybe_load_env();
    return (int)g_table.size();
}

extern "C" int sfairsc_tuning_lookup(int64_t n, int64_t nnz, int32_t k, int precision, int normalized, double tol,
                                     int32_t* block_width, int32_t* max_basis, int32_t* spmm_rows) {
    if (n < 1 || nnz < 0 || k < 1 || !block_width || !max_basis || !spmm_rows)
        return set_error(SFAIRSC_E_ARG, "bad tuning lookup arguments");
    const bool dbl = precision == SFAIRSC_PREC_FP64 || tol < kFloatTolFloor;
    Cfg c = default_cfg(n, nnz, k, dbl);
    const bool hit = lookup_cfg(n, nnz, k, dbl, normalized, &c);
    *block_width = c.b;
    *max_basis = c.ncv;
    *spmm_rows = std::min(c.rows, max_rows(c.b, dbl));
    return hit ? 1 : 0;
}
