// Batched fair eigensolves: many independent graphs in one persistent launch.
//
// Every graph of a batch gets the whole method of the single-graph solver:
// the deflated operator L^sigma = P (L_n - sigma I) P + sigma I (eq. asigma)
// applied through the group-sum form of P (eq. mv-Pw, Section 3.4), a block
// Krylov-Schur (thick-restart Lanczos) iteration, classical Gram-Schmidt
// twice and Cholesky-QR twice on the FP64 matrix cores, a Rayleigh-Ritz
// step and the fair output H (Alg. 3 step 3, Proposition 3.3).
//
// Design.  One workgroup of 512 threads (8 wavefronts) owns one graph at a
// time and runs its entire state machine: the Krylov basis and the sparse
// product blocks live in HBM, while the projected matrix T_m, the
// Rayleigh-Ritz eigenvectors, the coefficient matrices and all reductions
// live in the workgroup's LDS (about 130 KB, so one workgroup per compute
// unit).  Workgroups take graphs from a device work queue (an atomic
// counter over a list sorted by estimated cost, largest first), so uneven
// sizes balance over the compute units.  The small symmetric eigenproblem is
// solved in LDS by cyclic Jacobi with a round-robin ordering (all m/2
// disjoint rotations of a round are applied together).  Every reduction has
// a fixed order: results are bitwise reproducible.
//
// The block width b, the basis size and the rows handled together by a
// wavefront in the sparse product are chosen per graph, by default from a
// tuning table filled by timed trials (sfairsc_autotune).
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

namespace sfairsc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int NT = 1024;                    // threads of a workgroup
constexpr int NW = NT / 64;                 // wavefronts
constexpr int BMAX = 16;                    // widest block
constexpr int NCVMAX = 80;                  // basis columns before a restart
constexpr int LDT = NCVMAX + 1;             // LDS row stride of T and Z
constexpr int RTMAX = (NCVMAX + 15) / 16;   // row tiles of a Gram product
constexpr int KCH = (NCVMAX + BMAX + 15) / 16;  // 16-column chunks of an update input
constexpr int HMAX = kMaxGroups;            // groups
constexpr int KMAXB = 48;                   // wanted pairs (3 column tiles)
constexpr int WPART = NW * 8 * 16;          // group-sum wave partials
constexpr int WTILES = 2048;                // offset of reduced tiles in W

// Per-graph descriptor (device).
struct Task {
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
    double* theta;       // output eigenvalues [k]
    int64_t n;
    int32_t h, k, b, ncv, ld, rows, max_restarts, certify;
    double sigma, tol;
    double tol_conv;  // Ritz residual target (below tol with float products)
    uint64_t seed;
};

struct TaskStat {
    int32_t status;  // 0 converged, 1 not converged, 2 breakdown, 3 certification failed, 4 bad shape
    int32_t restarts, block_steps, converged;
    double max_rel_residual;  // certified (FP64 operator) or estimated
    double est_residual;      // Krylov-Schur estimate at the last Rayleigh-Ritz
    double gap_ratio;
    uint64_t t_begin, t_end;  // wall clock ticks
    uint64_t phase[8];        // wall clock ticks per phase (see kPhaseNames)
};

struct Shared {
    double T[NCVMAX * LDT];  // projected matrix; Jacobi workspace; rotation matrix
    double W[NCVMAX * LDT];  // Ritz eigenvectors; coefficient matrices and reduced tiles; group-sum partials
    double gA[HMAX * 16], gS[HMAX * 16], gR[HMAX * 16], gZ[HMAX * 16];
    double R1[256], Ri[256], R2[256], Rc[256];
    double theta[NCVMAX], res[NCVMAX];
    double red[NW * 16];
    double jc[NCVMAX / 2], js[NCVMAX / 2];
    int jp[NCVMAX / 2], jq[NCVMAX / 2];
    int perm[NCVMAX];
    int iflag[4];
    int cur;
    uint64_t ph[8], tmark;
    Task task;  // the graph being solved
};
static_assert(sizeof(Shared) <= 150 * 1024, "LDS budget");
static_assert(sizeof(Task) % 4 == 0, "task copy");

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

// Sum of v over the workgroup (fixed order).
__device__ double wg_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Phases of a graph's solve timed by the workgroup's wall clock:
// 0 operator, 1 pass A, 2 pass B, 3 pass C, 4 pass D, 5 Rayleigh-Ritz,
// 6 restart rotation, 7 start block and output.
__device__ __forceinline__ void phase_mark(Shared& S, int idx) {
    if (threadIdx.x == 0) {
        const uint64_t now = wall_clock64();
        S.ph[idx] += now - S.tmark;
        S.tmark = now;
    }
}

// Add the wavefronts' register tiles (nt tiles of 16 x 16, MFMA D layout)
// into out[nt * 256] in wavefront order.
template <int NTL>
__device__ void sum_tiles(const d4 (&acc)[NTL], int nt, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < NW; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < NTL; ++t) {
                if (t < nt) {
                    double* p = out + ((size_t)t * 64 + lane) * 4;
                    if (w == 0) {
                        p[0] = acc[t][0];
                        p[1] = acc[t][1];
                        p[2] = acc[t][2];
                        p[3] = acc[t][3];
                    } else {
                        p[0] += acc[t][0];
                        p[1] += acc[t][1];
                        p[2] += acc[t][2];
                        p[3] += acc[t][3];
                    }
                }
            }
        }
        __syncthreads();
    }
}

// As sum_tiles for nt Gram tiles acc[0 .. nt) followed by the Syrk tile
// acc[NTL - 1], stored at out[nt * 256].
template <int NTL>
__device__ void sum_tiles_gs(const d4 (&acc)[NTL], int nt, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int w = 0; w < NW; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < NTL; ++t) {
                const bool last = t == NTL - 1;
                if (t < nt || last) {
                    double* p = out + ((size_t)(last ? nt : t) * 64 + lane) * 4;
                    if (w == 0) {
                        p[0] = acc[t][0];
                        p[1] = acc[t][1];
                        p[2] = acc[t][2];
                        p[3] = acc[t][3];
                    } else {
                        p[0] += acc[t][0];
                        p[1] += acc[t][1];
                        p[2] += acc[t][2];
                        p[3] += acc[t][3];
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Element (i, j) (j < 16) of a column of 16 x 16 tiles in MFMA D layout.
__device__ __forceinline__ double tile_el(const double* t, int i, int j) {
    return t[((size_t)(i >> 4) * 64 + j + 16 * (i & 3)) * 4 + ((i & 15) >> 2)];
}

// A[s][j] = sum over rows i of group s of c_i X[i][j], j < b (b in {4, 8, 16}).
template <class XT>
__device__ __noinline__ void group_sums(const XT* X, int64_t ldx, int64_t n, int b, int h, const int32_t* __restrict__ grp,
                           const double* __restrict__ cs, double* part, double* A) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & (b - 1), rl = lane >> ilog2(b), rpw = 64 / b;
    for (int g0 = 0; g0 < h; g0 += 8) {
        double acc[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) acc[s] = 0.0;
        const int64_t st = (int64_t)NW * rpw;
        int64_t i = (int64_t)wave * rpw + rl;
        for (; i + 3 * st < n; i += 4 * st) {
            int gi[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t r = i + u * st;
                gi[u] = grp[r] - g0;
                v[u] = (cs ? cs[r] : 1.0) * (double)X[r * ldx + col];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int s = 0; s < 8; ++s) acc[s] += (gi[u] == s) ? v[u] : 0.0;
        }
        for (; i < n; i += st) {
            const int gi = grp[i] - g0;
            const double v = (cs ? cs[i] : 1.0) * (double)X[i * ldx + col];
#pragma unroll
            for (int s = 0; s < 8; ++s) acc[s] += (gi == s) ? v : 0.0;
        }
        for (int off = b; off < 64; off <<= 1)
#pragma unroll
            for (int s = 0; s < 8; ++s) acc[s] += __shfl_xor(acc[s], off);
        if (rl == 0)
#pragma unroll
            for (int s = 0; s < 8; ++s) part[(wave * 8 + s) * 16 + col] = acc[s];
        __syncthreads();
        if (threadIdx.x < 128) {
            const int s = threadIdx.x >> 4, j = threadIdx.x & 15;
            if (j < b && g0 + s < h) {
                double t = 0.0;
                for (int w = 0; w < NW; ++w) t += part[(w * 8 + s) * 16 + j];
                A[(g0 + s) * 16 + j] = t;
            }
        }
        __syncthreads();
    }
}

// From the group sums A of a block Z: S = C^T Z (A_s - p_s sum_t A_t,
// s < h-1), optionally stored in Sout; then S -= sigma * Ssub; U = Ginv S;
// R_s = U_s - q (s < h-1), R_{h-1} = -q, q = sum_s p_s U_s, so that
// (C U)_i = c_i R_{g_i}.
__device__ __noinline__ void group_finalize(const double* A, int h, int b, const double* __restrict__ gpar, double* Sout,
                               const double* Ssub, double sigma, double* zs, double* R) {
    const int j = threadIdx.x;
    if (j < b) {
        const int m = h - 1;
        const double* p = gpar;
        const double* Ginv = gpar + h;
        double tot = 0.0;
        for (int s = 0; s < h; ++s) tot += A[s * 16 + j];
        for (int s = 0; s < m; ++s) {
            double z = A[s * 16 + j] - p[s] * tot;
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

// out_i = X_i - c_i R_{g_i} (columns j < b), out typed OT with row stride ldo.
template <class OT>
__device__ __noinline__ void proj_apply(const double* X, int64_t ldx, int64_t n, int b, const int32_t* __restrict__ grp,
                           const double* __restrict__ cs, const double* R, OT* out, int64_t ldo) {
    const int lb = ilog2(b);
    const int64_t tot = n * b;
    int64_t idx = threadIdx.x;
    for (; idx + 3 * NT < tot; idx += 4 * NT) {
        double x[4], c[4], r[4];
        int64_t ii[4];
        int jj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = idx + u * NT;
            ii[u] = e >> lb;
            jj[u] = (int)(e & (b - 1));
            x[u] = X[ii[u] * ldx + jj[u]];
            c[u] = cs ? cs[ii[u]] : 1.0;
            r[u] = R[grp[ii[u]] * 16 + jj[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) out[ii[u] * ldo + jj[u]] = (OT)(x[u] - c[u] * r[u]);
    }
    for (; idx < tot; idx += NT) {
        const int64_t i = idx >> lb;
        const int j = (int)(idx & (b - 1));
        const double c = cs ? cs[i] : 1.0;
        out[i * ldo + j] = (OT)(X[i * ldx + j] - c * R[grp[i] * 16 + j]);
    }
}

// T_i = diag_i X_i - sum_e val_e X_{col_e} (CSR rows; X, T compact n x b).
// A wavefront handles `rows` rows at once, 64 / rows lanes each; within a
// row, lanes split into nonzero slots of b / VEC lanes (one 16-byte vector).
template <class VT>
__device__ __noinline__ void spmm_rows(const Task& t, const VT* __restrict__ X, VT* __restrict__ T, int b, int rows) {
    using V = Vec16<VT>;
    constexpr int VEC = V::N;
    const VT* __restrict__ val = pick<VT>(t.val32, t.val64);
    const VT* __restrict__ diag = pick<VT>(t.diag32, t.diag64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int LPR = b / VEC;
    rows = min(rows, 64 / LPR);  // at least one nonzero slot per row
    const int G = 64 / rows;
    const int sub = lane / G, sl = lane - sub * G;
    const int NS = G / LPR;
    const int slot = sl / LPR, cl = sl - slot * LPR;
    const int64_t n = t.n;
    for (int64_t base = (int64_t)wave * rows; base < n; base += (int64_t)NW * rows) {
        const int64_t row = base + sub;
        VT acc[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] = VT(0);
        if (row < n) {
            const int e0 = t.rowptr[row], e1 = t.rowptr[row + 1];
            int e = e0 + slot;
            // four gathers in flight
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
        if (row < n && slot == 0) {
            const V xi = V::load(X + row * b + cl * VEC);
            const VT dg = diag[row];
            V o;
#pragma unroll
            for (int v = 0; v < VEC; ++v) o.v[v] = dg * xi.v[v] - acc[v];
            o.store(T + row * b + cl * VEC);
        }
    }
}

// Pass A: Y0 = T - C U2 (deflation) into V[:, cv : cv + b]; reduced tiles
// of V[:, 0:cv]^T Y0 into out.
template <class SpT>
__device__ __noinline__ void pass_a(const Task& t, double* V, int ld, int cv, int b, const SpT* __restrict__ T, const double* R2,
                       double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nrt = (cv + 15) >> 4;
    d4 acc[RTMAX];
#pragma unroll
    for (int r = 0; r < RTMAX; ++r) acc[r] = d4{0, 0, 0, 0};
    const int64_t n = t.n, ntile = (n + 15) >> 4;
    for (int64_t tile = wave; tile < ntile; tile += NW) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = tile * 16 + 4 * q + lk;
            const bool rv = row < n;
            double y = 0.0;
            if (rv && li < b) {
                const double c = t.cs ? t.cs[row] : 1.0;
                y = (double)T[row * b + li] - c * R2[t.grp[row] * 16 + li];
                V[row * ld + cv + li] = y;
            }
#pragma unroll
            for (int rt = 0; rt < RTMAX; ++rt) {
                if (rt < nrt) {
                    const int col = rt * 16 + li;
                    const double a = (rv && col < cv) ? V[row * ld + col] : 0.0;
                    acc[rt] = mfma16(a, y, acc[rt]);
                }
            }
        }
    }
    sum_tiles(acc, nrt, out);
}

// Ynew = V[:, coff : coff + kin] M (M: kin x 16 in LDS, columns >= b zero)
// into V[:, yoff : yoff + b], in place (each 16-row tile is read completely
// by its wavefront before it is written).  GRAM: reduced tiles of
// V[:, 0:cv]^T Ynew into out[0 : nrt * 256]; SYRK: Ynew^T Ynew into the
// tile after them.
template <bool GRAM, bool SYRK>
__device__ __noinline__ void pass_upd(int64_t n, double* V, int ld, int coff, int kin, int yoff, int b, int cv, const double* M,
                         double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nrt = GRAM ? (cv + 15) >> 4 : 0;
    constexpr int NG = (GRAM ? RTMAX : 0) + 1;  // Gram tiles, then the Syrk tile
    d4 acc[NG];
#pragma unroll
    for (int r = 0; r < NG; ++r) acc[r] = d4{0, 0, 0, 0};
    const int64_t ntile = (n + 15) >> 4;
    for (int64_t tile = wave; tile < ntile; tile += NW) {
        const int64_t row0 = tile * 16;
        d4 D = d4{0, 0, 0, 0};
        {
            const int64_t row = row0 + li;
            const bool rv = row < n;
            const double* src = V + row * ld + coff + 4 * lk;
            double4 x[KCH];
#pragma unroll
            for (int c = 0; c < KCH; ++c) {
                x[c] = make_double4(0, 0, 0, 0);
                if (rv && c * 16 + 4 * lk < kin) x[c] = *reinterpret_cast<const double4*>(src + c * 16);
            }
#pragma unroll
            for (int c = 0; c < KCH; ++c) {
                if (c * 16 < kin) {
                    const double xs[4] = {x[c].x, x[c].y, x[c].z, x[c].w};
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int kr = c * 16 + 4 * lk + s;
                        const double bm = kr < kin ? M[kr * 16 + li] : 0.0;
                        D = mfma16(xs[s], bm, D);
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
                const int64_t row = row0 + 4 * q + lk;
                const bool rv = row < n;
#pragma unroll
                for (int rt = 0; rt < RTMAX; ++rt) {
                    if (rt < nrt) {
                        const int col = rt * 16 + li;
                        const double a = (rv && col < cv) ? V[row * ld + col] : 0.0;
                        acc[rt] = mfma16(a, D[q], acc[rt]);
                    }
                }
            }
        }
        if (GRAM || SYRK)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[NG - 1] = mfma16(D[q], D[q], acc[NG - 1]);
    }
    if (GRAM || SYRK) sum_tiles_gs(acc, nrt, out);
}

// V[:, 0:p] = V[:, 0:m] Z (Z: m x p in LDS, row stride ldz) and, if nb > 0,
// V[:, p : p + nb] = V[:, src : src + nb]; in place (p + nb <= src or nb = 0,
// every tile read before it is written).
__device__ __noinline__ void rotate(int64_t n, double* V, int ld, int m, const double* Z, int ldz, int p, int src, int nb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nct = (p + 15) >> 4;
    const int64_t ntile = (n + 15) >> 4;
    for (int64_t tile = wave; tile < ntile; tile += NW) {
        const int64_t row0 = tile * 16;
        // the tile's input rows (lane (li, lk): row row0 + li, columns 16 c + 4 lk ..)
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
            nx[q] = (row < n && li < nb) ? V[row * ld + src + li] : 0.0;
        }
        // every input of the tile is in registers before its first store
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
                        const double bm = (kr < m && col < p) ? Z[kr * ldz + col] : 0.0;
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

// Load the b x b block of a reduced tile into wavefront 0 (padded with the
// identity to 16 x 16), factor it, store R (row-major 16 x 16) and R^{-1}.
// Returns false on every thread if a pivot is <= thresh.
template <int B>
__device__ bool chol_wave(const double* tile, int b, double thresh, double* R, double* Rinv) {
    const int j = threadIdx.x;
    double g[B], ri[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        double v = 0.0;
        if (j < B) v = (i < b && j < b) ? tile_el(tile, i, j) : (i == j ? 1.0 : 0.0);
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
// b x b block of a reduced tile, by wavefront 0.  Returns false on every
// thread if a pivot is <= thresh.
__device__ __noinline__ bool chol16(const double* tile, int b, double thresh, double* R, double* Rinv, Shared& S) {
    if (threadIdx.x < 64) {
        const bool ok = b <= 4   ? chol_wave<4>(tile, b, thresh, R, Rinv)
                        : b <= 8 ? chol_wave<8>(tile, b, thresh, R, Rinv)
                                 : chol_wave<16>(tile, b, thresh, R, Rinv);
        if (threadIdx.x == 0) S.iflag[0] = ok ? 1 : 0;
    }
    __syncthreads();
    const bool ok = S.iflag[0] != 0;
    __syncthreads();
    return ok;
}

// Cholesky-QR twice of the block V[:, c : c + b] in place.
__device__ __noinline__ bool cholqr2(int64_t n, double* V, int ld, int c, int b, double thresh, Shared& S) {
    double* M = S.W;
    double* out = S.W + WTILES;
    for (int e = threadIdx.x; e < 16 * 16; e += NT) M[e] = ((e >> 4) == (e & 15)) ? 1.0 : 0.0;
    __syncthreads();
    pass_upd<false, true>(n, V, ld, c, b, c, b, 0, M, out);
    if (!chol16(out, b, thresh, S.R1, S.Ri, S)) return false;
    for (int e = threadIdx.x; e < 16 * 16; e += NT) M[e] = S.Ri[e];
    __syncthreads();
    pass_upd<false, true>(n, V, ld, c, b, c, b, 0, M, out);
    if (!chol16(out, b, 0.25, S.R2, S.Ri, S)) return false;
    for (int e = threadIdx.x; e < 16 * 16; e += NT) M[e] = S.Ri[e];
    __syncthreads();
    pass_upd<false, false>(n, V, ld, c, b, c, b, 0, M, out);
    __syncthreads();
    return true;
}

// Eigen-decomposition of the symmetric m x m matrix A (LDS, stride lda) by
// cyclic Jacobi, round-robin ordering.  On return diag(A) holds the
// eigenvalues and Z (LDS, stride ldz) the eigenvectors as columns.
__device__ __noinline__ void jacobi(double* A, int lda, int m, double* Z, int ldz, Shared& S) {
    const int t = threadIdx.x;
    for (int idx = t; idx < m * m; idx += NT) {
        const int i = idx / m, j = idx - i * m;
        Z[i * ldz + j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int mm = m + (m & 1), np = mm / 2, rr = mm - 1;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int idx = t; idx < m * m; idx += NT) {
            const int i = idx / m, j = idx - i * m;
            const double v = A[i * lda + j];
            if (i != j)
                off += v * v;
            else
                dg += v * v;
        }
        off = wg_sum(off, S.red);
        dg = wg_sum(dg, S.red);
        if (!(off > 1e-30 * dg)) break;
        for (int r = 0; r < rr; ++r) {
            if (t < np) {
                int p, q;
                if (t == 0) {
                    p = r;
                    q = rr;
                } else {
                    p = (r + t) % rr;
                    q = (r - t + rr) % rr;
                }
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[p * lda + q];
                    if (apq != 0.0) {
                        const double th = (A[q * lda + q] - A[p * lda + p]) / (2.0 * apq);
                        const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                S.jp[t] = p;
                S.jq[t] = q;
                S.jc[t] = c;
                S.js[t] = s;
            }
            __syncthreads();
            for (int idx = t; idx < m * np; idx += NT) {
                const int i = idx / np, pr = idx - i * np;
                const double s = S.js[pr];
                if (s == 0.0) continue;
                const int p = S.jp[pr], q = S.jq[pr];
                const double c = S.jc[pr];
                double* a = A + i * lda;
                const double ap = a[p], aq = a[q];
                a[p] = c * ap - s * aq;
                a[q] = s * ap + c * aq;
                double* z = Z + i * ldz;
                const double zp = z[p], zq = z[q];
                z[p] = c * zp - s * zq;
                z[q] = s * zp + c * zq;
            }
            __syncthreads();
            for (int idx = t; idx < m * np; idx += NT) {
                const int j = idx / np, pr = idx - j * np;
                const double s = S.js[pr];
                if (s == 0.0) continue;
                const int p = S.jp[pr], q = S.jq[pr];
                const double c = S.jc[pr];
                const double ap = A[p * lda + j], aq = A[q * lda + j];
                A[p * lda + j] = c * ap - s * aq;
                A[q * lda + j] = s * ap + c * aq;
            }
            __syncthreads();
        }
    }
}

// Y = L^sigma X for the block X = V[:, c : c + bw] (bw in {4, 8, 16}):
// on return the sparse product sits in tt, its deflation table in S.gR
// (Y_i = T_i - c_i R_{g_i}) and C^T X in S.gS.
template <class VT>
__device__ __noinline__ void apply_operator(const Task& t, const double* X, int ld, int bw, int rows, Shared& S) {
    const int64_t n = t.n;
    VT* xp = static_cast<VT*>(t.xp);
    VT* tt = static_cast<VT*>(t.tt);
    group_sums(X, ld, n, bw, t.h, t.grp, t.cs, S.W, S.gA);
    group_finalize(S.gA, t.h, bw, t.gpar, S.gS, nullptr, 0.0, S.gZ, S.gR);
    proj_apply<VT>(X, ld, n, bw, t.grp, t.cs, S.gR, xp, bw);
    __syncthreads();
    spmm_rows<VT>(t, xp, tt, bw, rows);
    __syncthreads();
    group_sums(tt, bw, n, bw, t.h, t.grp, t.cs, S.W, S.gA);
    group_finalize(S.gA, t.h, bw, t.gpar, nullptr, S.gS, t.sigma, S.gZ, S.gR);
}

// Fair output: V[:, 0:k] already holds the Ritz vectors.  Project them onto
// null(C^T), certify (optional), fix signs, scale and write H.
__device__ __noinline__ void finish(const Task& t, TaskStat& st, double* V, int ld, Shared& S) {
    const int64_t n = t.n;
    const int k = t.k;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, rl = lane >> 4;
    double maxres = 0.0;
    for (int c0 = 0; c0 < k; c0 += 16) {
        double* X = V + c0;
        group_sums(X, ld, n, 16, t.h, t.grp, t.cs, S.W, S.gA);
        group_finalize(S.gA, t.h, 16, t.gpar, nullptr, nullptr, 0.0, S.gZ, S.gR);
        proj_apply<double>(X, ld, n, 16, t.grp, t.cs, S.gR, X, ld);
        __syncthreads();
        if (t.certify) {
            apply_operator<double>(t, X, ld, 16, 8, S);
            const double* T = static_cast<const double*>(t.tt);
            const double th = (c0 + col < k) ? S.theta[c0 + col] : 0.0;
            double acc = 0.0;
            for (int64_t i = (int64_t)wave * 4 + rl; i < n; i += NW * 4) {
                const double c = t.cs ? t.cs[i] : 1.0;
                const double y = T[i * 16 + col] - c * S.gR[t.grp[i] * 16 + col];
                const double r = y - th * X[i * ld + col];
                acc += r * r;
            }
            acc += __shfl_xor(acc, 16);
            acc += __shfl_xor(acc, 32);
            if (rl == 0) S.W[wave * 16 + col] = acc;
            __syncthreads();
            if (threadIdx.x < 16 && c0 + threadIdx.x < k) {
                double s2 = 0.0;
                for (int w = 0; w < NW; ++w) s2 += S.W[w * 16 + threadIdx.x];
                S.res[threadIdx.x] = sqrt(s2) / t.sigma;
            }
            __syncthreads();
            if (threadIdx.x == 0)
                for (int j = 0; j < 16 && c0 + j < k; ++j) maxres = fmax(maxres, S.res[j]);
        }
        // sign: the largest-magnitude entry of each column of H positive
        // (lowest row on ties)
        double best = -1.0;
        int64_t bi = 0;
        double bv = 0.0;
        for (int64_t i = (int64_t)wave * 4 + rl; i < n; i += NW * 4) {
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
        double* Wb = S.W;
        int64_t* Wi = reinterpret_cast<int64_t*>(S.W + NW * 16);
        double* Wv = S.W + 2 * NW * 16;
        if (rl == 0) {
            Wb[wave * 16 + col] = best;
            Wi[wave * 16 + col] = bi;
            Wv[wave * 16 + col] = bv;
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            double b0 = -1.0, v0 = 0.0;
            int64_t i0 = 0;
            for (int w = 0; w < NW; ++w) {
                const double ob = Wb[w * 16 + threadIdx.x];
                const int64_t oi = Wi[w * 16 + threadIdx.x];
                if (ob > b0 || (ob == b0 && oi < i0)) {
                    b0 = ob;
                    i0 = oi;
                    v0 = Wv[w * 16 + threadIdx.x];
                }
            }
            S.res[16 + threadIdx.x] = v0 < 0.0 ? -1.0 : 1.0;
        }
        __syncthreads();
        const int kc = min(16, k - c0);
        for (int64_t idx = threadIdx.x; idx < n * kc; idx += NT) {
            const int j = (int)(idx / n);
            const int64_t i = idx - (int64_t)j * n;
            const double c = t.cs ? t.cs[i] : 1.0;
            t.H[(int64_t)(c0 + j) * n + i] = S.res[16 + j] * c * X[i * ld + j];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && t.certify) st.max_rel_residual = maxres;
}

template <class SpT>
__device__ __noinline__ void solve(const Task& t, TaskStat* stp, Shared& S, uint64_t seed) {
    const int tid = threadIdx.x;
    const int64_t n = t.n;
    const int b = t.b, ld = t.ld, ncv = t.ncv, k = t.k;
    double* V = t.V;
    TaskStat st{};
    if (tid == 0) {
        st.t_begin = wall_clock64();
        S.tmark = st.t_begin;
        for (int i = 0; i < 8; ++i) S.ph[i] = 0;
    }
    const double thresh = (1e-10 * t.sigma) * (1e-10 * t.sigma);
    const double tolabs = t.tol_conv * t.sigma;
    int status = 0;
    int m = 0, restarts = 0, steps = 0, nconv = 0;

    if (!(b == 4 || b == 8 || b == 16) || ncv > NCVMAX || ncv % 4 != 0 || ld < ncv + b || ld % 4 != 0 ||
        k < 1 || k > KMAXB || k + b >= ncv || ld < ((k + 15) / 16) * 16 || t.h < 1 || t.h > HMAX || t.rows < 1 ||
        t.rows > 64 || (t.rows & (t.rows - 1)) != 0 || n < 2 * (int64_t)ld) {
        status = 4;
        goto done;
    }

    // random start block, projected onto null(C^T), orthonormalised
    for (int64_t idx = tid; idx < n * b; idx += NT) {
        const int64_t i = idx / b;
        const int j = (int)(idx - i * b);
        V[i * ld + j] = rnd_pm1(seed, (uint64_t)idx);
    }
    __syncthreads();
    group_sums(V, ld, n, b, t.h, t.grp, t.cs, S.W, S.gA);
    group_finalize(S.gA, t.h, b, t.gpar, nullptr, nullptr, 0.0, S.gZ, S.gR);
    proj_apply<double>(V, ld, n, b, t.grp, t.cs, S.gR, V, ld);
    __syncthreads();
    if (!cholqr2(n, V, ld, 0, b, 0.0, S)) {
        status = 2;
        goto done;
    }

    for (;;) {
        // expansions: basis [0, m), current block [m, m + b)
        phase_mark(S, 7);
        while (m + b <= ncv) {
            const int cv = m + b;
            apply_operator<SpT>(t, V + m, ld, b, t.rows, S);
            phase_mark(S, 0);
            double* out = S.W + WTILES;
            double* M = S.W;
            pass_a<SpT>(t, V, ld, cv, b, static_cast<const SpT*>(t.tt), S.gR, out);
            // H1 -> T column block, M1 = [-H1; I]
            for (int e = tid; e < (cv + b) * 16; e += NT) {
                const int q = e >> 4, j = e & 15;
                if (q < cv) {
                    const double hv = j < b ? tile_el(out, q, j) : 0.0;
                    M[e] = -hv;
                    if (j < b) {
                        S.T[q * LDT + m + j] = hv;
                        if (q < m) S.T[(m + j) * LDT + q] = hv;
                    }
                } else {
                    M[e] = (q - cv == j) ? 1.0 : 0.0;
                }
            }
            __syncthreads();
            phase_mark(S, 1);
            pass_upd<true, true>(n, V, ld, 0, cv + b, cv, b, cv, M, out);
            // T column block += H2, symmetrised diagonal block
            for (int e = tid; e < cv * b; e += NT) {
                const int q = e / b, j = e - q * b;
                const double hv = tile_el(out, q, j);
                S.T[q * LDT + m + j] += hv;
                if (q < m) S.T[(m + j) * LDT + q] += hv;
            }
            __syncthreads();
            for (int e = tid; e < b * b; e += NT) {
                const int i = e / b, j = e - i * b;
                if (j > i) {
                    const double a = S.T[(m + i) * LDT + m + j], c = S.T[(m + j) * LDT + m + i];
                    const double mv = 0.5 * (a + c);
                    S.T[(m + i) * LDT + m + j] = mv;
                    S.T[(m + j) * LDT + m + i] = mv;
                }
            }
            const int nrt = (cv + 15) >> 4;
            if (!chol16(out + (size_t)nrt * 256, b, thresh, S.R1, S.Ri, S)) {
                status = 2;
                goto done;
            }
            // M2 = [-H2 R1^{-1}; R1^{-1}]
            for (int e = tid; e < (cv + b) * 16; e += NT) {
                const int q = e >> 4, j = e & 15;
                double acc = 0.0;
                if (j < b) {
                    if (q < cv) {
                        for (int u = 0; u <= j; ++u) acc -= tile_el(out, q, u) * S.Ri[u * 16 + j];
                    } else {
                        acc = S.Ri[(q - cv) * 16 + j];
                    }
                }
                M[e] = acc;
            }
            __syncthreads();
            phase_mark(S, 2);
            pass_upd<false, true>(n, V, ld, 0, cv + b, cv, b, cv, M, out);
            if (!chol16(out, b, 0.25, S.R2, S.Ri, S)) {
                status = 2;
                goto done;
            }
            // Rc = R2 R1; M3 = R2^{-1}
            for (int e = tid; e < 256; e += NT) {
                const int i = e >> 4, j = e & 15;
                double acc = 0.0;
                for (int u = i; u <= j; ++u) acc += S.R2[i * 16 + u] * S.R1[u * 16 + j];
                S.Rc[e] = acc;
                M[e] = S.Ri[e];
            }
            __syncthreads();
            phase_mark(S, 3);
            pass_upd<false, false>(n, V, ld, cv, b, cv, b, 0, M, out);
            __syncthreads();
            phase_mark(S, 4);
            m = cv;
            ++steps;
        }

        // Rayleigh-Ritz on T[0:m, 0:m]
        jacobi(S.T, LDT, m, S.W, LDT, S);
        if (tid < m) S.perm[tid] = tid;
        __syncthreads();
        if (tid < m) {
            const double w = S.T[tid * LDT + tid];
            int rank = 0;
            for (int j = 0; j < m; ++j) {
                const double o = S.T[j * LDT + j];
                rank += (o < w || (o == w && j < tid)) ? 1 : 0;
            }
            S.perm[rank] = tid;
            S.theta[rank] = w;
        }
        if (tid == 0) {
            bool finite = true;
            for (int r = 0; r < m; ++r) finite &= isfinite(S.theta[r]);
            S.iflag[1] = finite ? 1 : 0;
        }
        __syncthreads();
        if (!S.iflag[1]) {
            status = 2;
            goto done;
        }
        // residual estimates ||Rc z_last|| of the Ritz pairs
        if (tid < m) {
            const int c = S.perm[tid];
            double s2 = 0.0;
            for (int i = 0; i < b; ++i) {
                double v = 0.0;
                for (int j = i; j < b; ++j) v += S.Rc[i * 16 + j] * S.W[(m - b + j) * LDT + c];
                s2 += v * v;
            }
            S.res[tid] = sqrt(s2);
        }
        __syncthreads();
        nconv = 0;
        double est = 0.0;
        for (int r = 0; r < k; ++r) {
            nconv += S.res[r] <= tolabs ? 1 : 0;
            est = fmax(est, S.res[r]);
        }
        phase_mark(S, 5);
        st.est_residual = est / t.sigma;
        st.gap_ratio = m > k ? (S.theta[k] - S.theta[k - 1]) / t.sigma : 0.0;
        if (nconv == k || restarts >= t.max_restarts) break;

        // thick restart: keep p Ritz vectors (a multiple of 4, k < p <= m - b)
        const int ptarget = max(k + 1, (m + k) / 2);
        const int nd = max(1, (m - ptarget) / b);
        const int p = m - nd * b;
        for (int e = tid; e < m * p; e += NT) {
            const int q = e / p, r = e - q * p;
            S.T[q * LDT + r] = S.W[q * LDT + S.perm[r]];
        }
        __syncthreads();
        rotate(n, V, ld, m, S.T, LDT, p, m, b);
        __syncthreads();
        for (int e = tid; e < p * p; e += NT) {
            const int i = e / p, j = e - i * p;
            S.T[i * LDT + j] = (i == j) ? S.theta[i] : 0.0;
        }
        __syncthreads();
        phase_mark(S, 6);
        m = p;
        ++restarts;
    }

    // Ritz vectors V[:, 0:k] = V[:, 0:m] Z[:, 0:k]
    for (int e = tid; e < m * k; e += NT) {
        const int q = e / k, r = e - q * k;
        S.T[q * LDT + r] = S.W[q * LDT + S.perm[r]];
    }
    __syncthreads();
    rotate(n, V, ld, m, S.T, LDT, k, 0, 0);
    __syncthreads();
    if (tid == 0) st.max_rel_residual = st.est_residual;
    finish(t, st, V, ld, S);
    for (int r = tid; r < k; r += NT) t.theta[r] = S.theta[r];
    if (nconv < k)
        status = 1;
    else if (t.certify && st.max_rel_residual > t.tol)
        status = 3;

done:
    __syncthreads();
    if (tid == 0) {
        st.status = status;
        st.restarts = restarts;
        st.block_steps = steps;
        st.converged = nconv;
        st.t_end = wall_clock64();
        S.ph[7] += st.t_end - S.tmark;
        for (int i = 0; i < 8; ++i) st.phase[i] = S.ph[i];
        *stp = st;
    }
    __syncthreads();
}

template <class SpT>
__global__ __launch_bounds__(NT) void k_batched(const Task* __restrict__ tasks, TaskStat* __restrict__ stats,
                                                const int* __restrict__ order, int count, int* queue,
                                                uint64_t seed) {
    __shared__ Shared S;
    for (;;) {
        if (threadIdx.x == 0) S.cur = atomicAdd(queue, 1);
        __syncthreads();
        const int qi = S.cur;
        __syncthreads();
        if (qi >= count) break;
        const int ti = order[qi];
        {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(tasks + ti);
            uint32_t* dst = reinterpret_cast<uint32_t*>(&S.task);
            for (int w = threadIdx.x; w < (int)(sizeof(Task) / 4); w += NT) dst[w] = src[w];
        }
        __syncthreads();
        solve<SpT>(S.task, stats + ti, S, seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(ti + 1)));
    }
}

__global__ void k_set_i32(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
// host side

constexpr double kFloatTolFloor = 5e-7;  // tolerances below: double products

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

Cfg default_cfg(int64_t n, int64_t nnz, int k, bool dbl) {
    Cfg c;
    c.b = k <= 4 ? 4 : (k <= 8 ? 8 : 16);
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
    void* pin = nullptr;
    size_t pin_bytes = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int cus = 0;
    int wall_khz = 0;
};
std::mutex g_bw_mu;
BatchWork g_bw[64];

struct RunItem {
    sfairsc_graph* g;
    int k;
    Cfg cfg;
    double* H;  // device output (nullptr: workspace scratch)
};

struct RunOut {
    std::vector<TaskStat> st;
    std::vector<double> theta;  // [count][KMAXB]
    double kernel_ms = 0.0;
    double tick_ms = 0.0;  // ms per wall-clock tick
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Launch one persistent kernel over the items (each on its own workgroup
// when count <= compute units).  Synchronises `stream`.
int run_items(const std::vector<RunItem>& items, double tol, bool dbl, double sigma_override, int max_restarts,
              int certify, uint64_t seed, hipStream_t stream, RunOut* ro) {
    int dev = 0;
    SF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(SFAIRSC_E_ARG, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_bw_mu);
    BatchWork& w = g_bw[dev];
    if (!w.cus) {
        hipDeviceProp_t prop;
        SF_HIP(hipGetDeviceProperties(&prop, dev));
        w.cus = prop.multiProcessorCount;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        w.wall_khz = khz;
        SF_HIP(hipEventCreate(&w.e0));
        SF_HIP(hipEventCreate(&w.e1));
    }
    const int count = (int)items.size();
    // workspace layout
    std::vector<size_t> offV(count), offX(count), offT(count), offH(count);
    size_t tot = 0;
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) {
        const RunItem& it = items[i];
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
        cost[i] = (double)it.g->nnz + 8.0 * (double)n * it.cfg.ncv;
    }
    SF_TRY(w.big.ensure(std::max<size_t>(tot, 256)));
    const size_t meta_bytes = align256(sizeof(Task) * count) + align256(sizeof(TaskStat) * count) +
                              align256(sizeof(double) * KMAXB * count) + align256(sizeof(int) * count) + 256;
    SF_TRY(w.meta.ensure(meta_bytes));
    if (w.pin_bytes < meta_bytes) {
        if (w.pin) (void)hipHostFree(w.pin);
        w.pin = nullptr;
        w.pin_bytes = 0;
        SF_HIP(hipHostMalloc(&w.pin, meta_bytes, 0));
        w.pin_bytes = meta_bytes;
    }
    char* base = w.big.as<char>();
    char* mb = w.meta.as<char>();
    Task* d_tasks = reinterpret_cast<Task*>(mb);
    TaskStat* d_stats = reinterpret_cast<TaskStat*>(mb + align256(sizeof(Task) * count));
    double* d_theta = reinterpret_cast<double*>(reinterpret_cast<char*>(d_stats) + align256(sizeof(TaskStat) * count));
    int* d_order = reinterpret_cast<int*>(reinterpret_cast<char*>(d_theta) + align256(sizeof(double) * KMAXB * count));
    int* d_queue = reinterpret_cast<int*>(reinterpret_cast<char*>(d_order) + align256(sizeof(int) * count));

    char* hp = static_cast<char*>(w.pin);
    Task* h_tasks = reinterpret_cast<Task*>(hp);
    int* h_order = reinterpret_cast<int*>(hp + ((char*)d_order - mb));
    for (int i = 0; i < count; ++i) {
        const RunItem& it = items[i];
        sfairsc_graph* g = it.g;
        Task t{};
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
        t.n = g->n;
        t.h = g->h;
        t.k = it.k;
        t.b = it.cfg.b;
        t.ncv = it.cfg.ncv;
        t.ld = std::max(it.cfg.ncv + it.cfg.b, round_up(it.k, 16));
        t.rows = std::min(it.cfg.rows, max_rows(it.cfg.b, dbl));
        t.max_restarts = max_restarts;
        t.certify = certify;
        t.sigma = sigma_override > 0 ? sigma_override : g->sigma;
        t.tol = tol;
        // float products: converge the Ritz residuals to half the tolerance
        // so that the FP64 certification (which sees the float rounding of
        // the operator) meets tol
        t.tol_conv = dbl ? tol : std::max(0.5 * tol, kFloatTolFloor);
        t.seed = seed;
        h_tasks[i] = t;
        h_order[i] = i;
    }
    std::stable_sort(h_order, h_order + count, [&](int a, int b) { return cost[a] > cost[b]; });
    SF_HIP(hipMemcpyAsync(d_tasks, h_tasks, sizeof(Task) * count, hipMemcpyHostToDevice, stream));
    SF_HIP(hipMemcpyAsync(d_order, h_order, sizeof(int) * count, hipMemcpyHostToDevice, stream));
    k_set_i32<<<1, 64, 0, stream>>>(d_queue, 0);
    const int grid = std::max(1, std::min(count, w.cus));
    SF_HIP(hipEventRecord(w.e0, stream));
    if (dbl)
        k_batched<double><<<grid, NT, 0, stream>>>(d_tasks, d_stats, d_order, count, d_queue, seed);
    else
        k_batched<float><<<grid, NT, 0, stream>>>(d_tasks, d_stats, d_order, count, d_queue, seed);
    SF_HIP(hipGetLastError());
    SF_HIP(hipEventRecord(w.e1, stream));
    // results back through the pinned buffer (the task table is no longer needed)
    TaskStat* h_stats = reinterpret_cast<TaskStat*>(hp);
    double* h_theta = reinterpret_cast<double*>(hp + align256(sizeof(TaskStat) * count));
    SF_HIP(hipStreamSynchronize(stream));
    SF_HIP(hipMemcpyAsync(h_stats, d_stats, sizeof(TaskStat) * count, hipMemcpyDeviceToHost, stream));
    SF_HIP(hipMemcpyAsync(h_theta, d_theta, sizeof(double) * KMAXB * count, hipMemcpyDeviceToHost, stream));
    SF_HIP(hipStreamSynchronize(stream));
    float ms = 0.0f;
    SF_HIP(hipEventElapsedTime(&ms, w.e0, w.e1));
    ro->kernel_ms = ms;
    ro->tick_ms = 1.0 / (double)w.wall_khz;
    ro->st.assign(h_stats, h_stats + count);
    ro->theta.assign(h_theta, h_theta + (size_t)KMAXB * count);
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
        const int64_t kmax = std::min<int64_t>(kMaxK, graphs[i]->n - graphs[i]->h + 1);
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
        const bool ok = cfg_valid(c, k[i]) && k[i] <= KMAXB && g->n >= 2 * (int64_t)ld;
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
        SF_TRY(run_items(items, tol, dbl, o.sigma, max_restarts, o.certify ? 1 : 0, o.seed, stream, &ro));

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
        if (it >= 0) {
            const TaskStat& s = ro.st[it];
            inf.batch_status = s.status;
            inf.restarts = s.restarts;
            inf.block_steps = s.block_steps;
            inf.converged = s.converged;
            inf.max_rel_residual = s.max_rel_residual;
            inf.gap_ratio = s.gap_ratio;
            inf.sigma = o.sigma > 0 ? o.sigma : graphs[i]->sigma;
            inf.graph_ms = (double)(s.t_end - s.t_begin) * ro.tick_ms;
            for (int p = 0; p < 8; ++p) inf.phase_ms[p] = (double)s.phase[p] * ro.tick_ms;
            if (s.status == 0)
                std::memcpy(eigvals[i], ro.theta.data() + (size_t)it * KMAXB, sizeof(double) * k[i]);
            else
                need_single = true;
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
            if (r != SFAIRSC_OK && r != SFAIRSC_E_NOT_CONVERGED) {
                if (infos) infos[i] = inf;
                return r;
            }
            if (r == SFAIRSC_E_NOT_CONVERGED) ret = SFAIRSC_E_NOT_CONVERGED;
        }
        if (infos) infos[i] = inf;
    }
    if (ret != SFAIRSC_OK) set_error(ret, "some graphs did not converge (see their status)");
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
        if (k[i] > KMAXB) continue;
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
        SF_TRY(run_items(items, tol, dbl, 0.0, 500, 1, 0, stream, &ro));
        for (size_t t = 0; t < trials.size(); ++t) {
            double s = 0.0;
            bool ok = !trials[t].item_idx.empty();
            for (int ii : trials[t].item_idx) {
                const TaskStat& st = ro.st[ii];
                if (st.status != 0) ok = false;
                s += (double)(st.t_end - st.t_begin) * ro.tick_ms;
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
