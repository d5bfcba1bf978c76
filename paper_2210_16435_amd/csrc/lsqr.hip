// Inexact projection by LSQR for a sparse membership matrix with many
// columns (the inner-outer iteration of Section 3.4 (ii)).
//
// C = D^{-1/2} (G - 1 z^T) (normalized) or G - 1 z^T, G the n x m 0/1
// membership matrix (a vertex may belong to several groups, m up to
// kMaxMembers), z = G^T 1 / n (or 0 without centring).  P w = w - C x with
// x the least-squares solution of C x = w, computed by LSQR (Paige and
// Saunders' bidiagonalisation with Givens rotations), one solve per column
// of the block, all columns in one launch.  Products:
//   (C v)_i   = c_i ((G v)_i - z^T v)                  gather over i's groups
//   (C^T u)_t = sum_{i in V_t} c_i u_i - z_t sum_i c_i u_i
// The member lists V_t are cut into segments of at most kSegMembers
// vertices (short, so that a few large groups still spread over many
// wavefronts); one wavefront sums a segment and a group adds its segments in
// order, so every reduction has a fixed order.
//
// One cooperative launch runs a whole solve: three grid barriers per LSQR
// step (after the n-space update of u, after the segment sums, after the
// m-space update of v).  The sums of u's partials are reduced by workgroup 0
// while the grid computes the segment sums and published for the next
// barrier; those of v (and the final ones) are reduced by every workgroup
// itself, the grid being small.  Either way the order is fixed, so every
// workgroup holds bitwise the same scalars and leaves the loop at the same
// step (converged columns, or max_inner).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace cg = cooperative_groups;

namespace sfairsc {

constexpr int kLsThreads = 256;
constexpr int kLsWaves = kLsThreads / 64;
constexpr int kSegMembers = 128;
constexpr int kLsMaxGrid = 512;
#ifndef SF_LSQR_RPT
#define SF_LSQR_RPT 32
#endif
constexpr int kLsRowsPerThread = SF_LSQR_RPT;

enum { LS_IN = 0, LS_OUT = 1, LS_PROJ = 2 };

struct LsqrArgs {
    int64_t n;
    int m, b, BWc, BW;
    const void* W;  // input block, type TT, leading dimension ldw
    int ldw;
    void* out;  // LS_IN: compact stride BW (type OT); LS_OUT: double, ldo; LS_PROJ: W itself
    int ldo;
    double sigma;  // LS_OUT: Y = W - C (x - sigma x1)
    const int32_t* grow;
    const int32_t* gcol;
    const double* cs;
    const double* z;
    const int32_t* seg_start;
    const int32_t* seg_group;
    const int32_t* gseg;
    const int32_t* tcol;
    int nseg;
    double* u;       // n x 32
    double* v;       // m x 32 (raw, alpha v-hat)
    double* d;       // m x 32 search directions
    double* x;       // m x 32 solution
    double* x1;      // m x 32 solution of the last LS_IN solve
    double* zx1;     // [32] z^T x1
    double* segsum;  // nseg x 32
    // Per-workgroup partials, gridDim x 64 each.  n-space reductions use
    // part, m-space ones part2: a workgroup overwrites a buffer only after a
    // grid barrier that follows every other workgroup's read of it.
    double* part;
    double* part2;
    double* res;  // [2][64]: the reduced sums, written by workgroup 0
    double atol;
    int maxit;
    long long* stats;  // calls, steps, max steps, unconverged columns
    const int* skip;   // device flag: nonzero makes the launch a no-op
};

// Block partials of two per-column quantities (q0, q1 of column jc) into
// part[block][q * 32 + j]; the row slots of a wavefront are combined with
// shuffles, the wavefronts in LDS.
__device__ __forceinline__ void ls_block_partials(double q0, double q1, int BWc, int b, double* red,
                                                  double* part) {
    for (int off = BWc; off < 64; off <<= 1) {
        q0 += __shfl_xor(q0, off);
        q1 += __shfl_xor(q1, off);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane < BWc) {
        red[(w * 2 + 0) * 32 + lane] = q0;
        red[(w * 2 + 1) * 32 + lane] = q1;
    }
    __syncthreads();
    if ((int)threadIdx.x < 64) {
        const int q = threadIdx.x >> 5, j = threadIdx.x & 31;
        double s = 0.0;
        if (j < b)
            for (int ww = 0; ww < kLsWaves; ++ww) s += red[(ww * 2 + q) * 32 + j];
        part[(size_t)threadIdx.x * kLsMaxGrid + blockIdx.x] = s;  // [quantity][block]
    }
}

// Every workgroup: r0[j], r1[j] = sums over all workgroups.  Partials are
// stored [quantity][block] (row length kLsMaxGrid): each of the 64 outputs is
// summed by four threads, each over a contiguous quarter of the blocks read
// as 16-byte vectors into two accumulators, then combined in a fixed order,
// so every workgroup obtains bitwise the same values.  scratch: 256 doubles
// of LDS.
__device__ __forceinline__ void ls_grid_reduce(const double* part, int b, double* r0, double* r1,
                                               double* scratch) {
    const int e = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int G = gridDim.x;
    const int per = ((G + 7) / 8) * 2;  // blocks per quarter, even
    const int lo = min(G, sub * per), hi = min(G, lo + per);
    const double* p = part + (size_t)e * kLsMaxGrid;
    double s0 = 0.0, s1 = 0.0;
    int blk = lo;
    for (; blk + 1 < hi; blk += 2) {
        const double2 v = *reinterpret_cast<const double2*>(p + blk);
        s0 += v.x;
        s1 += v.y;
    }
    if (blk < hi) s0 += p[blk];
    scratch[threadIdx.x] = s0 + s1;
    __syncthreads();
    if ((int)threadIdx.x < 64) {
        const int q = e >> 5, j = e & 31;
        if (j < b) (q ? r1 : r0)[j] = ((scratch[e] + scratch[64 + e]) + scratch[128 + e]) + scratch[192 + e];
    }
    __syncthreads();
}

// Workgroup 0 reduces the partials into out[64] (the others go on); after
// the next grid barrier every workgroup reads them with ls_read.  Only one
// workgroup reads the G x 64 partials, instead of all G of them.
__device__ __forceinline__ void ls_reduce_by_first(const double* part, int b, double* out, double* r0, double* r1,
                                                   double* scratch) {
    if (blockIdx.x != 0) return;
    ls_grid_reduce(part, b, r0, r1, scratch);
    if ((int)threadIdx.x < b) {
        out[threadIdx.x] = r0[threadIdx.x];
        out[32 + threadIdx.x] = r1[threadIdx.x];
    }
}

__device__ __forceinline__ void ls_read(const double* in, int b, double* r0, double* r1) {
    if ((int)threadIdx.x < b) {
        r0[threadIdx.x] = in[threadIdx.x];
        r1[threadIdx.x] = in[32 + threadIdx.x];
    }
    __syncthreads();
}

template <class TT, class OT, int MODE>
__global__ __launch_bounds__(kLsThreads) void k_lsqr(LsqrArgs a) {
    // every workgroup reads the same flag before the first barrier
    if (a.skip && *a.skip) return;
    cg::grid_group grid = cg::this_grid();
    __shared__ double red[kLsWaves * 2 * 32];
    __shared__ double r0[32], r1[32];
    __shared__ double alpha[32], beta[32], su[32], zv[32], ccu[32];
    __shared__ double rhobar[32], phibar[32], anorm2[32], aphi[32], athe[32];
    __shared__ int live[32], pend[32], any_live;
    const int tid = threadIdx.x, lane = tid & 63;
    const int BWc = a.BWc, b = a.b;
    const int jc = tid & (BWc - 1);
    const int slot = tid / BWc;
    const int slots = kLsThreads / BWc;
    const int64_t rstride = (int64_t)gridDim.x * slots;
    const int64_t rfirst = (int64_t)blockIdx.x * slots + slot;
    const TT* W = static_cast<const TT*>(a.W);
    const int64_t n = a.n;
    const int m = a.m;

    // segment sums of c_i u_i (all waves of the grid, one segment each)
    auto seg_phase = [&]() {
        const int wid = blockIdx.x * kLsWaves + (tid >> 6);
        const int ms = lane / BWc, nms = 64 / BWc;
        for (int s = wid; s < a.nseg; s += gridDim.x * kLsWaves) {
            double acc = 0.0;
            if (jc < b) {
                const int e1 = a.seg_start[s + 1];
#pragma unroll 4
                for (int p = a.seg_start[s] + ms; p < e1; p += nms) {
                    const int64_t i = a.tcol[p];
                    acc += (a.cs ? a.cs[i] : 1.0) * a.u[i * 32 + jc];
                }
            }
            for (int off = BWc; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
            if (lane < BWc && jc < b) a.segsum[(size_t)s * 32 + jc] = acc;
        }
    };
    // v <- su (C^T u-raw) - coef v / alpha_old; partials ||v||^2, z^T v.
    // One wavefront per group: its segment sums spread over the lanes (64 /
    // BWc slots per column) and are combined by shuffles.
    auto group_phase = [&](bool first) {
        double q0 = 0.0, q1 = 0.0;
        const int wid = blockIdx.x * kLsWaves + (tid >> 6);
        const int ss = lane / BWc, nss = 64 / BWc;
        const bool col_live = jc < b && live[jc];
        for (int t = wid; t < m; t += gridDim.x * kLsWaves) {
            double acc = 0.0;
            if (col_live)
                for (int q = a.gseg[t] + ss; q < a.gseg[t + 1]; q += nss) acc += a.segsum[(size_t)q * 32 + jc];
            for (int off = BWc; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
            if (lane < BWc && col_live) {
                const double zt = a.z[t];
                double vn = su[jc] * (acc - zt * ccu[jc]);
                if (!first) vn -= (beta[jc] / alpha[jc]) * a.v[(int64_t)t * 32 + jc];
                a.v[(int64_t)t * 32 + jc] = vn;
                q0 += vn * vn;
                q1 += zt * vn;
            }
        }
        ls_block_partials(q0, q1, BWc, b, red, a.part2);
    };

    // ---- u = w, beta_1 = ||w||, sum_i c_i w_i
    {
        double q0 = 0.0, q1 = 0.0;
        if (jc < b)
            for (int64_t i = rfirst; i < n; i += rstride) {
                const double val = (double)W[i * a.ldw + jc];
                a.u[i * 32 + jc] = val;
                const double c = a.cs ? a.cs[i] : 1.0;
                q0 += val * val;
                q1 += c * val;
            }
        ls_block_partials(q0, q1, BWc, b, red, a.part);
    }
    grid.sync();
    ls_reduce_by_first(a.part, b, a.res, r0, r1, red);
    seg_phase();  // needs only u
    grid.sync();
    ls_read(a.res, b, r0, r1);
    if (tid < b) {
        beta[tid] = std::sqrt(r0[tid]);
        ccu[tid] = r1[tid];
        live[tid] = beta[tid] > 0.0;
        su[tid] = beta[tid] > 0.0 ? 1.0 / beta[tid] : 0.0;
        phibar[tid] = beta[tid];
        pend[tid] = 0;
    }
    __syncthreads();

    group_phase(true);
    grid.sync();
    ls_grid_reduce(a.part2, b, r0, r1, red);
    if (tid < b) {
        alpha[tid] = std::sqrt(r0[tid]);
        zv[tid] = r1[tid];
        if (!(alpha[tid] > 0.0)) live[tid] = 0;
        rhobar[tid] = alpha[tid];
        anorm2[tid] = alpha[tid] * alpha[tid];
    }
    __syncthreads();
    if (tid == 0) {
        int l = 0;
        for (int j = 0; j < b; ++j) l |= live[j];
        any_live = l;
    }
    __syncthreads();
    // x = 0, d = v-hat
    if (jc < b)
        for (int64_t t = rfirst; t < m; t += rstride) {
            a.x[t * 32 + jc] = 0.0;
            a.d[t * 32 + jc] = live[jc] ? a.v[t * 32 + jc] / alpha[jc] : 0.0;
        }

    int it = 0;
    while (any_live && it < a.maxit) {
        ++it;
        // pending solution/direction update of the last step, then
        // u <- C v-hat - alpha u-hat
        if (jc < b && pend[jc]) {
            const double ap = aphi[jc], at = athe[jc], al = alpha[jc];
            const bool lv = live[jc];
            for (int64_t t = rfirst; t < m; t += rstride) {
                const double dt = a.d[t * 32 + jc];
                a.x[t * 32 + jc] += ap * dt;
                if (lv) a.d[t * 32 + jc] = a.v[t * 32 + jc] / al - at * dt;
            }
        }
        {
            double q0 = 0.0, q1 = 0.0;
            if (jc < b && live[jc]) {
                const double al = alpha[jc], zvh = zv[jc], us = alpha[jc] * su[jc];
                for (int64_t i = rfirst; i < n; i += rstride) {
                    double s = 0.0;
                    for (int e = a.grow[i]; e < a.grow[i + 1]; ++e) s += a.v[(int64_t)a.gcol[e] * 32 + jc];
                    const double c = a.cs ? a.cs[i] : 1.0;
                    const double un = c * ((s - zvh) / al) - us * a.u[i * 32 + jc];
                    a.u[i * 32 + jc] = un;
                    q0 += un * un;
                    q1 += c * un;
                }
            }
            ls_block_partials(q0, q1, BWc, b, red, a.part);
        }
        grid.sync();
        ls_reduce_by_first(a.part, b, a.res, r0, r1, red);
        seg_phase();  // needs only u
        grid.sync();
        ls_read(a.res, b, r0, r1);
        if (tid < b) {
            pend[tid] = 0;
            if (live[tid]) {
                beta[tid] = std::sqrt(r0[tid]);
                ccu[tid] = r1[tid];
                su[tid] = beta[tid] > 0.0 ? 1.0 / beta[tid] : 0.0;
            }
        }
        __syncthreads();
        group_phase(false);
        grid.sync();
        ls_grid_reduce(a.part2, b, r0, r1, red);
        if (tid < b && live[tid]) {
            const double an = std::sqrt(r0[tid]), bn = beta[tid];
            const double rho = std::sqrt(rhobar[tid] * rhobar[tid] + bn * bn);
            const double c = rhobar[tid] / rho, s = bn / rho;
            const double theta = s * an;
            rhobar[tid] = -c * an;
            const double phi = c * phibar[tid];
            phibar[tid] = s * phibar[tid];
            anorm2[tid] += an * an + bn * bn;
            aphi[tid] = phi / rho;
            athe[tid] = theta / rho;
            pend[tid] = 1;
            const double test = phibar[tid] > 0.0 ? an * std::fabs(c) / std::sqrt(anorm2[tid]) : 0.0;
            alpha[tid] = an;
            zv[tid] = r1[tid];
            if (test <= a.atol || !(an > 0.0) || !(bn > 0.0)) live[tid] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            int l = 0;
            for (int j = 0; j < b; ++j) l |= live[j];
            any_live = l;
        }
        __syncthreads();
    }

    // last pending update of x, then z^T x
    {
        double q0 = 0.0;
        if (jc < b)
            for (int64_t t = rfirst; t < m; t += rstride) {
                double xv = a.x[t * 32 + jc];
                if (pend[jc]) {
                    xv += aphi[jc] * a.d[t * 32 + jc];
                    a.x[t * 32 + jc] = xv;
                }
                if (MODE == LS_OUT) xv -= a.sigma * a.x1[t * 32 + jc];
                if (MODE == LS_IN) a.x1[t * 32 + jc] = xv;
                q0 += a.z[t] * xv;
            }
        ls_block_partials(q0, 0.0, BWc, b, red, a.part);
    }
    grid.sync();
    ls_grid_reduce(a.part, b, r0, r1, red);
    if (MODE == LS_IN && blockIdx.x == 0 && tid < b) a.zx1[tid] = r0[tid];

    // output rows: W - C x (LS_OUT: x - sigma x1)
    for (int64_t i = rfirst; i < n; i += rstride) {
        double val = 0.0;
        if (jc < b) {
            double s = 0.0;
            for (int e = a.grow[i]; e < a.grow[i + 1]; ++e) {
                const int64_t t = a.gcol[e];
                double xt = a.x[t * 32 + jc];
                if (MODE == LS_OUT) xt -= a.sigma * a.x1[t * 32 + jc];
                s += xt;
            }
            const double c = a.cs ? a.cs[i] : 1.0;
            val = (double)W[i * a.ldw + jc] - c * (s - r0[jc]);
        }
        if (MODE == LS_IN) {
            OT* o = static_cast<OT*>(a.out);
            for (int jj = jc; jj < a.BW; jj += BWc) o[i * a.BW + jj] = (OT)(jj < b ? val : 0.0);
        } else if (jc < b) {
            static_cast<double*>(a.out)[i * a.ldo + jc] = val;
        }
    }
    if (blockIdx.x == 0 && tid == 0) {
        int left = 0;
        for (int j = 0; j < b; ++j) left += live[j];
        a.stats[0] += 1;
        a.stats[1] += it;
        if (it > a.stats[2]) a.stats[2] = it;
        a.stats[3] += left;
    }
}

// ---- host ---------------------------------------------------------------------

static int pow2_at_least(int b) {
    int p = 1;
    while (p < b) p <<= 1;
    return p;
}

template <class TT, class OT, int MODE>
static int launch_lsqr(sfairsc_graph* g, LsqrArgs& a, hipStream_t s) {
    // blocks per CU of this kernel, per device (calls on distinct handles
    // may come from several host threads)
    static std::map<int, int> occ_of_device;
    static std::mutex occ_mutex;
    int dev = 0;
    SF_HIP(hipGetDevice(&dev));
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(occ_mutex);
        auto it = occ_of_device.find(dev);
        if (it != occ_of_device.end()) per_cu = it->second;
    }
    if (per_cu == 0) {
        SF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_lsqr<TT, OT, MODE>),
                                                           kLsThreads, 0));
        if (per_cu < 1) return set_error(SFAIRSC_E_HIP, "LSQR kernel cannot be resident");
        std::lock_guard<std::mutex> lock(occ_mutex);
        occ_of_device[dev] = per_cu;
    }
    int cus = 0;
    SF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // every kernel variant is held to the smallest residency of the five
    const int resident = std::max(1, std::min(per_cu, 2) * cus);
    // A grid barrier costs more the more workgroups take part, and a solve
    // has four per step: few workgroups, each with about kLsRowsPerThread
    // rows per thread (wavefronts loop over the segments and groups).
    const int64_t want = (a.n * a.BWc + kLsRowsPerThread * kLsThreads - 1) / (kLsRowsPerThread * kLsThreads);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>({want, (int64_t)resident, (int64_t)kLsMaxGrid}));
    void* args[] = {&a};
    SF_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_lsqr<TT, OT, MODE>), dim3(grid), dim3(kLsThreads),
                                      args, 0, s));
    (void)g;
    return SFAIRSC_OK;
}

static void fill_args(sfairsc_graph* g, LsqrArgs& a, int b) {
    Memb& M = *g->memb;
    a.n = g->n;
    a.m = M.m;
    a.b = b;
    a.BWc = pow2_at_least(b);
    a.grow = M.grow;
    a.gcol = M.gcol;
    a.cs = g->normalized ? g->cs : nullptr;
    a.z = M.z;
    a.seg_start = M.seg_start;
    a.seg_group = M.seg_group;
    a.gseg = M.gseg;
    a.tcol = M.tcol;
    a.nseg = M.nseg;
    double* wk = M.work.as<double>();
    a.u = wk;
    a.v = a.u + (size_t)g->n * 32;
    a.d = a.v + (size_t)M.m * 32;
    a.x = a.d + (size_t)M.m * 32;
    a.x1 = a.x + (size_t)M.m * 32;
    a.zx1 = a.x1 + (size_t)M.m * 32;
    a.segsum = a.zx1 + 32;
    a.part = a.segsum + (size_t)M.nseg * 32;
    a.part2 = a.part + (size_t)kLsMaxGrid * 64;
    a.res = a.part2 + (size_t)kLsMaxGrid * 64;
    a.atol = M.inner_tol;
    a.maxit = M.max_inner;
    a.stats = M.stats;
    a.sigma = 0.0;
}

int lsqr_project_in(sfairsc_graph* g, const double* X, int ldx, int b, int BW, bool to_float, void* Xp,
                    hipStream_t s, const int* skip) {
    LsqrArgs a{};
    fill_args(g, a, b);
    a.skip = skip;
    a.W = X;
    a.ldw = ldx;
    a.out = Xp;
    a.BW = BW;
    if (to_float) return launch_lsqr<double, float, LS_IN>(g, a, s);
    return launch_lsqr<double, double, LS_IN>(g, a, s);
}

int lsqr_correct(sfairsc_graph* g, const void* T, bool t_float, int BW, int b, double sigma, double* Y, int ldy,
                 hipStream_t s, const int* skip) {
    LsqrArgs a{};
    fill_args(g, a, b);
    a.skip = skip;
    a.W = T;
    a.ldw = BW;
    a.out = Y;
    a.ldo = ldy;
    a.BW = BW;
    a.sigma = sigma;
    if (t_float) return launch_lsqr<float, double, LS_OUT>(g, a, s);
    return launch_lsqr<double, double, LS_OUT>(g, a, s);
}

int lsqr_project(sfairsc_graph* g, double* X, int ldx, int b, hipStream_t s) {
    LsqrArgs a{};
    fill_args(g, a, b);
    a.W = X;
    a.ldw = ldx;
    a.out = X;
    a.ldo = ldx;
    a.BW = b;
    return launch_lsqr<double, double, LS_PROJ>(g, a, s);
}

void free_memb(sfairsc_graph* g) {
    if (!g->memb) return;
    Memb& M = *g->memb;
    (void)hipFree(M.grow);
    (void)hipFree(M.gcol);
    (void)hipFree(M.z);
    (void)hipFree(M.seg_start);
    (void)hipFree(M.seg_group);
    (void)hipFree(M.gseg);
    (void)hipFree(M.tcol);
    (void)hipFree(M.stats);
    M.work.release();
    delete g->memb;
    g->memb = nullptr;
}

template <class T>
static int dev_copy(T** dst, const std::vector<T>& src, hipStream_t s) {
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    if (hipMalloc((void**)dst, bytes + 16) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return set_error(SFAIRSC_E_NOMEM, "hipMalloc(%zu) failed", bytes);
    }
    if (!src.empty()) SF_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return SFAIRSC_OK;
}

static int set_memb_impl(sfairsc_graph* g, int m, const int32_t* mrow, const int32_t* mcol, int center,
                         double inner_tol, int max_inner, hipStream_t s) {
    const int64_t n = g->n;
    std::vector<int32_t> row(n + 1);
    SF_HIP(hipStreamSynchronize(s));
    SF_HIP(hipMemcpy(row.data(), mrow, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (row[0] != 0) return set_error(SFAIRSC_E_ARG, "membership rowptr[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (row[i + 1] < row[i]) return set_error(SFAIRSC_E_ARG, "membership rowptr decreases at %lld", (long long)i);
    const int64_t nnz = row[n];
    if (nnz < 1) return set_error(SFAIRSC_E_ARG, "no memberships");
    std::vector<int32_t> col(nnz);
    SF_HIP(hipMemcpy(col.data(), mcol, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> cnt(m, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = row[i]; e < row[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= m) return set_error(SFAIRSC_E_ARG, "membership column %d outside [0, %d)", col[e], m);
            if (e > row[i] && col[e] <= col[e - 1])
                return set_error(SFAIRSC_E_ARG, "membership columns of vertex %lld not strictly increasing", (long long)i);
            ++cnt[col[e]];
        }
    // member lists by group, cut into segments
    std::vector<int32_t> start(m + 1, 0);
    for (int t = 0; t < m; ++t) start[t + 1] = start[t] + (int32_t)cnt[t];
    std::vector<int32_t> tcol(nnz), fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = row[i]; e < row[i + 1]; ++e) tcol[fill[col[e]]++] = (int32_t)i;
    std::vector<int32_t> seg_start, seg_group, gseg(m + 1);
    for (int t = 0; t < m; ++t) {
        gseg[t] = (int32_t)seg_group.size();
        for (int32_t p = start[t]; p < start[t + 1]; p += kSegMembers) {
            seg_start.push_back(p);
            seg_group.push_back(t);
        }
    }
    gseg[m] = (int32_t)seg_group.size();
    seg_start.push_back((int32_t)nnz);
    std::vector<double> z(m, 0.0);
    if (center)
        for (int t = 0; t < m; ++t) z[t] = (double)cnt[t] / (double)n;

    g->memb = new (std::nothrow) Memb();
    if (!g->memb) return set_error(SFAIRSC_E_NOMEM, "host allocation failed");
    Memb& M = *g->memb;
    M.m = m;
    M.nseg = (int)seg_group.size();
    M.inner_tol = inner_tol;
    M.max_inner = max_inner;
    SF_TRY(dev_copy(&M.grow, row, s));
    SF_TRY(dev_copy(&M.gcol, col, s));
    SF_TRY(dev_copy(&M.z, z, s));
    SF_TRY(dev_copy(&M.seg_start, seg_start, s));
    SF_TRY(dev_copy(&M.seg_group, seg_group, s));
    SF_TRY(dev_copy(&M.gseg, gseg, s));
    SF_TRY(dev_copy(&M.tcol, tcol, s));
    SF_TRY(dev_copy(&M.stats, std::vector<long long>(4, 0), s));
    const size_t work = (size_t)n * 32 + (size_t)m * 32 * 4 + 32 + (size_t)M.nseg * 32 + (size_t)kLsMaxGrid * 64 * 2 + 128;
    SF_TRY(M.work.ensure(work * sizeof(double)));
    SF_HIP(hipStreamSynchronize(s));
    return SFAIRSC_OK;
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" int sfairsc_graph_set_memberships(sfairsc_graph_t g, int32_t m, const int32_t* rowptr,
                                             const int32_t* colidx, int32_t center, double inner_tol,
                                             int32_t max_inner, hipStream_t stream) {
    if (!g || !rowptr || !colidx) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (m < 1 || m > kMaxMembers) return set_error(SFAIRSC_E_ARG, "m=%d outside [1, %d]", m, kMaxMembers);
    if (m >= g->n) return set_error(SFAIRSC_E_ARG, "m=%d leaves no free direction (n=%lld)", m, (long long)g->n);
    if (center != 0 && center != 1) return set_error(SFAIRSC_E_ARG, "center must be 0 or 1");
    if (inner_tol == 0.0) inner_tol = 1e-12;
    if (!(inner_tol >= 1e-15 && inner_tol < 1.0))
        return set_error(SFAIRSC_E_ARG, "inner_tol=%g outside [1e-15, 1)", inner_tol);
    if (max_inner == 0) max_inner = 200;
    if (max_inner < 1 || max_inner > 100000) return set_error(SFAIRSC_E_ARG, "max_inner=%d outside [1, 1e5]", max_inner);
    (void)hipStreamSynchronize(stream);
    free_memb(g);
    if (g->qbas) (void)hipFree(g->qbas);
    g->qbas = nullptr;
    g->qrank = g->qld = 0;
    const int st = set_memb_impl(g, m, rowptr, colidx, center, inner_tol, max_inner, stream);
    if (st != SFAIRSC_OK) {
        (void)hipStreamSynchronize(stream);
        free_memb(g);
    }
    return st;
}

extern "C" int sfairsc_lsqr_stats(sfairsc_graph_t g, int64_t* out, hipStream_t stream) {
    if (!g || !out) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (!g->memb) return set_error(SFAIRSC_E_ARG, "the handle has no membership constraint");
    long long h[4];
    SF_HIP(hipStreamSynchronize(stream));
    SF_HIP(hipMemcpy(h, g->memb->stats, sizeof h, hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) out[i] = h[i];
    return SFAIRSC_OK;
}
