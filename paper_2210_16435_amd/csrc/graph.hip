// Graph set-up: validation, degrees, normalisation, the shift sigma and the
// closed form of C^T C (Alg. 3 steps 1-2; Lemma 2.1; Appendix B.3).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include <atomic>

#include "internal.h"

namespace sfairsc {

static thread_local std::string t_last_error;

int set_error(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return code;
}

int DevBuf::ensure(size_t need) {
    if (need <= bytes && p) return SFAIRSC_OK;
    if (p) {
        (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    if (need == 0) need = 256;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return set_error(SFAIRSC_E_NOMEM, "hipMalloc(%zu) failed: %s", need, hipGetErrorString(e));
    }
    bytes = need;
    return SFAIRSC_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

// ---------------------------------------------------------------------------
// Set-up kernels.  Pass 1 validates the CSR and forms the degrees, pass 2
// checks symmetry and writes the operator's values, pass 3 sums the group
// statistics.  Every block leaves one partial record (no atomics: thousands
// of blocks updating one address serialise) and a last kernel folds them into
// the small record the host reads once.  Each CSR row is handled by LPR lanes
// (a power of two from 8 to 64, from the mean degree), each lane taking
// kUnroll entries at a time so that their loads are in flight together; each
// per-row sum is a fixed shuffle tree, so degrees and values are
// reproducible.
enum : int {
    kBadRowptr = 1,
    kBadCol = 2,
    kDiag = 4,
    kBadValue = 8,
    kAsym = 16,
    kBadGroup = 32,
};

constexpr int kSetupThreads = 256;
constexpr int kSetupBlocksMax = 8192;  // passes 1 and 2
constexpr int kStatBlocksMax = 1024;   // pass 3
constexpr int kFoldThreads = 1024;
constexpr int kUnroll = 4;  // entries per lane whose loads are issued together

// One block's partial of pass 1 (flags, min and max degree) or pass 2 (flags,
// max row sum in hi, stored entries above the diagonal minus those below).
struct RowPart {
    int flags;
    int pad;
    double lo, hi;
    long long updown;
};

// What the host reads back.
struct SetupSums {
    int flags;
    int pad;
    double dmin, dmax, rsmax;
    long long updown;
    double cnt[kMaxGroups];   // |V_s|
    double esum[kMaxGroups];  // sum over V_s of 1/d_i
};

template <int LPR>
__device__ __forceinline__ double row_sum(double v) {
    for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LPR);
    return v;
}

// Block-wide OR, min, max and integer sum; NT threads.  The result is valid
// in thread 0.  Each of these is exact in any order.
template <int NT>
__device__ void block_reduce(int& f, double& lo, double& hi, long long& ud) {
    __shared__ int sf[NT / 64];
    __shared__ double slo[NT / 64], shi[NT / 64];
    __shared__ long long sud[NT / 64];
    for (int o = 32; o > 0; o >>= 1) {
        f |= __shfl_xor(f, o);
        lo = fmin(lo, __shfl_xor(lo, o));
        hi = fmax(hi, __shfl_xor(hi, o));
        ud += __shfl_xor(ud, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sf[w] = f;
        slo[w] = lo;
        shi[w] = hi;
        sud[w] = ud;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < NT / 64; ++t) {
            f |= sf[t];
            lo = fmin(lo, slo[t]);
            hi = fmax(hi, shi[t]);
            ud += sud[t];
        }
    }
}

__device__ __forceinline__ void write_part(RowPart* out, int f, double lo, double hi, long long ud) {
    block_reduce<kSetupThreads>(f, lo, hi, ud);
    if (threadIdx.x == 0) {
        RowPart r;
        r.flags = f;
        r.pad = 0;
        r.lo = lo;
        r.hi = hi;
        r.updown = ud;
        out[blockIdx.x] = r;
    }
}

// Pass 1: row pointers, column range and order, no stored diagonal, finite
// non-negative weights, group labels in [0, h); d_i = sum_j w_ij (Section
// 2.1).  Every access stays inside the arrays whatever the input holds: a
// row whose pointers are out of order or range is flagged and skipped.
template <class VT, int LPR>
__global__ __launch_bounds__(kSetupThreads) void k_check_rows(const int32_t* __restrict__ rowptr,
                                                              const int32_t* __restrict__ col,
                                                              const VT* __restrict__ val,
                                                              const int32_t* __restrict__ grp, int64_t n,
                                                              int64_t nnz, int h, double* __restrict__ deg,
                                                              RowPart* __restrict__ part) {
    const int lane = threadIdx.x & (LPR - 1);
    const int64_t stride = (int64_t)gridDim.x * (kSetupThreads / LPR);
    int f = 0;
    double lo = INFINITY, hi = 0.0;
    for (int64_t i = (blockIdx.x * (int64_t)kSetupThreads + threadIdx.x) / LPR; i < n; i += stride) {
        const int32_t a = rowptr[i], b = rowptr[i + 1];
        double d = 0.0;
        if (a < 0 || a > b || b > nnz || (i == 0 && a != 0) || (i == n - 1 && b != nnz)) {
            f |= kBadRowptr;
        } else {
            for (int64_t e0 = (int64_t)a + lane; e0 < b; e0 += kUnroll * LPR) {
                bool ok[kUnroll];
                int32_t j[kUnroll], jp[kUnroll];
                double w[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int64_t e = e0 + u * LPR;
                    ok[u] = e < b;
                    j[u] = 0;
                    jp[u] = INT32_MIN;
                    w[u] = 0.0;
                    if (ok[u]) {
                        j[u] = col[e];
                        if (e > a) jp[u] = col[e - 1];
                        w[u] = (double)val[e];
                    }
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    if (!ok[u]) continue;
                    if (j[u] < 0 || j[u] >= n || jp[u] >= j[u]) f |= kBadCol;
                    if (j[u] == i) f |= kDiag;
                    if (!(w[u] >= 0.0) || !isfinite(w[u])) f |= kBadValue;
                    d += w[u];
                }
            }
        }
        d = row_sum<LPR>(d);
        if (lane == 0) {
            deg[i] = d;
            const int32_t s = grp[i];
            if (s < 0 || s >= h) f |= kBadGroup;
            lo = fmin(lo, d);
            hi = fmax(hi, d);
        }
    }
    write_part(part, f, lo, hi, 0);
}

// Pass 2: symmetry and the operator's values.  Each stored (i, j, w) above
// the diagonal looks up (j, i) by binary search in row j and needs an equal
// weight; the stored entries above and below the diagonal must also be
// equally many.  Columns strictly increasing in a row make (i, j) -> (j, i)
// one-to-one from the entries above into those below, so with equal counts it
// is onto as well: W is symmetric, at half the lookups of checking every
// entry.  Unnormalized:
// off-diagonal w, diagonal d.  Normalized (Alg. 3 step 2): w / sqrt(d_i d_j),
// diagonal 1, c_i = d_i^{-1/2}; the row sums of the scaled weights give sigma.
// Safe on any input (pass 1's flags decide what is reported).
template <class VT, int LPR>
__global__ __launch_bounds__(kSetupThreads) void k_setup_values(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col, const VT* __restrict__ val,
    const double* __restrict__ deg, int64_t n, int64_t nnz, int normalized, double* __restrict__ val64,
    float* __restrict__ val32, double* __restrict__ diag64, float* __restrict__ diag32, double* __restrict__ cs,
    RowPart* __restrict__ part) {
    const int lane = threadIdx.x & (LPR - 1);
    const int64_t stride = (int64_t)gridDim.x * (kSetupThreads / LPR);
    int f = 0;
    double rsmax = 0.0;
    long long ud = 0;
    for (int64_t i = (blockIdx.x * (int64_t)kSetupThreads + threadIdx.x) / LPR; i < n; i += stride) {
        const int32_t a = rowptr[i], b = rowptr[i + 1];
        const bool rowok = a >= 0 && a <= b && b <= nnz;
        const double di = deg[i];
        const double si = normalized ? 1.0 / sqrt(di) : 1.0;
        double rs = 0.0;
        for (int64_t e0 = rowok ? (int64_t)a + lane : (int64_t)b; e0 < b; e0 += kUnroll * LPR) {
            bool ok[kUnroll], act[kUnroll];
            int32_t j[kUnroll];
            VT wv[kUnroll];
            int64_t lo[kUnroll], hi[kUnroll], hit[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t e = e0 + u * LPR;
                j[u] = e < b ? col[e] : -1;
                ok[u] = j[u] >= 0 && j[u] < n;
                wv[u] = ok[u] ? val[e] : VT(0);
            }
            // the searches of the entries above the diagonal, interleaved so
            // that their loads are in flight together; each probe stays in
            // [rowptr[j], rowptr[j+1]) and each step shrinks it or ends
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                act[u] = ok[u] && j[u] > i;
                lo[u] = 0;
                hi[u] = -1;
                hit[u] = -1;
                if (act[u]) {
                    ++ud;
                    lo[u] = rowptr[j[u]];
                    hi[u] = (int64_t)rowptr[j[u] + 1] - 1;
                } else if (ok[u] && j[u] < i) {
                    --ud;
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) act[u] = act[u] && lo[u] >= 0 && hi[u] < nnz && lo[u] <= hi[u];
            for (;;) {
                bool any = false;
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) any |= act[u];
                if (!any) break;
                int64_t mid[kUnroll];
                int32_t c[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    mid[u] = (lo[u] + hi[u]) >> 1;
                    c[u] = act[u] ? col[mid[u]] : 0;
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    if (!act[u]) continue;
                    if (c[u] == (int32_t)i) {
                        hit[u] = mid[u];
                        act[u] = false;
                    } else {
                        if (c[u] < (int32_t)i)
                            lo[u] = mid[u] + 1;
                        else
                            hi[u] = mid[u] - 1;
                        act[u] = lo[u] <= hi[u];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (!(ok[u] && j[u] > i)) continue;
                if (!(hit[u] >= 0 && val[hit[u]] == wv[u])) f |= kAsym;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (!ok[u]) continue;
                double w = (double)wv[u];
                if (normalized) w = w * si * (1.0 / sqrt(deg[j[u]]));
                const int64_t e = e0 + u * LPR;
                val64[e] = w;
                val32[e] = (float)w;
                rs += w;
            }
        }
        rs = row_sum<LPR>(rs);
        if (lane == 0) {
            const double dg = normalized ? 1.0 : di;
            diag64[i] = dg;
            diag32[i] = (float)dg;
            if (normalized) cs[i] = si;
            rsmax = fmax(rsmax, rs);
        }
    }
    write_part(part, f, INFINITY, rsmax, ud);
}

// Pass 3: per group the count |V_s| and e_s = sum over V_s of 1/d_i (the
// closed form of C^T C below needs both).  Each block sums a contiguous
// chunk, wavefront by wavefront, in a fixed order; one partial per block.
__global__ __launch_bounds__(kSetupThreads) void k_group_stats(const int32_t* __restrict__ grp,
                                                               const double* __restrict__ deg, int64_t n, int h,
                                                               int64_t chunk, double* __restrict__ part) {
    constexpr int NW = kSetupThreads / 64;
    __shared__ double acc[NW][2 * kMaxGroups];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int t = threadIdx.x; t < NW * 2 * kMaxGroups; t += kSetupThreads) (&acc[0][0])[t] = 0.0;
    __syncthreads();
    const int64_t r0 = blockIdx.x * chunk, r1 = r0 + chunk < n ? r0 + chunk : n;
    for (int64_t base = r0 + 64 * w; base < r1; base += kSetupThreads) {
        const int64_t i = base + lane;
        int s = -1;
        double r = 0.0;
        if (i < r1) {
            s = grp[i];
            const double d = deg[i];
            r = d > 0.0 ? 1.0 / d : 0.0;
        }
        for (int t = 0; t < h; ++t) {
            double c = s == t ? 1.0 : 0.0, e = s == t ? r : 0.0;
            for (int o = 32; o > 0; o >>= 1) {
                c += __shfl_xor(c, o);
                e += __shfl_xor(e, o);
            }
            if (lane == 0) {
                acc[w][t] += c;
                acc[w][kMaxGroups + t] += e;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kMaxGroups) {
        double v = 0.0;
        for (int t = 0; t < NW; ++t) v += acc[t][threadIdx.x];
        part[(int64_t)blockIdx.x * 2 * kMaxGroups + threadIdx.x] = v;
    }
}

// Folds the partials: order-free operations for passes 1 and 2; the group
// sums of pass 3 in a fixed order (16 slices of the blocks, each summed in
// block order with eight loads in flight, then the slices in order).
__global__ __launch_bounds__(kFoldThreads) void k_setup_fold(const RowPart* __restrict__ p1,
                                                             const RowPart* __restrict__ p2, int nrow,
                                                             const double* __restrict__ gpart, int nstat,
                                                             SetupSums* S) {
    int f = 0;
    double lo = INFINITY, hi = 0.0, rs = 0.0;
    long long ud = 0;
    for (int q = threadIdx.x; q < nrow; q += kFoldThreads) {
        const RowPart a = p1[q], b = p2[q];
        f |= a.flags | b.flags;
        lo = fmin(lo, a.lo);
        hi = fmax(hi, a.hi);
        rs = fmax(rs, b.hi);
        ud += b.updown;
    }
    block_reduce<kFoldThreads>(f, lo, hi, ud);
    __syncthreads();  // the reduction's shared arrays are used again
    int f2 = 0;
    double inf = INFINITY;
    long long zero = 0;
    block_reduce<kFoldThreads>(f2, inf, rs, zero);
    if (threadIdx.x == 0) {
        S->flags = f;
        S->pad = 0;
        S->dmin = lo;
        S->dmax = hi;
        S->rsmax = rs;
        S->updown = ud;
    }

    constexpr int NS = kFoldThreads / (2 * kMaxGroups);
    __shared__ double red[NS][2 * kMaxGroups];
    const int fld = threadIdx.x % (2 * kMaxGroups), q0 = threadIdx.x / (2 * kMaxGroups);
    double v = 0.0;
    int q = q0;
    for (; q + 7 * NS < nstat; q += 8 * NS) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = gpart[(int64_t)(q + u * NS) * 2 * kMaxGroups + fld];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += x[u];
    }
    for (; q < nstat; q += NS) v += gpart[(int64_t)q * 2 * kMaxGroups + fld];
    red[q0][fld] = v;
    __syncthreads();
    if (threadIdx.x < 2 * kMaxGroups) {
        double t = 0.0;
        for (int r = 0; r < NS; ++r) t += red[r][threadIdx.x];
        if (threadIdx.x < kMaxGroups)
            S->cnt[threadIdx.x] = t;
        else
            S->esum[threadIdx.x - kMaxGroups] = t;
    }
}

// Lanes per CSR row from the mean degree: about kUnroll entries per lane.
static int lanes_per_row(int64_t n, int64_t nnz) {
    const double m = (double)nnz / (double)n;
    return m >= 256 ? 64 : m >= 128 ? 32 : m >= 64 ? 16 : 8;
}

static int row_grid(int64_t n, int lpr) {
    int64_t g = (n * lpr + kSetupThreads - 1) / kSetupThreads;
    if (g > kSetupBlocksMax) g = kSetupBlocksMax;
    if (g < 1) g = 1;
    return (int)g;
}

template <class VT>
static void launch_setup_rows(const sfairsc_graph* g, const VT* val, int lpr, int gr, RowPart* p1, RowPart* p2,
                              hipStream_t s) {
#define SF_ROWS(L)                                                                                          \
    do {                                                                                                    \
        k_check_rows<VT, L><<<gr, kSetupThreads, 0, s>>>(g->rowptr, g->col, val, g->grp, g->n, g->nnz, g->h, \
                                                         g->deg, p1);                                       \
        k_setup_values<VT, L><<<gr, kSetupThreads, 0, s>>>(g->rowptr, g->col, val, g->deg, g->n, g->nnz,   \
                                                           g->normalized, g->val64, g->val32, g->diag64,    \
                                                           g->diag32, g->cs, p2);                           \
    } while (0)
    switch (lpr) {
        case 64: SF_ROWS(64); break;
        case 32: SF_ROWS(32); break;
        case 16: SF_ROWS(16); break;
        default: SF_ROWS(8); break;
    }
#undef SF_ROWS
}

// Cholesky-based inverse of a small SPD matrix (row-major m x m), host.
static bool spd_inverse(int m, const std::vector<double>& A, std::vector<double>& inv) {
    std::vector<double> Lf(m * m, 0.0);
    for (int j = 0; j < m; ++j) {
        double s = A[j * m + j];
        for (int t = 0; t < j; ++t) s -= Lf[j * m + t] * Lf[j * m + t];
        if (!(s > 0.0)) return false;
        double ljj = std::sqrt(s);
        Lf[j * m + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            double r = A[i * m + j];
            for (int t = 0; t < j; ++t) r -= Lf[i * m + t] * Lf[j * m + t];
            Lf[i * m + j] = r / ljj;
        }
    }
    inv.assign(m * m, 0.0);
    // columns of A^{-1}: solve L L^T x = e_c
    std::vector<double> y(m);
    for (int c = 0; c < m; ++c) {
        for (int i = 0; i < m; ++i) {
            double r = (i == c) ? 1.0 : 0.0;
            for (int t = 0; t < i; ++t) r -= Lf[i * m + t] * y[t];
            y[i] = r / Lf[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double r = y[i];
            for (int t = i + 1; t < m; ++t) r -= Lf[t * m + i] * inv[t * m + c];
            inv[i * m + c] = r / Lf[i * m + i];
        }
    }
    return true;
}

static std::atomic<int> g_live_graphs{0};

static void free_graph(sfairsc_graph* g) {
    if (!g) return;
    (void)hipFree(g->rowptr);
    (void)hipFree(g->col);
    (void)hipFree(g->grp);
    (void)hipFree(g->val64);
    (void)hipFree(g->val32);
    (void)hipFree(g->diag64);
    (void)hipFree(g->diag32);
    (void)hipFree(g->cs);
    (void)hipFree(g->deg);
    (void)hipFree(g->gpar);
    auto& o = g->op;
    o.part_in.release();
    o.part_out.release();
    o.small.release();
    o.xp.release();
    o.t.release();
    o.xpad.release();
    o.ypad.release();
    o.lc.release();
    o.ctlc.release();
    if (o.ev0) (void)hipEventDestroy(o.ev0);
    if (o.ev1) (void)hipEventDestroy(o.ev1);
    auto& w = g->eig;
    w.V.release();
    w.V2.release();
    w.T.release();
    w.part.release();
    w.small.release();
    w.Q.release();
    w.X.release();
    w.opart.release();
    w.osmall.release();
    w.rr.release();
    if (w.ev_fork) (void)hipEventDestroy(w.ev_fork);
    if (w.ev_join) (void)hipEventDestroy(w.ev_join);
    if (w.ev_wait) (void)hipEventDestroy(w.ev_wait);
    if (w.s2) (void)hipStreamDestroy(w.s2);
    if (w.pin) (void)hipHostFree(w.pin);
    w.pin = nullptr;
    auto& k = g->km;
    k.d2.release();
    k.cs.release();
    k.cent.release();
    k.lab.release();
    k.best.release();
    k.part.release();
    k.misc.release();
    g->gw.hrow.release();
    (void)hipFree(g->qbas);
    free_memb(g);
    g->cw.part.release();
    g->cw.small.release();
    g->cw.cbuf.release();
    delete g;
}

template <class T>
static int dmalloc(T** p, size_t count) {
    hipError_t e = hipMalloc((void**)p, count * sizeof(T) + 16);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(SFAIRSC_E_NOMEM, "hipMalloc(%zu) failed", count * sizeof(T));
    }
    return SFAIRSC_OK;
}

static int create_impl(sfairsc_graph* g, int64_t n, int64_t nnz, const int32_t* rowptr,
                       const int32_t* colidx, const void* values, int value_dtype,
                       const int32_t* group, int h, int normalized, hipStream_t s) {
    g->n = n;
    g->nnz = nnz;
    g->h = h;
    g->normalized = normalized;
    g->value_dtype = value_dtype;
    SF_HIP(hipGetDevice(&g->device));

    SF_TRY(dmalloc(&g->rowptr, n + 1));
    SF_TRY(dmalloc(&g->col, nnz));
    SF_TRY(dmalloc(&g->grp, n));
    SF_TRY(dmalloc(&g->val64, nnz));
    SF_TRY(dmalloc(&g->val32, nnz));
    SF_TRY(dmalloc(&g->diag64, n));
    SF_TRY(dmalloc(&g->diag32, n));
    SF_TRY(dmalloc(&g->deg, n));
    if (normalized) SF_TRY(dmalloc(&g->cs, n));
    SF_TRY(dmalloc(&g->gpar, (size_t)h + (size_t)h * h));

    SF_HIP(hipMemcpyAsync(g->rowptr, rowptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (nnz) SF_HIP(hipMemcpyAsync(g->col, colidx, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    SF_HIP(hipMemcpyAsync(g->grp, group, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    // the per-block partials of the three passes, then the folded record
    const int lpr = lanes_per_row(n, nnz);
    const int gr = row_grid(n, lpr);
    int nstat = (int)std::min<int64_t>(kStatBlocksMax, (n + 2047) / 2048);
    const int64_t chunk = (n + nstat - 1) / nstat;
    nstat = (int)((n + chunk - 1) / chunk);
    const size_t o_p2 = (size_t)gr * sizeof(RowPart), o_g = 2 * o_p2,
                 o_s = o_g + (size_t)nstat * 2 * kMaxGroups * sizeof(double);
    void* tmp = nullptr;
    SF_HIP(hipMalloc(&tmp, o_s + sizeof(SetupSums)));
    struct Free1 {
        void** p;
        ~Free1() {
            if (*p) (void)hipFree(*p);
        }
    } free_tmp{&tmp};
    RowPart* p1 = (RowPart*)tmp;
    RowPart* p2 = (RowPart*)((char*)tmp + o_p2);
    double* gpart = (double*)((char*)tmp + o_g);
    SetupSums* dS = (SetupSums*)((char*)tmp + o_s);

    if (value_dtype == SFAIRSC_F32)
        launch_setup_rows(g, (const float*)values, lpr, gr, p1, p2, s);
    else
        launch_setup_rows(g, (const double*)values, lpr, gr, p1, p2, s);
    k_group_stats<<<nstat, kSetupThreads, 0, s>>>(g->grp, g->deg, n, h, chunk, gpart);
    k_setup_fold<<<1, kFoldThreads, 0, s>>>(p1, p2, gr, gpart, nstat, dS);
    SF_HIP(hipGetLastError());
    SetupSums hs;
    SF_HIP(hipMemcpyAsync(&hs, dS, sizeof hs, hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    const int hflags = hs.flags;
    if (hflags & kBadRowptr) return set_error(SFAIRSC_E_ARG, "malformed CSR row pointers");
    if (hflags & kBadGroup) return set_error(SFAIRSC_E_ARG, "group label outside [0, h)");
    if (hflags & kBadCol) return set_error(SFAIRSC_E_ARG, "column index out of range or not strictly increasing");
    if (hflags & kDiag) return set_error(SFAIRSC_E_ARG, "stored diagonal entry (w_ii must be 0 and not stored)");
    if (hflags & kBadValue) return set_error(SFAIRSC_E_ARG, "negative or non-finite weight");
    if ((hflags & kAsym) || hs.updown != 0) return set_error(SFAIRSC_E_ASYM, "W is not symmetric");
    std::vector<unsigned long long> cnt(h);
    for (int t = 0; t < h; ++t) cnt[t] = (unsigned long long)hs.cnt[t];
    for (int t = 0; t < h; ++t)
        if (cnt[t] == 0) return set_error(SFAIRSC_E_EMPTY_GROUP, "group %d is empty", t);
    const double dmin = hs.dmin, dmax = hs.dmax;
    g->dmin = dmin;
    g->dmax = dmax;
    if (normalized && !(dmin > 0.0))
        return set_error(SFAIRSC_E_ISOLATED, "isolated vertex: the normalized variant needs d_i > 0");

    // sigma = ||L_n||_1 = max_j sum_i |(L_n)_ij|; W symmetric with zero diagonal
    // gives 1 + max_j sum_i w-hat_ij (normalized) or 2 max_j d_j.
    double sig = normalized ? 1.0 + hs.rsmax : 2.0 * dmax;
    if (!(sig > 0.0)) sig = 1.0;  // edgeless graph: any positive shift works
    g->sigma = sig;

    // group fractions and (C^T C)^{-1} over the first h-1 groups.
    g->count.assign(h, 0);
    g->p.assign(h, 0.0);
    for (int t = 0; t < h; ++t) {
        g->count[t] = (int64_t)cnt[t];
        g->p[t] = (double)cnt[t] / (double)n;
    }
    const int m = h - 1;
    g->ginv.clear();
    if (m > 0) {
        std::vector<double> G(m * m, 0.0);
        if (!normalized) {
            // F^T F = diag(|V_s|) - |V_s| |V_t| / n
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b)
                    G[a * m + b] = (a == b ? (double)cnt[a] : 0.0) - (double)cnt[a] * (double)cnt[b] / (double)n;
        } else {
            // C^T C = diag(e_s) - e p^T - p e^T + E p p^T, e_s = sum_{V_s} 1/d_i
            std::vector<double> e(h, 0.0);
            double E = 0.0;
            for (int t = 0; t < h; ++t) {
                e[t] = hs.esum[t];
                E += e[t];
            }
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b)
                    G[a * m + b] = (a == b ? e[a] : 0.0) - e[a] * g->p[b] - g->p[a] * e[b] + E * g->p[a] * g->p[b];
        }
        if (!spd_inverse(m, G, g->ginv))
            return set_error(SFAIRSC_E_ARG, "C^T C is singular (degenerate group structure)");
    }
    std::vector<double> gp(h + m * m, 0.0);
    for (int t = 0; t < h; ++t) gp[t] = g->p[t];
    for (int t = 0; t < m * m; ++t) gp[h + t] = g->ginv[t];
    SF_HIP(hipMemcpyAsync(g->gpar, gp.data(), gp.size() * sizeof(double), hipMemcpyHostToDevice, s));
    SF_TRY(op_prepare_lc(g, s));
    SF_HIP(hipStreamSynchronize(s));
    return SFAIRSC_OK;
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" int sfairsc_graph_create(sfairsc_graph_t* out, int64_t n, int64_t nnz, const int32_t* rowptr,
                                    const int32_t* colidx, const void* values, int value_dtype,
                                    const int32_t* group, int32_t h, int normalized, hipStream_t stream) {
    if (!out) return set_error(SFAIRSC_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || nnz < 0 || nnz > INT32_MAX || n > INT32_MAX - 1)
        return set_error(SFAIRSC_E_ARG, "bad sizes n=%lld nnz=%lld", (long long)n, (long long)nnz);
    if (h < 1 || h > kMaxGroups) return set_error(SFAIRSC_E_ARG, "h=%d outside [1, %d]", h, kMaxGroups);
    if (value_dtype != SFAIRSC_F32 && value_dtype != SFAIRSC_F64)
        return set_error(SFAIRSC_E_ARG, "unknown value dtype %d", value_dtype);
    if (!rowptr || !group || (nnz > 0 && (!colidx || !values)))
        return set_error(SFAIRSC_E_ARG, "NULL input pointer");
    if (normalized != 0 && normalized != 1) return set_error(SFAIRSC_E_ARG, "normalized must be 0 or 1");
    sfairsc_graph* g = new (std::nothrow) sfairsc_graph();
    if (!g) return set_error(SFAIRSC_E_NOMEM, "host allocation failed");
    int r = create_impl(g, n, nnz, rowptr, colidx, values, value_dtype, group, h, normalized, stream);
    if (r != SFAIRSC_OK) {
        (void)hipStreamSynchronize(stream);
        free_graph(g);
        return r;
    }
    g_live_graphs.fetch_add(1);
    *out = g;
    return SFAIRSC_OK;
}

extern "C" void sfairsc_graph_destroy(sfairsc_graph_t g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    free_graph(g);
    // The library's process-wide workspaces (batched launches) live while
    // any handle does: freed with the last one, so nothing of the library
    // is left for the runtime's own teardown at exit.
    if (g_live_graphs.fetch_sub(1) == 1) batched_release_workspaces();
}

extern "C" int sfairsc_graph_query(sfairsc_graph_t g, sfairsc_graph_stats* out) {
    if (!g || !out) return set_error(SFAIRSC_E_ARG, "NULL argument");
    out->n = g->n;
    out->nnz = g->nnz;
    out->h = g->h;
    out->normalized = g->normalized;
    out->value_dtype = g->value_dtype;
    out->constraint_rank = g->memb ? g->memb->m : g->qbas ? g->qrank : g->h - 1;
    out->sigma = g->sigma;
    out->min_degree = g->dmin;
    out->max_degree = g->dmax;
    return SFAIRSC_OK;
}

extern "C" const char* sfairsc_last_error(void) { return t_last_error.c_str(); }

extern "C" const char* sfairsc_version(void) { return "sfairsc 0.1 (gfx950)"; }
