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
// validation kernels.  Error bits written with atomicOr into flags[0].
enum : int {
    kBadRowptr = 1,
    kBadCol = 2,
    kDiag = 4,
    kBadValue = 8,
    kAsym = 16,
    kBadGroup = 32,
};

__global__ void k_check_rowptr(const int32_t* __restrict__ rowptr, int64_t n, int64_t nnz,
                               int* flags) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        int32_t a = rowptr[i], b = rowptr[i + 1];
        bool bad = a > b || a < 0 || b > nnz;
        if (i == 0 && a != 0) bad = true;
        if (i == n - 1 && b != nnz) bad = true;
        if (bad) atomicOr(flags, kBadRowptr);
    }
}

__global__ void k_check_groups(const int32_t* __restrict__ grp, int64_t n, int h, int* flags,
                               unsigned long long* counts) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        int32_t s = grp[i];
        if (s < 0 || s >= h)
            atomicOr(flags, kBadGroup);
        else
            atomicAdd(&counts[s], 1ull);
    }
}

// Rows: column range, order, diagonal, values; degree by a sequential sum.
template <class VT>
__global__ void k_check_rows(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             const VT* __restrict__ val, int64_t n, int* flags,
                             double* __restrict__ deg) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        int32_t a = rowptr[i], b = rowptr[i + 1];
        double d = 0.0;
        int32_t prev = -1;
        int f = 0;
        for (int32_t e = a; e < b; ++e) {
            int32_t j = col[e];
            if (j < 0 || j >= n || j <= prev) f |= kBadCol;
            if (j == i) f |= kDiag;
            prev = j;
            double w = (double)val[e];
            if (!(w >= 0.0) || !isfinite(w)) f |= kBadValue;
            d += w;
        }
        deg[i] = d;
        if (f) atomicOr(flags, f);
    }
}

// Symmetry: every (i, j, w) has a bitwise-equal (j, i, w).
template <class VT>
__global__ void k_check_sym(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const VT* __restrict__ val, int64_t n, int* flags) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        int32_t a = rowptr[i], b = rowptr[i + 1];
        for (int32_t e = a; e < b; ++e) {
            int32_t j = col[e];
            int32_t lo = rowptr[j], hi = rowptr[j + 1] - 1;
            bool found = false;
            while (lo <= hi) {
                int32_t mid = (lo + hi) >> 1;
                int32_t c = col[mid];
                if (c == (int32_t)i) {
                    found = (val[mid] == val[e]);
                    break;
                }
                if (c < i)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            if (!found) {
                atomicOr(flags, kAsym);
                return;
            }
        }
    }
}

// Operator values.  Unnormalized: off-diagonal w, diagonal d.  Normalized:
// w-hat = w / sqrt(d_i d_j), diagonal 1, c_i = d_i^{-1/2}; rowsum = sum_j w-hat.
template <class VT>
__global__ void k_setup_values(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const VT* __restrict__ val, const double* __restrict__ deg, int64_t n,
                               int normalized, double* __restrict__ val64, float* __restrict__ val32,
                               double* __restrict__ diag64, float* __restrict__ diag32,
                               double* __restrict__ cs, double* __restrict__ rowsum) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        int32_t a = rowptr[i], b = rowptr[i + 1];
        double di = deg[i];
        double si = normalized ? 1.0 / sqrt(di) : 1.0;
        double rs = 0.0;
        for (int32_t e = a; e < b; ++e) {
            double w = (double)val[e];
            if (normalized) w = w * si * (1.0 / sqrt(deg[col[e]]));
            val64[e] = w;
            val32[e] = (float)w;
            rs += w;
        }
        double dg = normalized ? 1.0 : di;
        diag64[i] = dg;
        diag32[i] = (float)dg;
        if (normalized) cs[i] = si;
        rowsum[i] = rs;
    }
}

static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
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
    const size_t vsz = value_dtype == SFAIRSC_F32 ? 4 : 8;

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
    // the original values are kept in the val64 buffer's storage until
    // k_setup_values has read them: copy them into a temporary first
    void* wtmp = nullptr;
    SF_HIP(hipMalloc(&wtmp, nnz * vsz + 16));
    if (nnz) SF_HIP(hipMemcpyAsync(wtmp, values, nnz * vsz, hipMemcpyDeviceToDevice, s));

    int* dflags = nullptr;
    unsigned long long* dcounts = nullptr;
    double* rowsum = nullptr;
    struct Cleanup {
        void** ptrs[3];
        ~Cleanup() {
            for (auto p : ptrs)
                if (*p) (void)hipFree(*p);
        }
    } cleanup{{&wtmp, (void**)&dflags, (void**)&dcounts}};
    SF_HIP(hipMalloc(&dflags, 64));
    SF_HIP(hipMalloc(&dcounts, kMaxGroups * sizeof(unsigned long long)));
    SF_HIP(hipMemsetAsync(dflags, 0, 64, s));
    SF_HIP(hipMemsetAsync(dcounts, 0, kMaxGroups * sizeof(unsigned long long), s));

    const int gr = grid_for(n);
    k_check_rowptr<<<gr, 256, 0, s>>>(g->rowptr, n, nnz, dflags);
    k_check_groups<<<gr, 256, 0, s>>>(g->grp, n, h, dflags, dcounts);
    SF_HIP(hipGetLastError());
    int hflags = 0;
    SF_HIP(hipMemcpyAsync(&hflags, dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    if (hflags & kBadRowptr) return set_error(SFAIRSC_E_ARG, "malformed CSR row pointers");
    if (hflags & kBadGroup) return set_error(SFAIRSC_E_ARG, "group label outside [0, h)");

    if (value_dtype == SFAIRSC_F32)
        k_check_rows<float><<<gr, 256, 0, s>>>(g->rowptr, g->col, (const float*)wtmp, n, dflags, g->deg);
    else
        k_check_rows<double><<<gr, 256, 0, s>>>(g->rowptr, g->col, (const double*)wtmp, n, dflags, g->deg);
    SF_HIP(hipGetLastError());
    SF_HIP(hipMemcpyAsync(&hflags, dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    if (hflags & kBadCol) return set_error(SFAIRSC_E_ARG, "column index out of range or not strictly increasing");
    if (hflags & kDiag) return set_error(SFAIRSC_E_ARG, "stored diagonal entry (w_ii must be 0 and not stored)");
    if (hflags & kBadValue) return set_error(SFAIRSC_E_ARG, "negative or non-finite weight");

    if (value_dtype == SFAIRSC_F32)
        k_check_sym<float><<<gr, 256, 0, s>>>(g->rowptr, g->col, (const float*)wtmp, n, dflags);
    else
        k_check_sym<double><<<gr, 256, 0, s>>>(g->rowptr, g->col, (const double*)wtmp, n, dflags);
    SF_HIP(hipGetLastError());
    SF_HIP(hipMemcpyAsync(&hflags, dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<unsigned long long> cnt(kMaxGroups);
    SF_HIP(hipMemcpyAsync(cnt.data(), dcounts, kMaxGroups * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    std::vector<double> hdeg(n);
    SF_HIP(hipMemcpyAsync(hdeg.data(), g->deg, n * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<int32_t> hgrp(n);
    SF_HIP(hipMemcpyAsync(hgrp.data(), g->grp, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    if (hflags & kAsym) return set_error(SFAIRSC_E_ASYM, "W is not symmetric");
    for (int t = 0; t < h; ++t)
        if (cnt[t] == 0) return set_error(SFAIRSC_E_EMPTY_GROUP, "group %d is empty", t);
    double dmin = INFINITY, dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        dmin = std::min(dmin, hdeg[i]);
        dmax = std::max(dmax, hdeg[i]);
    }
    g->dmin = dmin;
    g->dmax = dmax;
    if (normalized && !(dmin > 0.0))
        return set_error(SFAIRSC_E_ISOLATED, "isolated vertex: the normalized variant needs d_i > 0");

    SF_HIP(hipMalloc(&rowsum, n * sizeof(double) + 16));
    struct Free1 {
        double** p;
        ~Free1() {
            if (*p) (void)hipFree(*p);
        }
    } free_rowsum{&rowsum};
    if (value_dtype == SFAIRSC_F32)
        k_setup_values<float><<<gr, 256, 0, s>>>(g->rowptr, g->col, (const float*)wtmp, g->deg, n, normalized,
                                                 g->val64, g->val32, g->diag64, g->diag32, g->cs, rowsum);
    else
        k_setup_values<double><<<gr, 256, 0, s>>>(g->rowptr, g->col, (const double*)wtmp, g->deg, n, normalized,
                                                  g->val64, g->val32, g->diag64, g->diag32, g->cs, rowsum);
    SF_HIP(hipGetLastError());
    std::vector<double> hrs(n);
    SF_HIP(hipMemcpyAsync(hrs.data(), rowsum, n * sizeof(double), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));

    // sigma = ||L_n||_1 = max_j sum_i |(L_n)_ij|; W symmetric with zero diagonal
    // gives 1 + max_j sum_i w-hat_ij (normalized) or 2 max_j d_j.
    double sig = 0.0;
    if (normalized) {
        double m = 0.0;
        for (int64_t i = 0; i < n; ++i) m = std::max(m, hrs[i]);
        sig = 1.0 + m;
    } else {
        sig = 2.0 * dmax;
    }
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
            for (int64_t i = 0; i < n; ++i) {
                double r = 1.0 / hdeg[i];
                e[hgrp[i]] += r;
                E += r;
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
