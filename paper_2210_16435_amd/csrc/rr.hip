// Rayleigh-Ritz step of the block Krylov-Schur solver on the GPU, in FP64:
// the eigenvalues and the wanted eigenvectors of the symmetric projected
// matrix T_c (order c <= 192), which Alg. 3 step 3 needs at every restart of
// the Krylov eigensolver (the paper's eigs/ARPACK solves the same small
// problem on the CPU), plus the residual estimates of the Ritz pairs and the
// thick-restart selection.  One workgroup of 1024 threads (16 wavefronts),
// in four stages of textbook dense symmetric eigensolver methods (Golub and
// Van Loan, Matrix Computations, 4th ed., Sections 8.3-8.4; Wilkinson, The
// Algebraic Eigenvalue Problem, Chapter 5):
//
//  1. Householder reduction to tridiagonal form, T = Q Tri Q^T with
//     Q = H_0 H_1 ... H_{c-3}, H_j = I - tau_j v_j v_j^T.  The matrix stays in
//     registers, lanes holding rows and wavefronts holding columns (lane l,
//     wavefront w: rows l + 64 t, columns w + 16 q).  The product T v then
//     needs no cross-lane reduction: each thread sums its columns, the
//     sixteen wavefront partials meet in LDS.  Three workgroup barriers per
//     column; the wavefront that owns the next column builds its reflector
//     right after its own update.
//  2. the eigenvalues that the restart needs, by Sturm counts (signs of the
//     leading principal minors of Tri - x I, three-term recurrence with
//     power-of-two rescaling every four steps): four lanes per eigenvalue
//     split its interval in five until the interval holds it alone; then
//     one lane finishes with Laguerre's method on the characteristic
//     polynomial (value and two derivatives by the same recurrence), whose
//     steps never pass the eigenvalue.
//     Eigenvalues that multisection cannot separate from a neighbour are
//     bisected to a few ulps of ||T||.
//  3. eigenvectors of Tri for the m smallest eigenvalues by inverse
//     iteration, one lane per vector: Gaussian elimination with partial
//     pivoting of Tri - s I (tiny pivots replaced by eps ||T||) and solves
//     from a pseudo-random start, the factors kept in rows shared by the
//     lanes and read eight rows ahead.  Eigenvalues closer than the
//     clustering distance are solved three times and orthonormalised
//     together after each solve (modified Gram-Schmidt, one wavefront per
//     cluster), as in LAPACK's inverse iteration; the others twice.
//  4. back-transformation Z = Q Y, sixteen lanes per column, the reflectors
//     applied in reverse order from LDS (kept there from stage 1 up to order
//     96, else staged sixteen at a time).
//
// The matrix is first scaled by a power of two (max |T_ij| in [1/2, 1)).
// Every reduction has a fixed order, so results are bitwise reproducible.
#include <cfloat>
#include <cmath>

#include "internal.h"
#include "rr.h"

namespace sfairsc {
namespace {

constexpr int kRrT = 1024;
constexpr int kRrW = kRrT / 64;    // wavefronts
constexpr int kRrMax = kMaxBasis;  // largest order
constexpr int kRrLd = kRrMax;      // leading dimension of the per-vector scratch

// scratch layout (doubles)
constexpr size_t kOffHV = 0;                               // Householder vectors [j][kRrMax]
constexpr size_t kOffY = kOffHV + (size_t)kRrMax * kRrMax;  // iterates [row][kRrLd]
constexpr size_t kOffU1 = kOffY + (size_t)kRrMax * kRrLd;   // reciprocal pivots
constexpr size_t kOffU2 = kOffU1 + (size_t)kRrMax * kRrLd;  // first superdiagonal of U
constexpr size_t kOffU3 = kOffU2 + (size_t)kRrMax * kRrLd;  // second superdiagonal of U
constexpr size_t kOffL = kOffU3 + (size_t)kRrMax * kRrLd;   // multipliers
constexpr size_t kOffPV = kOffL + (size_t)kRrMax * kRrLd;   // 1: rows interchanged
constexpr size_t kOffZ = kOffPV + (size_t)kRrMax * kRrLd;   // Ritz vectors [row][kRrLd]
constexpr size_t kWork = kOffZ + (size_t)kRrMax * kRrLd;

// Lane permutation of a double by the data-parallel primitives (DPP).
template <int CTRL>
__device__ inline double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Uniform copy of lane l's value.
__device__ inline double rdl(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
// Sum over each row of 16 lanes, in every lane of the row: exchanges with
// lane ^ 1, lane ^ 2 (quad permutations), then the mirrored lane within 8
// and within 16.
__device__ inline double sum16(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return v;
}
__device__ inline double wsum(double v) {
    v = sum16(v);
    return (rdl(v, 0) + rdl(v, 16)) + (rdl(v, 32) + rdl(v, 48));
}
__device__ inline double wmin(double v) {
    v = fmin(v, dpp_d<0xB1>(v));
    v = fmin(v, dpp_d<0x4E>(v));
    v = fmin(v, dpp_d<0x141>(v));
    v = fmin(v, dpp_d<0x140>(v));
    return fmin(fmin(rdl(v, 0), rdl(v, 16)), fmin(rdl(v, 32), rdl(v, 48)));
}
__device__ inline double wmax(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    return fmax(fmax(rdl(v, 0), rdl(v, 16)), fmax(rdl(v, 32), rdl(v, 48)));
}

// Uniform(-1, 1) start entry (SplitMix64 output function of the counter).
__device__ inline double start_entry(int vec, int row) {
    uint64_t z = 0x9E3779B97F4A7C15ull * (uint64_t)(((uint64_t)vec << 32) + (uint64_t)row + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-52 - 1.0;
}

// One step of the leading-minor recurrence p_i = (d - x) p_{i-1} - e^2 p_{i-2}
// with its sign-change count (sign bits compared).  Every e^2 is at least
// 2^-600, so a zero minor is never followed by another; a zero then counts
// one sign change across the pair whichever sign it carries, which is the
// count of the usual rule (a zero takes the sign opposite to its
// predecessor) without a test on the critical path.
__device__ inline void sturm_step(double2 de, double x, double& p, double& pm, int& cnt) {
    const double pn = (de.x - x) * p - de.y * pm;
    cnt += (int)((unsigned)(__double2hiint(pn) ^ __double2hiint(p)) >> 31);
    pm = p;
    p = pn;
}

// The scale factor that brings max(|p|, |pm|) back into [2^-200, 2^200]
// (a power of two, exact); within four steps the minors grow by at most a
// factor 5^4.
__device__ inline double sturm_scale(double p, double pm) {
    const double a = fmax(fabs(p), fabs(pm));
    return a > 0x1p200 ? 0x1p-200 : (a < 0x1p-200 ? 0x1p200 : 1.0);
}

// Number of eigenvalues of the tridiagonal matrix below x; de[i] = {d_i,
// e_{i-1}^2} (de[0].y unused; readable up to index c + 3).  The next four
// rows are read while the current four are used.
__device__ int sturm_count(const double2* __restrict__ de, int c, double x) {
    double pm = 1.0, p = de[0].x - x;
    int cnt = (int)((unsigned)__double2hiint(p) >> 31);
    int i = 1;
    double2 n0 = de[1], n1 = de[2], n2 = de[3], n3 = de[4];
    for (; i + 3 < c; i += 4) {
        const double2 d0 = n0, d1 = n1, d2 = n2, d3 = n3;
        n0 = de[i + 4];
        n1 = de[i + 5];
        n2 = de[i + 6];
        n3 = de[i + 7];
        sturm_step(d0, x, p, pm, cnt);
        sturm_step(d1, x, p, pm, cnt);
        sturm_step(d2, x, p, pm, cnt);
        sturm_step(d3, x, p, pm, cnt);
        const double sc = sturm_scale(p, pm);
        p *= sc;
        pm *= sc;
    }
    for (; i < c; ++i) sturm_step(de[i], x, p, pm, cnt);
    return cnt;
}

// The same count plus the characteristic polynomial f = p_c and its first
// two derivatives (p'_i = (d - x) p'_{i-1} - p_{i-1} - e^2 p'_{i-2},
// p''_i = (d - x) p''_{i-1} - 2 p'_{i-1} - e^2 p''_{i-2}), all scaled by the
// same power of two.
__device__ inline void lag_step(double2 de, double x, double& p, double& pm, double& q, double& qm, double& r,
                                double& rm, int& cnt) {
    const double t = de.x - x;
    const double pn = t * p - de.y * pm;
    const double qn = t * q - p - de.y * qm;
    const double rn = t * r - 2.0 * q - de.y * rm;
    cnt += (int)((unsigned)(__double2hiint(pn) ^ __double2hiint(p)) >> 31);
    pm = p;
    p = pn;
    qm = q;
    q = qn;
    rm = r;
    r = rn;
}
__device__ int sturm_laguerre(const double2* __restrict__ de, int c, double x, double& f, double& f1, double& f2) {
    double pm = 1.0, p = de[0].x - x;
    double qm = 0.0, q = -1.0, rm = 0.0, r = 0.0;
    int cnt = (int)((unsigned)__double2hiint(p) >> 31);
    int i = 1;
    for (; i + 3 < c; i += 4) {
        const double2 d0 = de[i], d1 = de[i + 1], d2 = de[i + 2], d3 = de[i + 3];
        lag_step(d0, x, p, pm, q, qm, r, rm, cnt);
        lag_step(d1, x, p, pm, q, qm, r, rm, cnt);
        lag_step(d2, x, p, pm, q, qm, r, rm, cnt);
        lag_step(d3, x, p, pm, q, qm, r, rm, cnt);
        const double a = fmax(fmax(fmax(fabs(p), fabs(pm)), fmax(fabs(q), fabs(qm))), fmax(fabs(r), fabs(rm)));
        const double sc = a > 0x1p200 ? 0x1p-200 : (a < 0x1p-200 ? 0x1p200 : 1.0);
        p *= sc;
        pm *= sc;
        q *= sc;
        qm *= sc;
        r *= sc;
        rm *= sc;
    }
    for (; i < c; ++i) lag_step(de[i], x, p, pm, q, qm, r, rm, cnt);
    f = p;
    f1 = q;
    f2 = r;
    return cnt;
}

template <int NR, int NC>
__global__ __launch_bounds__(kRrT) void k_rr(RrArgs a) {
    if (a.mode == 0 && a.rec && threadIdx.x < 3) a.rec[kRrRecFlag + threadIdx.x] = a.skip ? (double)a.skip[threadIdx.x] : 0.0;
    if (a.mode == 0 && a.rot_skip && threadIdx.x == 0) *a.rot_skip = 1;
    if (a.skip && *a.skip) return;
    constexpr int NT = 4 * NC;  // rows per lane in the back-transformation
    __shared__ double vs[2][kRrMax];
    __shared__ double ps[kRrMax];
    __shared__ double part[kRrW][kRrMax];
    __shared__ double tau_s[kRrMax];
    __shared__ double dd[kRrMax], ee[kRrMax];
    __shared__ double2 de[kRrMax + 8];
    __shared__ double th[kRrMax], sh[kRrMax], res_s[kRrMax], ysc[kRrMax];
    __shared__ int cl_start[kRrMax + 1];
    __shared__ int s_ncl, s_multi, s_p, s_m, s_nev, s_pcap;
    __shared__ double s_gl, s_gu;
    __shared__ double red[kRrW];
    // orders up to 96: the reflectors stay in LDS (the back-transformation
    // reads them there); larger orders keep them in the global scratch
    constexpr bool kHvLds = NR <= 6;
    constexpr int kHvLd = 96;
    __shared__ double hvs[kHvLds ? kHvLd * kHvLd : 1];

    const int c = a.c;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double* HV = a.work + kOffHV;
    double* Y = a.work + kOffY;
    double* U1 = a.work + kOffU1;
    double* U2 = a.work + kOffU2;
    double* U3 = a.work + kOffU3;
    double* Lm = a.work + kOffL;
    double* PV = a.work + kOffPV;
    double* Zs = a.work + kOffZ;

    // ---- stage 1: Householder tridiagonalisation --------------------------
    // A[q][t] = T[lane + 64 t][w + 16 q] (symmetrised: both triangles averaged)
    double A[NR][NC];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int col = w + 16 * q;
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            const int row = lane + 64 * t;
            A[q][t] = (row < c && col < c) ? 0.5 * (a.T[(size_t)row * a.ldt + col] + a.T[(size_t)col * a.ldt + row])
                                           : 0.0;
        }
    }
    for (int i = tid; i < kRrMax; i += kRrT) {
        vs[0][i] = vs[1][i] = ps[i] = 0.0;
        tau_s[i] = dd[i] = ee[i] = 0.0;
    }
    for (int i = tid; i < kRrMax + 8; i += kRrT) de[i] = make_double2(0.0, 0.0);
    // scale by a power of two (exact) so that max |T_ij| lies in [1/2, 1):
    // no overflow or underflow in the squares and Sturm recurrences below;
    // eigenvalues are scaled back on output, eigenvectors are unchanged
    bool finite;
    {
        // fmax drops NaNs; a scaled sum keeps them (and infinities) without
        // overflowing on finite entries
        double mx = 0.0, sm = 0.0;
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                mx = fmax(mx, fabs(A[q][t]));
                sm += A[q][t] * 0x1p-1000;
            }
        finite = isfinite(sm);
        mx = wmax(mx);
        if (lane == 0) red[w] = mx;
    }
    // a non-finite entry: every output is NaN (the residual estimates
    // infinite, no pair converged, no vector kept)
    if (!__syncthreads_and(finite)) {
        const double nan = __builtin_nan("");
        for (int i = tid; i < c; i += kRrT) a.theta[i] = nan;
        if (a.mode == 1) {
            for (int idx = tid; idx < c * a.mreq; idx += kRrT) a.Zout[idx] = nan;
            return;
        }
        if (a.Zk)
            for (int idx = tid; idx < c * a.k; idx += kRrT) a.Zk[idx] = nan;
        if (tid == 0) {
            a.rec[0] = 0.0;
            a.rec[1] = -1.0;
            a.rec[2] = 0.0;
            a.rec[3] = nan;
        }
        for (int i = tid; i < a.k; i += kRrT) {
            a.rec[kRrRecHead + i] = nan;
            a.rec[kRrRecHead + a.k + i] = INFINITY;
        }
        return;
    }
    int sexp = 0;
    {
        double mx = 0.0;
        for (int i = 0; i < kRrW; ++i) mx = fmax(mx, red[i]);
        if (mx > 0.0 && isfinite(mx)) frexp(mx, &sexp);
        const double sc = ldexp(1.0, -sexp);
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int t = 0; t < NC; ++t) A[q][t] *= sc;
    }
    // The reflector H_j = I - tau v v^T that zeroes T[j+2:, j], built by the
    // wavefront owning column j (w == j mod 16) from its registers.
    auto reflector = [&](int j) {
        const int qj = j >> 4;
        double x[NC];
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (q == qj) v = A[q][t];
            x[t] = v;
        }
        double ss = 0.0, xa = 0.0, xd = 0.0;
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            const int row = lane + 64 * t;
            if (row > j + 1 && row < c) ss += x[t] * x[t];
            if (t == ((j + 1) >> 6)) xa = x[t];
            if (t == (j >> 6)) xd = x[t];
        }
        ss = wsum(ss);
        const double al = rdl(xa, (j + 1) & 63);
        const double dj = rdl(xd, j & 63);
        double tau = 0.0, beta = al, scale = 0.0;
        if (ss > 0.0) {
            // tau = (beta - al) / beta and 1 / (al - beta) from one division
            beta = -copysign(sqrt(al * al + ss), al);
            const double g = al - beta, r = 1.0 / (beta * g);
            tau = -g * g * r;
            scale = beta * r;
        }
        double* hv = kHvLds ? hvs + (size_t)j * kHvLd : HV + (size_t)j * kRrMax;
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            const int row = lane + 64 * t;
            const double v = row == j + 1 ? 1.0 : (row > j + 1 && row < c ? x[t] * scale : 0.0);
            vs[j & 1][row] = v;
            if (row < c) hv[row] = v;
        }
        if (lane == 0) {
            dd[j] = dj;
            ee[j] = beta;
            tau_s[j] = tau;
        }
    };
    const int nwr = (c + 63) >> 6;  // wavefronts holding the rows in the reduction below
    if (c >= 2 && w == 0) reflector(0);
    for (int j = 0; j + 1 < c; ++j) {
        __syncthreads();  // reflector j in vs[j & 1] and tau_s[j]
        const double tau = tau_s[j];
        const double* v = vs[j & 1];
        if (tau != 0.0) {
            // p = tau T v: this wavefront's columns, then the sum of the
            // sixteen partials per row
            // the largest order has no registers to spare: its column
            // values of v are read again after the barriers
            constexpr bool keep = NR <= 8;
            double vc[keep ? NR : 1], vr[NC];
            auto vcol = [&](int q) { return keep ? vc[keep ? q : 0] : v[w + 16 * q]; };
            if (keep)
#pragma unroll
                for (int q = 0; q < NR; ++q) vc[keep ? q : 0] = v[w + 16 * q];
#pragma unroll
            for (int t = 0; t < NC; ++t) vr[t] = v[lane + 64 * t];
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < NR; ++q) s += A[q][t] * vcol(q);
                part[w][lane + 64 * t] = s;
            }
            __syncthreads();
            if (w < nwr) {
                double pv = 0.0;
                if (tid < c) {
                    double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0;
#pragma unroll
                    for (int u = 0; u < kRrW; u += 4) {
                        h0 += part[u][tid];
                        h1 += part[u + 1][tid];
                        h2 += part[u + 2][tid];
                        h3 += part[u + 3][tid];
                    }
                    const double pr = tid > j ? tau * ((h0 + h1) + (h2 + h3)) : 0.0;
                    ps[tid] = pr;
                    pv = pr * v[tid];
                }
                pv = wsum(pv);
                if (lane == 0) red[w] = pv;
            }
            __syncthreads();
            // K = tau/2 v^T p, w = p - K v, T -= v w^T + w v^T (rows and
            // columns above j are untouched: v and p vanish there)
            double pr[NC];
#pragma unroll
            for (int t = 0; t < NC; ++t) pr[t] = ps[lane + 64 * t];
            double K = 0.0;
            for (int u = 0; u < nwr; ++u) K += red[u];
            K *= 0.5 * tau;
            double wr[NC];
#pragma unroll
            for (int t = 0; t < NC; ++t) wr[t] = pr[t] - K * vr[t];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const double vq = vcol(q);
                const double wq = ps[w + 16 * q] - K * vq;
#pragma unroll
                for (int t = 0; t < NC; ++t) A[q][t] -= vr[t] * wq + wr[t] * vq;
            }
        }
        if (j + 2 < c && w == ((j + 1) & 15)) reflector(j + 1);
    }
    // the last diagonal entry
    if (w == ((c - 1) & 15)) {
        const int ql = (c - 1) >> 4;
        double xd = 0.0;
#pragma unroll
        for (int t = 0; t < NC; ++t)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (q == ql && t == ((c - 1) >> 6)) xd = A[q][t];
        const double dl = rdl(xd, (c - 1) & 63);
        if (lane == 0) dd[c - 1] = dl;
    }
    __syncthreads();

    // ---- stage 2: eigenvalues ------------------------------------------------------
    if (w == 0) {
        double lo = INFINITY, hi = -INFINITY;
        for (int i = lane; i < c; i += 64) {
            const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < c ? fabs(ee[i]) : 0.0);
            lo = fmin(lo, dd[i] - r);
            hi = fmax(hi, dd[i] + r);
            de[i] = make_double2(dd[i], i > 0 ? fmax(ee[i - 1] * ee[i - 1], 0x1p-600) : 0.0);
        }
        lo = wmin(lo);
        hi = wmax(hi);
        if (lane == 0) {
            s_gl = lo;
            s_gu = hi;
        }
    } else if (tid == 64) {
        // how many of the smallest eigenvalues the restart can use: the kept
        // count p (before its extension over equal eigenvalues and its
        // rounding to a multiple of 4) plus room for both, and theta_{k+1}
        int nev = c, pcap = c;
        if (a.mode == 0) {
            const int k = a.k, b = a.b, ncv = a.ncv;
            int p0 = a.keep > 0 ? a.keep : max(k + b, k + (c - k) / 2);
            p0 = min(p0, ncv - b);
            p0 = max(p0, min(k, ncv - b));
            nev = min(c, max(k + 1, p0 + 12));
            pcap = nev < c ? nev - 4 : c;
        } else {
            nev = c;
        }
        s_nev = nev;
        s_pcap = pcap;
    }
    __syncthreads();
    const double tn = fmax(fmax(fabs(s_gl), fabs(s_gu)), DBL_MIN);
    const double atol = 4.0 * DBL_EPSILON * tn;
    const int nev = s_nev;
    {
        // multisection: G lanes per eigenvalue (a group inside one
        // wavefront), until the interval holds lambda_i alone
        // (counts i at lo and i + 1 at hi) or is narrower than atol.  Wider
        // groups take fewer steps but keep more wavefronts busy on the FP64
        // units; four is as fast as eight or sixteen here.
        const int G = 4;
        const int i = tid / G, u = tid % G, base = lane & ~(G - 1);
        const bool act = i < nev;
        double lo = s_gl - 2.0 * atol, hi = s_gu + 2.0 * atol;
        int clo = 0, chi = c;
        for (int it = 0; it < 64; ++it) {
            const bool go = act && (clo != i || chi != i + 1) && hi - lo > atol;
            if (!__syncthreads_or(go)) break;
            if (go) {
                const double x = lo + (hi - lo) * ((double)(u + 1) / (double)(G + 1));
                const int cnt = sturm_count(de, c, x);
                // first point of the group whose count exceeds i
                const uint64_t bal = __ballot(cnt > i);
                const uint64_t gm = (bal >> base) & ((1ull << G) - 1ull);
                const int first = gm ? (__ffsll((unsigned long long)gm) - 1) : G;
                const int sl = base + (first > 0 ? first - 1 : 0), sh = base + (first < G ? first : G - 1);
                const double xl = __shfl(x, sl, 64), xh = __shfl(x, sh, 64);
                const int cl = __shfl(cnt, sl, 64), ch = __shfl(cnt, sh, 64);
                if (first > 0) {
                    lo = xl;
                    clo = cl;
                }
                if (first < G) {
                    hi = xh;
                    chi = ch;
                }
            }
        }
        // Laguerre's method (one lane of the group) from the middle of the
        // isolating interval.  The characteristic polynomial has only real
        // roots; from x left of lambda_i with no root in between, the right
        // Laguerre point x + n / (s - G) (G = f'/f, H = G^2 - f''/f,
        // s = sqrt((n-1)(nH - G^2))) lies in (x, lambda_i], and from the right
        // the left point x - n / (s + G) in [lambda_i, x): the iterates
        // approach lambda_i monotonically, cubically near it.  The count at x
        // says which side x is on; a step that crossed lambda_i (rounding)
        // only moves the bracket, the next one starts from its middle.
        if (act && u == 0) {
            double x = 0.5 * (lo + hi);
            if (clo == i && chi == i + 1 && hi - lo > atol) {
                const double nn = (double)c;
                for (int it = 0; it < 48; ++it) {
                    double f, f1, f2;
                    const int cnt = sturm_laguerre(de, c, x, f, f1, f2);
                    const bool right = cnt > i;  // x above lambda_i
                    if (right)
                        hi = x;
                    else
                        lo = x;
                    if (hi - lo <= atol) {
                        x = 0.5 * (lo + hi);
                        break;
                    }
                    // within atol / 4 of a root by the Newton distance
                    if (fabs(f) <= 0.25 * atol * fabs(f1)) break;
                    const double G = f1 / f, H = G * G - f2 / f;
                    const double sq = sqrt(fmax(0.0, (nn - 1.0) * (nn * H - G * G)));
                    // n / (s -+ G) in the form without cancellation:
                    // (s - G)(s + G) = n ((n - 1) H - G^2)
                    const double den = (nn - 1.0) * H - G * G;
                    double step;
                    if (!right)
                        step = G <= 0.0 ? nn / (sq - G) : (sq + G) / den;
                    else
                        step = -(G >= 0.0 ? nn / (sq + G) : (sq - G) / den);
                    double xn = x + step;
                    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
                    const double d = fabs(xn - x);
                    x = xn;
                    if (d <= 0.25 * atol) break;
                }
            }
            // inside the Gershgorin interval (exactly 0 for a zero matrix)
            th[i] = fmin(fmax(x, s_gl), s_gu);
        }
    }
    __syncthreads();

    // ---- selection, shifts and clusters (one thread) ------------------------
    if (tid == 0) {
        int p, m;
        if (a.mode == 0) {
            const int k = a.k, b = a.b, ncv = a.ncv;
            p = a.keep > 0 ? a.keep : max(k + b, k + (c - k) / 2);
            p = min(p, ncv - b);
            p = max(p, min(k, ncv - b));
            while (p < ncv - b && p < c && p < s_pcap &&
                   fabs(ldexp(th[p], sexp) - ldexp(th[p - 1], sexp)) <= 1e-10 * a.sigma)
                ++p;
            p = min((p + 3) & ~3, ncv - b);
            m = min(c, max(p, k));
        } else {
            p = a.mreq;
            m = a.mreq;
        }
        s_p = p;
        s_m = m;
        // Clustering distance: inverse iteration alone gives a vector whose
        // angle to the eigenvector is about eps ||T|| / gap, so eigenvalues
        // closer than 100 eps / tol ||T|| (at most LAPACK's 1e-3 ||T||) are
        // orthogonalised together, which keeps the restarted Krylov
        // relation accurate to a small fraction of the tolerance.
        double rel = 1e-3;
        if (a.mode == 0 && a.tol > 0.0) rel = fmin(rel, 100.0 * DBL_EPSILON / a.tol);
        const double ortol = rel * tn, pertol = 10.0 * DBL_EPSILON * tn;
        int ncl = 0, multi = 0;
        cl_start[0] = 0;
        double prev = 0.0;
        for (int i = 0; i < m; ++i) {
            double s = th[i];
            if (i > 0) {
                if (th[i] - th[i - 1] > ortol) {
                    multi |= (i - cl_start[ncl]) > 1;
                    cl_start[++ncl] = i;
                }
                if (s - prev < pertol) s = prev + pertol;
            }
            sh[i] = s;
            prev = s;
        }
        if (m > 0) multi |= (m - cl_start[ncl]) > 1;
        cl_start[++ncl] = m;
        s_ncl = ncl;
        s_multi = multi;
    }
    __syncthreads();
    const int m = s_m;
    const int ncl = s_ncl;

    // ---- stage 3: inverse iteration --------------------------------------------
    const double pivmin = DBL_EPSILON * tn;
    if (tid < m) {
        const double s = sh[tid];
        double ai = dd[0] - s, bi = c > 1 ? ee[0] : 0.0;
        for (int i = 0; i + 1 < c; ++i) {
            const double ci = ee[i];
            const double an = dd[i + 1] - s;
            const double bn = i + 2 < c ? ee[i + 1] : 0.0;
            const size_t o = (size_t)i * kRrLd + tid;
            // partial pivoting: rows i and i+1 swap when |ci| > |ai|
            // (selects, one reciprocal per row)
            const bool sw = fabs(ai) < fabs(ci);
            double piv = sw ? ci : ai;
            if (fabs(piv) < pivmin) piv = piv < 0.0 ? -pivmin : pivmin;
            const double rp = 1.0 / piv;
            const double l = (sw ? ai : ci) * rp;
            U1[o] = rp;
            U2[o] = sw ? an : bi;
            U3[o] = sw ? bn : 0.0;
            Lm[o] = l;
            PV[o] = sw ? 1.0 : 0.0;
            const double na = sw ? bi - l * an : an - l * bi;
            bi = sw ? -l * bn : bn;
            ai = na;
            Y[o] = start_entry(tid, i);
        }
        double piv = ai;
        if (fabs(piv) < pivmin) piv = piv < 0.0 ? -pivmin : pivmin;
        U1[(size_t)(c - 1) * kRrLd + tid] = 1.0 / piv;
        Y[(size_t)(c - 1) * kRrLd + tid] = start_entry(tid, c - 1);
    }
    // my cluster has more than one member?
    bool clustered = false;
    if (tid < m) {
        int cl = 0;
        while (cl_start[cl + 1] <= tid) ++cl;
        clustered = cl_start[cl + 1] - cl_start[cl] > 1;
    }
    const int nsolve = s_multi ? 3 : 2;
    for (int it = 0; it < nsolve; ++it) {
        if (tid < m && (it < 2 || clustered)) {
            // forward: the row interchanges and multipliers (rows read eight ahead)
            double cur = Y[tid];
            int i = 0;
            for (; i + 8 < c; i += 8) {
                double ny[8], lm[8], pv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const size_t o = (size_t)(i + u) * kRrLd + tid;
                    ny[u] = Y[o + kRrLd];
                    lm[u] = Lm[o];
                    pv[u] = PV[o];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const size_t o = (size_t)(i + u) * kRrLd + tid;
                    const bool sw = pv[u] != 0.0;
                    const double nxt = ny[u];
                    Y[o] = sw ? nxt : cur;
                    cur = sw ? cur - lm[u] * nxt : nxt - lm[u] * cur;
                }
            }
            for (; i + 1 < c; ++i) {
                const size_t o = (size_t)i * kRrLd + tid;
                const double nxt = Y[o + kRrLd];
                const double l = Lm[o];
                const bool sw = PV[o] != 0.0;
                Y[o] = sw ? nxt : cur;
                cur = sw ? cur - l * nxt : nxt - l * cur;
            }
            Y[(size_t)(c - 1) * kRrLd + tid] = cur;
            // backward substitution with U; the sum of squares of the result
            double y1 = 0.0, y2 = 0.0, nn = 0.0;
            int r = c - 1;
            for (; r >= 7; r -= 8) {
                double yv[8], u1[8], u2[8], u3[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const size_t o = (size_t)(r - u) * kRrLd + tid;
                    yv[u] = Y[o];
                    u1[u] = U1[o];
                    u2[u] = U2[o];
                    u3[u] = U3[o];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double yi = (yv[u] - u2[u] * y1 - u3[u] * y2) * u1[u];
                    Y[(size_t)(r - u) * kRrLd + tid] = yi;
                    nn += yi * yi;
                    y2 = y1;
                    y1 = yi;
                }
            }
            for (; r >= 0; --r) {
                const size_t o = (size_t)r * kRrLd + tid;
                const double yi = (Y[o] - U2[o] * y1 - U3[o] * y2) * U1[o];
                Y[o] = yi;
                nn += yi * yi;
                y2 = y1;
                y1 = yi;
            }
            // a vector alone in its cluster is normalised in the
            // back-transformation (three solves stay far from overflow:
            // each grows the vector by at most about 1 / (eps ||T||))
            if (!clustered) ysc[tid] = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        }
        if (!s_multi) continue;
        __syncthreads();
        // orthonormalise each cluster with more than one member
        for (int cl = w; cl < ncl; cl += kRrW) {
            const int s0 = cl_start[cl], s1 = cl_start[cl + 1];
            if (s1 - s0 < 2) continue;
            for (int jv = s0; jv < s1; ++jv) {
                double yv[NC];
#pragma unroll
                for (int t = 0; t < NC; ++t) {
                    const int r = 64 * t + lane;
                    yv[t] = r < c ? Y[(size_t)r * kRrLd + jv] : 0.0;
                }
                // the scale of a fresh solve can be ~1/eps: normalise first
                {
                    double mx = 0.0;
#pragma unroll
                    for (int t = 0; t < NC; ++t) mx = fmax(mx, fabs(yv[t]));
                    mx = wmax(mx);
                    const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
#pragma unroll
                    for (int t = 0; t < NC; ++t) yv[t] *= inv;
                }
                const int passes = it == nsolve - 1 ? 2 : 1;
                for (int pass = 0; pass < passes; ++pass)
                    for (int qv = s0; qv < jv; ++qv) {
                        double yq[NC], dp = 0.0;
#pragma unroll
                        for (int t = 0; t < NC; ++t) {
                            const int r = 64 * t + lane;
                            yq[t] = r < c ? Y[(size_t)r * kRrLd + qv] : 0.0;
                            dp += yv[t] * yq[t];
                        }
                        dp = wsum(dp);
#pragma unroll
                        for (int t = 0; t < NC; ++t) yv[t] -= dp * yq[t];
                    }
                double nn = 0.0;
#pragma unroll
                for (int t = 0; t < NC; ++t) nn += yv[t] * yv[t];
                nn = wsum(nn);
                const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
                for (int t = 0; t < NC; ++t) {
                    const int r = 64 * t + lane;
                    if (r < c) Y[(size_t)r * kRrLd + jv] = yv[t] * inv;
                }
                if (lane == 0) ysc[jv] = 1.0;
            }
        }
        __syncthreads();
    }
    __syncthreads();

    // ---- stage 4: back-transformation Z = Q Y ------------------------------------
    // Sixteen lanes per column (rows sl + 16 t), two columns per group of
    // sixteen lanes (c0 and c0 + 64; one for the largest orders, where the
    // registers would not hold two), 64 CS columns per pass.  The
    // reflectors are staged through LDS sixteen at a time, last first.
    {
        constexpr int CS = NC == 3 ? 1 : 2;
        const int sl = lane & 15, gi = 4 * w + (lane >> 4);
        for (int pbase = 0; pbase < m; pbase += 64 * CS) {
            const int c0 = pbase + gi, c1 = CS == 2 ? pbase + 64 + gi : m;
            const bool any0 = pbase + 4 * w < m, any1 = CS == 2 && pbase + 64 + 4 * w < m;  // uniform per wavefront
            const double sc0 = c0 < m ? ysc[c0] : 0.0, sc1 = c1 < m ? ysc[c1] : 0.0;
            double y0[NT], y1[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int r = sl + 16 * t;
                y0[t] = (c0 < m && r < c) ? Y[(size_t)r * kRrLd + c0] * sc0 : 0.0;
                y1[t] = (c1 < m && r < c) ? Y[(size_t)r * kRrLd + c1] * sc1 : 0.0;
            }
            // reflectors from LDS: all of them (orders up to 96) or sixteen
            // at a time staged from the global scratch
            const int chunk = kHvLds ? c : kRrW;
            for (int jc = c - 3; jc >= 0; jc -= chunk) {
                const int nj = min(chunk, jc + 1);
                if (!kHvLds) {
                    __syncthreads();
                    for (int idx = tid; idx < nj * c; idx += kRrT) {
                        const int jj = idx / c, r = idx - jj * c;
                        part[jj][r] = HV[(size_t)(jc - jj) * kRrMax + r];
                    }
                    __syncthreads();
                }
                if (!any0) continue;
                for (int jj = 0; jj < nj; ++jj) {
                    const double tau = tau_s[jc - jj];
                    if (tau == 0.0) continue;
                    const double* hr = kHvLds ? hvs + (size_t)(jc - jj) * kHvLd : &part[jj][0];
                    double v[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int r = sl + 16 * t;
                        v[t] = r < c ? hr[r] : 0.0;
                    }
                    double s0 = 0.0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) s0 += v[t] * y0[t];
                    if (any1) {
                        double s1 = 0.0;
#pragma unroll
                        for (int t = 0; t < NT; ++t) s1 += v[t] * y1[t];
                        s1 = tau * sum16(s1);
#pragma unroll
                        for (int t = 0; t < NT; ++t) y1[t] -= s1 * v[t];
                    }
                    s0 = tau * sum16(s0);
#pragma unroll
                    for (int t = 0; t < NT; ++t) y0[t] -= s0 * v[t];
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int r = sl + 16 * t;
                if (r < c) {
                    if (c0 < m) Zs[(size_t)r * kRrLd + c0] = y0[t];
                    if (c1 < m) Zs[(size_t)r * kRrLd + c1] = y1[t];
                }
            }
        }
    }
    __syncthreads();

    // ---- outputs ------------------------------------------------------------------
    for (int i = tid; i < nev; i += kRrT) a.theta[i] = ldexp(th[i], sexp);
    if (a.mode == 1) {
        for (int idx = tid; idx < c * m; idx += kRrT) {
            const int r = idx / m, col = idx - r * m;
            a.Zout[idx] = Zs[(size_t)r * kRrLd + col];
        }
        return;
    }
    const int p = s_p, b = a.b, k = a.k;
    // residual estimate of Ritz pair i: ||Rc Z[c-b:c, i]|| (Rc upper triangular)
    if (tid < m) {
        double ss = 0.0;
        for (int r = 0; r < b; ++r) {
            double acc = 0.0;
            for (int q = r; q < b; ++q) acc += a.Rc[r * b + q] * Zs[(size_t)(c - b + q) * kRrLd + tid];
            ss += acc * acc;
        }
        res_s[tid] = sqrt(ss);
    }
    // the rotation's factor in the layout rot_whole selects: the kept Ritz
    // vectors, then the next block unchanged
    if (rot_whole(c, b)) {
        // M = [Z[:, 0:p] 0; 0 I_b] in 48-column slices ((c + b) x wt each)
        const int kin = c + b, pw = p + b;
        for (int idx = tid; idx < kin * pw; idx += kRrT) {
            const int j0 = (idx / (kin * 48)) * 48;
            const int wt = min(48, pw - j0);
            const int rem = idx - kin * j0;
            const int r = rem / wt, j = j0 + (rem - r * wt);
            a.Qch[idx] = j < p ? (r < c ? Zs[(size_t)r * kRrLd + j] : 0.0) : (r - c == j - p ? 1.0 : 0.0);
        }
    } else {
        // Z[:, 0:p] in 32-column slices (c x wt each), then the identity
        for (int idx = tid; idx < c * p; idx += kRrT) {
            const int j0 = (idx / (c * 32)) * 32;
            const int wt = min(32, p - j0);
            const int rem = idx - c * j0;
            const int r = rem / wt, q = rem - r * wt;
            a.Qch[idx] = Zs[(size_t)r * kRrLd + j0 + q];
        }
        for (int idx = tid; idx < b * b; idx += kRrT) a.Qch[(size_t)c * p + idx] = (idx / b == idx % b) ? 1.0 : 0.0;
    }
    if (a.Zk)
        for (int idx = tid; idx < c * k; idx += kRrT) {
            const int r = idx / k, q = idx - r * k;
            a.Zk[idx] = Zs[(size_t)r * kRrLd + q];
        }
    __syncthreads();
    if (tid == 0) {
        int nconv = 0;
        for (int i = 0; i < k && i < m; ++i) nconv += res_s[i] <= a.tol * a.sigma;
        a.rec[0] = (double)nconv;
        a.rec[1] = (double)p;
        a.rec[2] = (double)m;
        if (a.rot_skip) *a.rot_skip = (nconv < k && p == a.p_pred) ? 0 : 1;
        a.rec[3] = c > k ? (ldexp(th[k], sexp) - ldexp(th[k - 1], sexp)) / a.sigma : 0.0;
    }
    for (int i = tid; i < k; i += kRrT) {
        a.rec[kRrRecHead + i] = i < c ? ldexp(th[i], sexp) : 0.0;
        a.rec[kRrRecHead + k + i] = i < m ? res_s[i] : INFINITY;
    }
}

}  // namespace

size_t rr_work_doubles() { return kWork; }

int rr_buffers(sfairsc_graph* g, RrBufs* out) {
    const size_t nw = kWork, nth = kRrMax, nzk = (size_t)kRrMax * kMaxK, nrec = rr_rec_doubles(kMaxK);
    const size_t nz = (size_t)kRrMax * kRrMax;
    SF_TRY(g->eig.rr.ensure((nw + nth + nzk + nrec + nz) * sizeof(double)));
    double* p = g->eig.rr.as<double>();
    out->work = p;
    out->theta = p + nw;
    out->zk = out->theta + nth;
    out->rec = out->zk + nzk;
    out->zout = out->rec + nrec;
    return SFAIRSC_OK;
}

int small_eig_host(sfairsc_graph* g, const double* dT, int c, int ldt, double* w, double* Z, hipStream_t s) {
    RrBufs rb;
    SF_TRY(rr_buffers(g, &rb));
    RrArgs a;
    a.T = dT;
    a.ldt = ldt;
    a.c = c;
    a.work = rb.work;
    a.mode = 1;
    a.mreq = c;
    a.theta = rb.theta;
    a.Zout = rb.zout;
    SF_TRY(rr_launch(a, s));
    SF_HIP(hipMemcpyAsync(w, rb.theta, sizeof(double) * c, hipMemcpyDeviceToHost, s));
    SF_HIP(hipMemcpyAsync(Z, rb.zout, sizeof(double) * c * c, hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    return SFAIRSC_OK;
}

int rr_launch(const RrArgs& a, hipStream_t s) {
    if (a.c < 1 || a.c > kRrMax || !a.T || !a.work || !a.theta)
        return set_error(SFAIRSC_E_ARG, "internal: Rayleigh-Ritz order %d outside [1, %d]", a.c, kRrMax);
    if (a.mode == 0) {
        if (!a.Rc || !a.Qch || !a.rec || a.b < 1 || a.k < 1 || a.b > a.c || a.k > kMaxK)
            return set_error(SFAIRSC_E_ARG, "internal: bad restart-mode Rayleigh-Ritz arguments");
    } else if (a.mode == 1) {
        if (a.mreq < 0 || a.mreq > a.c || (a.mreq > 0 && !a.Zout))
            return set_error(SFAIRSC_E_ARG, "internal: bad Rayleigh-Ritz vector count %d", a.mreq);
    } else {
        return set_error(SFAIRSC_E_ARG, "internal: Rayleigh-Ritz mode %d", a.mode);
    }
    if (a.c <= 64)
        k_rr<4, 1><<<1, kRrT, 0, s>>>(a);
    else if (a.c <= 80)
        k_rr<5, 2><<<1, kRrT, 0, s>>>(a);
    else if (a.c <= 96)
        k_rr<6, 2><<<1, kRrT, 0, s>>>(a);
    else if (a.c <= 128)
        k_rr<8, 2><<<1, kRrT, 0, s>>>(a);
    else
        k_rr<12, 3><<<1, kRrT, 0, s>>>(a);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

}  // namespace sfairsc

using namespace sfairsc;

extern "C" int sfairsc_symeig(const double* T, int32_t c, int32_t ldt, int32_t m, double* w, double* Z,
                              hipStream_t stream) {
    if (!T || !w || (m > 0 && !Z)) return set_error(SFAIRSC_E_ARG, "NULL argument");
    if (c < 1 || c > kMaxBasis) return set_error(SFAIRSC_E_ARG, "order %d outside [1, %d]", c, kMaxBasis);
    if (ldt < c) return set_error(SFAIRSC_E_ARG, "leading dimension %d below the order %d", ldt, c);
    if (m < 0 || m > c) return set_error(SFAIRSC_E_ARG, "m = %d outside [0, c]", m);
    DevBuf work;
    SF_TRY(work.ensure(rr_work_doubles() * sizeof(double)));
    RrArgs a;
    a.T = T;
    a.ldt = ldt;
    a.c = c;
    a.work = work.as<double>();
    a.mode = 1;
    a.mreq = m;
    a.theta = w;
    a.Zout = Z;
    int rc = rr_launch(a, stream);
    if (rc == SFAIRSC_OK && hipStreamSynchronize(stream) != hipSuccess)
        rc = set_error(SFAIRSC_E_HIP, "hipStreamSynchronize failed");
    work.release();
    return rc;
}
