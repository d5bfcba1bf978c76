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
//     registers: wavefront w holds rows w, w + 16, ..., lane l columns l,
//     l + 64, l + 128, so every row sum of a product is a wavefront
//     reduction.  Two workgroup barriers per column.
//  2. every eigenvalue of Tri by multisection: a group of G lanes per
//     eigenvalue evaluates G Sturm counts (signs of the leading principal
//     minors of Tri - x I, by their three-term recurrence with power-of-two
//     rescaling) and keeps the subinterval that holds the eigenvalue, until
//     its width is a few ulps of ||T||.
//  3. eigenvectors of Tri for the m smallest eigenvalues by inverse
//     iteration, one lane per vector: Gaussian elimination with partial
//     pivoting of Tri - s I (tiny pivots replaced by eps ||T||), three solves
//     from a pseudo-random start; after each solve the vectors whose
//     eigenvalues lie within 1e-3 ||T|| of each other are orthonormalised
//     together (modified Gram-Schmidt, one wavefront per such cluster), as in
//     LAPACK's inverse iteration.
//  4. back-transformation Z = Q Y, the reflectors applied in reverse order,
//     one wavefront per set of columns (no barriers).
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

__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wmin(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Uniform(-1, 1) start entry (SplitMix64 output function of the counter).
__device__ inline double start_entry(int vec, int row) {
    uint64_t z = 0x9E3779B97F4A7C15ull * (uint64_t)(((uint64_t)vec << 32) + (uint64_t)row + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-52 - 1.0;
}

// Number of eigenvalues of the tridiagonal matrix (d, e) below x: the sign
// changes of p_0 = 1, p_i = det of the leading i x i block of Tri - x I
// (p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}).  A zero p_i takes the sign
// opposite to p_{i-1}; both terms are rescaled by 2^-400 or 2^400 when the
// newest leaves [2^-400, 2^400].
__device__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int c, double x) {
    double pm = 1.0, p = d[0] - x;
    if (p == 0.0) p = -0x1p-60;
    int cnt = p < 0.0;
    for (int i = 1; i < c; ++i) {
        double pn = (d[i] - x) * p - e2[i - 1] * pm;
        if (pn == 0.0) pn = -p * 0x1p-60;
        cnt += (pn < 0.0) != (p < 0.0);
        const double a = fabs(pn);
        if (a > 0x1p400) {
            pn *= 0x1p-400;
            p *= 0x1p-400;
        } else if (a < 0x1p-400) {
            pn *= 0x1p400;
            p *= 0x1p400;
        }
        pm = p;
        p = pn;
    }
    return cnt;
}

template <int NR, int NC>
__global__ __launch_bounds__(kRrT) void k_rr(RrArgs a) {
    if (a.skip && *a.skip) return;
    __shared__ double vs[2][kRrMax];
    __shared__ double ps[2][kRrMax];
    __shared__ double tau_s[kRrMax];
    __shared__ double dd[kRrMax], ee[kRrMax], ee2[kRrMax];
    __shared__ double th[kRrMax], sh[kRrMax], res_s[kRrMax];
    __shared__ int cl_start[kRrMax + 1];
    __shared__ int s_ncl, s_p, s_m;
    __shared__ double s_gl, s_gu;
    __shared__ double red16[16];

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
    double A[NR][NC];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int r = 16 * q + w;
#pragma unroll
        for (int t = 0; t < NC; ++t) {
            const int col = 64 * t + lane;
            A[q][t] = (r < c && col < c) ? 0.5 * (a.T[(size_t)r * a.ldt + col] + a.T[(size_t)col * a.ldt + r]) : 0.0;
        }
    }
    for (int i = tid; i < kRrMax; i += kRrT) {
        vs[0][i] = vs[1][i] = ps[0][i] = ps[1][i] = 0.0;
        tau_s[i] = dd[i] = ee[i] = ee2[i] = 0.0;
    }
    // scale by a power of two (exact) so that max |T_ij| lies in [1/2, 1):
    // no overflow or underflow in the squares and Sturm recurrences below;
    // eigenvalues are scaled back on output, eigenvectors are unchanged
    {
        double mx = 0.0;
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int t = 0; t < NC; ++t) mx = fmax(mx, fabs(A[q][t]));
        mx = wmax(mx);
        if (lane == 0) red16[w] = mx;
    }
    __syncthreads();
    int sexp = 0;
    {
        double mx = 0.0;
        for (int i = 0; i < 16; ++i) mx = fmax(mx, red16[i]);
        if (mx > 0.0 && isfinite(mx)) frexp(mx, &sexp);
        const double sc = ldexp(1.0, -sexp);
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int t = 0; t < NC; ++t) A[q][t] *= sc;
    }
    for (int j = 0; j + 2 < c; ++j) {
        const int buf = j & 1;
        if (w == (j & 15)) {
            // the wavefront holding row j builds the reflector that zeroes
            // T[j, j+2:] (= T[j+2:, j])
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
            double ss = 0.0, al = 0.0, dj = 0.0;
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                const int col = 64 * t + lane;
                if (col > j + 1 && col < c) ss += x[t] * x[t];
                if (col == j + 1) al = x[t];
                if (col == j) dj = x[t];
            }
            ss = wsum(ss);
            al = wsum(al);
            dj = wsum(dj);
            double tau = 0.0, beta = al, scale = 0.0;
            if (ss > 0.0) {
                beta = -copysign(sqrt(al * al + ss), al);
                tau = (beta - al) / beta;
                scale = 1.0 / (al - beta);
            }
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                const int col = 64 * t + lane;
                if (col < c) {
                    const double v = col == j + 1 ? 1.0 : (col > j + 1 ? x[t] * scale : 0.0);
                    vs[buf][col] = v;
                    HV[(size_t)j * kRrMax + col] = v;
                }
            }
            if (lane == 0) {
                dd[j] = dj;
                ee[j] = beta;
                tau_s[j] = tau;
            }
        }
        __syncthreads();
        const double tau = tau_s[j];
        if (tau != 0.0) {
            // p = tau T v on the rows below j
            double vc[NC];
#pragma unroll
            for (int t = 0; t < NC; ++t) vc[t] = vs[buf][64 * t + lane];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const int r = 16 * q + w;
                if (16 * q < c) {
                    double s = 0.0;
#pragma unroll
                    for (int t = 0; t < NC; ++t) s += A[q][t] * vc[t];
                    s = wsum(s);
                    if (lane == 0 && r < c) ps[buf][r] = r > j ? tau * s : 0.0;
                }
            }
        }
        __syncthreads();
        if (tau != 0.0) {
            // K = tau/2 v^T p, w = p - K v, T -= v w^T + w v^T
            double part = 0.0;
#pragma unroll
            for (int t = 0; t < NC; ++t) part += vs[buf][64 * t + lane] * ps[buf][64 * t + lane];
            const double K = 0.5 * tau * wsum(part);
            double vc[NC], wc[NC];
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                vc[t] = vs[buf][64 * t + lane];
                wc[t] = ps[buf][64 * t + lane] - K * vc[t];
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const int r = 16 * q + w;
                if (r > j && r < c) {
                    const double vr = vs[buf][r];
                    const double wr = ps[buf][r] - K * vr;
#pragma unroll
                    for (int t = 0; t < NC; ++t) A[q][t] -= vr * wc[t] + wr * vc[t];
                }
            }
        }
    }
    // the trailing 2 x 2 (or 1 x 1) block
    for (int r = (c >= 2 ? c - 2 : 0); r < c; ++r) {
        if (w == (r & 15)) {
            const int qr = r >> 4;
            double dg = 0.0, of = 0.0;
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                double v = 0.0;
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    if (q == qr) v = A[q][t];
                const int col = 64 * t + lane;
                if (col == r) dg = v;
                if (col == r + 1 && col < c) of = v;
            }
            dg = wsum(dg);
            of = wsum(of);
            if (lane == 0) {
                dd[r] = dg;
                if (r + 1 < c) ee[r] = of;
            }
        }
    }
    __syncthreads();

    // ---- stage 2: eigenvalues by multisection ------------------------------
    if (w == 0) {
        double lo = INFINITY, hi = -INFINITY;
        for (int i = lane; i < c; i += 64) {
            const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < c ? fabs(ee[i]) : 0.0);
            lo = fmin(lo, dd[i] - r);
            hi = fmax(hi, dd[i] + r);
            if (i + 1 < c) ee2[i] = ee[i] * ee[i];
        }
        lo = wmin(lo);
        hi = wmax(hi);
        if (lane == 0) {
            s_gl = lo;
            s_gu = hi;
        }
    }
    __syncthreads();
    const double tn = fmax(fmax(fabs(s_gl), fabs(s_gu)), DBL_MIN);
    {
        const int G = c <= 64 ? 16 : (c <= 128 ? 8 : 4);
        const int i = tid / G, u = tid % G;
        const double atol = 4.0 * DBL_EPSILON * tn;
        double lo = s_gl - 2.0 * atol, hi = s_gu + 2.0 * atol;
        // iterations to shrink [lo, hi] to atol (uniform over the workgroup;
        // bounded also for non-finite input)
        const double nd = ceil(log2((hi - lo) / atol) / log2((double)(G + 1)));
        const int nit = (nd >= 0.0 && nd <= 128.0) ? (int)nd + 1 : 129;
        const int base = (lane / G) * G;
        const uint64_t gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
        for (int it = 0; it < nit; ++it) {
            const double x = lo + (hi - lo) * ((double)(u + 1) / (double)(G + 1));
            const int cnt = i < c ? sturm_count(dd, ee2, c, x) : 0;
            const uint64_t bal = __ballot(i < c && cnt > i);
            const uint64_t gm = (bal >> base) & gmask;
            const int first = gm ? (__ffsll((unsigned long long)gm) - 1) : G;
            const double xl = __shfl(x, base + (first > 0 ? first - 1 : 0), 64);
            const double xh = __shfl(x, base + (first < G ? first : G - 1), 64);
            if (first > 0) lo = xl;
            if (first < G) hi = xh;
        }
        if (i < c && u == 0) th[i] = 0.5 * (lo + hi);
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
            while (p < ncv - b && p < c && fabs(ldexp(th[p], sexp) - ldexp(th[p - 1], sexp)) <= 1e-10 * a.sigma)
                ++p;
            p = min((p + 3) & ~3, ncv - b);
            m = min(c, max(p, k));
        } else {
            p = a.mreq;
            m = a.mreq;
        }
        s_p = p;
        s_m = m;
        const double ortol = 1e-3 * tn, pertol = 10.0 * DBL_EPSILON * tn;
        int ncl = 0;
        cl_start[0] = 0;
        double prev = 0.0;
        for (int i = 0; i < m; ++i) {
            double s = th[i];
            if (i > 0) {
                if (th[i] - th[i - 1] > ortol) cl_start[++ncl] = i;
                if (s - prev < pertol) s = prev + pertol;
            }
            sh[i] = s;
            prev = s;
        }
        cl_start[++ncl] = m;
        s_ncl = ncl;
    }
    __syncthreads();
    const int m = s_m;

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
            if (fabs(ai) >= fabs(ci)) {
                double piv = ai;
                if (fabs(piv) < pivmin) piv = piv < 0.0 ? -pivmin : pivmin;
                const double l = ci / piv;
                U1[o] = 1.0 / piv;
                U2[o] = bi;
                U3[o] = 0.0;
                Lm[o] = l;
                PV[o] = 0.0;
                ai = an - l * bi;
                bi = bn;
            } else {
                double piv = ci;
                if (fabs(piv) < pivmin) piv = piv < 0.0 ? -pivmin : pivmin;
                const double l = ai / piv;
                U1[o] = 1.0 / piv;
                U2[o] = an;
                U3[o] = bn;
                Lm[o] = l;
                PV[o] = 1.0;
                ai = bi - l * an;
                bi = -l * bn;
            }
        }
        double piv = ai;
        if (fabs(piv) < pivmin) piv = piv < 0.0 ? -pivmin : pivmin;
        U1[(size_t)(c - 1) * kRrLd + tid] = 1.0 / piv;
        for (int r = 0; r < c; ++r) Y[(size_t)r * kRrLd + tid] = start_entry(tid, r);
    }
    const int ncl = s_ncl;
    for (int it = 0; it < 3; ++it) {
        if (tid < m) {
            // forward: the row interchanges and multipliers
            double cur = Y[tid];
            for (int i = 0; i + 1 < c; ++i) {
                const size_t o = (size_t)i * kRrLd + tid;
                double nxt = Y[o + kRrLd];
                const double l = Lm[o];
                if (PV[o] != 0.0) {
                    Y[o] = nxt;
                    nxt = cur - l * nxt;
                } else {
                    Y[o] = cur;
                    nxt = nxt - l * cur;
                }
                cur = nxt;
            }
            Y[(size_t)(c - 1) * kRrLd + tid] = cur;
            // backward substitution with U
            double y1 = 0.0, y2 = 0.0;
            for (int i = c - 1; i >= 0; --i) {
                const size_t o = (size_t)i * kRrLd + tid;
                const double yi = (Y[o] - U2[o] * y1 - U3[o] * y2) * U1[o];
                Y[o] = yi;
                y2 = y1;
                y1 = yi;
            }
        }
        __syncthreads();
        // orthonormalise each cluster (a singleton is only normalised)
        for (int cl = w; cl < ncl; cl += 16) {
            const int s0 = cl_start[cl], s1 = cl_start[cl + 1];
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
                const int passes = it == 2 ? 2 : 1;
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
            }
        }
        __syncthreads();
    }

    // ---- stage 4: back-transformation Z = Q Y ------------------------------------
    {
        double y[NR][NC];
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int col = w + 16 * u;
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                const int r = 64 * t + lane;
                y[u][t] = (col < m && r < c) ? Y[(size_t)r * kRrLd + col] : 0.0;
            }
        }
        for (int j = c - 3; j >= 0; --j) {
            const double tau = tau_s[j];
            if (tau == 0.0) continue;
            double v[NC];
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                const int r = 64 * t + lane;
                v[t] = r < c ? HV[(size_t)j * kRrMax + r] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                if (w + 16 * u < m) {
                    double s = 0.0;
#pragma unroll
                    for (int t = 0; t < NC; ++t) s += v[t] * y[u][t];
                    s = tau * wsum(s);
#pragma unroll
                    for (int t = 0; t < NC; ++t) y[u][t] -= s * v[t];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int col = w + 16 * u;
#pragma unroll
            for (int t = 0; t < NC; ++t) {
                const int r = 64 * t + lane;
                if (col < m && r < c) Zs[(size_t)r * kRrLd + col] = y[u][t];
            }
        }
    }
    __syncthreads();

    // ---- outputs ------------------------------------------------------------------
    for (int i = tid; i < c; i += kRrT) a.theta[i] = ldexp(th[i], sexp);
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
    // Z[:, 0:p] in 32-column slices (slice s: c x wt row-major at c * 32 s)
    for (int idx = tid; idx < c * p; idx += kRrT) {
        const int j0 = (idx / (c * 32)) * 32;
        const int wt = min(32, p - j0);
        const int rem = idx - c * j0;
        const int r = rem / wt, q = rem - r * wt;
        a.Qch[idx] = Zs[(size_t)r * kRrLd + j0 + q];
    }
    // then the b x b identity (the next block moves unchanged)
    for (int idx = tid; idx < b * b; idx += kRrT) a.Qch[(size_t)c * p + idx] = (idx / b == idx % b) ? 1.0 : 0.0;
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
