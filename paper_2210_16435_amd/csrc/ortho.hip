// Tall-skinny block orthogonalisation on the FP64 matrix cores (gfx950
// v_mfma_f64_16x16x4f64).  One Krylov expansion (block classical
// Gram-Schmidt twice, then Cholesky-QR twice) runs as four row passes over
// the row-major basis V (n x ld):
//
//   A  Y0 = T - C G^{-1}(C^T T - sigma S)  (deflation, Section 3.4), stored in
//      the Y slot;  partial H1 = V[:, 0:cv]^T Y0
//   B  Y' = [V | Y0] [-H1; I];  partial [H2; G] = [V | Y']^T Y'
//   C  Y1 = [V | Y'] [-H2 R1^{-1}; R1^{-1}],  R1^T R1 = G;
//      partial G2 = Y1^T Y1
//   D  Y2 = Y1 R2^{-1},  R2^T R2 = G2            (the next block V_next)
//
// so that Y0 = V (H1 + H2) + Y2 (R2 R1): the projected matrix gets the
// column block H1 + H2 and the coupling is R = R2 R1.
//
// MFMA operand layout (measured on gfx950): A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4), register i / 4.
//  * Gram products (K = rows): lane (i, k) loads V[row0 + k][c0 + i], four
//    rows of 16 consecutive columns per instruction (coalesced).
//  * Updates (K = columns): lane (i, g) loads 4 consecutive columns
//    V[row0 + i][c0 + 4g .. 4g + 3] as one 32-byte load and feeds four MFMAs;
//    step s uses columns {c0 + 4g + s}, so the B operand reads the matching
//    rows of the coefficient matrix.  The update's D register q holds rows
//    4q..4q+3 in exactly the operand layout of a Gram step, so the new block
//    feeds the following Gram/Syrk products straight from registers.
//
// Each block has kOrWaves waves; a wave owns 16-row tiles (grid-stride) and
// keeps its products in registers; the waves' tiles are summed in LDS in wave
// order and the block writes one partial (tile layout: [tile][lane][4]).
// Partials are summed in a fixed order by k_reduce_partials: bitwise
// reproducible results.
#include <algorithm>

#include <type_traits>

#include "internal.h"
#include "ortho.h"
#include "reduce.h"
#include "wave_chol.h"

namespace sfairsc {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

#ifndef SF_ORTHO_THREADS
#define SF_ORTHO_THREADS 512
#endif
constexpr int kOrThreads = SF_ORTHO_THREADS;
constexpr int kOrWaves = kOrThreads / 64;
constexpr int kMaxRT = (kLdMax + 15) / 16;  // 14 row tiles of the Gram products

// A block partial of ntile tiles is summed either from one LDS slot per
// wave (one barrier; kOrWaves x ntile x 2 KiB of LDS, at most 96 KiB) or
// wave after wave in one area (a barrier per wave).  Either way each
// element is w_0 + w_1 + ... in wave order, so the two give the same bits.
__host__ __device__ inline bool store_wide(int ntile) { return ntile * kOrWaves * 256 * 8 <= 96 * 1024; }
inline size_t store_lds_bytes(int ntile) {
    return (size_t)(store_wide(ntile) ? kOrWaves : 1) * ntile * 256 * sizeof(double);
}

// Sum the block's waves' register tiles (na tiles of acca, then nb of accb,
// each 64 x d4) in LDS in wave order and write the block partial (out may be
// null); the sums are left in lds[0 : (na + nb) * 256] for every thread.
// WIDE: the one-barrier form may be taken (compiled for small register sets
// only: with the wide passes' 28 tiles a second copy of the stores costs
// registers, which those kernels spill).
template <bool WIDE, int NA, int NB>
__device__ __forceinline__ void block_store_tiles2(d4 (&acca)[NA], int na, d4 (&accb)[NB], int nb, double* lds,
                                                   double* __restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tot = (na + nb) * 256;
    auto put = [&](double* base, bool add) {
#pragma unroll
        for (int t = 0; t < NA + NB; ++t) {
            const bool first = t < NA;
            const int tt = first ? t : t - NA;
            if (first ? tt < na : tt < nb) {
                const d4 v = first ? acca[first ? tt : 0] : accb[first ? 0 : tt];
                double* p = base + ((size_t)(first ? tt : na + tt) * 64 + lane) * 4;
                if (add) {
                    p[0] += v[0];
                    p[1] += v[1];
                    p[2] += v[2];
                    p[3] += v[3];
                } else {
                    p[0] = v[0];
                    p[1] = v[1];
                    p[2] = v[2];
                    p[3] = v[3];
                }
            }
        }
    };
    if (WIDE && store_wide(na + nb)) {
        put(lds + (size_t)wave * tot, false);
        __syncthreads();
        for (int e = threadIdx.x; e < tot; e += kOrThreads) {
            double sum = lds[e];
            for (int w = 1; w < kOrWaves; ++w) sum += lds[(size_t)w * tot + e];
            lds[e] = sum;
            if (out) out[e] = sum;
        }
        __syncthreads();
        return;
    }
    for (int w = 0; w < kOrWaves; ++w) {
        if (wave == w) put(lds, w != 0);
        __syncthreads();
    }
    if (out)
        for (int e = threadIdx.x; e < tot; e += kOrThreads) out[e] = lds[e];
}

template <bool WIDE, int NT>
__device__ __forceinline__ void block_store_tiles(d4 (&acc)[NT], int ntile, double* lds, double* __restrict__ out) {
    if constexpr (WIDE) {
        d4 none[1] = {d4{0, 0, 0, 0}};
        block_store_tiles2<true>(acc, ntile, none, 0, lds, out);
    } else {
        // wave after wave only (the same sums)
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int w = 0; w < kOrWaves; ++w) {
            if (wave == w) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (t < ntile) {
                        double* p = lds + ((size_t)t * 64 + lane) * 4;
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
        if (out)
            for (int e = threadIdx.x; e < ntile * 256; e += kOrThreads) out[e] = lds[e];
    }
}

// Element (i, j) of a tile-layout matrix with BJ column tiles.
__device__ __forceinline__ double tile_at(const double* __restrict__ t, int BJ, int i, int j) {
    const int tile = (i >> 4) * BJ + (j >> 4);
    const int ii = i & 15, jj = j & 15;
    return t[((size_t)tile * 64 + jj + 16 * (ii & 3)) * 4 + (ii >> 2)];
}

// Pass A.  Y0 from the sparse product T (compact stride BW, type TT) and the
// deflation tables: Y0_i = T_i - c_i Rtab[g_i] - sum_{s<m} LC[i][s] Utab[s]
// (the last term only with LC, the reassociated operator); partial
// V[:, 0:cv]^T Y0 (nrt x BJ tiles).  RT bounds nrt (4, 8 or kMaxRT): the
// accumulators and the loads in flight are sized by it, so the common small
// bases keep their registers for loads.  The L C term of a 16-row tile,
// LC[16 x m] Utab[m x b], is a matrix-core product whose output registers
// are already laid out as the tile's Y0 values (row 4q + lk of the tile in
// register q of lane li + 16 lk): each lane loads one LC value per 4 of the
// m columns (lcw, a multiple of 4, keeps the loads in bounds; LC's padding
// columns and the table's rows from m on are zero).
template <int BJ, class TT, int RT>
__global__ __launch_bounds__(kOrThreads) void k_pass_a(double* __restrict__ V, int ld, int64_t n, int cv, int b,
                                                        const TT* __restrict__ T, int BW,
                                                        const int32_t* __restrict__ grp,
                                                        const double* __restrict__ cs,
                                                        const double* __restrict__ Rtab,
                                                        const double* __restrict__ LC, int lcw, int m,
                                                        const double* __restrict__ Utab, double* __restrict__ part,
                                                        const int* skip) {
    if (skip && *skip) return;
    extern __shared__ double lds[];
    // the deflation tables (kMaxGroups x 32 doubles; the rows past h are read
    // but never used), so that their lookups wait for no global load
    // (the L C term is compiled for one column tile of the block only: the
    // reassociated operator serves widths up to 16, and the two-tile
    // variants have no registers to spare)
    constexpr bool kLC = BJ == 1;
    __shared__ double rtab_s[BJ == 1 ? kMaxGroups * 32 : 1];
    __shared__ double utab_s[kLC ? kMaxGroups * 32 : 1];
    if constexpr (BJ == 1) {
        if (Rtab)
            for (int e = threadIdx.x; e < kMaxGroups * 32; e += kOrThreads) rtab_s[e] = Rtab[e];
        if (LC)
            for (int e = threadIdx.x; e < kMaxGroups * 32; e += kOrThreads) utab_s[e] = e < m * 32 ? Utab[e] : 0.0;
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nrt = (cv + 15) >> 4;
    d4 acc[RT * BJ];
#pragma unroll
    for (int t = 0; t < RT * BJ; ++t) acc[t] = d4{0, 0, 0, 0};
    const int64_t ntiles = (n + 15) >> 4;
    const int64_t wstride = (int64_t)gridDim.x * kOrWaves;
    for (int64_t tile = (int64_t)blockIdx.x * kOrWaves + (threadIdx.x >> 6); tile < ntiles; tile += wstride) {
        // the tile's L C term (see above): corr[jt][q] for row 4q + lk,
        // column jt * 16 + li
        d4 corr[1] = {d4{0, 0, 0, 0}};
        if constexpr (kLC) {
            if (LC) {
                const int64_t ra = tile * 16 + li;
                const int64_t rsa = ra < n ? ra : 0;
                for (int k0 = 0; k0 < m; k0 += 4) {
                    const double av = LC[rsa * lcw + k0 + lk];
                    corr[0] = mfma(av, utab_s[(k0 + lk) * 32 + li], corr[0]);
                }
            }
        }
        if constexpr (BJ == 1 && RT <= 8) {
            // a small basis: every load of the tile (4 steps) first
            double yraw[4];
            double araw[4][RT];
            double cq[4];
            int gq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = tile * 16 + q * 4 + lk;
                const int64_t rs = row < n ? row : 0;
                cq[q] = (cs && Rtab) ? cs[rs] : 1.0;
                gq[q] = Rtab ? grp[rs] : 0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = tile * 16 + q * 4 + lk;
                const int64_t rs = row < n ? row : 0;
                yraw[q] = (double)T[rs * BW + (li < b ? li : 0)];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const int col = rt * 16 + li;
                    araw[q][rt] = V[rs * ld + (rt < nrt && col < cv ? col : 0)];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = tile * 16 + q * 4 + lk;
                const bool rv = row < n;
                double y = 0.0;
                if (rv && li < b) {
                    y = yraw[q];
                    if (Rtab) y -= cq[q] * rtab_s[gq[q] * 32 + li];
                    if (LC) y -= corr[0][q];
                    V[row * ld + cv + li] = y;
                }
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (rt < nrt) {
                        const double a = (rv && rt * 16 + li < cv) ? araw[q][rt] : 0.0;
                        acc[rt] = mfma(a, y, acc[rt]);
                    }
                }
            }
        } else if constexpr (BJ == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // every load of the step first, so that they are in flight
                // together: rows past n read row 0 and columns past b or cv
                // read column 0 (always in bounds), and the value is replaced
                // by zero only where it is used (a select right after a load
                // would wait for it)
                const int64_t row = tile * 16 + q * 4 + lk;
                const bool rv = row < n;
                const int64_t rs = rv ? row : 0;
                double yraw[BJ];
                double araw[RT];
                // the row's scale and group first: the table lookup waits
                // for them only
                const double c = (cs && Rtab) ? cs[rs] : 1.0;
                const int gi = Rtab ? grp[rs] : 0;
#pragma unroll
                for (int jt = 0; jt < BJ; ++jt) {
                    const int col = jt * 16 + li;
                    yraw[jt] = (double)T[rs * BW + (col < b ? col : 0)];
                }
                // unconditional loads (no branch between them): a tile past
                // nrt re-reads the row's first element, in tile 0's line
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const int col = rt * 16 + li;
                    araw[rt] = V[rs * ld + (rt < nrt && col < cv ? col : 0)];
                }
                // Y0 = T - c_i Rtab[g_i] (Rtab == nullptr: T already holds Y, a
                // general constraint) into the new block's columns
                double y[BJ];
#pragma unroll
                for (int jt = 0; jt < BJ; ++jt) {
                    const int col = jt * 16 + li;
                    double v = 0.0;
                    if (rv && col < b) {
                        v = yraw[jt];
                        if (Rtab) v -= c * rtab_s[gi * 32 + col];
                        if (LC) v -= corr[0][q];
                        V[row * ld + cv + col] = v;
                    }
                    y[jt] = v;
                }
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (rt < nrt) {
                        const bool ok = rv && rt * 16 + li < cv;
                        const double a = ok ? araw[rt] : 0.0;
#pragma unroll
                        for (int jt = 0; jt < BJ; ++jt) acc[rt * BJ + jt] = mfma(a, y[jt], acc[rt * BJ + jt]);
                    }
                }
            }
        } else {
            // two column tiles of the block: the registers of the hoisted
            // form above would spill
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = tile * 16 + q * 4 + lk;
                const bool rv = row < n;
                double y[BJ];
                // Rtab == nullptr: T already holds Y (general constraint)
                const double c = (rv && cs && Rtab) ? cs[row] : 1.0;
                const int gi = (rv && Rtab) ? grp[row] : 0;
#pragma unroll
                for (int jt = 0; jt < BJ; ++jt) {
                    const int col = jt * 16 + li;
                    double v = 0.0;
                    if (rv && col < b) {
                        v = (double)T[row * BW + col];
                        if (Rtab) v -= c * Rtab[gi * 32 + col];
                        V[row * ld + cv + col] = v;
                    }
                    y[jt] = v;
                }
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (rt < nrt) {
                        const int col = rt * 16 + li;
                        const double a = (rv && col < cv) ? V[row * ld + col] : 0.0;
#pragma unroll
                        for (int jt = 0; jt < BJ; ++jt) acc[rt * BJ + jt] = mfma(a, y[jt], acc[rt * BJ + jt]);
                    }
                }
            }
        }
    }
    block_store_tiles<RT * BJ <= 8>(acc, nrt * BJ, lds, part + (size_t)blockIdx.x * nrt * BJ * 256);
}

// Passes B, C, D (and the restart rotation).  Ynew = In M with
// In = V[:, coff : coff + kin] (kin a multiple of 4) and M (kin x b,
// row-major) staged in LDS; Ynew replaces Vout[:, yoff : yoff + b] (Vout may
// be V itself: every row is read completely before it is written, by the
// same wavefront).
//   GRAM: partial [V[:, 0:cv]^T Ynew (nrt x BJ tiles); Ynew^T Ynew (BJ x BJ)]
//   SYRK: partial Ynew^T Ynew
//
// With CB > 0 the pass first does the small finalisation that precedes it
// (F.mode 1: the one before pass C, 2: before pass D), every workgroup
// alike, instead of a single-workgroup kernel between the two: one
// wavefront factors the CB x CB Gram block (R = chol(G), R^{-1}) from the
// reduced tiles, M is built in LDS from them, and workgroup 0 also writes
// what the solver keeps (the projected matrix's new column block and R1 in
// mode 1, the coupling R2 R1 in mode 2, the Gram of the block and the
// failure flag).  A failed factorisation fails alike in every workgroup:
// all return, workgroup 0 raises the flag.
struct FoldArgs {
    int mode;
    const double* sumA;  // mode 1: pass A's reduced tiles (H1)
    const double* sumB;  // mode 1: pass B's (H2, then G); mode 2: pass C's (G2)
    int BJ, cv, cact, ldt;
    double thresh;
    double* R1g;  // mode 1: written; mode 2: read
    double* Gsave;
    double* T;
    double* Rc;
    int* flag;
    // mode 2 with gpart: G2 not yet reduced; the per-block partials (B x B
    // row-major each, gnblk blocks) are summed here by every workgroup
    const double* gpart;
    int gnblk;
    // pass D with XPT > 0: the next operator input (see OrthoArgs)
    void* xp;
    double* xsum;
    const int32_t* grp;
    const double* cs;
    int h;
};

template <int BJ, bool GRAM, bool SYRK, int RT = kMaxRT, int CB = 0, bool SCALE = false, int XPT = 0>
__global__ __launch_bounds__(kOrThreads) void k_pass_upd(double* V, int ld, int64_t n, int coff, int kin, int yoff,
                                                          int b, int cv, const double* __restrict__ M,
                                                          double* __restrict__ part, const int* skip, double* Vout,
                                                          int ldo, const double* __restrict__ Htiles,
                                                          const double* __restrict__ rscale, FoldArgs F) {
    if (skip && *skip) return;
    extern __shared__ double lds[];
    double* Ms = lds;                                   // [kin][BJ * 16]
    const int mld = BJ * 16;
    if constexpr (CB > 0) {
        constexpr int B = CB;
        __shared__ double Rs[B * B], Ris[B * B];
        __shared__ int bad;
        const int nrtf = (F.cv + 15) >> 4;
        const double* H2 = F.sumB;
        const double* gt = F.mode == 1 ? F.sumB + (size_t)nrtf * F.BJ * 256 : F.sumB;
        const bool w0 = blockIdx.x == 0;
        // mode 2 from the partials: every thread sums a fixed slice of the
        // blocks for one entry (eight loads in flight), the slices then in
        // order, so that every workgroup forms the same G2
        constexpr int NSL = kOrThreads / (B * B);
        __shared__ double gsl[NSL][B * B];
        if (F.gpart) {
            const int v = threadIdx.x % (B * B), q = threadIdx.x / (B * B);
            double acc = 0.0;
            int blk = q;
            for (; blk + 7 * NSL < F.gnblk; blk += 8 * NSL) {
                double x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = F.gpart[(size_t)(blk + u * NSL) * (B * B) + v];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc += x[u];
            }
            for (; blk < F.gnblk; blk += NSL) acc += F.gpart[(size_t)blk * (B * B) + v];
            gsl[q][v] = acc;
            __syncthreads();
        }
        if (threadIdx.x < 64) {
            const int j = threadIdx.x;
            double g[B], ri[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                double gv = 0.0;
                if (j < B) {
                    if (F.gpart) {
                        for (int q = 0; q < NSL; ++q) gv += gsl[q][i * B + j];
                    } else {
                        gv = tile_at(gt, F.BJ, i, j);
                    }
                }
                g[i] = gv;
                ri[i] = 0.0;
                if (w0 && j < B) F.Gsave[i * B + j] = g[i];
            }
            const bool ok = wave_chol_inv<B>(g, ri, F.thresh);
            if (j < B) {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    Rs[i * B + j] = g[i];
                    Ris[i * B + j] = ri[i];
                    if (w0 && F.mode == 1) F.R1g[i * B + j] = g[i];
                }
            }
            if (j == 0) {
                bad = ok ? 0 : 1;
                if (!ok && w0) {
                    F.flag[0] = 1;
                    F.flag[1] = F.cact;
                    F.flag[2] = F.mode;
                }
            }
        } else if (F.mode == 1 && w0) {
            // the projected matrix's new column block H1 + H2 (and its mirror
            // row block)
            for (int e = threadIdx.x - 64; e < F.cv * B; e += kOrThreads - 64) {
                const int q = e / B, j = e - q * B;
                const double h = tile_at(F.sumA, F.BJ, q, j) + tile_at(H2, F.BJ, q, j);
                F.T[(size_t)q * F.ldt + F.cact + j] = h;
                if (q < F.cact) F.T[(size_t)(F.cact + j) * F.ldt + q] = h;
            }
        }
        __syncthreads();
        if (F.mode == 1 && w0) {
            // symmetrise the diagonal block (its two triangles came from two
            // different sums)
            for (int e = threadIdx.x; e < B * B; e += kOrThreads) {
                const int i = e / B, j = e - i * B;
                if (j > i) {
                    double* x = F.T + (size_t)(F.cact + i) * F.ldt + F.cact + j;
                    double* y = F.T + (size_t)(F.cact + j) * F.ldt + F.cact + i;
                    const double mm = 0.5 * (*x + *y);
                    *x = mm;
                    *y = mm;
                }
            }
        }
        if (bad) return;
        if (F.mode == 2 && w0)
            for (int e = threadIdx.x; e < B * B; e += kOrThreads) {
                const int i = e / B, j = e - i * B;
                double acc = 0.0;
                for (int q = i; q <= j; ++q) acc += Rs[i * B + q] * F.R1g[q * B + j];
                F.Rc[e] = acc;
            }
        // M: mode 1 [-H2 R^{-1}; R^{-1}] (kin = cv + B rows), mode 2 R^{-1}
        for (int e = threadIdx.x; e < kin * mld; e += kOrThreads) {
            const int q = e / mld, j = e - q * mld;
            double acc = 0.0;
            if (j < B) {
                if (F.mode == 1 && q < F.cv) {
                    for (int t = 0; t <= j; ++t) acc -= tile_at(H2, F.BJ, q, t) * Ris[t * B + j];
                } else {
                    const int r = F.mode == 1 ? q - F.cv : q;
                    acc = Ris[r * B + j];
                }
            }
            Ms[e] = acc;
        }
    } else if (Htiles) {
        // M = [-H1; I] straight from pass A's reduced tiles (rows < cv)
        for (int e = threadIdx.x; e < kin * mld; e += kOrThreads) {
            const int r = e / mld, j = e - r * mld;
            double v = 0.0;
            if (j < b) v = r < cv ? -tile_at(Htiles, BJ, r, j) : (r - cv == j ? 1.0 : 0.0);
            Ms[e] = v;
        }
    } else {
        for (int e = threadIdx.x; e < kin * mld; e += kOrThreads) {
            const int r = e / mld, j = e - r * mld;
            Ms[e] = j < b ? M[r * b + j] : 0.0;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nrt = GRAM ? (cv + 15) >> 4 : 0;
    constexpr int NG = GRAM ? RT * BJ : 1;
    d4 accg[NG];
    d4 accs[BJ * BJ];
    d4 accx[2] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};  // XPT: group sums, groups 0-15 and 16-31
#pragma unroll
    for (int t = 0; t < NG; ++t) accg[t] = d4{0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < BJ * BJ; ++t) accs[t] = d4{0, 0, 0, 0};
    const int64_t ntiles = (n + 15) >> 4;
    const int64_t wstride = (int64_t)gridDim.x * kOrWaves;
    for (int64_t tile = (int64_t)blockIdx.x * kOrWaves + (threadIdx.x >> 6); tile < ntiles; tile += wstride) {
        const int64_t row0 = tile * 16;
        // XPT: groups and scales of the rows this lane feeds to the sums
        [[maybe_unused]] int gq[4];
        [[maybe_unused]] double cq[4];
        if constexpr (XPT > 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = row0 + 4 * q + lk;
                const int64_t rs = row < n ? row : 0;
                gq[q] = row < n ? F.grp[rs] : -1;
                cq[q] = F.cs ? F.cs[rs] : 1.0;
            }
        }
        // update: D[jt] (16 rows x 16 cols) = In(rows) M
        d4 D[BJ];
#pragma unroll
        for (int jt = 0; jt < BJ; ++jt) D[jt] = d4{0, 0, 0, 0};
        {
            const int64_t row = row0 + li;
            const bool rv = row < n;
            const double* src = V + row * ld + coff + 4 * lk;
            auto step = [&](const double4 x, int c0) {
                const double xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int kr = c0 + 4 * lk + s;
                    const double* mrow = Ms + (size_t)(kr < kin ? kr : 0) * mld;
#pragma unroll
                    for (int jt = 0; jt < BJ; ++jt) {
                        const double bm = kr < kin ? mrow[jt * 16 + li] : 0.0;
                        D[jt] = mfma(xs[s], bm, D[jt]);
                    }
                }
            };
            // two 16-column chunks per iteration: both loads in flight first
            for (int c0 = 0; c0 < kin; c0 += 32) {
                double4 x0 = make_double4(0, 0, 0, 0), x1 = make_double4(0, 0, 0, 0);
                if (rv && c0 + 4 * lk < kin) x0 = *reinterpret_cast<const double4*>(src + c0);
                if (rv && c0 + 16 + 4 * lk < kin) x1 = *reinterpret_cast<const double4*>(src + c0 + 16);
                step(x0, c0);
                step(x1, c0 + 16);
            }
        }
        // store Ynew: lane holds rows row0 + 4q + lk, column jt*16 + li
        // (optionally scaled by row: Ritz vectors in the D^{-1/2} basis)
        const int col_in_tile = li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = row0 + 4 * q + lk;
            if (row < n) {
                // (SCALE only: a conditional load here would make the
                // stores wait for the loads already in flight)
                const double rs = SCALE ? rscale[row] : 1.0;
#pragma unroll
                for (int jt = 0; jt < BJ; ++jt) {
                    const int col = jt * 16 + col_in_tile;
                    if (col < b) Vout[row * ldo + yoff + col] = SCALE ? D[jt][q] * rs : D[jt][q];
                }
            }
        }
        if constexpr (XPT > 0) {
            // the operator's next input: the compact copy, and on the matrix
            // cores S += C_tile^T X~_tile with C_tile[r][s] = c_r [g_r = s]
            // (A operand: group li, row lk of the step; B operand: this
            // lane's own output value, already in place)
            using OT = typename std::conditional<XPT == 1, float, double>::type;
            OT* xo = static_cast<OT*>(F.xp);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = row0 + 4 * q + lk;
                const OT xv = (OT)D[0][q];
                if (row < n && li < b) xo[row * b + li] = xv;
                accx[0] = mfma(gq[q] == li ? cq[q] : 0.0, (double)xv, accx[0]);
                if (F.h > 16) accx[1] = mfma(gq[q] == li + 16 ? cq[q] : 0.0, (double)xv, accx[1]);
            }
        }
        // Gram and Syrk from registers (rows past n hold zeros)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (GRAM && BJ == 1) {
                // the step's loads first, unconditionally (row 0 / column 0
                // stand in past n or cv), zeroed only where used, so that
                // they are all in flight together
                const int64_t row = row0 + 4 * q + lk;
                const bool rv = row < n;
                const int64_t rs = rv ? row : 0;
                double araw[RT];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const int col = rt * 16 + li;
                    araw[rt] = V[rs * ld + (rt < nrt && col < cv ? col : 0)];
                }
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (rt < nrt) {
                        const double a = (rv && rt * 16 + li < cv) ? araw[rt] : 0.0;
                        accg[rt] = mfma(a, D[0][q], accg[rt]);
                    }
                }
            } else if constexpr (GRAM) {
                const int64_t row = row0 + 4 * q + lk;
                const bool rv = row < n;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (rt < nrt) {
                        const int col = rt * 16 + li;
                        const double a = (rv && col < cv) ? V[row * ld + col] : 0.0;
#pragma unroll
                        for (int jt = 0; jt < BJ; ++jt) accg[rt * BJ + jt] = mfma(a, D[jt][q], accg[rt * BJ + jt]);
                    }
                }
            }
            if (GRAM || SYRK) {
#pragma unroll
                for (int i1 = 0; i1 < BJ; ++i1)
#pragma unroll
                    for (int i2 = 0; i2 < BJ; ++i2) accs[i1 * BJ + i2] = mfma(D[i1][q], D[i2][q], accs[i1 * BJ + i2]);
            }
        }
    }
    if constexpr (XPT > 0) {
        // the waves' sum tiles in wave order, one partial per block
        __shared__ double xs[kOrWaves][2 * 256];
        const int wv = threadIdx.x >> 6;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) xs[wv][t * 256 + (4 * r + lk) * 16 + li] = accx[t][r];
        __syncthreads();
        const int rowlen = xcd_row(gridDim.x), sl = xcd_slot(blockIdx.x, gridDim.x);
        for (int o = threadIdx.x; o < F.h * b; o += kOrThreads) {
            const int g = o / b, j = o - g * b;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < kOrWaves; ++w) sum += xs[w][g * 16 + j];
            F.xsum[(size_t)o * rowlen + sl] = sum;
        }
    }
    if constexpr (CB > 0 && SYRK && !GRAM) {
        // the folded pass C: its block's B x B Gram, row-major, for the next
        // pass to sum (no separate reduction)
        __syncthreads();
        block_store_tiles<true>(accs, 1, lds, nullptr);
        for (int e = threadIdx.x; e < CB * CB; e += kOrThreads)
            part[(size_t)blockIdx.x * (CB * CB) + e] = tile_at(lds, 1, e / CB, e % CB);
    } else if (GRAM || SYRK) {
        __syncthreads();  // Ms no longer needed: reuse LDS for the block sums
        const size_t gsz = (size_t)nrt * BJ * 256;
        double* dst = part + (size_t)blockIdx.x * (gsz + BJ * BJ * 256);
        if constexpr (GRAM && NG <= 8) {
            block_store_tiles2<true>(accg, nrt * BJ, accs, BJ * BJ, lds, dst);
        } else if constexpr (GRAM) {
            // (the wide Gram: the two sets one after the other, as in its
            // tuned form)
            block_store_tiles<false>(accg, nrt * BJ, lds, dst);
            __syncthreads();
            block_store_tiles<false>(accs, BJ * BJ, lds, dst + gsz);
        } else {
            block_store_tiles<true>(accs, BJ * BJ, lds, dst + gsz);
        }
    }
}

// After pass B: H2 and G = Y'^T Y' from the summed tiles.  T column block
// = H1 + H2 (pass A's and pass B's tiles; and the mirror), diagonal block
// symmetrised; R1 = chol(G) (pivot test against thresh: flag[0] = 1,
// flag[1] = cact on failure; G saved for the repair path);
// M2 = [-H2 R1^{-1}; R1^{-1}].  (H2 is O(eps) relative to the first
// projection, so G - H2^T H2 and G differ at rounding level; the second
// Cholesky-QR pass absorbs the difference.)  For B <= 16 the H2 tiles are
// first staged in LDS.
template <int B>
__global__ __launch_bounds__(256) void k_fin_b(const double* __restrict__ sumA, const double* __restrict__ sumB,
                                                int BJ, int cv, double thresh, double* __restrict__ M2,
                                                double* __restrict__ R1g, double* __restrict__ Gsave,
                                                double* __restrict__ T, int ldt, int cact, int* flag,
                                                const int* skip) {
    if (skip && *skip) return;
    constexpr int b = B;
    constexpr bool kStage = B <= 16;
    __shared__ double Ri[B * B];
    __shared__ double Hs[kStage ? (kMaxRT + 1) * 256 : 1];
    __shared__ int bad;
    const int nrt = (cv + 15) >> 4;
    const double* gt = sumB + (size_t)nrt * BJ * 256;
    const double* H2 = sumB;
    if (kStage) {
        for (int e = threadIdx.x; e < (nrt + 1) * 256; e += blockDim.x) Hs[e] = sumB[e];
        __syncthreads();
        H2 = Hs;
        gt = Hs + (size_t)nrt * 256;
    }
    for (int e = threadIdx.x; e < cv * b; e += blockDim.x) {
        const int q = e / b, j = e - q * b;
        const double h = tile_at(sumA, BJ, q, j) + tile_at(H2, BJ, q, j);
        T[(size_t)q * ldt + cact + j] = h;
        if (q < cact) T[(size_t)(cact + j) * ldt + q] = h;
    }
    __syncthreads();  // T updates (global, this workgroup) visible
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e - i * b;
        if (j > i) {
            double* a = T + (size_t)(cact + i) * ldt + cact + j;
            double* c = T + (size_t)(cact + j) * ldt + cact + i;
            const double m = 0.5 * (*a + *c);
            *a = m;
            *c = m;
        }
    }
    if (threadIdx.x < 64) {
        const int j = threadIdx.x;
        double g[B], ri[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            g[i] = j < B ? tile_at(gt, BJ, i, j) : 0.0;
            ri[i] = 0.0;
            if (j < B) Gsave[i * b + j] = g[i];
        }
        const bool ok = wave_chol_inv<B>(g, ri, thresh);
        if (j < B) {
#pragma unroll
            for (int i = 0; i < B; ++i) {
                R1g[i * b + j] = g[i];
                Ri[i * b + j] = ri[i];
            }
        }
        if (j == 0) {
            bad = ok ? 0 : 1;
            if (!ok) {
                flag[0] = 1;
                flag[1] = cact;
                flag[2] = 1;
            }
        }
    }
    __syncthreads();
    if (bad) return;
    for (int e = threadIdx.x; e < (cv + b) * b; e += blockDim.x) {
        const int q = e / b, j = e - q * b;
        double acc;
        if (q < cv) {
            acc = 0.0;
            for (int t = 0; t <= j; ++t) acc -= tile_at(H2, BJ, q, t) * Ri[t * b + j];
        } else {
            acc = Ri[(q - cv) * b + j];
        }
        M2[e] = acc;
    }
}

// After pass C: R2 = chol(G2) from the summed tiles, M3 = R2^{-1},
// coupling Rc = R2 R1.  Wavefront 0 factors while the others stage R1;
// the product Rc runs over the whole block from LDS.
template <int B>
__global__ __launch_bounds__(256) void k_fin_c(const double* __restrict__ sumC, int BJ,
                                                const double* __restrict__ R1g, double* __restrict__ M3,
                                                double* __restrict__ Rc, double* __restrict__ Gsave, int cact,
                                                int* flag, const int* skip, double thresh) {
    if (skip && *skip) return;
    constexpr int b = B;
    __shared__ double R1s[B * B], R2s[B * B];
    __shared__ int bad;
    if (threadIdx.x < 64) {
        const int j = threadIdx.x;
        double g[B], ri[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            g[i] = j < B ? tile_at(sumC, BJ, i, j) : 0.0;
            ri[i] = 0.0;
            if (j < B) Gsave[i * b + j] = g[i];
        }
        const bool ok = wave_chol_inv<B>(g, ri, thresh);
        if (j < B) {
#pragma unroll
            for (int i = 0; i < B; ++i) {
                R2s[i * b + j] = g[i];
                M3[i * b + j] = ri[i];
            }
        }
        if (j == 0) {
            bad = ok ? 0 : 1;
            if (!ok) {
                flag[0] = 1;
                flag[1] = cact;
                flag[2] = 2;
            }
        }
    } else {
        for (int e = threadIdx.x - 64; e < b * b; e += blockDim.x - 64) R1s[e] = R1g[e];
    }
    __syncthreads();
    if (bad) return;
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e - i * b;
        double acc = 0.0;
        for (int q = i; q <= j; ++q) acc += R2s[i * b + q] * R1s[q * b + j];
        Rc[e] = acc;
    }
}

// ---------------------------------------------------------------------------
// host side

// One 16-row tile per wavefront, at most 256 blocks of 512 threads (a
// block's partial tiles are reduced afterwards in a fixed order).  The Gram
// passes hold ~200 registers per lane, so a compute unit takes one block:
// fewer than 256 blocks leave compute units idle (two tiles per wavefront
// gave 196 blocks at n = 50,000 and a 0.7% slower solve).
#ifndef SF_ORTHO_TILES_PER_WAVE
#define SF_ORTHO_TILES_PER_WAVE 1
#endif
#ifndef SF_ORTHO_MAX_BLOCKS
#define SF_ORTHO_MAX_BLOCKS 256
#endif
// the operator's input-sum buffer, which the last pass may fill, holds the
// sums of at most 256 blocks
static_assert(((SF_ORTHO_MAX_BLOCKS + 7) & ~7) <= 256, "ortho_nblk() exceeds the operator's input-sum rows");
static int nblk_for(int64_t n) {
    const int64_t ntiles = (n + 15) / 16;
    constexpr int per = kOrWaves * SF_ORTHO_TILES_PER_WAVE;  // 16-row tiles per block
    int64_t g = (ntiles + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, SF_ORTHO_MAX_BLOCKS));
}

size_t ortho_part_doubles(int64_t n) {
    return (size_t)nblk_for(n) * ((size_t)kMaxRT * 2 * 256 + 4 * 256);
}

double* ortho_r1(double* small) {
    return small + (size_t)(kMaxRT * 2 + 4) * 256 * 2 + (size_t)kLdMax * kMaxBlock * 3;
}

size_t ortho_small_doubles() {
    // sumA, sumB tiles; H1; M1, M2 ((ld) x 32); R1; M3; Gsave
    return (size_t)(kMaxRT * 2 + 4) * 256 * 2 + (size_t)kLdMax * kMaxBlock * 3 + 4 * kMaxBlock * kMaxBlock;
}

// Row-tile bound of the Gram products for cv basis columns.
static int rt_bound(int cv) {
    const int nrt = (cv + 15) / 16;
    return nrt <= 4 ? 4 : nrt <= 8 ? 8 : kMaxRT;
}

template <class TT>
static void launch_a(int BJ, dim3 g, size_t lds, hipStream_t s, double* V, int ld, int64_t n, int cv, int b,
                     const TT* T, int BW, const int32_t* grp, const double* cs, const double* Rtab,
                     const double* LC, int lcw, int m, const double* Utab, double* part, const int* skip) {
#define SF_PASS_A(BJV, RTV)                                                                                 \
    k_pass_a<BJV, TT, RTV><<<g, kOrThreads, lds, s>>>(V, ld, n, cv, b, T, BW, grp, cs, Rtab, LC, lcw, m, Utab, \
                                                      part, skip)
    const int rt = rt_bound(cv);
    if (BJ == 1) {
        if (rt == 4)
            SF_PASS_A(1, 4);
        else if (rt == 8)
            SF_PASS_A(1, 8);
        else
            SF_PASS_A(1, kMaxRT);
    } else {
        if (rt == 4)
            SF_PASS_A(2, 4);
        else if (rt == 8)
            SF_PASS_A(2, 8);
        else
            SF_PASS_A(2, kMaxRT);
    }
#undef SF_PASS_A
}

template <bool GRAM, bool SYRK>
static void launch_upd(int BJ, dim3 g, size_t lds, hipStream_t s, double* V, int ld, int64_t n, int coff, int kin,
                       int yoff, int b, int cv, const double* M, double* part, const int* skip,
                       double* Vout = nullptr, int ldo = 0, const double* Htiles = nullptr,
                       const double* rscale = nullptr) {
    if (!Vout) {
        Vout = V;
        ldo = ld;
    }
#define SF_PASS_U(BJV, RTV)                                                                                   \
    do {                                                                                                        \
        if (!GRAM && !SYRK && rscale)                                                                           \
            k_pass_upd<BJV, GRAM, SYRK, RTV, 0, true><<<g, kOrThreads, lds, s>>>(                               \
                V, ld, n, coff, kin, yoff, b, cv, M, part, skip, Vout, ldo, Htiles, rscale, FoldArgs{});        \
        else                                                                                                    \
            k_pass_upd<BJV, GRAM, SYRK, RTV><<<g, kOrThreads, lds, s>>>(V, ld, n, coff, kin, yoff, b, cv, M, part, \
                                                                        skip, Vout, ldo, Htiles, nullptr,       \
                                                                        FoldArgs{});                            \
    } while (0)
    // the row-tile bound matters only for the Gram product
    const int rt = GRAM ? rt_bound(cv) : kMaxRT;
    if constexpr (!GRAM && !SYRK) {
        // up to 48 output columns (the restart rotation's slices)
        if (BJ == 3) {
            SF_PASS_U(3, kMaxRT);
            return;
        }
    }
    if (BJ == 1) {
        if (rt == 4)
            SF_PASS_U(1, 4);
        else if (rt == 8)
            SF_PASS_U(1, 8);
        else
            SF_PASS_U(1, kMaxRT);
    } else {
        if (rt == 4)
            SF_PASS_U(2, 4);
        else if (rt == 8)
            SF_PASS_U(2, 8);
        else
            SF_PASS_U(2, kMaxRT);
    }
#undef SF_PASS_U
}

// Pass C (SYRK) or D with the finalisation before it folded in (CB = b <= 8).
// xpt (pass D only): 1 or 2 also writes the operator's next input, its
// compact copy in float or double and the group sums.
template <bool SYRK>
static void launch_fold(int b, dim3 g, size_t lds, hipStream_t s, double* V, int ld, int64_t n, int coff, int kin,
                        int yoff, int cv, double* part, const int* skip, const FoldArgs& F, int xpt = 0) {
#define SF_FOLD(BJV, CBV, XP)                                                                                   \
    k_pass_upd<BJV, false, SYRK, kMaxRT, CBV, false, XP><<<g, kOrThreads, lds, s>>>(                           \
        V, ld, n, coff, kin, yoff, b, cv, nullptr, part, skip, V, ld, nullptr, nullptr, F)
#define SF_FOLD_X(CBV)                     \
    do {                                   \
        if (SYRK || xpt == 0)              \
            SF_FOLD(1, CBV, 0);            \
        else if (xpt == 1)                 \
            SF_FOLD(1, CBV, SYRK ? 0 : 1); \
        else                               \
            SF_FOLD(1, CBV, SYRK ? 0 : 2); \
    } while (0)
    if (b == 4)
        SF_FOLD_X(4);
    else
        SF_FOLD_X(8);
#undef SF_FOLD_X
#undef SF_FOLD
}

// (a multiple of 8, so that every slot of the output-major sums is written:
// their reader then keeps eight loads in flight)
int ortho_nblk(int64_t n) { return (nblk_for(n) + 7) & ~7; }

int ortho_expand(const OrthoArgs& a) {
    const int b = a.b, cv = a.cv, BJ = b > 16 ? 2 : 1;
    const int64_t n = a.n;
    if (cv % 4 != 0 || a.ld % 4 != 0 || cv + 2 * b > a.ld + b || cv > kLdMax)
        return set_error(SFAIRSC_E_ARG, "internal: bad orthogonalisation shape cv=%d ld=%d b=%d", cv, a.ld, b);
    const int nblk = nblk_for(n);
    const int nrt = (cv + 15) / 16;
    hipStream_t s = a.stream;
    double* sumA = a.small;
    double* sumB = sumA + (size_t)(kMaxRT * 2 + 4) * 256;
    double* H1 = sumB + (size_t)(kMaxRT * 2 + 4) * 256;
    double* M1 = H1 + (size_t)kLdMax * kMaxBlock;
    double* M2 = M1 + (size_t)kLdMax * kMaxBlock;
    double* R1 = M2 + (size_t)kLdMax * kMaxBlock;
    double* M3 = R1 + kMaxBlock * kMaxBlock;
    const int cact = cv - b;

    // pass A
    const int OA = nrt * BJ * 256;
    size_t ldsA = store_lds_bytes(nrt * BJ);
    if (a.lc && (b > 16 || a.lcw < 4 || a.lcw % 4 != 0 || a.m > a.lcw || a.m > kMaxGroups - 1 || !a.utab))
        return set_error(SFAIRSC_E_ARG, "internal: bad constraint image lcw=%d m=%d", a.lcw, a.m);
    if (a.t_is_float)
        launch_a<float>(BJ, nblk, ldsA, s, a.V, a.ld, n, cv, b, (const float*)a.t, a.BW, a.grp, a.cs, a.rtab, a.lc,
                        a.lcw, a.m, a.utab, a.part, a.flag);
    else
        launch_a<double>(BJ, nblk, ldsA, s, a.V, a.ld, n, cv, b, (const double*)a.t, a.BW, a.grp, a.cs, a.rtab,
                         a.lc, a.lcw, a.m, a.utab, a.part, a.flag);
    k_reduce_partials<<<reduce_grid(OA), kRedElems * kRedSlices, 0, s>>>(a.part, nblk, OA, sumA, a.flag);

    // pass B: Y' = [V | Y0] [-H1; I] (built from pass A's tiles), Gram + Syrk
    const int kin = cv + b;
    const int OB = (nrt * BJ + BJ * BJ) * 256;
    size_t ldsB = std::max((size_t)kin * BJ * 16 * sizeof(double), store_lds_bytes(nrt * BJ + BJ * BJ));
    launch_upd<true, true>(BJ, nblk, ldsB, s, a.V, a.ld, n, 0, kin, cv, b, cv, nullptr, a.part, a.flag, nullptr, 0,
                           sumA);
    k_reduce_partials<<<reduce_grid(OB), kRedElems * kRedSlices, 0, s>>>(a.part, nblk, OB, sumB, a.flag);

    const int OC = BJ * BJ * 256;
    size_t ldsC = std::max((size_t)kin * BJ * 16 * sizeof(double), store_lds_bytes(BJ * BJ));
    size_t ldsD = (size_t)b * BJ * 16 * sizeof(double);
    if (b <= 8) {
        // pass C: R1 = chol(G) and M2 = [-H2 R1^{-1}; R1^{-1}] (folded in),
        // then Y1 = [V | Y'] M2 and its Syrk
        FoldArgs F{1, sumA, sumB, BJ, cv, cact, a.ldt, a.thresh, R1, a.gsave, a.T, a.rc, a.flag};
        launch_fold<true>(b, nblk, ldsC, s, a.V, a.ld, n, 0, kin, cv, cv, a.part, a.flag, F);
        // pass D: G2 summed from pass C's block partials, R2 = chol(G2), the
        // coupling R2 R1 (folded in), Y2 = Y1 R2^{-1}
        F.mode = 2;
        F.sumB = nullptr;
        F.gpart = a.part;
        F.gnblk = nblk;
        F.thresh = 0.25;
        int xpt = 0;
        if (a.xp) {
            if (!a.xsum || !a.grp || a.h < 2 || a.h > kMaxGroups)
                return set_error(SFAIRSC_E_ARG, "internal: bad operator-input request h=%d", a.h);
            F.xp = a.xp;
            F.xsum = a.xsum;
            F.grp = a.grp;
            F.cs = a.cs;
            F.h = a.h;
            xpt = a.xp_float ? 1 : 2;
        }
        launch_fold<false>(b, xpt ? ortho_nblk(n) : nblk, ldsD, s, a.V, a.ld, n, cv, b, cv, cv, nullptr, a.flag, F,
                           xpt);
        SF_HIP(hipGetLastError());
        return SFAIRSC_OK;
    }
    // wider blocks: the factorisations in single-workgroup kernels (one
    // wavefront per SIMD; folded into a pass their registers would spill)
#define SF_FINB(BB) \
    k_fin_b<BB><<<1, 256, 0, s>>>(sumA, sumB, BJ, cv, a.thresh, M2, R1, a.gsave, a.T, a.ldt, cact, a.flag, a.flag)
    if (b == 16)
        SF_FINB(16);
    else
        SF_FINB(32);
#undef SF_FINB
    launch_upd<false, true>(BJ, nblk, ldsC, s, a.V, a.ld, n, 0, kin, cv, b, cv, M2, a.part, a.flag);
    k_reduce_partials<<<reduce_grid(OC), kRedElems * kRedSlices, 0, s>>>(a.part, nblk, OC, sumA, a.flag);
    if (b == 16)
        k_fin_c<16><<<1, 256, 0, s>>>(sumA, BJ, R1, M3, a.rc, a.gsave, cact, a.flag, a.flag, 0.25);
    else
        k_fin_c<32><<<1, 256, 0, s>>>(sumA, BJ, R1, M3, a.rc, a.gsave, cact, a.flag, a.flag, 0.25);
    // pass D: Y2 = Y1 R2^{-1}
    launch_upd<false, false>(BJ, nblk, ldsD, s, a.V, a.ld, n, cv, b, cv, b, cv, M3, nullptr, a.flag);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

// Start block: Cholesky-QR twice of V[:, 0:b] in place on the matrix
// cores (Syrk pass, Cholesky, update + Syrk, Cholesky, update).  ident is
// the b x b identity, R1 receives the first factor (its pivot test uses
// thresh), flag[0] = 1 and flag[1] = -1 (no expansion's column) if either
// factorisation fails.
int ortho_start(double* V, int ld, int64_t n, int b, const double* ident, double thresh, double* part, double* small,
                double* gsave, double* rc, int* flag, hipStream_t s) {
    const int BJ = b > 16 ? 2 : 1;
    const int nblk = nblk_for(n);
    double* sumA = small;
    double* R1 = ortho_r1(small);
    double* M3 = R1 + kMaxBlock * kMaxBlock;
    double* M = sumA + (size_t)(kMaxRT * 2 + 4) * 256 * 2;  // the H1 slot: b x b
    const int OS = BJ * BJ * 256;
    const size_t lds = std::max((size_t)b * BJ * 16 * sizeof(double), store_lds_bytes(BJ * BJ));
#define SF_FINC(BB, R1IN, MOUT, TH)                                                                            \
    k_fin_c<BB><<<1, 256, 0, s>>>(sumA, BJ, R1IN, MOUT, rc, gsave, -1, flag, flag, TH)
#define SF_FINC_B(R1IN, MOUT, TH)                \
    switch (b) {                                 \
        case 4: SF_FINC(4, R1IN, MOUT, TH); break;   \
        case 8: SF_FINC(8, R1IN, MOUT, TH); break;   \
        case 16: SF_FINC(16, R1IN, MOUT, TH); break; \
        default: SF_FINC(32, R1IN, MOUT, TH); break; \
    }
    // G = Y^T Y (Y unchanged: multiplied by the identity)
    launch_upd<false, true>(BJ, nblk, lds, s, V, ld, n, 0, b, 0, b, 0, ident, part, flag);
    k_reduce_partials<<<reduce_grid(OS), kRedElems * kRedSlices, 0, s>>>(part, nblk, OS, sumA, flag);
    // R = chol(G) (coupling against the identity), M = R^{-1}
    SF_FINC_B(ident, M, thresh);
    // Y <- Y M with the Gram of the result, then the second factor
    launch_upd<false, true>(BJ, nblk, lds, s, V, ld, n, 0, b, 0, b, 0, M, part, flag);
    k_reduce_partials<<<reduce_grid(OS), kRedElems * kRedSlices, 0, s>>>(part, nblk, OS, sumA, flag);
    SF_FINC_B(ident, M3, 0.25);
    launch_upd<false, false>(BJ, nblk, (size_t)b * BJ * 16 * sizeof(double), s, V, ld, n, 0, b, 0, b, 0, M3,
                             nullptr, flag);
#undef SF_FINC_B
#undef SF_FINC
    (void)R1;
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

// Thick restart: Vout[:, 0:p] = V[:, 0:c] Z[:, 0:p] and Vout[:, p:p+b] =
// V[:, c:c+b], with the factor laid out as rot_whole selects: one
// matrix-core update per slice of the whole factor [Z 0; 0 I] (V read once
// per slice), or per 32-column slice of Z plus one update that moves the
// next block.
int ortho_rotate(double* V, double* Vout, int ld, int64_t n, int c, int p, int b, const double* Mchunks,
                 hipStream_t s, const int* skip) {
    if (c % 4 != 0 || b % 4 != 0 || ld % 4 != 0 || c + b > kLdMax || p + b > ld || c + b > ld)
        return set_error(SFAIRSC_E_ARG, "internal: bad rotation shape c=%d p=%d b=%d", c, p, b);
    const int nblk = nblk_for(n);
    const double* q = Mchunks;
    if (rot_whole(c, b)) {
        const int kin = c + b, pw = p + b;
        for (int j0 = 0; j0 < pw; j0 += 48) {
            const int wt = std::min(48, pw - j0);
            const int BJ = (wt + 15) / 16;
            const size_t lds = (size_t)kin * BJ * 16 * sizeof(double);
            launch_upd<false, false>(BJ, nblk, lds, s, V, ld, n, 0, kin, j0, wt, kin, q, nullptr, skip, Vout, ld);
            q += (size_t)kin * wt;
        }
    } else {
        for (int j0 = 0; j0 < p; j0 += 32) {
            const int wt = std::min(32, p - j0);
            const int BJ = wt > 16 ? 2 : 1;
            const size_t lds = (size_t)c * BJ * 16 * sizeof(double);
            launch_upd<false, false>(BJ, nblk, lds, s, V, ld, n, 0, c, j0, wt, c, q, nullptr, skip, Vout, ld);
            q += (size_t)c * wt;
        }
        const int BJ = b > 16 ? 2 : 1;
        launch_upd<false, false>(BJ, nblk, (size_t)b * BJ * 16 * sizeof(double), s, V, ld, n, c, b, p, b, c, q,
                                 nullptr, skip, Vout, ld);
    }
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

int ortho_product(double* V, int ld, int64_t n, int kin, const double* M, int b, double* Out, int ldo,
                  const double* rscale, hipStream_t s) {
    if (kin % 4 != 0 || ld % 4 != 0 || kin > kLdMax || b < 1 || b > 32)
        return set_error(SFAIRSC_E_ARG, "internal: bad product shape kin=%d b=%d", kin, b);
    const int BJ = b > 16 ? 2 : 1;
    // no partial sums here: one 16-row tile per wavefront, for latency
    const int64_t g = ((n + 15) / 16 + kOrWaves - 1) / kOrWaves;
    const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
    launch_upd<false, false>(BJ, nblk, (size_t)kin * BJ * 16 * sizeof(double), s, V, ld, n, 0, kin, 0, b, kin, M,
                             nullptr, nullptr, Out, ldo, nullptr, rscale);
    SF_HIP(hipGetLastError());
    return SFAIRSC_OK;
}

}  // namespace sfairsc
