/*
 * sfairsc.h — C ABI of the s-FairSC GPU library (AMD MI355X / gfx950).
 *
 * Scalable fair spectral clustering (Wang, Lu, Davidson and Bai, "Scalable
 * Spectral Clustering with Group Fairness Constraints", AISTATS 2023).
 *
 * Problem (Section 2.2, eq. normal-prob-fair): given an undirected graph with
 * weighted adjacency W (w_ij >= 0, w_ii = 0), degrees d = W 1, Laplacian
 * L = D - W and a partition of the vertices into h groups, find the k
 * eigenpairs of smallest eigenvalue of L restricted to null(F^T), where F is
 * the n x (h-1) group-fairness matrix of Lemma 2.1 (F_0 = G - 1 z^T with
 * z = G^T 1 / n, first h-1 columns).
 *
 *   normalized = 1: the paper's Alg. 3.  X = D^{1/2} H, C = D^{-1/2} F,
 *                   L_n = D^{-1/2} L D^{-1/2}; outputs H = D^{-1/2} X
 *                   (H^T D H = I, F^T H = 0).
 *   normalized = 0: the same derivation with D replaced by I in the
 *                   constraint: C = F, operator L, H = X (H^T H = I).
 *
 * Method (Section 3.3-3.4, Alg. 3): the k smallest eigenpairs of the deflated
 * operator L^sigma = P (L_n - sigma I) P + sigma I (eq. asigma), with
 * P = I - C (C^T C)^{-1} C^T applied from the group labels (eq. mv-Pw;
 * or from an orthonormal basis of range(C) for a general F, see
 * sfairsc_graph_set_constraint) and
 * sigma = ||L_n||_1 (Appendix B.3), found by a block Krylov-Schur
 * (thick-restart Lanczos) eigensolver; then k-means on the rows of H
 * (Alg. 3 step 4).  Proposition 3.3 makes these exactly the fair solution.
 *
 * Conventions shared by every entry point:
 *   - Pointers documented "device" must point to GPU memory on the current
 *     HIP device; "host" pointers to CPU memory.
 *   - Dense blocks: "row-major n x b" means element (i, j) at [i * b + j];
 *     "column-major n x k" means element (i, j) at [j * n + i].
 *   - All work is enqueued on `stream` (0 = the null stream) and is
 *     asynchronous unless stated; functions that return host values
 *     synchronise `stream` before returning.
 *   - Every function returns SFAIRSC_OK (0) or a negative status; on error
 *     sfairsc_last_error() gives a message (per host thread).  No C++
 *     exception crosses this interface.
 *   - A graph handle is not thread-safe: calls on one handle must not
 *     overlap.  Calls on distinct handles may.
 */
#ifndef SFAIRSC_H
#define SFAIRSC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
enum {
    SFAIRSC_OK = 0,
    SFAIRSC_E_ARG = -1,           /* invalid argument or malformed CSR           */
    SFAIRSC_E_ASYM = -2,          /* W not symmetric (structure or value)        */
    SFAIRSC_E_EMPTY_GROUP = -3,   /* some group has no vertex (eq. groupdef)     */
    SFAIRSC_E_ISOLATED = -4,      /* d_i = 0 with normalized = 1 (D must be p.d.) */
    SFAIRSC_E_NOT_CONVERGED = -5, /* outputs hold the best current pairs         */
    SFAIRSC_E_DEGENERATE = -6,    /* theta_k ~ theta_{k+1}: outputs written, the
                                     k-dimensional subspace is not determined   */
    SFAIRSC_E_HIP = -7,           /* a HIP runtime call failed                   */
    SFAIRSC_E_NOMEM = -8          /* device allocation failed                    */
};

enum { SFAIRSC_F32 = 0, SFAIRSC_F64 = 1 };              /* value dtypes */
enum { SFAIRSC_PREC_FP64 = 0, SFAIRSC_PREC_MIXED = 1 }; /* arithmetic   */

typedef struct sfairsc_graph* sfairsc_graph_t;

/* ---- graph ----------------------------------------------------------- */

/*
 * Build a graph handle (Alg. 3 steps 1-2: L, L_n and C; Lemma 2.1: F).
 *
 * rowptr  device int32[n+1]   CSR row pointers of W, rowptr[0] = 0,
 *                             rowptr[n] = nnz, non-decreasing.
 * colidx  device int32[nnz]   column indices, strictly increasing in a row,
 *                             no diagonal entry (w_ii = 0).
 * values  device [nnz]        w_ij >= 0, finite; float (value_dtype =
 *                             SFAIRSC_F32) or double (SFAIRSC_F64).  Both
 *                             stored copies (i,j) and (j,i) must be present
 *                             and bitwise equal.
 * group   device int32[n]     group label of each vertex in [0, h); every
 *                             group non-empty.  h >= 1 (h = 1 is plain
 *                             spectral clustering, Alg. 1).
 * normalized                  1: Alg. 3 (L_n, C = D^{-1/2} F); 0: L, C = F.
 *
 * The library copies every input into its own device buffers, so the caller
 * may free them once this returns.  Validation runs on the device; the call
 * synchronises `stream`.  Errors: E_ARG (sizes, ranges, CSR structure,
 * non-finite or negative weights, h > 32), E_ASYM, E_EMPTY_GROUP,
 * E_ISOLATED (normalized only), E_NOMEM, E_HIP.  *out is NULL on error.
 */
int sfairsc_graph_create(sfairsc_graph_t* out, int64_t n, int64_t nnz,
                         const int32_t* rowptr, const int32_t* colidx,
                         const void* values, int value_dtype,
                         const int32_t* group, int32_t h, int normalized,
                         hipStream_t stream);

/* Release every device buffer of the handle (synchronises the device). */
void sfairsc_graph_destroy(sfairsc_graph_t g);

/*
 * Replace the handle's constraint by a general matrix F (n x m): the fair
 * problem becomes min tr(H^T L H) under F^T H = 0 (eq. normal-prob-fair
 * with any F), as in the paper's random-Laplacian workload, whose F is a
 * random placeholder (Section 5), and in overlapping groups (Section 6).
 * The group labels given at creation are no longer used by any solve.
 *
 * F          device double, column-major n x m, leading dimension ldf >= n;
 *            read during the call only.  1 <= m <= 32.
 * center     1: use F_0 = F - 1 mu^T with mu the column means (for 0/1
 *            memberships G, possibly overlapping, this is Lemma 2.1's
 *            G - 1 z^T with every column kept); 0: use F as given.
 * rank_tol   singular values of C = D^{-1/2} F (normalized) or C = F below
 *            rank_tol times the largest are treated as zero, the
 *            rank-revealing step for a rank-deficient F; 0 selects 1e-6.
 *            Must lie in [1e-7, 1) (the rank is read from the Gram matrix).
 * rank       host int32 (may be NULL): the rank r kept.  Solves then allow
 *            k <= n - r and sfairsc_graph_query reports r.
 *
 * The handle keeps an orthonormal basis Q (n x r, padded to 4, 8, 16 or 32
 * columns) of range(C); the operator applies P = I - Q Q^T.  Batched solves
 * hand such handles to the single-graph solver.  Synchronises `stream`.
 * Errors: E_ARG (sizes, rank_tol, F zero or non-finite, r >= n; the handle
 * then has no general constraint, its group constraint applies again),
 * E_NOMEM, E_HIP.
 */
int sfairsc_graph_set_constraint(sfairsc_graph_t g, const double* F,
                                 int64_t ldf, int32_t m, int32_t center,
                                 double rank_tol, int32_t* rank,
                                 hipStream_t stream);

/*
 * Replace the handle's constraint by a sparse 0/1 membership matrix G
 * (n x m, a vertex may belong to several groups, m up to 2^20) whose
 * projection is computed iteratively: P w = w - C x with x from LSQR on
 * min ||C x - w||_2 (Section 3.4 (ii): an iterative least-squares solver
 * inside the eigensolver, an inner-outer iteration), where
 * C = D^{-1/2} (G - 1 z^T) (normalized) or G - 1 z^T, z = G^T 1 / n
 * (center = 1, Lemma 2.1's centring with every column kept) or z = 0.
 * For many groups this replaces both the closed form of the group path
 * (h <= 32) and the dense basis of sfairsc_graph_set_constraint (m <= 32).
 *
 * rowptr, colidx  device int32 CSR of G: rowptr[n+1] (rowptr[0] = 0,
 *            non-decreasing), colidx[nnz] in [0, m), strictly increasing
 *            within a row.  Read during the call only (copied to the host
 *            to build the member lists).
 * inner_tol  LSQR stops a column when its estimate of
 *            ||C^T r|| / (||C||_est ||r||) falls to inner_tol; 0 selects
 *            1e-12.  The projection error is then about
 *            inner_tol * cond(C) * ||r||: the eigensolver's tolerance
 *            should stay above it.  Must lie in [1e-15, 1).
 * max_inner  LSQR steps per solve (0 selects 200), at most 1e5.
 *
 * Each projection is one cooperative launch (every step's reductions in a
 * fixed order).  Solves allow k <= n - m (m bounds the rank of C from
 * above; LSQR needs no rank).  sfairsc_graph_query reports m.  Batched
 * solves hand such handles to the single-graph solver.  Synchronises
 * `stream`.  Errors: E_ARG (sizes, CSR structure, tolerances; the handle
 * then has no membership constraint, its group constraint applies again),
 * E_NOMEM, E_HIP.
 */
int sfairsc_graph_set_memberships(sfairsc_graph_t g, int32_t m,
                                  const int32_t* rowptr, const int32_t* colidx,
                                  int32_t center, double inner_tol,
                                  int32_t max_inner, hipStream_t stream);

/*
 * LSQR counters of a handle with a membership constraint, accumulated over
 * every projection since the constraint was set: out[0] solves (one per
 * projection of a block), out[1] LSQR steps in total, out[2] the most steps
 * of one solve, out[3] columns that reached max_inner unconverged.
 * Synchronises `stream`.  Errors: E_ARG (no membership constraint), E_HIP.
 */
int sfairsc_lsqr_stats(sfairsc_graph_t g, int64_t* out, hipStream_t stream);

typedef struct sfairsc_graph_stats {
    int64_t n, nnz;
    int32_t h, normalized, value_dtype;
    int32_t constraint_rank; /* h - 1, or the rank of a general F          */
    double sigma;      /* ||L_n||_1 (normalized) or ||L||_1 = 2 max_i d_i   */
    double min_degree, max_degree;
} sfairsc_graph_stats;

/* Host copy of the handle's scalar properties (no device work). */
int sfairsc_graph_query(sfairsc_graph_t g, sfairsc_graph_stats* out);

/* ---- operator (Section 3.4, implementation issues (i)-(ii)) ----------- */

/*
 * Y = L^sigma X = P (L_n (P X)) - sigma P X + sigma X   (eq. asigma).
 *
 * X, Y   device double, row-major n x b, 1 <= b <= 32, must not overlap.
 * precision  SFAIRSC_PREC_FP64: all arithmetic in double.
 *            SFAIRSC_PREC_MIXED: P X is rounded to float and the sparse
 *            product L_n (P X) runs in float with float accumulation; the
 *            projections and the deflation stay in double.
 * sigma  shift; <= 0 selects the handle's ||L_n||_1.
 * Asynchronous.  Errors: E_ARG, E_NOMEM, E_HIP.
 */
int sfairsc_apply_operator(sfairsc_graph_t g, const double* X, double* Y,
                           int32_t b, int precision, double sigma,
                           hipStream_t stream);

/*
 * The same Y = L^sigma X as sfairsc_apply_operator, through the same
 * kernels, for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc.  Its
 * scratch (group-sum partials, the projected input and the sparse product,
 * the small tables) lives in a 64 MiB device array inside the library, one
 * copy per GPU, held until the process ends; nothing is allocated or freed
 * (the graph handle must already exist).
 *
 * Limits: the group constraint only (a handle with
 * sfairsc_graph_set_constraint or sfairsc_graph_set_memberships gives
 * E_ARG), and 2 n BW s plus the partials within 64 MiB, with BW = b rounded
 * up to 4, 8, 16 or 32 and s = 4 (mixed) or 8 (FP64) bytes: about n <= 2
 * million at b = 4 mixed, 500,000 at b = 8 FP64, 125,000 at b = 32 FP64.
 * A larger problem returns E_ARG and launches nothing.
 * All calls on one GPU share the array: calls that overlap in time on one
 * GPU (different streams or threads) race and must be serialised by the
 * caller.  Every scratch element a call reads is written earlier in the same
 * call, so nothing carries over from the previous call.
 * Arguments, layout and the other errors as sfairsc_apply_operator.
 */
int sfairsc_apply_operator_noalloc(sfairsc_graph_t g, const double* X,
                                   double* Y, int32_t b, int precision,
                                   double sigma, hipStream_t stream);

/*
 * T = L_n X (normalized) or T = L X (unnormalized) with no projection: the
 * sparse product alone (the matrix-vector product of Section 3.4 (i)).
 * X, T   device row-major n x b, 1 <= b <= 32, float for SFAIRSC_PREC_MIXED
 *        and double for SFAIRSC_PREC_FP64; must not overlap.
 * Asynchronous.  Errors: E_ARG, E_NOMEM, E_HIP.
 */
int sfairsc_spmm(sfairsc_graph_t g, const void* X, void* T, int32_t b,
                 int precision, hipStream_t stream);

/* ---- eigensolver (Alg. 3 step 3) -------------------------------------- */

typedef struct sfairsc_eigs_opts {
    int32_t block_width;   /* b in {4, 8, 16, 32}; 0 = automatic          */
    int32_t max_basis;     /* basis columns before a restart (<= 192);
                              0 = automatic                                */
    int32_t max_restarts;  /* 0 = automatic (2000)                        */
    int32_t keep;          /* Ritz vectors kept at a restart; 0 = auto:
                              k + 0.35 (basis - k) for an FP64 solve with
                              b <= 16, max(k + b, k + (basis - k) / 2)
                              otherwise (rounded up to a multiple of 4)   */
    uint64_t seed;         /* seed of the random start block              */
    double sigma;          /* Hotelling shift; <= 0 selects ||L_n||_1     */
    int32_t certify;       /* 1: recompute the final residuals with an
                              FP64 operator application                   */
    int32_t time_kernels;  /* 1: time every SpMM launch with HIP events
                              (reported in sfairsc_eigs_info)             */
    const double* x0;      /* optional device row-major n x b0 warm start */
    int32_t b0;            /* columns of x0 (0 = none), <= block width;
                              an automatic block width is widened to it   */
    int32_t reserved;
} sfairsc_eigs_opts;

typedef struct sfairsc_eigs_info {
    int32_t restarts;          /* Rayleigh-Ritz / restart cycles           */
    int32_t converged;         /* wanted pairs meeting the tolerance       */
    int32_t block_steps;       /* block Krylov expansions                  */
    int32_t breakdowns;        /* rank-deficient residual blocks repaired  */
    int64_t operator_applies;  /* columns multiplied by L^sigma            */
    int64_t spmm_launches[2];  /* [0] FP64 SpMM launches, [1] FP32         */
    double spmm_ms[2];         /* summed SpMM kernel time (time_kernels)   */
    double max_rel_residual;   /* max_i ||L^s x_i - theta_i x_i|| / sigma  */
    double sigma;              /* shift used                               */
    double gap_ratio;          /* (theta_{k+1} - theta_k) / sigma, last RR */
    double phase1_ms;          /* mixed precision: host wall time of the
                                  FP32-SpMM phase; 0 otherwise             */
    double rr_ms;              /* time_kernels: GPU time of the Rayleigh-
                                  Ritz kernels (small dense eigensolves,
                                  with the look-ahead operator application
                                  beside them on a second stream), all
                                  phases; 0 otherwise                       */
    /* time_kernels: summed GPU time between event pairs around the block
       steps' operator applications (projections, sparse product, C^T T),
       their orthogonalisation (CGS2 + Cholesky-QR) and the restart
       rotations; 0 otherwise */
    double operator_ms, ortho_ms, restart_ms;
    int32_t degenerate;        /* 1: gap_ratio <= 100 tol (the status is then
                                  SFAIRSC_E_DEGENERATE unless not converged) */
    int32_t restarts_unpredicted; /* restarts whose kept count the rule did
                                  not give (equal Ritz values extended it):
                                  their rotation waited for the host         */
} sfairsc_eigs_info;

/* Fill *opts with the defaults (all automatic, seed 0, certify 1). */
void sfairsc_eigs_opts_init(sfairsc_eigs_opts* opts);

/*
 * The k smallest eigenpairs of L^sigma (Proposition 3.3: for sigma above
 * the k-th fair eigenvalue they are the fair eigenpairs).
 *
 * k        1 <= k <= n - h + 1 and k <= 64.
 * tol      pair i is converged when ||L^sigma x_i - theta_i x_i||_2 <=
 *          tol * sigma (a backward error, as ||L^sigma||_2 = sigma).
 * precision SFAIRSC_PREC_FP64, or SFAIRSC_PREC_MIXED: the basis is built
 *          with float sparse products; if the FP64 residuals then miss tol
 *          the solve continues with double sparse products, warm-started
 *          from the float result, so both precisions meet the same tol.
 * opts     may be NULL (defaults).
 * eigvals  host double[k], ascending.
 * H        device double, column-major n x k: H = D^{-1/2} X (normalized)
 *          or X; each column's largest-magnitude entry is positive (lowest
 *          index on ties).
 * info     may be NULL.
 * Synchronises `stream`.  Returns SFAIRSC_E_NOT_CONVERGED (outputs and info
 * still written: the best current pairs) if max_restarts is reached, else
 * SFAIRSC_E_DEGENERATE (outputs and info written, info->degenerate = 1) when
 * the relative gap (theta_{k+1} - theta_k) / sigma of the last Rayleigh-Ritz
 * step is at most 100 tol: Proposition 3.3 and any subspace-angle bound need
 * lambda_k < lambda_{k+1}, so the returned k vectors are one basis of a
 * subspace that is not determined (a multiple eigenvalue split by k).  The
 * handle keeps its workspace for later calls (no allocation after the
 * first call of a given shape).  Errors also: E_ARG, E_NOMEM, E_HIP.
 */
int sfairsc_eigs(sfairsc_graph_t g, int32_t k, double tol, int precision,
                 const sfairsc_eigs_opts* opts, double* eigvals, double* H,
                 sfairsc_eigs_info* info, hipStream_t stream);

/* ---- batched solves (many independent graphs) -------------------------- */

/*
 * Per-graph outcome of sfairsc_eigs_batched.
 */
typedef struct sfairsc_batch_info {
    int32_t status;        /* SFAIRSC_OK, SFAIRSC_E_NOT_CONVERGED or
                              SFAIRSC_E_DEGENERATE (gap_ratio <= 100 tol)   */
    int32_t path;          /* 0: solved in the batched launch;
                              1: solved by sfairsc_eigs (the launch could
                              not take the graph or did not finish it)      */
    int32_t batch_status;  /* the launch's outcome: 0 converged, 1 not
                              converged, 2 rank-deficient block, 3 FP64
                              certification above tol, 4 shape not
                              supported, 5 handed off (one of the last
                              three graphs of a batch of >= 32: finished by
                              sfairsc_eigs from the launch's current Ritz
                              vectors); -1 not attempted                    */
    int32_t block_width;   /* configuration used in the launch             */
    int32_t max_basis;
    int32_t spmm_rows;     /* CSR rows a wavefront handles together        */
    int32_t from_table;    /* 1: configuration from the tuning table       */
    int32_t double_spmm;   /* 1: double sparse products in the launch      */
    int32_t restarts, block_steps, converged, reserved;
    double max_rel_residual;  /* max_i ||L^s x_i - theta_i x_i|| / sigma   */
    double sigma;
    double gap_ratio;      /* (theta_{k+1} - theta_k) / sigma              */
    double graph_ms;       /* wall time from the launch's start until the
                              graph left its block steps                   */
    double batch_ms;       /* wall time of the whole launch                */
    double phase_ms[8];    /* compute-unit milliseconds spent on this graph
                              (busy time of the workgroups that worked on
                              it; each holds a whole compute unit) by
                              phase: operator, Gram-Schmidt passes A, B,
                              C, D (with the next block's group sums),
                              Rayleigh-Ritz, restart rotation, start block
                              and output                                   */
} sfairsc_batch_info;

/*
 * The k[i] smallest fair eigenpairs of each of `count` independent graphs
 * (the problem of sfairsc_eigs for every graph), solved in ONE cooperative
 * persistent kernel launch (every workgroup resident): the block
 * Krylov-Schur iterations of all graphs (deflated operator of eq. asigma
 * with the group-sum projection of eq. mv-Pw, block Gram-Schmidt and
 * Cholesky-QR on the FP64 matrix cores, Rayleigh-Ritz by Jacobi rotations in
 * LDS, Proposition 3.3's output) advance together in phases separated by
 * grid barriers; row work is split into 1024-row items spread over all
 * compute units, per-graph reductions and small factorizations run on one
 * owner workgroup per graph.
 *
 * graphs     host array of `count` handles, all on the current device.
 * k          host int32[count], 1 <= k[i] <= min(64, n_i - h_i + 1).
 * tol        as for sfairsc_eigs (||r_i|| <= tol * sigma).
 * precision  SFAIRSC_PREC_MIXED: float sparse products with float
 *            accumulation (double below tol = 5e-7); SFAIRSC_PREC_FP64.
 * opts       may be NULL.  block_width (0, 4, 8 or 16) and max_basis (0 or
 *            a multiple of the block width <= 80) force one configuration
 *            for every graph; both 0 = per graph from the tuning table
 *            (sfairsc_autotune), else a built-in rule.  seed, sigma,
 *            certify and max_restarts (0 = 500) as for sfairsc_eigs; x0 must
 *            be NULL.
 * eigvals    host array of `count` host pointers to double[k[i]], ascending.
 * H          host array of `count` device pointers to column-major
 *            n_i x k[i] doubles (the layout and sign rule of sfairsc_eigs).
 * infos      host array of `count` records, or NULL.
 *
 * Graphs the launch cannot take (k[i] > 48, n_i below twice the basis
 * leading dimension) and graphs whose launch result misses tol are solved by
 * sfairsc_eigs on the same stream.  In a batch of at least 32 graphs, the
 * launch stops once at most three graphs are still iterating (they could
 * not fill the GPU); those are finished by sfairsc_eigs, warm-started from
 * their current Ritz vectors.  The library keeps a per-device
 * workspace between calls: calls on one device must not overlap.
 * Synchronises `stream`.  Returns SFAIRSC_OK, SFAIRSC_E_NOT_CONVERGED (some
 * graph's status), else SFAIRSC_E_DEGENERATE (some graph's status; all
 * outputs written), or E_ARG, E_NOMEM, E_HIP.
 */
int sfairsc_eigs_batched(const sfairsc_graph_t* graphs, int32_t count,
                         const int32_t* k, double tol, int precision,
                         const sfairsc_eigs_opts* opts,
                         double* const* eigvals, double* const* H,
                         sfairsc_batch_info* infos, hipStream_t stream);

/*
 * Autotuner of the batched solve.  Graphs are grouped into buckets by
 * (floor(log2 n), average degree class <16 / <32 / <64 / >=64, k class
 * <=4 / <=8 / <=16 / >16, sparse-product precision, normalized); for up to
 * per_bucket (1..16) graphs of each bucket, candidate configurations run as
 * batched launches, each graph scored by the compute-unit time spent on it
 * (phase_ms summed): first block width x basis size, then the CSR rows per
 * wavefront.  The cheapest configuration whose solves all converge is
 * stored in the process-wide tuning table (replacing that bucket's entry).
 * Synchronises
 * `stream`.  Errors: E_ARG, E_NOMEM, E_HIP.
 */
int sfairsc_autotune(const sfairsc_graph_t* graphs, int32_t count,
                     const int32_t* k, double tol, int precision,
                     int32_t per_bucket, hipStream_t stream);

/* Write the tuning table to `path` (JSON: an "entries" array of flat
 * objects n_log2, degree_bucket, k_bucket, double_spmm, normalized,
 * block_width, max_basis, spmm_rows, ms). */
int sfairsc_tuning_save(const char* path);

/* Replace the tuning table by the file's entries.  The environment variable
 * SFAIRSC_TUNING_FILE, if set, is loaded at the first table use instead. */
int sfairsc_tuning_load(const char* path);

/* Empty the tuning table. */
int sfairsc_tuning_clear(void);

/* Number of entries in the tuning table. */
int sfairsc_tuning_size(void);

/* The configuration a batched solve would use for a graph of this shape:
 * returns 1 if it comes from the table, 0 for the built-in rule, or a
 * negative status. */
int sfairsc_tuning_lookup(int64_t n, int64_t nnz, int32_t k, int precision,
                          int normalized, double tol, int32_t* block_width,
                          int32_t* max_basis, int32_t* spmm_rows);

/* ---- clustering (Alg. 3 step 4) -------------------------------------- */

/*
 * k-means on the n rows of H (device double, column-major n x kdim,
 * 1 <= kdim <= 64): k-means++ seeding driven by SplitMix64 uniforms
 * (restart r, draw t uses output r * 2^32 + t + 1 of the stream seeded with
 * `seed`), Lloyd iterations until no label changes or max_iter (0 = 300),
 * best inertia of n_restarts, labels renumbered by first appearance.
 * labels   device int32[n].
 * inertia  host double (may be NULL).
 * 2 <= n_clusters <= min(64, n).  Synchronises `stream`.
 * Errors: E_ARG, E_NOMEM, E_HIP.
 */
int sfairsc_labels(sfairsc_graph_t g, const double* H, int32_t kdim,
                   int32_t n_clusters, int32_t n_restarts, uint64_t seed,
                   int32_t max_iter, int32_t* labels, double* inertia,
                   hipStream_t stream);

/* ---- differentiation -------------------------------------------------- */

/*
 * Gradient of f(W) = sum_{i<=k} lambda_i (the k smallest fair eigenvalues)
 * with respect to every stored value w_ij, by the envelope theorem applied
 * to Theorem 2.1 / Proposition 3.3 (F does not depend on W; sigma is held
 * constant).  For stored entry e = (i, j):
 *   unnormalized:  grad[e] = 0.5 * sum_l (H[i,l] - H[j,l])^2
 *   normalized:    grad[e] = 0.5 * sum_l [(H[i,l] - H[j,l])^2
 *                                         - lambda_l (H[i,l]^2 + H[j,l]^2)]
 * (in the normalized variant w_ij also enters d_i and d_j; H is
 * D-orthonormal there), so the two stored copies of an edge together carry
 * d f / d w_ij and a stored diagonal entry carries its whole derivative.
 * Valid when lambda_k < lambda_{k+1}.
 * H            device double, column-major n x k (from sfairsc_eigs).
 * eigenvalues  host double[k], the eigenvalues matching the columns of H;
 *              required for normalized handles, ignored (may be NULL) for
 *              unnormalized ones.  Read before the call returns.
 * grad         device [nnz] in the handle's value dtype.
 * Errors: E_ARG, E_NOMEM, E_HIP.  Asynchronous.
 */
int sfairsc_eigsum_backward(sfairsc_graph_t g, const double* H, int32_t k,
                            const double* eigenvalues, void* grad,
                            hipStream_t stream);

/* ---- diagnostics ------------------------------------------------------ */

/*
 * The small dense symmetric eigensolver of the Rayleigh-Ritz step that the
 * eigensolver runs at every restart (Alg. 3 step 3: the eigenpairs of the
 * projected matrix), exposed for validation: all eigenvalues of the
 * symmetric c x c matrix T and the eigenvectors of its m smallest, in FP64
 * on the device (one workgroup: Householder tridiagonalisation, Sturm-count
 * multisection, inverse iteration, back-transformation).
 * T   device double, row-major c x c with leading dimension ldt >= c; the
 *     two triangles are averaged (T is meant to be symmetric).
 * w   device double[c], ascending.
 * Z   device double, row-major c x m: column j is the unit eigenvector of
 *     w[j] (may be NULL when m = 0).
 * 1 <= c <= 192, 0 <= m <= c.  Allocates its scratch and synchronises
 * `stream`.  Errors: E_ARG, E_NOMEM, E_HIP.
 */
int sfairsc_symeig(const double* T, int32_t c, int32_t ldt, int32_t m,
                   double* w, double* Z, hipStream_t stream);

/* Message for the last non-OK status returned on this host thread. */
const char* sfairsc_last_error(void);

/* Library version string. */
const char* sfairsc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SFAIRSC_H */
