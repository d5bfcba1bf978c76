// Rayleigh-Ritz step of the block Krylov-Schur solver on the GPU (FP64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace sfairsc {

// Record the kernel leaves for the host after a restart-mode call (doubles):
// [0] pairs among the k wanted meeting tol, [1] p (Ritz vectors kept),
// [2] m (Ritz vectors formed), [3] (theta_{k+1} - theta_k) / sigma (0 when
// c <= k), [4..6] the three words of the skip flag as the kernel found them
// (written also when it skipped, so that one download carries both), then
// theta[0:k] and the residual estimates res[0:k].
constexpr int kRrRecFlag = 4;
constexpr int kRrRecHead = 7;
inline size_t rr_rec_doubles(int k) { return (size_t)kRrRecHead + 2 * (size_t)k; }

struct RrArgs {
    // input: the symmetric projected matrix (order c, row-major with leading
    // dimension ldt; the two triangles are averaged on load)
    const double* T = nullptr;
    int ldt = 0;
    int c = 0;
    const int* skip = nullptr;  // device flag (3 words): nonzero = leave every output but
                                // the record's flag words untouched
    double* work = nullptr;     // rr_work_doubles() of scratch
    // mode 0 (restart): the Ritz vectors kept by the thick restart, chosen by
    // the rule of the solver, their residual estimates ||Rc Z[c-b:c, i]||
    // and the convergence count; mode 1: all eigenvalues and the
    // eigenvectors of the m = mreq smallest only.
    int mode = 0;
    int mreq = 0;
    // mode 0 inputs
    const double* Rc = nullptr;  // b x b coupling of the next block (upper triangle used)
    int b = 0, k = 0, ncv = 0, keep = 0;
    double tol = 0.0, sigma = 0.0;
    // outputs
    double* theta = nullptr;  // [c] all eigenvalues, ascending
    double* Qch = nullptr;    // mode 0: the restart rotation's factor (layout: rot_whole)
    double* Zk = nullptr;     // mode 0: Z[:, 0:k] row-major c x k (may be null)
    double* rec = nullptr;    // mode 0: rr_rec_doubles(k) (see above)
    double* Zout = nullptr;   // mode 1: Z[:, 0:m] row-major c x m
    // mode 0, optional: the solver may enqueue the restart rotation for a
    // predicted kept count p_pred before it reads the record; that work runs
    // only while *rot_skip is 0.  The kernel sets it to 1 first (so that it
    // stays 1 if the kernel skips or stops early) and at the end to 0 exactly
    // when the cycle did not converge and p == p_pred.
    int* rot_skip = nullptr;
    int p_pred = 0;
};

size_t rr_work_doubles();

// Enqueue the one-workgroup kernel on `s` (1 <= c <= kMaxBasis).
int rr_launch(const RrArgs& a, hipStream_t s);

}  // namespace sfairsc
