// Device kernels of the Jacobi-Davidson hot path (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "setup.h"

namespace jdmi {

constexpr int kBlock = 256;        // threads per workgroup for streaming kernels
constexpr int kRedBlocks = 1024;   // fixed grid of the deterministic reductions

// Device-resident scalar state of one simplified-QMR solve.
struct SqmrState {
    double rho, sigma, alpha, tau, tau0, theta, theta_old, c1, c2, beta, rr;
    double tol;       // stop when tau * sqrt(j+1) <= tol * tau0
    double shift;     // operator (A - shift I)
    int j;
    int done;         // set before this step: every kernel of the step is skipped
    int done_next;    // set during this step: the rest of the step is skipped
    int breakdown;
    int done_prev;    // the value of done before the beta step of the last step
};

// ---- K1 / K2 --------------------------------------------------------------------
void launch_gen_diag(int L, double W, uint64_t seed, double *eps, float *eps32, hipStream_t s);
// random bond values hop[d n + s] (bond from s to s + e_d), hop32 may be NULL
void launch_gen_hop(int L, double W, uint64_t seed, double *hop, float *hop32, hipStream_t s);
// bc: 0 periodic, 1 hard walls; hop: bond values (NULL: the constant coupling -1)
template <typename T>
void launch_stencil(int L, int bc, const T *eps, double shift, const T *x, T *y, hipStream_t s,
                    const int *skip = nullptr, const T *hop = nullptr);

// ---- multilevel apply ---------------------------------------------------------------
template <typename T>
struct DevLevel {
    int off, nB, n_after;
    const int64_t *g_ptr; const int *g_col; const T *g_val;
    const int64_t *gt_ptr; const int *gt_col; const T *gt_val;
    const T *bd, *bo; const int *bp;
};
template <typename T>
void launch_gather(int n, const int *perm, const T *b, T *w, hipStream_t s, const int *skip);
template <typename T>
void launch_scatter(int n, const int *perm, const T *x, T *out, hipStream_t s, const int *skip);
template <typename T>
void launch_down(const DevLevel<T> &lv, T *w, hipStream_t s, const int *skip);
template <typename T>
void launch_up(const DevLevel<T> &lv, const T *w, T *x, hipStream_t s, const int *skip);
// last level (dense inverse Cinv, row i at cinv + i * ld): x[off + i] = sum_j Cinv[i, j] w[off + j]
template <typename T>
void launch_coarse(int nc, int ld, int off, const T *cinv, const T *w, T *x, hipStream_t s, const int *skip);
// rows of the last level are padded to a multiple of kCoarseAlign (padding holds zeros)
constexpr int kCoarseAlign = 64;

// Product with the explicit inverse factor (y = Z w, or Z^T w) in the hybrid layout of
// jdmi::HybHost; workgroup b works on part b % kHybParts, so that on an 8-XCD device a
// part's gathers stay in one XCD's L2.  Values are stored in Tv and the vectors in Tx;
// products are accumulated in binary64 and the result rounded to Tx once, so that the
// binary32 products with Z and Z^T stay transposes of each other to one rounding.
// Summation order is fixed (per lane, then a fixed shuffle tree): results are
// reproducible.
template <typename Tv>
struct Hyb {
    int nlong = 0, nslices = 0;
    // per part: tasks (long rows, then slices), long rows, first long row, first slice
    int ntask[kHybParts] = {}, plong[kHybParts] = {}, long0[kHybParts] = {}, slice0[kHybParts] = {};
    const int *long_row = nullptr;     // row of each long row
    const int64_t *long_ptr = nullptr; // nlong + 1
    const int *long_col = nullptr;
    const Tv *long_val = nullptr;
    // 2 (nslices + 1) values: for slice s, [2 s] = its first entry (a multiple of 64) | shape
    // code and [2 s + 1] = its first rowidx entry (one 16-byte load per slice boundary)
    const int64_t *slice_desc = nullptr;
    const int *rowidx = nullptr;         // the slices' rows, -1 for padding rows (+ 64 entries -1)
    const int *col = nullptr;
    const Tv *val = nullptr;
};
// y[r] = (Z w)[r] for every row number r of the layout
template <typename Tv, typename Tx>
void launch_hyb_spmv(const Hyb<Tv> &A, const Tx *x, Tx *y, hipStream_t s, const int *skip);

// The block-diagonal step z[j] = dd[j] y[j] + dof[j] y[dp[j]] (j < m), then the last
// level with scattered unknowns, z[idx[i]] = sum_j Cinv[i, j] y[idx[j]]: the gather
// yc[i] = y[idx[i]] shares the first launch with the block-diagonal step (both only read
// y); ld is a multiple of kCoarseAlign, and Cinv's row padding and yc[nc .. ld) hold zeros
template <typename T>
void launch_dinv_coarse(int m, const T *dd, const T *dof, const int *dp, int nc, int ld, const int *idx,
                        const T *cinv, const T *y, T *yc, T *z, hipStream_t s, const int *skip);

// ---- reductions (deterministic two-stage; results stay on the device) ---------------
// partial[c * kRedBlocks + b] for c < ncols; out[c] = sum
template <typename T>
void launch_multidot(int n, int ncols, const T *Q, int64_t ldq, const T *y, double *partial,
                     double *out, hipStream_t s, const int *skip = nullptr);
template <typename T>
void launch_dot(int n, const T *x, const T *y, double *partial, double *out, hipStream_t s,
                const int *skip = nullptr);

// y -= Q c   (c on the device, ncols entries, double); optional skip flag
template <typename T>
void launch_sub_qc(int n, int ncols, const T *Q, int64_t ldq, const double *c, T *y, hipStream_t s,
                   const int *skip = nullptr, double alpha = 1.0);
// y = V s for an n x m column-major V (double); y may not alias V
void launch_gemv_vs(int n, int m, const double *V, int64_t ldv, const double *s, double *y, hipStream_t st);
// Vout[:, c] = V * S[:, c] for c < mout (S m x mout column-major, leading dim lds)
void launch_gemm_vs(int n, int m, int mout, const double *V, int64_t ldv, const double *S, int lds,
                    double *Vout, int64_t ldo, hipStream_t st);

// Dense inverse by Gauss-Jordan elimination with partial pivoting (the exactly inverted
// last level): a (n x n row-major) is destroyed, inv receives A^{-1}; colc is an n
// workspace; status[0] becomes 1 if a pivot column is zero.
void launch_gauss_jordan(int n, double *a, double *inv, double *colc, int *status, hipStream_t s);
// a[i, j] *= sc[i] sc[j]
void launch_scale_sym(int n, double *a, const double *sc, hipStream_t s);

// elementwise helpers
template <typename Tin, typename Tout>
void launch_convert(int n, const Tin *x, Tout *y, double scale, hipStream_t s);
void launch_axpby_d(int n, double a, const double *x, double b, double *y, hipStream_t s);
void launch_scale_by_inv_sqrt(int n, const double *nrm2, double *x, hipStream_t s);
void launch_random_vector(int n, uint64_t seed, double *x, hipStream_t s);

// ---- simplified QMR pieces (scalars read from SqmrState on the device) -----------------
template <typename T>
void launch_sqmr_init(int n, const T *b, T *r, T *x, T *d, hipStream_t s);
void launch_sqmr_params(SqmrState *st, double shift, double tol, hipStream_t s);
void launch_sqmr_scalar_start(SqmrState *st, const double *rr, const double *rho, hipStream_t s);
// t = (A - st->shift I) q with the binary64 operator (eps, bond values) applied to q and
// the result rounded once; skipped when st->done
template <typename T>
void launch_stencil_state(int L, int bc, const double *eps, const SqmrState *st, const T *x, T *y, hipStream_t s,
                          const double *hop = nullptr);
template <typename T>
void launch_copy(int n, const T *x, T *y, hipStream_t s);
// r -= alpha t; |r|^2 (stored in *rr) and, in the same final reduction, the theta / c / tau
// update and the stopping test (skipped when st->done)
template <typename T>
void launch_sqmr_update_r(int n, SqmrState *st, const T *t, T *r, double *partial, double *rr, hipStream_t s);
// t -= Qt c, then sigma = q.t (stored in *sigma) and, in the same final reduction,
// alpha = rho / sigma (skipped when st->done; a zero or non-finite sigma is a breakdown
// that stops the solve).  u -= Y g, then rho' = r.u (stored in *rho, skipped when
// st->done_next) and, in the same final reduction, beta = rho' / rho; then st->done
// takes the value of st->done_next.  ncols <= 128, 0 for no projection.
template <typename T>
void launch_sqmr_sub_dot_alpha(int n, int ncols, const T *Q, const double *c, T *t, const T *q, double *partial,
                               double *sigma, SqmrState *st, hipStream_t s);
template <typename T>
void launch_sqmr_sub_dot_beta(int n, int ncols, const T *Y, const double *g, T *u, const T *r, double *partial,
                              double *rho, SqmrState *st, hipStream_t s);
// the end of a step (after the beta step): d = c1 d + c2 q, x += d if the step was live
// before the beta step (st->done_prev == 0), then q = u + beta q if it still is
template <typename T>
void launch_sqmr_update_xdq(int n, SqmrState *st, const T *u, T *q, T *d, T *x, hipStream_t s);
// small dense product on the device: out = M c (p x p, double), skip if done
void launch_small_matvec(int p, const double *M, const double *c, double *out, const int *skip, hipStream_t s);

}  // namespace jdmi
