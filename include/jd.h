/*
 * jd.h -- C ABI of the MI355X (gfx950) shift-and-invert Jacobi-Davidson library
 * for the 3D Anderson model of localization.
 *
 * Method: Schenk, Bollhoefer & Roemer, "On large scale diagonalization techniques
 * for the Anderson model of localization".  The operator is the Anderson matrix of
 * section 3, eq. (eigenequation), on the periodic L x L x L lattice, written here
 * as A = -T + diag(eps) (hopping -1; for even L the staggered gauge maps it onto
 * the paper's +1 convention with the same spectrum).  eps_s = W (u_s - 1/2),
 * u_s the top 53 bits of output s+1 of SplitMix64 seeded with `seed`, site
 * s = i + L (j + L k) (x fastest, 0-based).
 *
 * Conventions for every entry point:
 *  - Return value: JD_OK (0) on success, JD_ENOCONV (1) for a partial result,
 *    a negative JD_E* code on failure; jd_last_error() then describes it
 *    (thread-local string owned by the library, valid until the next call on the
 *    same thread).  No C++ exception crosses this interface.
 *  - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *    pointers are HIP device memory on the current device, owned by the caller
 *    (the library never frees them).  Handles (jd_problem, jd_precond) are owned
 *    by the library and released by their *_free call.
 *  - Vectors over the lattice have length n = L^3 in site order; multi-column
 *    arrays are column-major with leading dimension n.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Device work of
 *    a call is ordered on that stream; calls returning host results synchronise it.
 *  - Distinct handles may be used from distinct threads; one handle must not be
 *    used by two threads at once.
 */
#ifndef JD_H
#define JD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    JD_OK = 0,
    JD_ENOCONV = 1,    /* partial result: fewer than k pairs met the tolerance */
    JD_EINVAL = -1,    /* invalid argument (sizes, non-finite values, NULL outputs) */
    JD_ENOMEM = -2,    /* device or host allocation failed */
    JD_EDEVICE = -3,   /* a HIP call failed (message names it) */
    JD_ESETUP = -4,    /* preconditioner construction failed (e.g. singular coarse level) */
    JD_ENOTIMPL = -5   /* option combination not provided */
};

enum { JD_FP64 = 0, JD_MIXED = 1, JD_MIXED_FACTORS = 2 };

/* Boundary conditions of the lattice (section 8.2): periodic (the paper's main
 * experiments; figure 1) or hard walls (the Table 6 variant: the box is embedded in
 * zeros, so a site on a face has no coupling across it). */
enum { JD_BC_PERIODIC = 0, JD_BC_HARDWALL = 1 };

/* The model (section 8.2, Table 6).  JD_MODEL_ANDERSON: random diagonal of width W,
 * couplings -1 (section 3).  JD_MODEL_OFFDIAG, the off-diagonal ("inverse") model:
 * constant diagonal 1.28 and a random value on every bond, uniform on [-W/2, W/2)
 * (W = 1: the paper's [-1/2, 1/2]); the bond from site s to its +x, +y, +z neighbour
 * (d = 0, 1, 2) takes output n + 3 s + d + 1 of the SplitMix64 stream of `seed`. */
enum { JD_MODEL_ANDERSON = 0, JD_MODEL_OFFDIAG = 1 };

/*
 * Options; a zero-initialised struct selects every default.
 *  precision  JD_FP64: every step in binary64.  JD_MIXED: inner SQMR vectors and
 *             preconditioner factors stored in binary32; the inner stencil product
 *             applies the binary64 operator to the binary32 vector, and dot products
 *             and factor products accumulate in binary64, each result rounded once
 *             (the level-by-level apply of JD_FLAG_LEVELS accumulates in binary32);
 *             Gram-Schmidt, Rayleigh-Ritz, residual norms
 *             and acceptance in binary64.  JD_MIXED_FACTORS: only the preconditioner
 *             factors stored in binary32; stencil product and SQMR vectors in binary64.
 *  drop_tol   epsilon of section 7.2: an entry of a factor column is dropped when
 *             its modulus is below drop_tol / kappa (0 -> 1/sqrt(n), the paper's
 *             choice in section 8.2; < 0 -> nothing dropped, exact factorisation).
 *  kappa      bound on ||L^{-1}|| of inverse-based pivoting, section 7.2 (0 -> 5).
 *             After a level that accepts fewer than 1% of its unknowns while more
 *             than 8192 remain, the bound (and with it drop_tol / kappa) doubles for
 *             the following levels, up to max(20, kappa).
 *  agg_tau    tau of the aggressive dropping rule of section 7.3 (0 -> 0.1).
 *  schur_tol  off-diagonal entries of a scaled Schur complement below this are
 *             dropped (0 -> drop_tol / 2).
 *  coarse_max the multilevel recursion (section 7.3) stops at this size and the
 *             last Schur complement is inverted exactly (0 -> 1536); it also stops
 *             once a level accepts fewer than 1% of its unknowns and at most 8192 remain.
 *  max_levels cap on the number of levels (0 -> 400).
 *  z_drop     the preconditioner is applied as P^T Z^T D^{-1} Z P with Z the inverse
 *             of the unit lower triangular factor of all levels, formed explicitly as a
 *             product of segments Z = Z_{S-1} ... Z_0, each the inverse of the factor of a
 *             consecutive range of levels; entries of each Z_s below z_drop (scaled
 *             domain) are dropped (0 -> min(1e-2, 10 drop_tol); < 0 -> none).
 *  z_parts    the number S of segments: level cuts at 1, 3, 9, 27, ... (0 -> 6 for
 *             n >= 2^19, 4 for n >= 2^16, else 3; 1 -> a single explicit inverse).
 *  jmin, jmax search-space sizes after / before a restart (0 -> after a setup that
 *             stalled (see kappa): max(k+20,30) and min(3 jmin, 120); else for
 *             n >= 2^19: max(k+10,20) and min(3 jmin, 120); else max(k+5,10) and
 *             min(2 jmin, 120)); jmin < 120, jmax <= 120, and
 *             jmin < jmax when both are given (JD_EINVAL otherwise); a jmin given
 *             alone raises the default jmax to at least jmin + 1.
 *  max_outer  outer Jacobi-Davidson iterations (0 -> 60 k + 200).
 *  max_inner  SQMR steps per correction equation (0 -> 50 with binary32 vectors; with
 *             binary64 ones 40, or 80 after a setup that stalled).
 *  switch_tol the correction operator uses sigma until ||r|| < switch_tol ||A||_inf,
 *             then the Ritz value theta; < 0: always sigma (0 -> 1e-3).
 *  flags      bit 0 (JD_FLAG_GRAPHS): replay the inner iteration as a captured HIP graph
 *             instead of launching it kernel by kernel (same kernels in the same order,
 *             same results; the serving workers always launch kernel by kernel).
 *             bit 1 (JD_FLAG_LEVELS): apply the factorisation level by level (two
 *             dependent sparse passes per level) instead of through Z.
 *  bc         JD_BC_PERIODIC (0) or JD_BC_HARDWALL.  ||A||_inf is the largest row sum
 *             of |entries| (6 + max|eps| for the diagonal model on the torus).
 *  model      JD_MODEL_ANDERSON (0) or JD_MODEL_OFFDIAG.
 *  inner_tol_min  floor of the relative tolerance rate^j of the j-th correction
 *             equation solved for the current pair (0 -> 1e-10); a solve-time option.
 *  inner_tol_rate the rate of that tolerance, in (0, 1) (0 -> 0.5 for JD_MIXED, whose
 *             binary32 vectors cannot resolve tighter inner solves, 0.25 for the splits
 *             with binary64 vectors); a solve-time option.
 *  stream     stream for the solve's device work (NULL: a library-created blocking stream).
 */
typedef struct jd_options {
    int precision;
    double drop_tol;
    double kappa;
    double agg_tau;
    double schur_tol;
    int coarse_max;
    int max_levels;
    double z_drop;
    int jmin, jmax;
    int max_outer, max_inner;
    double switch_tol;
    int flags;
    int z_parts;
    int bc;
    int model;
    double inner_tol_min;
    double inner_tol_rate;
    void *stream;
} jd_options;

enum { JD_FLAG_GRAPHS = 1, JD_FLAG_LEVELS = 2 };

/* Statistics of a solve (the paper's Tables 3-5 quantities plus timings). */
typedef struct jd_info {
    int n_converged;      /* eigenpairs that met the tolerance */
    int outer_its;        /* Jacobi-Davidson outer iterations */
    int inner_its;        /* SQMR steps summed over all correction equations */
    int levels;           /* multilevel factorisation: number of levels */
    int n_2x2;            /* 2x2 pivots over all levels */
    int coarse_n;         /* size of the exactly inverted last Schur complement */
    double setup_s;       /* host setup: matching, scaling, ordering, factorisation, upload */
    double solve_s;       /* device solve (outer + inner iterations) */
    double fill;          /* (nnz strict lower L + nnz D + coarse entries) / nnz lower(A) */
    double anorm;         /* ||A||_inf = 6 + max |eps| */
    size_t device_bytes;  /* device memory held by the problem */
} jd_info;

typedef struct jd_problem jd_problem;
typedef struct jd_precond jd_precond;

/*
 * jd_solve -- the k eigenpairs of A nearest sigma (abstract; section 4.2; the
 * experiments of section 8.2 ask for the five eigenvalues nearest 0).
 *  L >= 2 with L^3 < 2^31; W >= 0 finite; sigma finite; 1 <= k <= min(n, 64);
 *  tol in [1e-14, 1): a pair is accepted when ||A x - lambda x||_2 <= tol ||A||_inf
 *  with ||x||_2 = 1.
 *  evals [k] host (required): sorted by (|lambda - sigma|, lambda).
 *  evecs [n*k] host or NULL: column c is the unit eigenvector of evals[c].
 *  resid [k] host or NULL: ||A x - lambda x||_2 / ||A||_inf per pair (binary64).
 *  opt, info may be NULL.
 *  Returns JD_ENOCONV with the converged prefix filled and NaN in the rest when
 *  max_outer is exhausted.
 */
int jd_solve(int L, double W, uint64_t seed, double sigma, int k, double tol,
             double *evals, double *evecs, double *resid,
             const jd_options *opt, jd_info *info);

/* Split form: the setup (timed separately) keeps the factors resident. */
int jd_setup(int L, double W, uint64_t seed, double sigma, const jd_options *opt,
             jd_problem **out);
/* Same contract as jd_solve.  evecs_device, if not NULL, is a caller-owned device
 * array of n*k binary64 values that receives the eigenvectors. */
int jd_problem_solve(jd_problem *p, int k, double tol, double *evals, double *evecs_host,
                     void *evecs_device, double *resid, jd_info *info);
/*
 * jd_problem_lanczos -- the same k eigenpairs by shift-and-invert Lanczos (section 4.1;
 * the ARPACK runs of section 8.2, Tables 2-3): Lanczos on (A - sigma I)^{-1} with full
 * reorthogonalisation and restarts that keep the wanted Ritz vectors, each product an
 * SQMR solve with the problem's multilevel preconditioner stopped when its quasi-residual
 * bound reaches inner_tol times the right-hand side's norm (0 -> 1e-10, the paper's
 * setting).  Outputs as jd_problem_solve (no device vectors); info->outer_its counts the
 * products with (A - sigma I)^{-1}, info->inner_its the SQMR steps.  Options of the
 * problem: jmax is the largest basis (0 -> min(max(2(k+5), k+25), 120)), max_outer the
 * products (0 -> 60 k + 200), max_inner the SQMR steps of one product (0 -> 1000).
 * Needs binary64 vectors: JD_ENOTIMPL for JD_MIXED (binary32 inner solves cannot reach
 * 1e-10); JD_MIXED_FACTORS uses the binary32 factors with binary64 vectors.
 */
int jd_problem_lanczos(jd_problem *p, int k, double tol, double inner_tol, double *evals, double *evecs_host,
                       double *resid, jd_info *info);
/* Switch the precision of later jd_problem_solve calls (JD_FP64, JD_MIXED or
 * JD_MIXED_FACTORS); the setup keeps the factors in both precisions, so no new setup
 * is needed. */
int jd_problem_set_precision(jd_problem *p, int precision);
/* Replace the solve-time options of later jd_problem_solve calls: jmin, jmax,
 * max_outer, max_inner, switch_tol, inner_tol_min, inner_tol_rate and the JD_FLAG_GRAPHS bit of flags are taken from
 * *opt (0 -> the default, as in jd_setup); every setup option of *opt is ignored.
 * JD_EINVAL for out-of-range values, and the problem keeps its previous options. */
int jd_problem_set_solve_options(jd_problem *p, const jd_options *opt);
/* Setup statistics of a problem (levels, fill, timings so far). */
int jd_problem_info(const jd_problem *p, jd_info *info);
void jd_problem_free(jd_problem *p);

/*
 * Hot-path steps exposed on their own (used by the parity tests and the benchmark).
 *
 * jd_gen_diag -- K1: eps (n binary64) and its binary32 rounding into device arrays.
 *   d_eps32 may be NULL.
 */
int jd_gen_diag(int L, double W, uint64_t seed, double *d_eps, float *d_eps32, void *stream);

/*
 * jd_block_product -- out = V S, the dense tall-skinny products of Rayleigh-Ritz
 * (section 4.2: the restart V <- V S and the deflation after locking), on the FP64
 * matrix cores.  V: n x m, S: m x mout, out: n x mout, all binary64 device arrays in
 * column-major order with leading dimensions ldv >= n, lds >= m, ldo >= n; out must not
 * overlap V or S.
 */
int jd_block_product(int n, int m, int mout, const double *d_V, int64_t ldv, const double *d_S, int lds,
                     double *d_out, int64_t ldo, void *stream);

/* jd_gen_hop -- the bond values of the off-diagonal model (see JD_MODEL_OFFDIAG) into
 * a device array d_hop[d n + s] of 3 n binary64 values (bond from s to s + e_d), and
 * their binary32 rounding (d_hop32 may be NULL). */
int jd_gen_hop(int L, double W, uint64_t seed, double *d_hop, float *d_hop32, void *stream);

/*
 * jd_stencil_spmv -- y = (A - shift I) x on the lattice (section 3,
 * eq. (eigenequation)); only eps (and, for the off-diagonal model, the bond values)
 * is stored, the lattice structure is implicit.
 *   bc JD_BC_PERIODIC or JD_BC_HARDWALL (section 8.2).
 *   d_hop NULL: couplings -1; else 3 n bond values laid out as by jd_gen_hop.
 *   precision JD_FP64: d_eps, d_hop, d_x, d_y are double*; JD_MIXED: float*.
 */
int jd_stencil_spmv(int L, int bc, int precision, const void *d_eps, const void *d_hop, double shift,
                    const void *d_x, void *d_y, void *stream);

/*
 * jd_precond_create -- host setup of the matching-based multilevel incomplete
 * LDL^T of A - sigma I (sections 6 and 7): maximum weight matching, 1x1/2x2
 * cycle split, symmetric scaling, block independent-set ordering, inverse-based
 * pivot acceptance with bound kappa, dropping, explicit Schur complement, recursion,
 * exactly inverted last level; factors uploaded in binary64 and binary32.
 * With drop_tol < 0 nothing is dropped and kappa is ignored (exact factorisation
 * up to rounding: the apply then equals (A - sigma I)^{-1}).
 */
int jd_precond_create(int L, double W, uint64_t seed, double sigma, const jd_options *opt,
                      jd_precond **out);
/* out = K^{-1} in (device vectors of length n, double* for JD_FP64, float* for
 * JD_MIXED); in and out must not overlap. */
int jd_precond_apply(jd_precond *p, int precision, const void *d_in, void *d_out, void *stream);
/* Level structure: sizes[l] = unknowns entering level l (l < levels), sizes[levels] =
 * coarse size; nB[l] = pivots accepted at level l; nnzG[l] = stored coupling entries.
 * Arrays of length cap (host); returns the number of levels. */
int jd_precond_levels(const jd_precond *p, int cap, int *sizes, int *nB, long long *nnzG);
/* Release a preconditioner (a view obtained from jd_problem_precond leaves the
 * problem's factors alone). */
void jd_precond_free(jd_precond *p);
/* A view of the preconditioner held by a problem (valid while the problem lives;
 * release the view with jd_precond_free). */
int jd_problem_precond(jd_problem *p, jd_precond **out);
/* Number of stored entries of the inverse factor, all segments (and n). */
int jd_precond_factor_nnz(const jd_precond *p, long long *nnz, int *n);
/* Segments of the inverse factor: lev_begin[s] = first level of segment s, rows[s] =
 * rows of Z_s (unknowns entering that level), nnz[s] = its stored entries (arrays of
 * length cap, host; NULL entries skipped).  Returns the number of segments. */
int jd_precond_segments(const jd_precond *p, int cap, int *lev_begin, int *rows, long long *nnz);
/* The dominant kernel of the apply on its own: the sparse products with the segments.
 * transpose = 0: y = Z_{S-1} ... Z_0 x, x in the Morton order of the sites, y in the
 * middle numbering of the factorisation; transpose = 1: y = P^T Z_0^T ... Z_{S-1}^T x,
 * x in the middle numbering, y in site order.  Device vectors of length n (d_x is copied
 * into the preconditioner's workspace, the result copied out for transpose = 0).  With
 * d_x = d_y = NULL only the products run, on the values the workspace holds (timing
 * form: the kernels of one apply's direction and nothing else).  The workspace is the
 * one jd_precond_apply uses: calls on one preconditioner must not overlap. */
int jd_precond_factor_product(jd_precond *p, int precision, int transpose, const void *d_x, void *d_y,
                              void *stream);

/*
 * jd_problem_linear_solve -- the inner iteration on its own: simplified QMR with
 * the projected preconditioner (section 4.2) for
 *   (I - Q Q^T)(A - shift I)(I - Q Q^T) x = (I - Q Q^T) b,  x = (I - Q Q^T) x,
 * Q the p orthonormal binary64 columns of d_Q (p may be 0, d_Q then NULL).
 * d_b, d_x: device binary64 n-vectors.  Stops when the quasi-residual bound
 * reaches rtol ||b|| or after maxit steps; *its receives the step count.
 * pcols <= 64.  Runs on the problem's stream (jd_options.stream at jd_setup) and
 * synchronises it before returning; the caller orders its writes of d_Q and d_b
 * before the call.
 */
int jd_problem_linear_solve(jd_problem *p, double shift, const double *d_Q, int pcols,
                            const double *d_b, double *d_x, double rtol, int maxit, int *its);

/*
 * jd_problem_linear_solve_noalloc -- jd_problem_linear_solve for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, hosts that
 * forbid hipMalloc).  Same arguments, same kernels in the same order and the same result;
 * it allocates nothing: no hipMalloc / hipFree, no pinned host memory, no events or
 * graphs, and jd_set_allocator's hook is not called.  Its work buffers (the seven SQMR
 * vectors, the solver state and reduction partials, Q in the inner precision, K^{-1} Q
 * and the pcols x pcols projection matrix) live in one static device array of 64 MiB that
 * every GPU the library runs on holds until the process ends; JD_EINVAL when a call needs
 * more (about (7 + 2 pcols) n value-size bytes plus 2.1 MiB; e.g. n = 10^6 with binary32
 * inner vectors allows pcols <= 4).  All calls on one GPU share that array and it keeps
 * the last call's contents: calls that overlap on one GPU (from several threads or
 * streams) race and must be serialised by the caller.  The host reads the stop flag
 * synchronously every few steps.
 */
int jd_problem_linear_solve_noalloc(jd_problem *p, double shift, const double *d_Q, int pcols,
                                    const double *d_b, double *d_x, double rtol, int maxit, int *its);

/*
 * Serving: independent solve requests run concurrently (the disorder averaging
 * of section 3 needs many realisations).  A request is admitted when a worker is free
 * and its estimated device footprint fits the HBM budget; admitted requests run their
 * host setup and their device solve concurrently, each on its own stream, so work of
 * requests that arrived at different times overlaps on the GPU (each worker launches
 * on its own non-blocking stream).  Every request's
 * arithmetic is independent of the others (deterministic kernels and setup), so its
 * result is identical alone and in the mix.  All jd_server_* calls are thread-safe.
 */
typedef struct jd_request {
    int L;
    double W;
    uint64_t seed;
    double sigma;
    int k;            /* 1 .. 64 */
    double tol;
    int precision;    /* JD_FP64, JD_MIXED or JD_MIXED_FACTORS */
    int flags;        /* jd_options flags (JD_FLAG_LEVELS; JD_FLAG_GRAPHS is ignored) */
    int bc;           /* JD_BC_PERIODIC or JD_BC_HARDWALL */
    int model;        /* JD_MODEL_ANDERSON or JD_MODEL_OFFDIAG */
} jd_request;

typedef struct jd_result {
    int status;           /* JD_OK, JD_ENOCONV or a negative code */
    int k, n_converged, outer_its, inner_its;
    double evals[64];     /* sorted by (|lambda - sigma|, lambda); NaN past n_converged */
    double resid[64];     /* ||A x - lambda x|| / ||A||_inf */
    double queued_s;      /* submission -> admission */
    double setup_s;       /* host setup and upload */
    double solve_s;       /* device solve */
    double latency_s;     /* submission -> completion */
    size_t device_bytes;  /* footprint reserved for the request */
    char error[160];      /* message of a failed request ("" on success) */
} jd_result;

typedef struct jd_server jd_server;

/* hbm_budget_bytes: device memory the server may reserve (0 -> 80% of free memory);
 * workers: concurrently active requests (0 -> 8); setup_threads: host threads of one
 * setup.  Host setups are a resource of their own, drawn from the OpenMP thread budget
 * (OMP_NUM_THREADS); a setup waiting for threads counts its wait in setup_s, while
 * admitted solves all run.
 *   setup_threads > 0: every setup uses that many, and at most
 *     max(1, budget / setup_threads) run at once.
 *   setup_threads 0 (adaptive): a setup starts when a thread is free and takes
 *     budget / max(2, setups running or waiting) threads (at least 1, at most the free
 *     ones): two setups share the budget at light load, and a backlog runs more,
 *     narrower setups, which clear it faster.
 * Results do not depend on the split: the factors are identical for any thread count. */
int jd_server_create(size_t hbm_budget_bytes, int workers, int setup_threads, jd_server **out);
/* Queue a request (never blocks); *ticket identifies it.  JD_EINVAL for bad fields, or
 * a footprint larger than the whole budget. */
int jd_server_submit(jd_server *s, const jd_request *req, uint64_t *ticket);
/* 0: done (result filled, ticket released); 1: still queued or running; < 0: error. */
int jd_server_poll(jd_server *s, uint64_t ticket, jd_result *res);
/* Block until the request is done; returns 0 with the result, or a negative code. */
int jd_server_wait(jd_server *s, uint64_t ticket, jd_result *res);
/* Estimated device footprint of a request (the admission test). */
size_t jd_server_footprint(const jd_request *req);
/* Finish queued and running requests, then release everything. */
void jd_server_destroy(jd_server *s);

/*
 * Host setup steps on their own (no GPU involved), for checks of the setup logic.
 * The matrix is symmetric, CSR with sorted column indices and a diagonal entry in
 * every row (n rows, ptr[n + 1], col/val[ptr[n]]).
 *
 * jd_host_matching -- maximum-product transversal (section 6.1, eq. (1)-(2)):
 *   match[i] = column matched to row i; logd[i] = log of the symmetric scaling
 *   d_i (|d_i a_ij d_j| <= 1, = 1 on matched entries).  Returns the number of
 *   unmatched rows (0 for a structurally nonsingular matrix) or a negative code.
 */
int jd_host_matching(int n, const int64_t *ptr, const int *col, const double *val, int *match, double *logd);
/*
 * jd_host_split_cycles -- 1x1 / 2x2 blocks from the cycles of the matching
 * (section 6.2, figures 3-4): pairs[2 b], pairs[2 b + 1] are the members of block b
 * (second = -1 for a 1x1 block); *nblocks receives the count (<= n).
 */
int jd_host_split_cycles(int n, const int64_t *ptr, const int *col, const double *val, const int *match,
                         const double *logd, int *pairs, int *nblocks);
/*
 * jd_host_factor -- the multilevel factorisation of A (sections 6-7) on the host.
 * Fills, when non-NULL: perm[n] (position -> row), scale[n] (cumulative scaling of
 * each position), level_off/level_nb/level_n2x2[cap] per level; returns the number
 * of levels (or a negative code) and *coarse_n.  g_nnz[cap] receives the stored
 * coupling entries per level; g_min_scaled[cap] the smallest |entry| of each level's
 * coupling block in the scaled domain, g_max_colsum[cap] the largest 1 + column sum
 * of |entries| of a pivot's coupling column in the scaled domain (the ||L^{-1}||_1
 * bound of inverse-based pivoting).
 */
int jd_host_factor(int n, const int64_t *ptr, const int *col, const double *val, const jd_options *opt,
                   int *perm, double *scale, int cap, int *level_off, int *level_nb, int *level_n2x2,
                   long long *g_nnz, double *g_min_scaled, double *g_max_colsum, int *coarse_n);

/*
 * jd_host_precond_apply -- x = K^{-1} b for the multilevel preconditioner of A
 * (sections 6-7), on the host in binary64, through the very layouts the device products
 * read (the segments of the inverse factor, D^{-1}, the exactly inverted last level,
 * here inverted on the host), in the device's order.  A check of those layouts: every
 * row, column and task number is checked against the region of the 3n workspace it may
 * address, no product may read a value it writes, and no value may be read before it
 * is written; a failed check returns JD_ESETUP with the reason in jd_last_error().  n
 * must be L^3 (the layouts follow the Morton order of the lattice); b and x are host
 * arrays of n values in site order, b finite.  Options as for jd_setup (drop_tol < 0:
 * nothing dropped, so that K^{-1} A = I).  Returns the number of segments.
 */
int jd_host_precond_apply(int n, const int64_t *ptr, const int *col, const double *val, const jd_options *opt,
                          const double *b, double *x);

/*
 * jd_set_allocator -- device memory from the caller (for instance a framework's caching
 * allocator), so that the library's buffers share the caller's memory pool.  Every device
 * buffer the library allocates after the call -- a problem's operator and factors, the
 * search space and work vectors of each solve, the buffers of serving requests -- comes
 * from alloc(bytes, stream, ctx) and goes back through free_(ptr, stream, ctx); `stream`
 * is the hipStream_t whose work uses the buffer.  alloc returns device memory on the
 * current device, aligned to 256 bytes, or NULL (the calling entry point then fails with
 * JD_ENOMEM).  Before a buffer is handed to free_ the library synchronises that stream,
 * so free_ may reuse it at once.  Both functions may be called from any library thread
 * (serving workers) and must be thread-safe; they must not call into this library.
 * alloc = free_ = NULL restores hipMalloc / hipFree.  A buffer is always returned to the
 * allocator it came from, also after a later jd_set_allocator call; ctx must stay valid
 * while such buffers live.  JD_EINVAL if exactly one of alloc, free_ is NULL.
 * Not a step of the paper's method: it lets the host framework (PyTorch in the Python
 * binding) own the device memory.
 */
int jd_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx),
                     void (*free_)(void *ptr, void *stream, void *ctx), void *ctx);

const char *jd_last_error(void);
/* Library version string. */
const char *jd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JD_H */
