// Host-side construction of the matching-based multilevel incomplete LDL^T
// (sections 6 and 7 of Schenk, Bollhoefer & Roemer).  Everything here runs on
// the CPU once per problem; the factors it returns are uploaded and applied by
// the device kernels.
#pragma once
#include <cstdint>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

namespace jdmi {

// Allocator whose resize(n) leaves new elements uninitialised: the arrays of a
// matrix built level by level are filled by parallel loops right after they are
// sized, so zeroing them first would only add a serial pass over fresh pages.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() noexcept = default;
    template <typename U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    template <typename U>
    void construct(U *p) noexcept
    {
        ::new (static_cast<void *>(p)) U;
    }
    template <typename U, typename... Args>
    void construct(U *p, Args &&...args)
    {
        ::new (static_cast<void *>(p)) U(std::forward<Args>(args)...);
    }
};

// Large arrays filled in parallel right after they are sized.
template <typename T>
using BigVec = std::vector<T, NoInitAlloc<T>>;

// Symmetric sparse matrix, CSR with sorted column indices and an explicit
// (possibly zero) diagonal entry in every row.  resize() of its arrays does not
// initialise: every writer fills what it sizes.
struct Csr {
    int n = 0;
    BigVec<int64_t> ptr;
    BigVec<int> col;
    BigVec<double> val;
};

struct MatchResult {
    std::vector<int> match;     // row i -> column match[i] (-1: unmatched)
    std::vector<double> logd;   // symmetric scaling, log d_i
    int unmatched = 0;
};

// Maximum-product transversal (section 6.1, eq. (1)/(2)): minimise
// sum_i c_{i, match(i)} with c_ij = log max_k |a_ik| - log |a_ij| by shortest
// augmenting paths; the optimal duals give the symmetric scaling
// log d_i = (u_i - log max_k|a_ik| + v_i) / 2 (|d_i a_ij d_j| <= 1).
MatchResult max_product_matching(const Csr &A);

// Split the cycles of the matching permutation into 1x1 and 2x2 blocks
// (section 6.2, figures 3 and 4).  Returns blocks as (a, b) with b = -1 for 1x1.
// Values are those of the scaled matrix (scale = exp(logd)).
std::vector<std::pair<int, int>> split_cycles(const Csr &A, const std::vector<int> &match,
                                              const std::vector<double> &logd);

struct SetupParams {
    double drop_tol = 1e-2;   // epsilon (< 0: exact factorisation, nothing dropped)
    double kappa = 5.0;
    double agg_tau = 0.1;
    double schur_tol = 1e-2;
    int coarse_max = 1536;
    int max_levels = 64;
    double z_drop = 1e-2;     // relative drop tolerance of the explicit inverse factor (< 0: none)
    int z_parts = 0;          // segments of the inverse factor (0: default_z_parts(n))
    bool inverse_factor = true;
    bool host_coarse_inverse = true;  // false: leave the dense last level for the device to invert
};

// Device layout of a sparse product (built on the host; the kernel reads it as
// jdmi::Hyb).  The rows are cut into kHybParts contiguous parts of equal nonzero count;
// inside a part, rows with more than kLongRow entries are kept in CSR (longest first,
// one wave each) and the other rows form slices (one wave each).  The tasks of part k are
// its plong[k] long rows, numbered from long0[k], then its slices, numbered from
// slice0[k]: ntask[k] in all.  The slices of R = kSliceRows << c rows with
// g = kSliceLanes >> c lanes per row (c = 0..3: 8 x 8, 16 x 4, 32 x 2, 64 x 1, chosen
// per slice to pad its longest row least): entry j of the slice's row l sits at
// base + (j / g) * 64 + (j % g) * R + l, with base = slice_ptr[s] & ~63 and
// c = slice_ptr[s] & 3; the slice's rows are rowidx[slice_row[s] .. slice_row[s] + R)
// (padding: value 0 and the column of the slice's first entry, so that it reads a
// location the product reads anyway; row -1).  Short rows are sorted by decreasing
// length inside windows of 2048 consecutive rows, so a slice holds rows of similar
// length that are also neighbours in row order.  Row and column numbers are the element offsets the
// kernel writes and reads (see InverseFactor for the buffer they address).
constexpr int kHybParts = 8;
constexpr int kLongRow = 96;
constexpr int kSliceRows = 8;
constexpr int kSliceLanes = 64 / kSliceRows;
struct HybHost {
    int ntask[kHybParts] = {}, plong[kHybParts] = {}, long0[kHybParts] = {}, slice0[kHybParts] = {};
    std::vector<int> long_row;
    std::vector<int64_t> long_ptr{0};
    std::vector<int> long_col;
    std::vector<double> long_val;
    std::vector<int64_t> slice_ptr{0};     // in entries (multiples of 64) | shape code
    std::vector<int64_t> slice_row{0};     // first rowidx entry of each slice
    std::vector<int> rowidx, col;          // rowidx: R per slice, -1 for padding rows
    std::vector<double> val;
};
// CSR with nrows rows -> the hybrid layout; row i is written to row_code[i] (i when NULL).
HybHost to_hyb(int nrows, const int64_t *ptr, const int *col, const double *val, const int *row_code = nullptr);

// The inverse of the unit lower triangular factor of all levels, Z = L^{-1}, applied as
// a product of segments: with the levels cut into consecutive ranges [a, b),
// Z = Z_{S-1} ... Z_1 Z_0 and Z_s = (I - G_{b-1}) ... (I - G_a), each formed explicitly
// (with dropping in the scaled domain).  One explicit Z (S = 1) needs no dependent passes
// but its rows accumulate the fill of every chain through all levels (85 M entries at
// L = 100); cutting the chains at a few level boundaries keeps the apply at 2 S + 3
// launches and stores about a quarter of the entries.  K^{-1} = P^T Z^T D^{-1} Z P.
//
// Numbering.  The input vector is gathered in the Morton order of the lattice sites
// (site_of: Morton index -> site); every other vector uses the middle numbering: blocks
// of kMidBlock consecutive Morton ranks, the unknowns of a block ordered by elimination
// level.  The device works in one buffer of 3 n values, regions [0, n), [n, 2n),
// [2n, 3n):
//   down, segment s: reads region (s == 0 ? 2 (the gathered input, Morton numbering)
//     : the region segment s - 1 wrote); writes its own pivots (and, in the last
//     segment, the last level's unknowns) to region 0, its other rows to region
//     (s even ? 1 : 2);
//   D^{-1} and the last level: region 0 -> region 1;
//   up, segment s = S-1 .. 1: writes its pivots to region 2, reading a position from
//     region 2 when a later segment owns it, else from region 1;
//   up, segment 0: every position, its row numbers the lattice sites (the output vector).
// The layouts store these element offsets directly as row and column numbers.
constexpr int kMidBlock = 128;
struct ZSegment {
    int lev_begin = 0, lev_end = 0;   // levels [lev_begin, lev_end)
    int rows = 0;                      // rows of the down product (unknowns entering lev_begin)
    long long nnz = 0;                 // stored entries, unit diagonal included
    HybHost down, up;
};
struct InverseFactor {
    std::vector<int> site_of;         // n: Morton index -> lattice site
    std::vector<ZSegment> seg;
    std::vector<double> dd, dof;      // D^{-1} (middle numbering): z[q] = dd[q] y[q] + dof[q] y[dp[q]] (0 on the last level)
    std::vector<int> dp;
    std::vector<int> coarse_idx;      // coarse_n: middle index of each unknown of the last level
    long long nnz = 0;                // stored entries of all segments
    double seconds = 0.0;
};

// One level of the multilevel factorisation in global (permuted) positions, with
// every scaling folded into the stored values.
//   rows [off, off+nB) are this level's pivots, rows [off+nB, n) its complement.
//   down pass:  w[r] -= sum G[r, c] w[c]        r >= off+nB, c in [off, off+nB)
//   up pass:    x[j]  = bd[j] w[j] + bo[j] w[bp[j]] - sum GT[j, r] x[r]
struct Level {
    int off = 0, nB = 0, n_after = 0;          // n_after = unknowns of the next level
    int n2x2 = 0;
    std::vector<int64_t> g_ptr;                 // n_after + 1 (rows off+nB .. n-1)
    std::vector<int> g_col;
    std::vector<double> g_val;
    std::vector<int64_t> gt_ptr;                // nB + 1 (rows off .. off+nB-1)
    std::vector<int> gt_col;
    std::vector<double> gt_val;
    std::vector<double> bd, bo;                 // nB
    std::vector<int> bp;                        // nB, global partner position
    int cand_rejected = 0;                      // candidates refused by the kappa test
    double g_min_scaled = 0.0;                  // smallest stored |L21 entry|, scaled domain
    double g_max_colsum = 1.0;                  // largest 1 + sum_r |L21[r, j]| over pivots j
};

struct Multilevel {
    int n = 0;
    std::vector<int> perm;        // perm[position] = original site index
    std::vector<double> pos_scale;  // cumulative symmetric scaling of each position (pivots ~ +-1)
    std::vector<Level> levels;
    int coarse_off = 0, coarse_n = 0;
    int stalls = 0;               // levels after which kappa was raised (the recursion stalled)
    std::vector<double> coarse_inv;  // coarse_n x coarse_n row-major, scalings folded in
    std::vector<double> coarse_mat;  // the last Schur complement itself (when inverted on the device)
    std::vector<double> coarse_scale;  // its cumulative scaling: inverse = diag(s) S^{-1} diag(s)
    long long nnz_lower_A = 0;
    double fill = 0.0;
    double seconds = 0.0;
    InverseFactor z;               // filled when SetupParams::inverse_factor
};

// Default number of segments of the inverse factor for n unknowns.
int default_z_parts(int n);

// The segments of Z (see InverseFactor): level cuts at 1, 3, 9, 27, ... (at most
// `parts` segments); row r of Z_s is e_r - sum over the segment's levels before r's of
// G[r, c] (row c of Z_s), with entries |z_rc| s_r / s_c < z_drop dropped
// (s = pos_scale; z_drop < 0: none), then the device layouts of Z_s and Z_s^T.
void build_inverse_factor(Multilevel &ml, double z_drop, int L, int parts);

// Build the multilevel factorisation of the symmetric matrix A.
// Returns an empty string on success, else a message.
std::string build_multilevel(const Csr &A, const SetupParams &prm, Multilevel &out);

// x = K^{-1} b on the host, in binary64, through the device layouts of the segmented
// inverse factor and in the device's order of products: the input gathered in Morton
// order into region 2 of a 3n workspace, the down products, D^{-1}, the last level
// (ml.coarse_inv, so the setup must have inverted it on the host), the up products,
// the last one writing the lattice sites of x.  A check of the layouts: it returns a
// message if a row or column number leaves its region, a product reads a value it
// writes itself, a part's tasks do not cover its long rows and slices once each, or a
// value is read before any product wrote it; else an empty string.
std::string apply_inverse_factor_host(const Multilevel &ml, const double *b, double *x);

// Host threads used by the setup of the calling thread (OpenMP); <= 0 leaves the default.
void set_setup_threads(int threads);
// OpenMP threads available to the calling thread (OMP_NUM_THREADS when set).
int setup_thread_budget();

// A - sigma I for the Anderson lattice, CSR; bc 0: periodic, 1: hard walls; couplings -1,
// or the bond values hop[d n + s] (bond from site s to s + e_d) when hop is not NULL.
Csr anderson_shifted(int L, const double *eps, double sigma, int bc = 0, const double *hop = nullptr);



}  // namespace jdmi
