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
    bool inverse_factor = true;
    bool host_coarse_inverse = true;  // false: leave the dense last level for the device to invert
};

// Explicit inverse of the unit lower triangular factor of all levels, Z ~ L^{-1}
// (global positions), and the block diagonal D^{-1}: K^{-1} = P^T Z^T D^{-1} Z P.
// The apply does not need the elimination order, so the unknowns are renumbered:
// K^{-1} b = S^T Z^T D^{-1} Z S b with (S b)[q] = b[site_of[q]].  Z's columns (the
// input numbering, also Z^T's rows) follow the Morton order of the lattice sites, so
// that the gathers of neighbouring rows share cache lines; Z's rows (the middle
// numbering of D^{-1}, the last level and Z^T's columns) follow blocks of kMidBlock
// Morton ranks with the unknowns of each block ordered by elimination level.
constexpr int kMidBlock = 128;
struct InverseFactor {
    std::vector<int> site_of;         // n: input index -> lattice site
    BigVec<int64_t> ptr, tptr;        // CSR of Z (rows: middle, columns: input numbering) and of Z^T
    BigVec<int> col, tcol;
    BigVec<double> val, tval;
    std::vector<double> dd, dof;      // D^{-1} (middle numbering): z[q] = dd[q] y[q] + dof[q] y[dp[q]] (0 on the last level)
    std::vector<int> dp;
    std::vector<int> coarse_idx;      // coarse_n: middle index of each unknown of the last level
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

// Z = L^{-1} row by row (row r = e_r - sum over earlier levels of G[r, c] z_c), dropping
// entries with |z_rc| s_r / s_c < z_drop (s = pos_scale), and its transpose.
void build_inverse_factor(Multilevel &ml, double z_drop, int L);

// Build the multilevel factorisation of the symmetric matrix A.
// Returns an empty string on success, else a message.
std::string build_multilevel(const Csr &A, const SetupParams &prm, Multilevel &out);

// Host threads used by the setup of the calling thread (OpenMP); <= 0 leaves the default.
void set_setup_threads(int threads);
// OpenMP threads available to the calling thread (OMP_NUM_THREADS when set).
int setup_thread_budget();

// A - sigma I for the periodic Anderson lattice (hopping -1), CSR.
Csr anderson_shifted(int L, const double *eps, double sigma);

// Device layout of the explicit inverse factor's products (built on the host; the
// kernel reads it as jdmi::Hyb).  The rows (lattice sites in Morton order) are cut into
// kHybParts contiguous parts of equal nonzero count; inside a part, rows with more than
// kLongRow entries are kept in CSR (longest first, one wave each) and the other rows
// form slices of kSliceRows rows with kSliceLanes lanes per row: entry j of the slice's
// row l sits at slice_ptr[s] + (j / kSliceLanes) * 64 + (j % kSliceLanes) * kSliceRows + l
// (padding: index 0, value 0).  Short rows are sorted by decreasing length inside
// windows of 2048 consecutive rows, so a slice holds rows of similar length that are
// also neighbours in position order.
constexpr int kHybParts = 8;
constexpr int kLongRow = 96;
constexpr int kSliceRows = 8;
constexpr int kSliceLanes = 64 / kSliceRows;
struct HybHost {
    int tbeg[kHybParts] = {}, tend[kHybParts] = {};  // task range of each part
    std::vector<int> task;                 // >= 0: long row index; < 0: slice -1 - task
    std::vector<int> long_row;
    std::vector<int64_t> long_ptr{0};
    std::vector<int> long_col;
    std::vector<double> long_val;
    std::vector<int64_t> slice_ptr{0};     // in entries (multiples of 64)
    std::vector<int> rowidx, col;          // rowidx: kSliceRows per slice, -1 for padding rows
    std::vector<double> val;
};
HybHost to_hyb(int n, const int64_t *ptr, const int *col, const double *val);

}  // namespace jdmi
