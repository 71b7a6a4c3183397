// Host setup of the multilevel incomplete LDL^T (sections 6 and 7).
//
// GPU-first reading of the paper's level structure: the symmetric ordering Pi of
// each level (section 7.1) puts an independent set of the compressed 1x1/2x2 block
// graph first.  The leading block of that level is then exactly the block diagonal
// D11 of 1x1 and 2x2 pivots and L11 = I, so the factor of a level is the coupling
// block L21 = F D11^{-1} alone, and applying a level costs two fully parallel sparse
// passes instead of a level-scheduled triangular solve.  Everything else follows the
// paper's order: maximum weight matching, cycle split into 1x1/2x2 blocks, symmetric
// scaling, inverse-based acceptance of pivots with bound kappa (postponed pivots go
// to the next level), dropping with epsilon/kappa and the aggressive tau rule,
// explicit Schur complement of the postponed part, recursion, exact last level.
#include "setup.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <tuple>
#include <utility>
#include <cstdio>
#include <cstdlib>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace jdmi {

namespace {
constexpr double kInf = std::numeric_limits<double>::infinity();

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

inline double get(const Csr &A, int i, int j)
{
    auto b = A.col.begin() + A.ptr[i], e = A.col.begin() + A.ptr[i + 1];
    auto it = std::lower_bound(b, e, j);
    return (it != e && *it == j) ? A.val[it - A.col.begin()] : 0.0;
}
}  // namespace

int setup_thread_budget()
{
#ifdef _OPENMP
    return std::max(1, omp_get_max_threads());
#else
    return 1;
#endif
}

void set_setup_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

Csr anderson_shifted(int L, const double *eps, double sigma, int bc, const double *hop)
{
    const bool wall = bc != 0;
    const int64_t nn = int64_t(L) * L * L;
    // coupling of the bond from site a to a + e_d (d = 0, 1, 2), -1 without bond values
    auto t = [&](int d, int a) { return hop ? hop[d * nn + a] : -1.0; };
    const int n = L * L * L;
    Csr A;
    A.n = n;
    A.ptr.assign(n + 1, 0);
    A.col.reserve(size_t(n) * 7);
    A.val.reserve(size_t(n) * 7);
    for (int s = 0; s < n; ++s) {
        const int i = s % L, j = (s / L) % L, k = s / (L * L);
        std::pair<int, double> e[7];
        int m = 0;
        auto add = [&](int c, double v) {
            for (int t = 0; t < m; ++t)
                if (e[t].first == c) { e[t].second += v; return; }
            e[m++] = {c, v};
        };
        add(s, eps[s] - sigma);
        // with hard walls a neighbour across a face of the box is absent
        const int xm = (i + L - 1) % L + L * (j + L * k), ym = i + L * ((j + L - 1) % L + L * k);
        const int zm = i + L * (j + L * ((k + L - 1) % L));
        if (!wall || i < L - 1) add((i + 1) % L + L * (j + L * k), t(0, s));
        if (!wall || i > 0) add(xm, t(0, xm));
        if (!wall || j < L - 1) add(i + L * ((j + 1) % L + L * k), t(1, s));
        if (!wall || j > 0) add(ym, t(1, ym));
        if (!wall || k < L - 1) add(i + L * (j + L * ((k + 1) % L)), t(2, s));
        if (!wall || k > 0) add(zm, t(2, zm));
        std::sort(e, e + m);
        for (int t = 0; t < m; ++t) { A.col.push_back(e[t].first); A.val.push_back(e[t].second); }
        A.ptr[s + 1] = int64_t(A.col.size());
    }
    return A;
}

// ---------------------------------------------------------------------------------
// Maximum-product matching by shortest augmenting paths (Dijkstra on reduced costs).
// ---------------------------------------------------------------------------------
MatchResult max_product_matching(const Csr &A)
{
    const int n = A.n;
    std::vector<double> lmax(n, -kInf);
    std::vector<double> cost(A.val.size());
    std::vector<int64_t> first_tight(n);  // first entry of each row with zero cost (or -1)
#pragma omp parallel for schedule(dynamic, 4096)
    for (int i = 0; i < n; ++i) {
        double m = -kInf;
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            cost[p] = (A.val[p] != 0.0) ? std::log(std::fabs(A.val[p])) : -kInf;
            m = std::max(m, cost[p]);
        }
        lmax[i] = m;
        first_tight[i] = -1;
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            cost[p] = (A.val[p] != 0.0) ? m - cost[p] : kInf;
            if (cost[p] == 0.0 && first_tight[i] < 0) first_tight[i] = p;
        }
    }
    std::vector<double> u(n, 0.0), v(n, 0.0);  // c_ij >= 0 and min_j c_ij = 0: feasible
    std::vector<int> rmatch(n, -1), cmatch(n, -1);
    // greedy start on tight edges: each row, in order, takes its first tight entry whose
    // column is still free
    for (int i = 0; i < n; ++i) {
        if (first_tight[i] < 0) continue;
        for (int64_t p = first_tight[i]; p < A.ptr[i + 1]; ++p) {
            const int j = A.col[p];
            if (cost[p] == 0.0 && cmatch[j] < 0) { rmatch[i] = j; cmatch[j] = i; break; }
        }
    }
    std::vector<double> d(n, kInf);
    std::vector<int> pred(n, -1);
    std::vector<char> scanned(n, 0);
    std::vector<int> touched, scanned_list;
    using HE = std::pair<double, int>;
    std::vector<HE> heap;  // binary min-heap on (distance, column), reused by every search
    const std::greater<HE> later;
    int unmatched = 0;
    for (int i0 = 0; i0 < n; ++i0) {
        if (rmatch[i0] >= 0) continue;
        heap.clear();
        touched.clear();
        scanned_list.clear();
        auto relax_row = [&](int i, double base) {
            for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                if (cost[p] == kInf) continue;
                const int j = A.col[p];
                if (scanned[j]) continue;
                const double nd = base + cost[p] - u[i] - v[j];
                if (nd < d[j]) {
                    if (d[j] == kInf) touched.push_back(j);
                    d[j] = nd;
                    pred[j] = i;
                    heap.push_back({nd, j});
                    std::push_heap(heap.begin(), heap.end(), later);
                }
            }
        };
        relax_row(i0, 0.0);
        int sink = -1;
        double delta = 0.0;
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), later);
            const auto [dj, j] = heap.back();
            heap.pop_back();
            if (scanned[j] || dj > d[j]) continue;
            scanned[j] = 1;
            if (cmatch[j] < 0) { sink = j; delta = dj; break; }
            scanned_list.push_back(j);
            relax_row(cmatch[j], dj);
        }
        if (sink >= 0) {
            // dual update keeps c_ij - u_i - v_j >= 0, = 0 on the matching
            u[i0] += delta;
            for (int j : scanned_list) {
                const double t = delta - d[j];
                u[cmatch[j]] += t;
                v[j] -= t;
            }
            // augment along the predecessor chain
            int j = sink;
            while (true) {
                const int i = pred[j];
                const int nxt = rmatch[i];
                rmatch[i] = j;
                cmatch[j] = i;
                if (i == i0) break;
                j = nxt;
            }
        } else {
            ++unmatched;
        }
        for (int j : touched) { d[j] = kInf; pred[j] = -1; scanned[j] = 0; }
        if (sink >= 0) scanned[sink] = 0;
        for (int j : scanned_list) scanned[j] = 0;
    }
    MatchResult r;
    r.match = rmatch;
    r.unmatched = unmatched;
    r.logd.resize(n);
    for (int i = 0; i < n; ++i) {
        if (unmatched == 0)
            r.logd[i] = 0.5 * (u[i] - lmax[i] + v[i]);
        else
            r.logd[i] = -0.5 * lmax[i];  // no perfect matching: row-maximum equilibration
        if (!std::isfinite(r.logd[i])) r.logd[i] = 0.0;
    }
    return r;
}

// ---------------------------------------------------------------------------------
// Cycle split (section 6.2).  Tie rules (the paper names a structural criterion for
// choosing the pairs without defining it): minimise the summed size of the union of the two rows' patterns
// over the pairs, then maximise the product of the pairs' scaled couplings, then
// take the first candidate; in odd cycles the 1x1 element must have a nonzero
// diagonal when possible.
// ---------------------------------------------------------------------------------
std::vector<std::pair<int, int>> split_cycles(const Csr &A, const std::vector<int> &match,
                                              const std::vector<double> &logd)
{
    const int n = A.n;
    // the cycles (and open chains) of the matching, in order of their first unknown
    std::vector<int> nodes, cstart{0};
    std::vector<char> closed;
    {
        std::vector<char> seen(n, 0);
        for (int s = 0; s < n; ++s) {
            if (seen[s]) continue;
            int t = s;
            while (t >= 0 && !seen[t]) { seen[t] = 1; nodes.push_back(t); t = match[t]; }
            cstart.push_back(int(nodes.size()));
            closed.push_back(t == s);
        }
    }
    const int ncyc = int(closed.size());
    // blocks per cycle, known from its length and kind: the output keeps cycle order
    std::vector<int64_t> boff(ncyc + 1, 0);
    for (int c = 0; c < ncyc; ++c) {
        const int m = cstart[c + 1] - cstart[c];
        boff[c + 1] = boff[c] + (m == 1 ? 1 : (!closed[c] || m % 2 == 0) ? (m + 1) / 2 : 1 + (m - 1) / 2);
    }
    std::vector<std::pair<int, int>> blocks(boff[ncyc]);
    auto coupling = [&](int a, int b) {
        return std::fabs(get(A, a, b)) * std::exp(logd[a] + logd[b]);
    };
#pragma omp parallel
    {
        std::vector<int> mark(n, -1);
        int stamp = 0;
        auto union_size = [&](int a, int b) {
            ++stamp;
            int c = 0;
            for (int64_t p = A.ptr[a]; p < A.ptr[a + 1]; ++p) { mark[A.col[p]] = stamp; ++c; }
            for (int64_t p = A.ptr[b]; p < A.ptr[b + 1]; ++p)
                if (mark[A.col[p]] != stamp) { mark[A.col[p]] = stamp; ++c; }
            return c;
        };
        std::vector<double> pu, pc;
#pragma omp for schedule(dynamic, 256)
        for (int ci = 0; ci < ncyc; ++ci) {
            const int *cyc = nodes.data() + cstart[ci];
            const int m = cstart[ci + 1] - cstart[ci];
            std::pair<int, int> *out = blocks.data() + boff[ci];
            if (m == 1) { out[0] = {cyc[0], -1}; continue; }
            if (!closed[ci]) {
                // an open chain (only when the matching is not perfect): pair consecutively
                int q = 0;
                for (; q + 1 < m; q += 2) *out++ = {cyc[q], cyc[q + 1]};
                if (q < m) *out++ = {cyc[q], -1};
                continue;
            }
            // pair metrics for consecutive positions q -> q+1 (mod m)
            pu.assign(m, 0.0);
            pc.assign(m, 0.0);
            for (int q = 0; q < m; ++q) {
                const int a = cyc[q], b = cyc[(q + 1) % m];
                pu[q] = union_size(a, b);
                pc[q] = std::log(std::max(coupling(a, b), 1e-300));
            }
            if (m % 2 == 0) {
                double u0 = 0, u1 = 0, c0 = 0, c1 = 0;
                for (int q = 0; q < m; q += 2) { u0 += pu[q]; c0 += pc[q]; }
                for (int q = 1; q < m; q += 2) { u1 += pu[q]; c1 += pc[q]; }
                const int st = (u1 < u0 || (u1 == u0 && c1 > c0)) ? 1 : 0;
                for (int q = st; q < m + st; q += 2) *out++ = {cyc[q % m], cyc[(q + 1) % m]};
            } else {
                int best = -1;
                double bu = kInf, bc = -kInf;
                bool bnz = false;
                const int lim = std::min(m, 257);  // very long cycles: first choices only
                for (int sgl = 0; sgl < lim; ++sgl) {
                    const bool nz = get(A, cyc[sgl], cyc[sgl]) != 0.0;
                    double us = 0, cs = 0;
                    for (int q = sgl + 1; q < sgl + m; q += 2) { us += pu[q % m]; cs += pc[q % m]; }
                    bool better;
                    if (best < 0) better = true;
                    else if (nz != bnz) better = nz;
                    else if (us != bu) better = us < bu;
                    else better = cs > bc;
                    if (better) { best = sgl; bu = us; bc = cs; bnz = nz; }
                }
                *out++ = {cyc[best], -1};
                for (int q = best + 1; q < best + m; q += 2) *out++ = {cyc[q % m], cyc[(q + 1) % m]};
            }
        }
    }
    return blocks;
}

// ---------------------------------------------------------------------------------
// Dense inverse by LU with partial pivoting (last level).
// ---------------------------------------------------------------------------------
static bool dense_inverse(int n, std::vector<double> &a)
{
    std::vector<double> inv(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
    double amax = 0;
    for (double x : a) amax = std::max(amax, std::fabs(x));
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = std::fabs(a[size_t(c) * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[size_t(r) * n + c]) > best) { best = std::fabs(a[size_t(r) * n + c]); piv = r; }
        if (!(best > 1e-14 * std::max(amax, 1e-300))) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                std::swap(a[size_t(c) * n + k], a[size_t(piv) * n + k]);
                std::swap(inv[size_t(c) * n + k], inv[size_t(piv) * n + k]);
            }
        }
        const double pinv = 1.0 / a[size_t(c) * n + c];
        for (int k = 0; k < n; ++k) { a[size_t(c) * n + k] *= pinv; inv[size_t(c) * n + k] *= pinv; }
        const double *arow = &a[size_t(c) * n];
        const double *irow = &inv[size_t(c) * n];
#pragma omp parallel for schedule(static)
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a[size_t(r) * n + c];
            if (f == 0.0) continue;
            double *ar = &a[size_t(r) * n];
            double *ir = &inv[size_t(r) * n];
            for (int k = 0; k < n; ++k) { ar[k] -= f * arow[k]; ir[k] -= f * irow[k]; }
        }
    }
    // symmetrise (the exact inverse of a symmetric matrix is symmetric)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (inv[size_t(i) * n + j] + inv[size_t(j) * n + i]);
            inv[size_t(i) * n + j] = inv[size_t(j) * n + i] = s;
        }
    a.swap(inv);
    return true;
}

// ---------------------------------------------------------------------------------
// One level.
// ---------------------------------------------------------------------------------
namespace {

struct LevelLocal {
    // in level-local numbering (0..n-1 of this level's matrix)
    std::vector<int> B, C;           // pivots (block members adjacent), complement
    std::vector<int> partner;        // level-local partner (self for 1x1), for B members
    std::vector<double> bd, bo;      // scaled block inverse entries for B members
    // G over C rows (local C index) -> B local index, scaled domain
    std::vector<int64_t> g_ptr;
    std::vector<int> g_col;
    std::vector<double> g_val;
    int n2x2 = 0, rejected = 0;
    double g_min = 0.0, g_colsum = 1.0;
};

// scaled value
struct Scaled {
    const Csr &A;
    const std::vector<double> &d;
    double operator()(int64_t p, int i) const { return A.val[p] * d[i] * d[A.col[p]]; }
};

}  // namespace

// Transpose of an n x n CSR matrix, built in parallel from per-thread column counts
// over fixed row ranges: the rows of the transpose list their entries in increasing
// row order, exactly as a serial pass over the rows would.
static void transpose(int n, const BigVec<int64_t> &ptr, const BigVec<int> &col, const BigVec<double> &val,
                      BigVec<int64_t> &tptr, BigVec<int> &tcol, BigVec<double> &tval)
{
    tptr.assign(n + 1, 0);
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    std::vector<std::vector<int64_t>> cnt(nt, std::vector<int64_t>(n + 1, 0));
    auto range = [&](int t, int &a, int &b) {
        a = int(int64_t(n) * t / nt);
        b = int(int64_t(n) * (t + 1) / nt);
    };
    // one iteration per row range: every range is done whatever the team size
#pragma omp parallel for schedule(static, 1)
    for (int t = 0; t < nt; ++t) {
        int a, b;
        range(t, a, b);
        auto &c = cnt[t];
        for (int r = a; r < b; ++r)
            for (int64_t p = ptr[r]; p < ptr[r + 1]; ++p) ++c[col[p]];
    }
    // offsets: column c of thread t starts after the entries of c from threads < t
    for (int c = 0; c < n; ++c) {
        int64_t o = tptr[c];
        for (int t = 0; t < nt; ++t) {
            const int64_t k = cnt[t][c];
            cnt[t][c] = o;
            o += k;
        }
        tptr[c + 1] = o;
    }
    tcol.resize(tptr[n]);
    tval.resize(tptr[n]);
#pragma omp parallel for schedule(static, 1)
    for (int t = 0; t < nt; ++t) {
        int a, b;
        range(t, a, b);
        auto &fp = cnt[t];
        for (int r = a; r < b; ++r)
            for (int64_t p = ptr[r]; p < ptr[r + 1]; ++p) {
                const int c = col[p];
                tcol[fp[c]] = r;
                tval[fp[c]++] = val[p];
            }
    }
}

// (S + S^T) / 2 on the union pattern, rows sorted; the merge counts each output row,
// then writes it.
static Csr symmetrize(const Csr &S)
{
    const int n = S.n;
    Csr T;
    T.n = n;
    transpose(n, S.ptr, S.col, S.val, T.ptr, T.col, T.val);
    Csr U;
    U.n = n;
    U.ptr.assign(n + 1, 0);
    // merged length of row r of S and row r of T (both sorted)
    auto merge = [&](int r, int *col, double *val) {
        int64_t a = S.ptr[r], ae = S.ptr[r + 1], b = T.ptr[r], be = T.ptr[r + 1], k = 0;
        while (a < ae || b < be) {
            int c;
            double v;
            if (b >= be || (a < ae && S.col[a] < T.col[b])) { c = S.col[a]; v = 0.5 * S.val[a]; ++a; }
            else if (a >= ae || T.col[b] < S.col[a]) { c = T.col[b]; v = 0.5 * T.val[b]; ++b; }
            else { c = S.col[a]; v = 0.5 * (S.val[a] + T.val[b]); ++a; ++b; }
            if (col) { col[k] = c; val[k] = v; }
            ++k;
        }
        return k;
    };
#pragma omp parallel for schedule(dynamic, 256)
    for (int r = 0; r < n; ++r) U.ptr[r + 1] = merge(r, nullptr, nullptr);
    for (int r = 0; r < n; ++r) U.ptr[r + 1] += U.ptr[r];
    U.col.resize(U.ptr[n]);
    U.val.resize(U.ptr[n]);
#pragma omp parallel for schedule(dynamic, 256)
    for (int r = 0; r < n; ++r) merge(r, U.col.data() + U.ptr[r], U.val.data() + U.ptr[r]);
    return U;
}

static std::string factor_level(const Csr &A, const SetupParams &prm, const std::vector<double> &d,
                                const std::vector<std::pair<int, int>> &blocks, const std::vector<uint64_t> &key,
                                LevelLocal &lv, Csr &S_next)
{
    const int n = A.n;
    const bool exact = prm.drop_tol < 0;
    const double kappa = exact ? kInf : prm.kappa;
    auto sv = [&](int64_t p, int i) { return A.val[p] * d[i] * d[A.col[p]]; };
    auto sget = [&](int i, int j) { return get(A, i, j) * d[i] * d[j]; };

    // candidate pivots with their inverse-bound measure (1-norm of the L columns)
    struct Cand { int a, b; double q; int deg; double i00, i01, i11; };
    std::vector<Cand> cands;
    cands.reserve(blocks.size() + 16);
    auto colsum1 = [&](int i) {
        double s = 0;
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
            if (A.col[p] != i) s += std::fabs(sv(p, i));
        return s;
    };
    // every block is evaluated on its own (in parallel), then the candidates are
    // collected in block order
    std::vector<std::array<Cand, 2>> per(blocks.size());
    std::vector<int> nper(blocks.size(), 0);
#pragma omp parallel
    {
        std::vector<std::pair<int, double>> ra, rb;  // per-thread buffers, reused by every block
#pragma omp for schedule(dynamic, 2048)
        for (int64_t bi = 0; bi < int64_t(blocks.size()); ++bi) {
            const int a = blocks[bi].first, b = blocks[bi].second;
            auto put = [&](const Cand &c) { per[bi][nper[bi]++] = c; };
            auto push1l = [&](int i) {
                const double dii = sget(i, i);
                if (!(std::fabs(dii) > 0.0)) return;
                put({i, -1, colsum1(i) / std::fabs(dii), int(A.ptr[i + 1] - A.ptr[i]), 1.0 / dii, 0.0, 0.0});
            };
            if (b < 0) { push1l(a); continue; }
            const double saa = sget(a, a), sab = sget(a, b), sbb = sget(b, b);
            const double det = saa * sbb - sab * sab;
            const double scale = std::max({std::fabs(saa), std::fabs(sbb), std::fabs(sab)});
            double d2 = kInf, cs_a = 0, cs_b = 0;
            double i00 = 0, i01 = 0, i11 = 0;
            if (std::fabs(det) > 1e-12 * scale * scale) {
                i00 = sbb / det; i01 = -sab / det; i11 = saa / det;
                // rows of (s_r,a  s_r,b) S2^{-1} over the union of both columns' rows
                d2 = 0;
                ra.clear();
                rb.clear();
                for (int64_t p = A.ptr[a]; p < A.ptr[a + 1]; ++p)
                    if (A.col[p] != a && A.col[p] != b) ra.push_back({A.col[p], sv(p, a)});
                for (int64_t p = A.ptr[b]; p < A.ptr[b + 1]; ++p)
                    if (A.col[p] != a && A.col[p] != b) rb.push_back({A.col[p], sv(p, b)});
                size_t x = 0, y = 0;
                while (x < ra.size() || y < rb.size()) {
                    int r;
                    double va = 0, vb = 0;
                    if (y >= rb.size() || (x < ra.size() && ra[x].first < rb[y].first)) { r = ra[x].first; va = ra[x++].second; }
                    else if (x >= ra.size() || rb[y].first < ra[x].first) { r = rb[y].first; vb = rb[y++].second; }
                    else { r = ra[x].first; va = ra[x++].second; vb = rb[y++].second; }
                    (void)r;
                    const double za = va * i00 + vb * i01, zb = va * i01 + vb * i11;
                    d2 += std::max(std::fabs(za), std::fabs(zb));  // infinity norm of the row
                    cs_a += std::fabs(za);
                    cs_b += std::fabs(zb);
                }
            }
            const double d1a = (saa != 0.0) ? colsum1(a) / std::fabs(saa) : kInf;
            const double d1b = (sbb != 0.0) ? colsum1(b) / std::fabs(sbb) : kInf;
            if (d2 < std::min(d1a, d1b)) {
                int deg = int(A.ptr[a + 1] - A.ptr[a] + A.ptr[b + 1] - A.ptr[b]);
                put({a, b, std::max(cs_a, cs_b), deg, i00, i01, i11});
            } else {
                push1l(a);
                push1l(b);
            }
        }
    }
    for (size_t bi = 0; bi < blocks.size(); ++bi)
        for (int t = 0; t < nper[bi]; ++t) cands.push_back(per[bi][t]);
    // greedy independent set of the compressed graph: fewest couplings first, ties by
    // the smallest member.  Every unknown belongs to exactly one candidate, so the key
    // (couplings, smallest member) is distinct per candidate and fixes the order.
    std::vector<int> order(cands.size());
    {
        std::vector<int> cand_of_first(n, -1);
        std::vector<uint64_t> keyed(cands.size());
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const Cand &c = cands[ci];
            const int first = c.b < 0 ? c.a : std::min(c.a, c.b);
            cand_of_first[first] = int(ci);
            keyed[ci] = (uint64_t(uint32_t(c.deg)) << 32) | uint32_t(first);
        }
        std::sort(keyed.begin(), keyed.end());
        for (size_t k = 0; k < keyed.size(); ++k) order[k] = cand_of_first[uint32_t(keyed[k])];
    }
    enum : char { FREE = 0, INB = 1, INC = 2 };
    std::vector<char> state(n, FREE);
    std::vector<int> cand_of(n, -1);
    int rejected = 0;
    for (int ci : order) {
        const Cand &c = cands[ci];
        if (state[c.a] != FREE || (c.b >= 0 && state[c.b] != FREE)) continue;
        if (!(1.0 + c.q <= kappa)) { ++rejected; continue; }  // postponed
        state[c.a] = INB;
        cand_of[c.a] = ci;
        if (c.b >= 0) { state[c.b] = INB; cand_of[c.b] = ci; }
        for (int v : {c.a, c.b}) {
            if (v < 0) continue;
            for (int64_t p = A.ptr[v]; p < A.ptr[v + 1]; ++p)
                if (state[A.col[p]] == FREE) state[A.col[p]] = INC;
        }
    }
    lv.B.clear();
    lv.C.clear();
    std::vector<int> loc(n, -1);
    for (int i = 0; i < n; ++i) {
        if (state[i] == INB) lv.B.push_back(i);
        else { loc[i] = int(lv.C.size()); lv.C.push_back(i); }
    }
    // pivots of the level in Morton order of their lattice sites: the order only sets
    // memory positions, and keeps lattice neighbours close in the device vectors
    std::stable_sort(lv.B.begin(), lv.B.end(), [&](int a, int b) { return key[a] < key[b]; });
    for (size_t t = 0; t < lv.B.size(); ++t) loc[lv.B[t]] = int(t);
    const int nB = int(lv.B.size()), nC = int(lv.C.size());
    lv.rejected = rejected;
    lv.partner.assign(nB, 0);
    lv.bd.assign(nB, 0.0);
    lv.bo.assign(nB, 0.0);
    lv.n2x2 = 0;
    for (int t = 0; t < nB; ++t) {
        const int i = lv.B[t];
        const Cand &c = cands[cand_of[i]];
        if (c.b < 0) { lv.partner[t] = t; lv.bd[t] = c.i00; lv.bo[t] = 0.0; }
        else if (i == c.a) { lv.partner[t] = loc[c.b]; lv.bd[t] = c.i00; lv.bo[t] = c.i01; ++lv.n2x2; }
        else { lv.partner[t] = loc[c.a]; lv.bd[t] = c.i11; lv.bo[t] = c.i01; }
    }
    // G = F B^{-1} over C rows, scaled domain, then dropping
    std::vector<std::vector<std::pair<int, double>>> grow(nC);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int r = 0; r < nC; ++r) {
        const int i = lv.C[r];
        auto &row = grow[r];
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            const int j = A.col[p];
            if (state[j] != INB) continue;
            const double f = sv(p, i);
            const int tj = loc[j], tp = lv.partner[tj];
            auto add = [&](int c, double v) {
                for (auto &e : row) if (e.first == c) { e.second += v; return; }
                row.push_back({c, v});
            };
            add(tj, f * lv.bd[tj]);
            if (tp != tj) add(tp, f * lv.bo[tj]);
        }
        std::sort(row.begin(), row.end());
    }
    if (!exact) {
        const double thr = prm.drop_tol / prm.kappa;
        std::vector<int> cnt(nB, 0);
        for (auto &row : grow) {
            size_t w = 0;
            for (auto &e : row)
                if (std::fabs(e.second) >= thr) row[w++] = e;
            row.resize(w);
            for (auto &e : row) ++cnt[e.first];
        }
        // aggressive dropping: |l_rj| <= tau / (nu_r * nnz(column j)); nu_r = 1 for
        // rows of the complement since L^{-1} e_r = e_r there.
        for (auto &row : grow) {
            size_t w = 0;
            for (auto &e : row)
                if (std::fabs(e.second) > prm.agg_tau / std::max(cnt[e.first], 1)) row[w++] = e;
            row.resize(w);
        }
    }
    {
        // invariants of the stored factor columns (reported for checks)
        double mn = kInf;
        std::vector<double> cs(nB, 0.0);
        for (auto &row : grow)
            for (auto &e : row) { mn = std::min(mn, std::fabs(e.second)); cs[e.first] += std::fabs(e.second); }
        double mx = 1.0;
        for (double v : cs) mx = std::max(mx, 1.0 + v);
        lv.g_min = mn;
        lv.g_colsum = mx;
    }
    lv.g_ptr.assign(nC + 1, 0);
    for (int r = 0; r < nC; ++r) lv.g_ptr[r + 1] = lv.g_ptr[r] + int64_t(grow[r].size());
    lv.g_col.resize(lv.g_ptr[nC]);
    lv.g_val.resize(lv.g_ptr[nC]);
    for (int r = 0; r < nC; ++r) {
        int64_t p = lv.g_ptr[r];
        for (auto &e : grow[r]) { lv.g_col[p] = e.first; lv.g_val[p] = e.second; ++p; }
    }
    grow.clear();
    grow.shrink_to_fit();
    // H^T = B G^T by B rows: HT[t, r] = sum_{t' in block(t)} B[t, t'] G[r, t']
    //   with B the scaled pivot block itself (not its inverse).
    std::vector<int64_t> gt_ptr(nB + 1, 0);
    for (int r = 0; r < nC; ++r)
        for (int64_t p = lv.g_ptr[r]; p < lv.g_ptr[r + 1]; ++p) ++gt_ptr[lv.g_col[p] + 1];
    for (int t = 0; t < nB; ++t) gt_ptr[t + 1] += gt_ptr[t];
    std::vector<int> gt_col(gt_ptr[nB]);
    std::vector<double> gt_val(gt_ptr[nB]);
    {
        std::vector<int64_t> fillp(gt_ptr.begin(), gt_ptr.end() - 1);
        for (int r = 0; r < nC; ++r)
            for (int64_t p = lv.g_ptr[r]; p < lv.g_ptr[r + 1]; ++p) {
                const int t = lv.g_col[p];
                gt_col[fillp[t]] = r;
                gt_val[fillp[t]++] = lv.g_val[p];
            }
    }
    // scaled pivot block entries
    std::vector<double> Bd(nB), Bo(nB);
    for (int t = 0; t < nB; ++t) {
        const int i = lv.B[t];
        Bd[t] = sget(i, i);
        Bo[t] = (lv.partner[t] != t) ? sget(i, lv.B[lv.partner[t]]) : 0.0;
    }
    // Schur complement S = C - G B G^T (rows of C), row by row
    const double stol = exact ? -1.0 : prm.schur_tol;
    S_next.n = nC;
    std::vector<std::vector<std::pair<int, double>>> srow(nC);
#pragma omp parallel
    {
        std::vector<double> acc(nC, 0.0);
        std::vector<int> mark(nC, -1), list;
#pragma omp for schedule(dynamic, 64)
        for (int r = 0; r < nC; ++r) {
            list.clear();
            const int i = lv.C[r];
            auto put = [&](int c, double v) {
                if (mark[c] != r) { mark[c] = r; acc[c] = 0.0; list.push_back(c); }
                acc[c] += v;
            };
            put(r, 0.0);  // keep the diagonal
            for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
                const int j = A.col[p];
                if (state[j] == INB) continue;
                put(loc[j], sv(p, i));
            }
            for (int64_t p = lv.g_ptr[r]; p < lv.g_ptr[r + 1]; ++p) {
                const int t = lv.g_col[p];
                const double g = lv.g_val[p];
                const int tp = lv.partner[t];
                // (G B)[r, t'] for t' in block -> times G[c, t'] ... use HT rows
                // contribution: g * sum_{c} (B G^T)[t, c]
                for (int64_t q = gt_ptr[t]; q < gt_ptr[t + 1]; ++q) put(gt_col[q], -g * Bd[t] * gt_val[q]);
                if (tp != t)
                    for (int64_t q = gt_ptr[tp]; q < gt_ptr[tp + 1]; ++q) put(gt_col[q], -g * Bo[t] * gt_val[q]);
            }
            auto &out = srow[r];
            for (int c : list) {
                const double v = acc[c];
                if (c == r || std::fabs(v) >= stol) out.push_back({c, v});
            }
            std::sort(out.begin(), out.end());  // columns are distinct: sorts by column
        }
    }
    S_next.ptr.assign(nC + 1, 0);
    for (int r = 0; r < nC; ++r) S_next.ptr[r + 1] = S_next.ptr[r] + int64_t(srow[r].size());
    S_next.col.resize(S_next.ptr[nC]);
    S_next.val.resize(S_next.ptr[nC]);
#pragma omp parallel for schedule(dynamic, 256)
    for (int r = 0; r < nC; ++r) {
        int64_t p = S_next.ptr[r];
        for (auto &e : srow[r]) { S_next.col[p] = e.first; S_next.val[p] = e.second; ++p; }
        std::vector<std::pair<int, double>>().swap(srow[r]);
    }
    // the computed Schur complement is symmetric up to rounding; enforce it by
    // averaging mirrored entries and keeping the union pattern
    S_next = symmetrize(S_next);
    return "";
}

// Morton (bit-interleaved) code of the site s = i + L (j + L k)
static uint64_t morton(int s, int L)
{
    if (L <= 0) return uint64_t(s);
    const uint64_t i = uint64_t(s % L), j = uint64_t((s / L) % L), k = uint64_t(s / L / L);
    uint64_t m = 0;
    for (int b = 0; b < 21; ++b)
        m |= (((i >> b) & 1ull) << (3 * b)) | (((j >> b) & 1ull) << (3 * b + 1)) | (((k >> b) & 1ull) << (3 * b + 2));
    return m;
}

std::string build_multilevel(const Csr &A0, const SetupParams &prm, Multilevel &out)
{
    // lattice edge for the locality order (0 if n is not a cube)
    int L = int(std::lround(std::cbrt(double(A0.n))));
    if (int64_t(L) * L * L != A0.n) L = 0;
    const double t0 = now_s();
    const int n = A0.n;
    out = Multilevel();
    out.n = n;
    {
        long long low = 0;
        for (int i = 0; i < n; ++i)
            for (int64_t p = A0.ptr[i]; p < A0.ptr[i + 1]; ++p)
                if (A0.col[p] <= i) ++low;
        out.nnz_lower_A = low;
    }
    struct Pending {
        LevelLocal lv;
        std::vector<double> cum;   // cumulative scaling of this level's unknowns (incl. own d)
        int off;
    };
    std::vector<Pending> pend;
    Csr S = A0;
    std::vector<int> orig(n);
    std::iota(orig.begin(), orig.end(), 0);
    std::vector<double> cum_prev(n, 1.0);
    // level-local -> original sites of B members, per level, to build the permutation
    std::vector<std::vector<int>> level_orig;
    int off = 0;
    const bool verbose = std::getenv("JDMI_VERBOSE") != nullptr;
    double t_match = 0, t_split = 0, t_fact = 0;
    // kappa of the current level: doubled (up to kKappaMax) after a level that accepted
    // fewer than 1% of its unknowns while the rest is still too large for the exact last
    // level, so that a stalled recursion keeps shrinking.  A higher cap (1000) also ended
    // every recursion tried, but its pivots left preconditioners under which JD did not
    // converge at all (W = 12, L = 60)
    SetupParams lp = prm;
    constexpr double kKappaMax = 20.0;
    while (S.n > prm.coarse_max && int(pend.size()) < prm.max_levels) {
        double ta = now_s();
        MatchResult mr = max_product_matching(S);
        double tb = now_s();
        auto blocks = split_cycles(S, mr.match, mr.logd);
        double tc = now_s();
        std::vector<double> d(S.n);
        for (int i = 0; i < S.n; ++i) d[i] = std::exp(mr.logd[i]);
        Pending pl;
        Csr Snext;
        std::vector<uint64_t> key(S.n);
        for (int i = 0; i < S.n; ++i) key[i] = morton(orig[i], L);
        std::string err = factor_level(S, lp, d, blocks, key, pl.lv, Snext);
        double td = now_s();
        t_match += tb - ta; t_split += tc - tb; t_fact += td - tc;
        if (verbose)
            fprintf(stderr, "level %zu: n %d nnz %lld nB %zu 2x2 %d rej %d kappa %g | match %.3fs split %.3fs factor %.3fs\n",
                    pend.size(), S.n, (long long)S.col.size(), pl.lv.B.size(), pl.lv.n2x2, pl.lv.rejected, lp.kappa,
                    tb - ta, tc - tb, td - tc);
        if (!err.empty()) return err;
        // no acceptable pivot, or the level barely shrinks and the rest fits the
        // exactly inverted last level: stop the recursion here
        if (pl.lv.B.empty() || (int64_t(pl.lv.B.size()) * 100 < S.n && S.n <= 8192)) break;
        if (int64_t(pl.lv.B.size()) * 100 < S.n && lp.drop_tol >= 0) {
            lp.kappa = std::min(2.0 * lp.kappa, std::max(kKappaMax, prm.kappa));
            ++out.stalls;
        }
        pl.cum.resize(S.n);
        for (int i = 0; i < S.n; ++i) pl.cum[i] = cum_prev[i] * d[i];
        pl.off = off;
        std::vector<int> bo(pl.lv.B.size()), co(pl.lv.C.size());
        for (size_t t = 0; t < pl.lv.B.size(); ++t) bo[t] = orig[pl.lv.B[t]];
        for (size_t t = 0; t < pl.lv.C.size(); ++t) co[t] = orig[pl.lv.C[t]];
        std::vector<double> cum_next(pl.lv.C.size());
        for (size_t t = 0; t < pl.lv.C.size(); ++t) cum_next[t] = pl.cum[pl.lv.C[t]];
        level_orig.push_back(bo);
        off += int(pl.lv.B.size());
        orig.swap(co);
        cum_prev.swap(cum_next);
        pend.push_back(std::move(pl));
        S = std::move(Snext);
    }
    if (S.n > 8192) return "last Schur complement too large for the exact last level (" + std::to_string(S.n) + ")";
    // permutation: level pivots in order, then the last level
    out.perm.resize(n);
    {
        int p = 0;
        for (auto &lo : level_orig) for (int s : lo) out.perm[p++] = s;
        for (int s : orig) out.perm[p++] = s;
    }
    out.coarse_off = off;
    out.coarse_n = S.n;
    out.pos_scale.assign(n, 1.0);
    {
        int p = 0;
        for (auto &pl : pend)
            for (int b : pl.lv.B) out.pos_scale[p++] = pl.cum[b];
        for (int i = 0; i < S.n; ++i) out.pos_scale[p++] = cum_prev[i];
    }
    // global position of each level-local unknown, computed from the last level back
    // gpos for the current (last) level: coarse positions
    std::vector<int> gpos(S.n);
    for (int i = 0; i < S.n; ++i) gpos[i] = off + i;
    // last level: dense inverse with the cumulative scaling folded in
    {
        const int nc = S.n;
        std::vector<double> dense(size_t(nc) * nc, 0.0);
        for (int i = 0; i < nc; ++i)
            for (int64_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p) dense[size_t(i) * nc + S.col[p]] = S.val[p];
        if (prm.host_coarse_inverse) {
            if (nc > 0 && !dense_inverse(nc, dense)) return "singular last level";
            for (int i = 0; i < nc; ++i)
                for (int j = 0; j < nc; ++j) dense[size_t(i) * nc + j] *= cum_prev[i] * cum_prev[j];
            out.coarse_inv.swap(dense);
        } else {
            out.coarse_mat.swap(dense);
            out.coarse_scale = cum_prev;
        }
    }
    out.levels.resize(pend.size());
    long long nnz_fact = 0;
    for (int l = int(pend.size()) - 1; l >= 0; --l) {
        Pending &pl = pend[l];
        LevelLocal &lv = pl.lv;
        Level &G = out.levels[l];
        const int nB = int(lv.B.size()), nC = int(lv.C.size());
        G.off = pl.off;
        G.nB = nB;
        G.n_after = nC;
        G.n2x2 = lv.n2x2;
        G.cand_rejected = lv.rejected;
        G.g_min_scaled = lv.g_min;
        G.g_max_colsum = lv.g_colsum;
        // gpos (next level) -> this level
        std::vector<int> gl(lv.B.size() + lv.C.size());
        for (int t = 0; t < nB; ++t) gl[lv.B[t]] = pl.off + t;
        for (int r = 0; r < nC; ++r) gl[lv.C[r]] = gpos[r];
        const std::vector<double> &cum = pl.cum;
        // G rows ordered by global position of the C unknown: positions off+nB .. n-1
        std::vector<int> row_at(nC);  // global position - (off+nB) -> local C row
        for (int r = 0; r < nC; ++r) row_at[gpos[r] - (pl.off + nB)] = r;
        G.g_ptr.assign(nC + 1, 0);
        for (int q = 0; q < nC; ++q) {
            const int r = row_at[q];
            G.g_ptr[q + 1] = G.g_ptr[q] + (lv.g_ptr[r + 1] - lv.g_ptr[r]);
        }
        G.g_col.resize(G.g_ptr[nC]);
        G.g_val.resize(G.g_ptr[nC]);
        for (int q = 0; q < nC; ++q) {
            const int r = row_at[q];
            const int ci = lv.C[r];
            int64_t o = G.g_ptr[q];
            for (int64_t p = lv.g_ptr[r]; p < lv.g_ptr[r + 1]; ++p, ++o) {
                const int t = lv.g_col[p];
                G.g_col[o] = pl.off + t;
                G.g_val[o] = lv.g_val[p] * cum[lv.B[t]] / cum[ci];
            }
        }
        // G^T rows = pivots in order
        G.gt_ptr.assign(nB + 1, 0);
        for (int r = 0; r < nC; ++r)
            for (int64_t p = lv.g_ptr[r]; p < lv.g_ptr[r + 1]; ++p) ++G.gt_ptr[lv.g_col[p] + 1];
        for (int t = 0; t < nB; ++t) G.gt_ptr[t + 1] += G.gt_ptr[t];
        G.gt_col.resize(G.gt_ptr[nB]);
        G.gt_val.resize(G.gt_ptr[nB]);
        {
            std::vector<int64_t> fp(G.gt_ptr.begin(), G.gt_ptr.end() - 1);
            for (int q = 0; q < nC; ++q) {
                const int r = row_at[q];
                const int ci = lv.C[r];
                for (int64_t p = lv.g_ptr[r]; p < lv.g_ptr[r + 1]; ++p) {
                    const int t = lv.g_col[p];
                    G.gt_col[fp[t]] = gpos[r];
                    G.gt_val[fp[t]++] = lv.g_val[p] * cum[lv.B[t]] / cum[ci];
                }
            }
        }
        G.bd.resize(nB);
        G.bo.resize(nB);
        G.bp.resize(nB);
        for (int t = 0; t < nB; ++t) {
            const double ci = cum[lv.B[t]], cp = cum[lv.B[lv.partner[t]]];
            G.bd[t] = lv.bd[t] * ci * ci;
            G.bo[t] = lv.bo[t] * ci * cp;
            G.bp[t] = pl.off + lv.partner[t];
        }
        nnz_fact += G.g_ptr[nC] + nB + lv.n2x2;
        gpos.swap(gl);
    }
    nnz_fact += (long long)out.coarse_n * (out.coarse_n + 1) / 2;
    out.fill = double(nnz_fact) / double(std::max<long long>(out.nnz_lower_A, 1));
    if (verbose)
        fprintf(stderr, "levels %zu coarse %d: match %.2fs split %.2fs factor %.2fs total %.2fs\n", out.levels.size(),
                out.coarse_n, t_match, t_split, t_fact, now_s() - t0);
    if (prm.inverse_factor) build_inverse_factor(out, prm.z_drop, L, prm.z_parts > 0 ? prm.z_parts : default_z_parts(n));
    out.seconds = now_s() - t0;
    return "";
}

// ---------------------------------------------------------------------------------
// Explicit inverse factor, in segments.  Applying the levels one after the other needs
// one dependent pass per level and direction; the product of the passes of a range of
// levels is itself a unit lower triangular matrix, formed here (with dropping in the
// scaled domain), so that the device applies the whole preconditioner as
// P^T Z_0^T ... Z_{S-1}^T D^{-1} Z_{S-1} ... Z_0 P: 2 S sparse products, a block-diagonal
// solve and the exact last level.
// ---------------------------------------------------------------------------------
int default_z_parts(int n)
{
    // measured on the MI355X: the segments save bytes, each costs two launches
    if (n >= (1 << 19)) return 6;
    if (n >= (1 << 16)) return 4;
    return 3;
}

void build_inverse_factor(Multilevel &ml, double z_drop, int L, int parts)
{
    const double t0 = now_s();
    const int n = ml.n;
    const int nl = int(ml.levels.size());
    InverseFactor &Z = ml.z;
    const std::vector<double> &sc = ml.pos_scale;
    auto lev_off = [&](int l) { return l < nl ? ml.levels[l].off : ml.coarse_off; };
    // renumbering: position p -> Morton rank of its site
    std::vector<int> newidx(n);
    {
        std::vector<std::pair<uint64_t, int>> keyed(n);
        for (int p = 0; p < n; ++p) keyed[p] = {morton(ml.perm[p], L), p};
        std::sort(keyed.begin(), keyed.end());
        Z.site_of.resize(n);
        for (int q = 0; q < n; ++q) {
            newidx[keyed[q].second] = q;
            Z.site_of[q] = ml.perm[keyed[q].second];
        }
    }
    // middle numbering: blocks of kMidBlock consecutive Morton ranks, by elimination level
    // inside a block (a pivot's later-level dependants are then packed together, which
    // cuts the cache lines each gather of the transposed products touches)
    std::vector<int> level(n, nl), midx(n), pos_of(n);
    for (int l = 0; l < nl; ++l)
        for (int t = 0; t < ml.levels[l].nB; ++t) level[ml.levels[l].off + t] = l;
    {
        std::vector<std::tuple<int, int, int>> keyed(n);
        for (int p = 0; p < n; ++p) keyed[p] = {newidx[p] / kMidBlock, level[p], newidx[p]};
        std::vector<int> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int a, int b) { return keyed[a] < keyed[b]; });
        for (int m = 0; m < n; ++m) {
            midx[order[m]] = m;
            pos_of[m] = order[m];
        }
    }
    // segment cuts at levels 1, 3, 9, 27, ...
    std::vector<int> cuts{0};
    for (int c = 1; int(cuts.size()) < std::max(parts, 1) && c < nl; c *= 3) cuts.push_back(c);
    cuts.push_back(nl);
    const int S = int(cuts.size()) - 1;
    std::vector<int> seg_of(n, S);  // segment owning each position (S: the last level)
    for (int s = 0; s < S; ++s)
        for (int l = cuts[s]; l < cuts[s + 1]; ++l)
            for (int t = 0; t < ml.levels[l].nB; ++t) seg_of[ml.levels[l].off + t] = s;
    const int64_t n1 = n, n2 = 2 * int64_t(n);
    Z.seg.assign(S, ZSegment());
    Z.nnz = 0;
    for (int s = 0; s < S; ++s) {
        const int a = cuts[s], b = cuts[s + 1];
        const int off_a = lev_off(a);
        const int nr = n - off_a;
        ZSegment &zs = Z.seg[s];
        zs.lev_begin = a;
        zs.lev_end = b;
        zs.rows = nr;
        // rows of Z_s by position (p - off_a), level by level: a row needs the rows of
        // the segment's earlier pivots only
        std::vector<std::vector<std::pair<int, double>>> rows(nr);
#pragma omp parallel
        {
            std::vector<double> acc(n, 0.0);
            std::vector<int> mark(n, -1), list;
            for (int m = a; m <= nl; ++m) {
                const int r0 = lev_off(m);
                const int r1 = (m < nl) ? ml.levels[m].off + ml.levels[m].nB : n;
                const int lmax = std::min(m, b);
#pragma omp for schedule(dynamic, 16)
                for (int r = r0; r < r1; ++r) {
                    list.clear();
                    auto put = [&](int c, double v) {
                        if (mark[c] != r) { mark[c] = r; acc[c] = 0.0; list.push_back(c); }
                        acc[c] += v;
                    };
                    put(r, 1.0);
                    for (int l = a; l < lmax; ++l) {
                        const Level &Lv = ml.levels[l];
                        const int q = r - (Lv.off + Lv.nB);
                        for (int64_t p = Lv.g_ptr[q]; p < Lv.g_ptr[q + 1]; ++p) {
                            const double g = Lv.g_val[p];
                            for (const auto &e : rows[Lv.g_col[p] - off_a]) put(e.first, -g * e.second);
                        }
                    }
                    auto &out = rows[r - off_a];
                    size_t keep = 0;
                    for (int c : list)
                        if (c == r || z_drop < 0 || std::fabs(acc[c]) * sc[r] / sc[c] >= z_drop) ++keep;
                    out.reserve(keep);
                    for (int c : list) {
                        const double v = acc[c];
                        if (c == r || z_drop < 0 || std::fabs(v) * sc[r] / sc[c] >= z_drop) out.push_back({c, v});
                    }
                }
                // implicit barrier of the worksharing loop: level m is complete
            }
        }
        // down product: rows in the middle order, offsets into the 3 n buffer
        const int64_t w_off = (s % 2 == 0) ? n1 : n2;       // region of the rows passed on
        const int64_t r_off = (s % 2 == 1) ? n1 : n2;       // region segment s - 1 wrote
        std::vector<int> drow;                               // local row -> position
        drow.reserve(nr);
        for (int m = 0; m < n; ++m)
            if (pos_of[m] >= off_a) drow.push_back(pos_of[m]);
        BigVec<int64_t> ptr(nr + 1);
        ptr[0] = 0;
        for (int i = 0; i < nr; ++i) ptr[i + 1] = ptr[i] + int64_t(rows[drow[i] - off_a].size());
        const int64_t nnz = ptr[nr];
        BigVec<int> col(nnz);
        BigVec<double> val(nnz);
        std::vector<int> code(nr);
#pragma omp parallel for schedule(dynamic, 256)
        for (int i = 0; i < nr; ++i) {
            const int p = drow[i];
            const bool final_row = seg_of[p] == s || (s == S - 1 && seg_of[p] == S);
            code[i] = int(final_row ? midx[p] : w_off + midx[p]);
            auto row = rows[p - off_a];  // copy: the transposed product reads positions
            for (auto &e : row) e.first = int(s == 0 ? n2 + newidx[e.first] : r_off + midx[e.first]);
            std::sort(row.begin(), row.end());
            int64_t o = ptr[i];
            for (auto &e : row) { col[o] = e.first; val[o] = e.second; ++o; }
        }
        zs.nnz = nnz;
        Z.nnz += nnz;
        zs.down = to_hyb(nr, ptr.data(), col.data(), val.data(), code.data());
        // up product: Z_s^T restricted to this segment's pivots (segment 0: every position,
        // for the output permutation), rows in the middle order (segment 0: Morton order)
        std::vector<int> urow;  // up row -> position
        std::vector<int> uat(n, -1);
        if (s == 0) {
            urow.resize(n);
            for (int p = 0; p < n; ++p) urow[newidx[p]] = p;
        } else {
            for (int m = 0; m < n; ++m)
                if (seg_of[pos_of[m]] == s) urow.push_back(pos_of[m]);
        }
        const int nu = int(urow.size());
        for (int i = 0; i < nu; ++i) uat[urow[i]] = i;
        BigVec<int64_t> tptr(nu + 1);
        std::fill(tptr.begin(), tptr.end(), 0);
        for (int i = 0; i < nr; ++i)
            for (const auto &e : rows[drow[i] - off_a])
                if (uat[e.first] >= 0) ++tptr[uat[e.first] + 1];
        for (int i = 0; i < nu; ++i) tptr[i + 1] += tptr[i];
        BigVec<int> tcol(tptr[nu]);
        BigVec<double> tval(tptr[nu]);
        {
            std::vector<int64_t> fp(tptr.begin(), tptr.end() - 1);
            for (int i = 0; i < nr; ++i) {
                const int r = drow[i];
                // a later segment's pivot has its final value in region 2; this segment's
                // own pivots and the last level's unknowns are read from region 1
                const bool later = seg_of[r] > s && seg_of[r] < S;
                const int rc = int(later ? n2 + midx[r] : n1 + midx[r]);
                for (const auto &e : rows[r - off_a]) {
                    const int u = uat[e.first];
                    if (u < 0) continue;
                    tcol[fp[u]] = rc;
                    tval[fp[u]++] = e.second;
                }
            }
        }
        std::vector<int> ucode(nu);
#pragma omp parallel for schedule(dynamic, 256)
        for (int i = 0; i < nu; ++i) {
            // the first segment's transposed product is the last of the apply: its rows
            // are written straight to their lattice sites (the output permutation P^T)
            ucode[i] = int(s == 0 ? Z.site_of[newidx[urow[i]]] : n2 + midx[urow[i]]);
            std::vector<std::pair<int, double>> row(size_t(tptr[i + 1] - tptr[i]));
            for (int64_t o = tptr[i]; o < tptr[i + 1]; ++o) row[o - tptr[i]] = {tcol[o], tval[o]};
            std::sort(row.begin(), row.end());
            for (int64_t o = tptr[i]; o < tptr[i + 1]; ++o) { tcol[o] = row[o - tptr[i]].first; tval[o] = row[o - tptr[i]].second; }
        }
        zs.up = to_hyb(nu, tptr.data(), tcol.data(), tval.data(), ucode.data());
    }
    Z.dd.assign(n, 0.0);
    Z.dof.assign(n, 0.0);
    Z.dp.resize(n);
    for (int q = 0; q < n; ++q) Z.dp[q] = q;
    for (const auto &Lv : ml.levels)
        for (int t = 0; t < Lv.nB; ++t) {
            const int q = midx[Lv.off + t];
            Z.dd[q] = Lv.bd[t];
            Z.dof[q] = Lv.bo[t];
            Z.dp[q] = midx[Lv.bp[t]];
        }
    Z.coarse_idx.resize(ml.coarse_n);
    for (int i = 0; i < ml.coarse_n; ++i) Z.coarse_idx[i] = midx[ml.coarse_off + i];
    Z.seconds = now_s() - t0;
}

// CSR -> the hybrid device layout (see HybHost).  The parts are built on their own
// (in parallel) and then concatenated, with their long-row indices, slice codes and
// offsets shifted to the global numbering.
// One product of the layout h on the host (see apply_inverse_factor_host): rows are
// written to y, columns read from x; every number is checked against its limit, and no
// row the product writes may be read by it.
static std::string hyb_product_host(const HybHost &h, const std::vector<double> &x, int64_t xlim, double *y,
                                    int64_t ylim, std::vector<char> &mark)
{
    const int ns = int(h.slice_ptr.size()) - 1;
    if (ns < 0 || int64_t(h.slice_row.size()) != ns + 1 || int64_t(h.rowidx.size()) != h.slice_row[ns])
        return "slice arrays of inconsistent sizes";
    // the tasks of each part cover its long rows and its slices exactly once
    std::vector<int> seen_long(h.long_row.size(), 0), seen_slice(ns, 0);
    for (int p = 0; p < kHybParts; ++p)
        for (int i = 0; i < h.ntask[p]; ++i) {
            if (i < h.plong[p]) {
                const int c = h.long0[p] + i;
                if (c < 0 || c >= int(h.long_row.size())) return "long-row task out of range";
                ++seen_long[c];
            } else {
                const int c = h.slice0[p] + i - h.plong[p];
                if (c < 0 || c >= ns) return "slice task out of range";
                ++seen_slice[c];
            }
        }
    for (int v : seen_long) if (v != 1) return "long rows not covered once by the tasks";
    for (int v : seen_slice) if (v != 1) return "slices not covered once by the tasks";
    // the rows written, then every column read (a product never reads its own rows)
    std::vector<int64_t> written;
    for (int r : h.long_row) {
        if (r < 0 || r >= ylim) return "long row number out of range";
        written.push_back(r);
    }
    for (int r : h.rowidx) {
        if (r >= ylim) return "slice row number out of range";
        if (r >= 0) written.push_back(r);
    }
    if (y == x.data())
        for (int64_t r : written) mark[r] = 1;
    auto col_ok = [&](int c) { return c >= 0 && c < xlim && !(y == x.data() && mark[c]); };
    std::string err;
    for (size_t i = 0; i < h.long_row.size() && err.empty(); ++i) {
        double a = 0.0;
        for (int64_t q = h.long_ptr[i]; q < h.long_ptr[i + 1]; ++q) {
            if (!col_ok(h.long_col[q])) { err = "long-row column out of range or written by the product"; break; }
            a += h.long_val[q] * x[h.long_col[q]];
        }
        y[h.long_row[i]] = a;
    }
    for (int s = 0; s < ns && err.empty(); ++s) {
        const int64_t p0 = h.slice_ptr[s];
        const int R = kSliceRows << int(p0 & 3);
        const int64_t b = p0 & ~int64_t(63);
        const int64_t e = h.slice_ptr[s + 1] & ~int64_t(63);
        if (e <= b || e > int64_t(h.col.size()) || h.slice_row[s + 1] - h.slice_row[s] != R) {
            err = "slice extent";
            break;
        }
        const int groups = int((e - b) / 64), lanes = 64 / R;
        for (int l = 0; l < R && err.empty(); ++l) {
            double a = 0.0;
            for (int g = 0; g < groups; ++g)
                for (int j = 0; j < lanes; ++j) {
                    const int64_t at = b + int64_t(g) * 64 + int64_t(j) * R + l;
                    if (!col_ok(h.col[at])) { err = "slice column out of range or written by the product"; break; }
                    a += h.val[at] * x[h.col[at]];
                }
            const int r = h.rowidx[h.slice_row[s] + l];
            if (r >= 0) y[r] = a;
        }
    }
    if (y == x.data())
        for (int64_t r : written) mark[r] = 0;
    return err;
}

std::string apply_inverse_factor_host(const Multilevel &ml, const double *b, double *x)
{
    const int n = ml.n;
    const InverseFactor &Z = ml.z;
    const int S = int(Z.seg.size()), nc = ml.coarse_n;
    if (S == 0 || int(Z.site_of.size()) != n) return "no inverse factor";
    if (nc > 0 && ml.coarse_inv.size() != size_t(nc) * nc) return "last level not inverted on the host";
    const int64_t n3 = 3 * int64_t(n);
    // NaN marks a value no product has written: it reaches x if it is ever read
    std::vector<double> buf(n3, std::numeric_limits<double>::quiet_NaN());
    std::vector<char> mark(n3, 0);
    for (int q = 0; q < n; ++q) buf[2 * int64_t(n) + q] = b[Z.site_of[q]];
    std::string err;
    for (int s = 0; s < S && err.empty(); ++s) err = hyb_product_host(Z.seg[s].down, buf, n3, buf.data(), n3, mark);
    if (!err.empty()) return "down product: " + err;
    for (int j = 0; j < n; ++j) {
        if (Z.dp[j] < 0 || Z.dp[j] >= n) return "block partner out of range";
        buf[int64_t(n) + j] = Z.dd[j] * buf[j] + Z.dof[j] * buf[Z.dp[j]];
    }
    std::vector<double> yc(nc);
    for (int i = 0; i < nc; ++i) {
        if (Z.coarse_idx[i] < 0 || Z.coarse_idx[i] >= n) return "last-level index out of range";
        yc[i] = buf[Z.coarse_idx[i]];
    }
    for (int i = 0; i < nc; ++i) {
        double a = 0.0;
        for (int j = 0; j < nc; ++j) a += ml.coarse_inv[size_t(i) * nc + j] * yc[j];
        buf[int64_t(n) + Z.coarse_idx[i]] = a;
    }
    for (int s = S - 1; s >= 1 && err.empty(); --s) err = hyb_product_host(Z.seg[s].up, buf, n3, buf.data(), n3, mark);
    if (!err.empty()) return "up product: " + err;
    std::fill(x, x + n, std::numeric_limits<double>::quiet_NaN());
    err = hyb_product_host(Z.seg[0].up, buf, n3, x, n, mark);
    if (!err.empty()) return "first segment's up product: " + err;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return "a value was read before any product wrote it, or a site was not written";
    return "";
}

HybHost to_hyb(int n, const int64_t *ptr, const int *col, const double *val, const int *row_code)
{
    constexpr int P = kHybParts;
    constexpr size_t kWindow = 2048;
    auto len = [&](int r) { return ptr[r + 1] - ptr[r]; };
    auto rcode = [&](int r) { return row_code ? row_code[r] : r; };
    const int64_t nnz = ptr[n];
    // rows [rb[part], rb[part + 1]): the part's share of the nonzeros
    int rb[P + 1];
    rb[0] = 0;
    for (int part = 0; part < P; ++part) {
        int r1 = rb[part];
        const int64_t target = nnz * (part + 1) / P;
        while (r1 < n && (part == P - 1 || ptr[r1] < target)) ++r1;
        rb[part + 1] = r1;
    }
    HybHost parts[P];
#pragma omp parallel for schedule(dynamic, 1)
    for (int part = 0; part < P; ++part) {
        HybHost &h = parts[part];
        std::vector<int> longr, shortr;
        for (int r = rb[part]; r < rb[part + 1]; ++r) (len(r) > kLongRow ? longr : shortr).push_back(r);
        std::stable_sort(longr.begin(), longr.end(), [&](int a, int b) { return len(a) > len(b); });
        for (int r : longr) {
            h.long_row.push_back(rcode(r));
            h.long_col.insert(h.long_col.end(), col + ptr[r], col + ptr[r + 1]);
            h.long_val.insert(h.long_val.end(), val + ptr[r], val + ptr[r + 1]);
            h.long_ptr.push_back(int64_t(h.long_col.size()));
        }
        for (size_t w0 = 0; w0 < shortr.size(); w0 += kWindow) {
            auto b = shortr.begin() + w0, e = shortr.begin() + std::min(shortr.size(), w0 + kWindow);
            std::stable_sort(b, e, [&](int a, int c) { return len(a) > len(c); });
        }
        // slices of 8 << c rows with 8 >> c lanes per row: the lanes per row minimise the
        // padded slots of the slice's longest row (ceil(w / g) g) within 8 groups, larger
        // on ties; a slice does not cross a sorting window
        for (size_t s0 = 0; s0 < shortr.size();) {
            const size_t wend = std::min(shortr.size(), (s0 / kWindow + 1) * kWindow);
            const int64_t w0 = len(shortr[s0]);
            int g = kSliceLanes, code = 0;
            int64_t best = (w0 + g - 1) / g * g;
            for (int c = 1; c <= 3; ++c) {
                const int gc = kSliceLanes >> c;
                const int64_t grp = (w0 + gc - 1) / gc;
                if (grp <= 8 && grp * gc < best) {
                    best = grp * gc;
                    g = gc;
                    code = c;
                }
            }
            const int R = 64 / g;
            const size_t cnt = std::min<size_t>(size_t(R), wend - s0);
            int64_t w = 0;
            for (size_t l = 0; l < cnt; ++l) w = std::max(w, len(shortr[s0 + l]));
            const int64_t base = h.slice_ptr.back(), groups = (w + g - 1) / g;
            h.slice_ptr.back() = base | code;
            // padding reads the slice's first entry's location (a value the product reads anyway)
            const int pad = len(shortr[s0]) > 0 ? col[ptr[shortr[s0]]] : 0;
            h.slice_ptr.push_back(base + groups * 64);
            h.col.resize(size_t(base + groups * 64), pad);
            h.val.resize(size_t(base + groups * 64), 0.0);
            for (int l = 0; l < R; ++l) {
                if (size_t(l) >= cnt) {
                    h.rowidx.push_back(-1);
                    continue;
                }
                const int r = shortr[s0 + l];
                h.rowidx.push_back(rcode(r));
                for (int64_t j = 0; j < len(r); ++j) {
                    const int64_t at = base + (j / g) * 64 + (j % g) * R + l;
                    h.col[at] = col[ptr[r] + j];
                    h.val[at] = val[ptr[r] + j];
                }
            }
            h.slice_row.push_back(int64_t(h.rowidx.size()));
            s0 += cnt;
        }
    }
    // offsets of every part in the concatenated arrays
    struct Off { size_t long_row, long_ent, slice, slice_ent, rows; };
    Off off[P + 1];
    off[0] = {0, 0, 0, 0, 0};
    for (int part = 0; part < P; ++part) {
        const HybHost &q = parts[part];
        off[part + 1] = {off[part].long_row + q.long_row.size(), off[part].long_ent + q.long_col.size(),
                         off[part].slice + (q.slice_ptr.size() - 1), off[part].slice_ent + q.col.size(),
                         off[part].rows + q.rowidx.size()};
    }
    HybHost h;
    const Off &tot = off[P];
    h.long_row.resize(tot.long_row);
    h.long_ptr.resize(tot.long_row + 1);
    h.long_col.resize(tot.long_ent);
    h.long_val.resize(tot.long_ent);
    h.slice_ptr.resize(tot.slice + 1);
    h.slice_row.resize(tot.slice + 1);
    h.rowidx.resize(tot.rows);
    h.col.resize(tot.slice_ent);
    h.val.resize(tot.slice_ent);
    h.long_ptr[0] = 0;
    h.slice_ptr[0] = 0;
    h.slice_row[0] = 0;
    for (int part = 0; part < P; ++part) {
        const HybHost &q = parts[part];
        h.plong[part] = int(q.long_row.size());
        h.ntask[part] = int(q.long_row.size() + (q.slice_ptr.size() - 1));
        h.long0[part] = int(off[part].long_row);
        h.slice0[part] = int(off[part].slice);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int part = 0; part < P; ++part) {
        const HybHost &q = parts[part];
        const Off &o = off[part];
        std::copy(q.long_row.begin(), q.long_row.end(), h.long_row.begin() + o.long_row);
        for (size_t i = 1; i < q.long_ptr.size(); ++i) h.long_ptr[o.long_row + i] = int64_t(o.long_ent) + q.long_ptr[i];
        std::copy(q.long_col.begin(), q.long_col.end(), h.long_col.begin() + o.long_ent);
        std::copy(q.long_val.begin(), q.long_val.end(), h.long_val.begin() + o.long_ent);
        // each part writes the starts of its slices (the shift keeps the shape code in the
        // low bits: the offsets are multiples of 64); the common end is written below
        for (size_t i = 0; i + 1 < q.slice_ptr.size(); ++i) {
            h.slice_ptr[o.slice + i] = int64_t(o.slice_ent) + q.slice_ptr[i];
            h.slice_row[o.slice + i] = int64_t(o.rows) + q.slice_row[i];
        }
        std::copy(q.rowidx.begin(), q.rowidx.end(), h.rowidx.begin() + o.rows);
        std::copy(q.col.begin(), q.col.end(), h.col.begin() + o.slice_ent);
        std::copy(q.val.begin(), q.val.end(), h.val.begin() + o.slice_ent);
    }
    h.slice_ptr[tot.slice] = int64_t(tot.slice_ent);
    h.slice_row[tot.slice] = int64_t(tot.rows);
    return h;
}

}  // namespace jdmi
