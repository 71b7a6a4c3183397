// Device kernels of the Jacobi-Davidson hot path for gfx950 (wave64, 256 CUs).
//
// All streaming kernels are HBM-bound: one thread per row or site, unit-stride
// access along the fastest lattice direction, no host synchronisation.  Reductions
// are deterministic two-stage trees (wave shuffles, then LDS, then a fixed-order
// final pass), so a result never depends on what else runs on the device.
#include "kernels.h"

#include <algorithm>
#include <stdexcept>
#include <cmath>

namespace jdmi {

namespace {

__host__ __device__ inline int nblocks(int64_t n, int b = kBlock)
{
    return int((n + b - 1) / b);
}

inline int red_blocks(int64_t n)
{
    int b = nblocks(n);
    return b < 1 ? 1 : (b > kRedBlocks ? kRedBlocks : b);
}

// streamed-once matrix data: non-temporal loads keep the gathered vector in cache
template <typename T>
__device__ inline T nt_load(const T *p)
{
    return __builtin_nontemporal_load(p);
}

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// sum over a kBlock-thread workgroup, result in thread 0; fixed order
__device__ inline double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

}  // namespace

// ---------------------------------------------------------------------------------
// K1: the disorder eps_s = W (u_s - 1/2), u_s from SplitMix64 output s+1 (counter form:
// state = seed + (s+1) * 0x9E3779B97F4A7C15, then the two xor-shift-multiply rounds).
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_gen_diag(int n, double W, uint64_t seed, double *eps, float *eps32)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    uint64_t z = seed + uint64_t(s + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = double(z >> 11) * 0x1.0p-53;
    const double e = W * (u - 0.5);
    eps[s] = e;
    if (eps32) eps32[s] = float(e);
}

void launch_gen_diag(int L, double W, uint64_t seed, double *eps, float *eps32, hipStream_t s)
{
    const int n = L * L * L;
    hipLaunchKernelGGL(k_gen_diag, dim3(nblocks(n)), dim3(kBlock), 0, s, n, W, seed, eps, eps32);
}

// The off-diagonal model: bond (s, d) (site s to its +x, +y, +z neighbour) takes output
// n + 3 s + d + 1 of the same SplitMix64 stream, t = W (u - 1/2); stored as hop[d n + s].
__global__ void __launch_bounds__(kBlock) k_gen_hop(int n, double W, uint64_t seed, double *hop, float *hop32)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    for (int d = 0; d < 3; ++d) {
        const uint64_t m = uint64_t(n) + 3ull * uint64_t(s) + uint64_t(d) + 1ull;
        uint64_t z = seed + m * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double t = W * (double(z >> 11) * 0x1.0p-53 - 0.5);
        hop[size_t(d) * n + s] = t;
        if (hop32) hop32[size_t(d) * n + s] = float(t);
    }
}

void launch_gen_hop(int L, double W, uint64_t seed, double *hop, float *hop32, hipStream_t s)
{
    const int n = L * L * L;
    hipLaunchKernelGGL(k_gen_hop, dim3(nblocks(n)), dim3(kBlock), 0, s, n, W, seed, hop, hop32);
}

// ---------------------------------------------------------------------------------
// K2: y = (A - shift I) x with A = -T + diag(eps) on the periodic lattice, or on the box
// with hard walls (a neighbour outside the box contributes nothing).
// ---------------------------------------------------------------------------------
template <typename T>
__device__ inline T neighbour_sum(int L, int n, int s, const T *__restrict__ x, int bc)
{
    const int LL = L * L;
    const int i = s % L, jk = s / L, j = jk % L, k = jk / L;
    if (bc == 0) {
        const int xm = (i == 0) ? s + L - 1 : s - 1;
        const int xp = (i == L - 1) ? s - L + 1 : s + 1;
        const int ym = (j == 0) ? s + LL - L : s - L;
        const int yp = (j == L - 1) ? s - LL + L : s + L;
        const int zm = (k == 0) ? s + n - LL : s - LL;
        const int zp = (k == L - 1) ? s - n + LL : s + LL;
        return ((x[xm] + x[xp]) + (x[ym] + x[yp])) + (x[zm] + x[zp]);
    }
    const T xm = i > 0 ? x[s - 1] : T(0), xp = i < L - 1 ? x[s + 1] : T(0);
    const T ym = j > 0 ? x[s - L] : T(0), yp = j < L - 1 ? x[s + L] : T(0);
    const T zm = k > 0 ? x[s - LL] : T(0), zp = k < L - 1 ? x[s + LL] : T(0);
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// Random bond values (the off-diagonal model): sum over the site's bonds of t x, the
// bond to s + e_d stored at hop[d n + s], the bond to s - e_d at hop[d n + (s - e_d)].
template <typename T>
__device__ inline T bond_sum(int L, int n, int s, const T *__restrict__ x, const T *__restrict__ hop, int bc)
{
    const int LL = L * L;
    const int c[3] = {s % L, (s / L) % L, s / LL};
    const int stride[3] = {1, L, LL};
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T *t = hop + size_t(d) * n;
        const int up = c[d] == L - 1 ? s - (L - 1) * stride[d] : s + stride[d];
        const int dn = c[d] == 0 ? s + (L - 1) * stride[d] : s - stride[d];
        const bool has_up = bc == 0 || c[d] < L - 1, has_dn = bc == 0 || c[d] > 0;
        const T a = has_up ? t[s] * x[up] : T(0);
        const T b = has_dn ? t[dn] * x[dn] : T(0);
        acc += a + b;
    }
    return acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_stencil(int L, int n, int bc, const T *__restrict__ eps, T shift,
                                                    const T *__restrict__ x, T *__restrict__ y,
                                                    const int *skip, const T *__restrict__ hop)
{
    if (skip && *skip) return;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    if (hop) y[s] = (eps[s] - shift) * x[s] + bond_sum(L, n, s, x, hop, bc);
    else y[s] = (eps[s] - shift) * x[s] - neighbour_sum(L, n, s, x, bc);
}

template <typename T>
void launch_stencil(int L, int bc, const T *eps, double shift, const T *x, T *y, hipStream_t s, const int *skip,
                    const T *hop)
{
    const int n = L * L * L;
    hipLaunchKernelGGL(k_stencil<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, L, n, bc, eps, T(shift), x, y, skip,
                       hop);
}

// The product of the inner iteration, with the shift read from the solver state
// (graph-replayable).  The operator is the binary64 one (eps and bond values in
// binary64) applied to the stored vector x of either precision, and the result is
// rounded once: binary32 inner vectors then see rounding of the product only, not an
// operator perturbed by eps rounded to binary32 (near sigma that perturbation, of order
// 1e-7 ||A||, is not small against the eigenvalue spacing).
template <typename T>
__device__ inline double bond_sum64(int L, int n, int s, const T *__restrict__ x, const double *__restrict__ hop, int bc)
{
    const int LL = L * L;
    const int c[3] = {s % L, (s / L) % L, s / LL};
    const int stride[3] = {1, L, LL};
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *t = hop + size_t(d) * n;
        const int up = c[d] == L - 1 ? s - (L - 1) * stride[d] : s + stride[d];
        const int dn = c[d] == 0 ? s + (L - 1) * stride[d] : s - stride[d];
        const bool has_up = bc == 0 || c[d] < L - 1, has_dn = bc == 0 || c[d] > 0;
        const double a = has_up ? t[s] * double(x[up]) : 0.0;
        const double b = has_dn ? t[dn] * double(x[dn]) : 0.0;
        acc += a + b;
    }
    return acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_stencil_state(int L, int n, int bc, const double *__restrict__ eps,
                                                          const SqmrState *st, const T *__restrict__ x,
                                                          T *__restrict__ y, const double *__restrict__ hop)
{
    if (st->done) return;
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const double shift = st->shift;
    const double xs = double(x[s]);
    if (hop) {
        y[s] = T((eps[s] - shift) * xs + bond_sum64(L, n, s, x, hop, bc));
    } else {
        const int LL = L * L;
        const int i = s % L, jk = s / L, j = jk % L, k = jk / L;
        double nb;
        if (bc == 0) {
            const int xm = (i == 0) ? s + L - 1 : s - 1;
            const int xp = (i == L - 1) ? s - L + 1 : s + 1;
            const int ym = (j == 0) ? s + LL - L : s - L;
            const int yp = (j == L - 1) ? s - LL + L : s + L;
            const int zm = (k == 0) ? s + n - LL : s - LL;
            const int zp = (k == L - 1) ? s - n + LL : s + LL;
            nb = ((double(x[xm]) + double(x[xp])) + (double(x[ym]) + double(x[yp]))) + (double(x[zm]) + double(x[zp]));
        } else {
            const double xm = i > 0 ? double(x[s - 1]) : 0.0, xp = i < L - 1 ? double(x[s + 1]) : 0.0;
            const double ym = j > 0 ? double(x[s - L]) : 0.0, yp = j < L - 1 ? double(x[s + L]) : 0.0;
            const double zm = k > 0 ? double(x[s - LL]) : 0.0, zp = k < L - 1 ? double(x[s + LL]) : 0.0;
            nb = ((xm + xp) + (ym + yp)) + (zm + zp);
        }
        y[s] = T((eps[s] - shift) * xs - nb);
    }
}

template <typename T>
void launch_stencil_state(int L, int bc, const double *eps, const SqmrState *st, const T *x, T *y, hipStream_t s,
                          const double *hop)
{
    const int n = L * L * L;
    hipLaunchKernelGGL(k_stencil_state<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, L, n, bc, eps, st, x, y, hop);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy(int n, const T *__restrict__ x, T *__restrict__ y)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = x[i];
}
template <typename T>
void launch_copy(int n, const T *x, T *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, n, x, y);
}

// ---------------------------------------------------------------------------------
// Multilevel preconditioner apply (global permuted positions, scalings folded in).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather(int n, const int *__restrict__ perm, const T *__restrict__ b,
                                                   T *__restrict__ w, const int *skip)
{
    if (skip && *skip) return;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < n) w[p] = b[perm[p]];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scatter(int n, const int *__restrict__ perm, const T *__restrict__ x,
                                                    T *__restrict__ out, const int *skip)
{
    if (skip && *skip) return;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < n) out[perm[p]] = x[p];
}

// w[r] -= sum_c G[r, c] w[c] for the complement rows of one level
template <typename T>
__global__ void __launch_bounds__(kBlock) k_down(int row0, int nrows, const int64_t *__restrict__ ptr,
                                                 const int *__restrict__ col, const T *__restrict__ val,
                                                 T *__restrict__ w, const int *skip)
{
    if (skip && *skip) return;
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= nrows) return;
    const int64_t b = ptr[q], e = ptr[q + 1];
    if (b == e) return;
    T acc = T(0);
    for (int64_t p = b; p < e; ++p) acc += val[p] * w[col[p]];
    w[row0 + q] -= acc;
}

// x[j] = D^{-1} w (1x1 or 2x2 block) - sum_r G^T[j, r] x[r] for the pivots of one level
template <typename T>
__global__ void __launch_bounds__(kBlock) k_up(int off, int nB, const int64_t *__restrict__ ptr,
                                               const int *__restrict__ col, const T *__restrict__ val,
                                               const T *__restrict__ bd, const T *__restrict__ bo,
                                               const int *__restrict__ bp, const T *__restrict__ w,
                                               T *__restrict__ x, const int *skip)
{
    if (skip && *skip) return;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= nB) return;
    const int j = off + t;
    T acc = bd[t] * w[j] + bo[t] * w[bp[t]];
    for (int64_t p = ptr[t], e = ptr[t + 1]; p < e; ++p) acc -= val[p] * x[col[p]];
    x[j] = acc;
}

// 16-byte vector of T and its dot product, accumulated in binary64
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = f32x4;
    static constexpr int n = 4;
    __device__ static double dot(const f32x4 &a, const f32x4 &b)
    {
        return (double(a.x) * double(b.x) + double(a.y) * double(b.y)) +
               (double(a.z) * double(b.z) + double(a.w) * double(b.w));
    }
};
template <>
struct Vec16<double> {
    using type = f64x2;
    static constexpr int n = 2;
    __device__ static double dot(const f64x2 &a, const f64x2 &b) { return a.x * b.x + a.y * b.y; }
};

// x[off + i] = sum_j Cinv[i, j] w[off + j] (rows of Cinv ld apart): one wave per row
template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse(int nc, int ld, int off, const T *__restrict__ cinv,
                                                   const T *__restrict__ w, T *__restrict__ x, const int *skip)
{
    if (skip && *skip) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nc) return;
    const T *a = cinv + int64_t(row) * ld;
    double acc = 0.0;
    for (int c = lane; c < nc; c += 64) acc += double(a[c]) * double(w[off + c]);
    acc = wave_sum(acc);
    if (lane == 0) x[off + row] = T(acc);
}

// z[idx[i]] = sum_j Cinv[i, j] yc[j]: one wave per row, 16-byte loads (ld is a multiple
// of 64 and the padding of Cinv's rows and of yc holds zeros)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_rows(int nc, int ld, const int *__restrict__ idx,
                                                        const T *__restrict__ cinv, const T *__restrict__ yc,
                                                        T *__restrict__ z, const int *skip)
{
    if (skip && *skip) return;
    using V = typename Vec16<T>::type;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nc) return;
    const V *a = reinterpret_cast<const V *>(cinv + int64_t(row) * ld);
    const V *y = reinterpret_cast<const V *>(yc);
    const int nv = ld / Vec16<T>::n;
    double acc0 = 0.0, acc1 = 0.0;
    int c = lane;
    for (; c + 64 < nv; c += 128) {
        const V a0 = nt_load(a + c), a1 = nt_load(a + c + 64);
        acc0 += Vec16<T>::dot(a0, y[c]);
        acc1 += Vec16<T>::dot(a1, y[c + 64]);
    }
    for (; c < nv; c += 64) acc0 += Vec16<T>::dot(nt_load(a + c), y[c]);
    const double acc = wave_sum(acc0 + acc1);
    if (lane == 0) z[idx[row]] = T(acc);
}

// The block-diagonal step z = D^{-1} y (blocks [0, nbd)) and the gather of the last
// level's unknowns yc = y[idx] (the other blocks) in one launch: both read y only
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dinv_gather(int m, const T *__restrict__ dd, const T *__restrict__ dof,
                                                        const int *__restrict__ dp, const T *__restrict__ y,
                                                        T *__restrict__ z, int nc, const int *__restrict__ idx,
                                                        T *__restrict__ yc, int nbd, const int *skip)
{
    if (skip && *skip) return;
    if (int(blockIdx.x) < nbd) {
        const int j = blockIdx.x * kBlock + threadIdx.x;
        if (j < m) z[j] = dd[j] * y[j] + dof[j] * y[dp[j]];
    } else {
        const int p = (blockIdx.x - nbd) * kBlock + threadIdx.x;
        if (p < nc) yc[p] = y[idx[p]];
    }
}

template <typename T>
void launch_dinv_coarse(int m, const T *dd, const T *dof, const int *dp, int nc, int ld, const int *idx,
                        const T *cinv, const T *y, T *yc, T *z, hipStream_t s, const int *skip)
{
    const int nbd = m > 0 ? nblocks(m) : 0, nbg = nc > 0 ? nblocks(nc) : 0;
    if (nbd + nbg == 0) return;
    hipLaunchKernelGGL(k_dinv_gather<T>, dim3(nbd + nbg), dim3(kBlock), 0, s, m, dd, dof, dp, y, z, nc, idx, yc, nbd,
                       skip);
    if (nc > 0)
        hipLaunchKernelGGL(k_coarse_rows<T>, dim3(nblocks(nc, kBlock / 64)), dim3(kBlock), 0, s, nc, ld, idx, cinv,
                           yc, z, skip);
}

template <typename T>
void launch_gather(int n, const int *perm, const T *b, T *w, hipStream_t s, const int *skip)
{
    hipLaunchKernelGGL(k_gather<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, n, perm, b, w, skip);
}
template <typename T>
void launch_scatter(int n, const int *perm, const T *x, T *out, hipStream_t s, const int *skip)
{
    hipLaunchKernelGGL(k_scatter<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, n, perm, x, out, skip);
}
template <typename T>
void launch_down(const DevLevel<T> &lv, T *w, hipStream_t s, const int *skip)
{
    if (lv.n_after <= 0) return;
    hipLaunchKernelGGL(k_down<T>, dim3(nblocks(lv.n_after)), dim3(kBlock), 0, s, lv.off + lv.nB, lv.n_after,
                       lv.g_ptr, lv.g_col, lv.g_val, w, skip);
}
template <typename T>
void launch_up(const DevLevel<T> &lv, const T *w, T *x, hipStream_t s, const int *skip)
{
    if (lv.nB <= 0) return;
    hipLaunchKernelGGL(k_up<T>, dim3(nblocks(lv.nB)), dim3(kBlock), 0, s, lv.off, lv.nB, lv.gt_ptr, lv.gt_col,
                       lv.gt_val, lv.bd, lv.bo, lv.bp, w, x, skip);
}
template <typename T>
void launch_coarse(int nc, int ld, int off, const T *cinv, const T *w, T *x, hipStream_t s, const int *skip)
{
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_coarse<T>, dim3(nblocks(nc, kBlock / 64)), dim3(kBlock), 0, s, nc, ld, off, cinv, w, x,
                       skip);
}

// ---------------------------------------------------------------------------------
// Explicit inverse factor, hybrid layout (see kernels.h for the layout).
// ---------------------------------------------------------------------------------
template <typename Tv, typename Tx>
__global__ void __launch_bounds__(kBlock) k_hyb_spmv(Hyb<Tv> A, const Tx *__restrict__ x, Tx *__restrict__ y,
                                                     const int *skip)
{
    if (skip && *skip) return;
    const int part = blockIdx.x % kHybParts;
    // the wave's task within its part (the same for its 64 lanes)
    const int i = __builtin_amdgcn_readfirstlane(int(blockIdx.x / kHybParts) * (kBlock / 64) + int(threadIdx.x >> 6));
    if (i >= A.ntask[part]) return;
    const int lane = threadIdx.x & 63;
    // Four entries per lane in flight: every index and value load of a batch is issued
    // before its dependent gathers.  In a row's (or slice's) last batch a position past
    // the end reads the last entry again with weight 0, so a batch never runs serially.
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (i < A.plong[part]) {
        // one long row per wave: lanes stride over the row
        const int code = A.long0[part] + i;
        const int64_t b = A.long_ptr[code], e = A.long_ptr[code + 1];
        const int r = A.long_row[code];
        for (int64_t p = b + lane; p < e; p += 256) {
            const int64_t q1 = min(p + 64, e - 1), q2 = min(p + 128, e - 1), q3 = min(p + 192, e - 1);
            const int c0 = nt_load(A.long_col + p), c1 = nt_load(A.long_col + q1);
            const int c2 = nt_load(A.long_col + q2), c3 = nt_load(A.long_col + q3);
            const Tv v0 = nt_load(A.long_val + p), v1 = nt_load(A.long_val + q1);
            const Tv v2 = nt_load(A.long_val + q2), v3 = nt_load(A.long_val + q3);
            a0 += double(v0) * double(x[c0]);
            a1 += (p + 64 < e ? double(v1) : 0.0) * double(x[c1]);
            a2 += (p + 128 < e ? double(v2) : 0.0) * double(x[c2]);
            a3 += (p + 192 < e ? double(v3) : 0.0) * double(x[c3]);
        }
        double a = (a0 + a1) + (a2 + a3);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (lane == 0) y[r] = Tx(a);
        return;
    }
    // a slice of R = kSliceRows << sc short rows, 64 / R lanes per row
    const int slice = A.slice0[part] + (i - A.plong[part]);
    const longlong2 d0 = reinterpret_cast<const longlong2 *>(A.slice_desc)[slice];
    const longlong2 d1 = reinterpret_cast<const longlong2 *>(A.slice_desc)[slice + 1];
    const int64_t p0 = d0.x, p1 = d1.x, rr = d0.y;
    const int R = kSliceRows << int(p0 & 3);
    const int64_t b = p0 & ~int64_t(63);
    const int groups = int(((p1 & ~int64_t(63)) - b) >> 6);
    // the slice's row numbers are loaded with its first entries (every lane loads: the
    // array carries 64 entries of padding at its end)
    const int rl = A.rowidx[rr + lane];
    const int r = lane < R ? rl : -1;
    const int *c = A.col + b + lane;
    const Tv *v = A.val + b + lane;
    for (int j = 0; j < groups; j += 4) {
        const int64_t o0 = int64_t(j) * 64, o1 = int64_t(min(j + 1, groups - 1)) * 64;
        const int64_t o2 = int64_t(min(j + 2, groups - 1)) * 64, o3 = int64_t(min(j + 3, groups - 1)) * 64;
        const int c0 = nt_load(c + o0), c1 = nt_load(c + o1), c2 = nt_load(c + o2), c3 = nt_load(c + o3);
        const Tv v0 = nt_load(v + o0), v1 = nt_load(v + o1), v2 = nt_load(v + o2), v3 = nt_load(v + o3);
        a0 += double(v0) * double(x[c0]);
        a1 += (j + 1 < groups ? double(v1) : 0.0) * double(x[c1]);
        a2 += (j + 2 < groups ? double(v2) : 0.0) * double(x[c2]);
        a3 += (j + 3 < groups ? double(v3) : 0.0) * double(x[c3]);
    }
    double a = (a0 + a1) + (a2 + a3);
    // lanes l, l + R, l + 2 R, ... hold the pieces of row l
    for (int o = R; o < 64; o <<= 1) a += __shfl_xor(a, o, 64);
    if (r >= 0) y[r] = Tx(a);
}

template <typename Tv, typename Tx>
void launch_hyb_spmv(const Hyb<Tv> &A, const Tx *x, Tx *y, hipStream_t s, const int *skip)
{
    int most = 0;
    for (int k = 0; k < kHybParts; ++k) most = std::max(most, A.ntask[k]);
    if (most <= 0) return;
    const int blocks = kHybParts * ((most + kBlock / 64 - 1) / (kBlock / 64));
    hipLaunchKernelGGL((k_hyb_spmv<Tv, Tx>), dim3(blocks), dim3(kBlock), 0, s, A, x, y, skip);
}
template void launch_hyb_spmv<float, float>(const Hyb<float> &, const float *, float *, hipStream_t, const int *);
template void launch_hyb_spmv<double, double>(const Hyb<double> &, const double *, double *, hipStream_t,
                                              const int *);
template void launch_hyb_spmv<float, double>(const Hyb<float> &, const double *, double *, hipStream_t,
                                             const int *);


// ---------------------------------------------------------------------------------
// Reductions.
// ---------------------------------------------------------------------------------
constexpr int kDotChunk = 8;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_multidot_partial(int n, int ncols, const T *__restrict__ Q, int64_t ldq,
                                                             const T *__restrict__ y, double *__restrict__ partial,
                                                             int pstride, const int *skip)
{
    if (skip && *skip) return;
    __shared__ double sh[kBlock / 64];
    const int c0 = blockIdx.y * kDotChunk;
    const int nc = min(kDotChunk, ncols - c0);
    double acc[kDotChunk];
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c) acc[c] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const double yi = double(y[i]);
#pragma unroll
        for (int c = 0; c < kDotChunk; ++c)
            if (c < nc) acc[c] += double(Q[i + int64_t(c0 + c) * ldq]) * yi;
    }
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c) {
        if (c < nc) {
            const double r = block_sum(acc[c], sh);
            if (threadIdx.x == 0) partial[int64_t(c0 + c) * pstride + blockIdx.x] = r;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_final_sum(int nparts, int pstride, const double *__restrict__ partial,
                                                      double *__restrict__ out, const int *skip)
{
    if (skip && *skip) return;
    __shared__ double sh[kBlock / 64];
    const int c = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) a += partial[int64_t(c) * pstride + b];
    const double r = block_sum(a, sh);
    if (threadIdx.x == 0) out[c] = r;
}

template <typename T>
void launch_multidot(int n, int ncols, const T *Q, int64_t ldq, const T *y, double *partial, double *out,
                     hipStream_t s, const int *skip)
{
    if (ncols <= 0) return;
    const int nb = red_blocks(n);
    dim3 grid(nb, (ncols + kDotChunk - 1) / kDotChunk);
    hipLaunchKernelGGL(k_multidot_partial<T>, grid, dim3(kBlock), 0, s, n, ncols, Q, ldq, y, partial, kRedBlocks, skip);
    hipLaunchKernelGGL(k_final_sum, dim3(ncols), dim3(kBlock), 0, s, nb, kRedBlocks, partial, out, skip);
}

template <typename T>
void launch_dot(int n, const T *x, const T *y, double *partial, double *out, hipStream_t s, const int *skip)
{
    launch_multidot<T>(n, 1, x, n, y, partial, out, s, skip);
}

// y -= alpha * Q c
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sub_qc(int n, int ncols, const T *__restrict__ Q, int64_t ldq,
                                                   const double *__restrict__ c, T *__restrict__ y, double alpha,
                                                   const int *skip)
{
    if (skip && *skip) return;
    __shared__ double cs[128];
    for (int t = threadIdx.x; t < ncols; t += kBlock) cs[t] = c[t] * alpha;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < ncols; ++k) acc += double(Q[i + int64_t(k) * ldq]) * cs[k];
    y[i] = T(double(y[i]) - acc);
}

template <typename T>
void launch_sub_qc(int n, int ncols, const T *Q, int64_t ldq, const double *c, T *y, hipStream_t s,
                   const int *skip, double alpha)
{
    if (ncols <= 0) return;
    hipLaunchKernelGGL(k_sub_qc<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, n, ncols, Q, ldq, c, y, alpha, skip);
}

__global__ void __launch_bounds__(kBlock) k_gemv_vs(int n, int m, const double *__restrict__ V, int64_t ldv,
                                                    const double *__restrict__ sv, double *__restrict__ y)
{
    __shared__ double cs[128];
    for (int t = threadIdx.x; t < m; t += kBlock) cs[t] = sv[t];
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += V[i + int64_t(k) * ldv] * cs[k];
    y[i] = acc;
}

void launch_gemv_vs(int n, int m, const double *V, int64_t ldv, const double *s, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_gemv_vs, dim3(nblocks(n)), dim3(kBlock), 0, st, n, m, V, ldv, s, y);
}

// Vout[:, 0 .. mout) = V[:, 0 .. m) S (column-major, the restart and deflation products
// of Rayleigh-Ritz) on the FP64 matrix cores: v_mfma_f64_16x16x4 multiplies a 16 x 4
// block of V (lane l holds row l % 16, column l / 16) by a 4 x 16 block of S (lane l
// holds row l / 16, column l % 16) into a 16 x 16 tile of which lane l holds rows
// l / 16 + 4 j (j = 0..3) of column l % 16 (checked on the device).  A workgroup covers 128 rows (each wave
// two 16-row blocks) and a slab of 64 output columns (blockIdx.y), and stages S through
// LDS 16 rows at a time; V is read once per slab (once when mout <= 64).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kMmRows = 128, kMmCols = 64, kMmK = 16;

__global__ void __launch_bounds__(kBlock) k_gemm_vs(int n, int m, int mout, const double *__restrict__ V,
                                                    int64_t ldv, const double *__restrict__ S, int lds,
                                                    double *__restrict__ Vout, int64_t ldo)
{
    __shared__ double sb[kMmK][kMmCols];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane >> 4, r16 = lane & 15;
    const int c0 = blockIdx.y * kMmCols;
    const int64_t rbase = int64_t(blockIdx.x) * kMmRows + wave * 32;
    v4d acc[2][kMmCols / 16];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < kMmCols / 16; ++t) acc[h][t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < m; k0 += kMmK) {
        __syncthreads();
        for (int e = threadIdx.x; e < kMmK * kMmCols; e += kBlock) {
            const int kk = e / kMmCols, cc = e % kMmCols;
            const int k = k0 + kk, c = c0 + cc;
            sb[kk][cc] = (k < m && c < mout) ? S[k + int64_t(c) * lds] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kMmK; kk += 4) {
            const int k = k0 + kk + q;
            double a[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t row = rbase + h * 16 + r16;
                a[h] = (row < n && k < m) ? V[row + int64_t(k) * ldv] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < kMmCols / 16; ++t) {
                const double b = sb[kk + q][t * 16 + r16];
                acc[0][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b, acc[0][t], 0, 0, 0);
                acc[1][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b, acc[1][t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < kMmCols / 16; ++t) {
            const int col = c0 + t * 16 + r16;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = rbase + h * 16 + q + 4 * j;
                if (row < n && col < mout) Vout[row + int64_t(col) * ldo] = acc[h][t][j];
            }
        }
}

void launch_gemm_vs(int n, int m, int mout, const double *V, int64_t ldv, const double *S, int lds, double *Vout,
                    int64_t ldo, hipStream_t st)
{
    if (mout <= 0 || n <= 0) return;
    dim3 grid(unsigned((int64_t(n) + kMmRows - 1) / kMmRows), unsigned((mout + kMmCols - 1) / kMmCols));
    hipLaunchKernelGGL(k_gemm_vs, grid, dim3(kBlock), 0, st, n, m, mout, V, ldv, S, lds, Vout, ldo);
}

// ---------------------------------------------------------------------------------
// Gauss-Jordan inverse of the dense last level.  One step per pivot column: a single
// workgroup picks the pivot row (largest modulus, lowest index on ties), swaps it in,
// scales it and saves the column of factors; then every other row is updated.
// ---------------------------------------------------------------------------------
constexpr int kGJ = 1024;

__global__ void __launch_bounds__(kGJ) k_gj_pivot(int n, int c, double *__restrict__ a, double *__restrict__ inv,
                                                  double *__restrict__ colc, int *status)
{
    __shared__ double sv[kGJ];
    __shared__ int si[kGJ];
    const int t = threadIdx.x;
    double best = -1.0;
    int bi = n;
    for (int r = c + t; r < n; r += kGJ) {
        const double v = fabs(a[int64_t(r) * n + c]);
        if (v > best) { best = v; bi = r; }
    }
    sv[t] = best;
    si[t] = bi;
    __syncthreads();
    for (int o = kGJ / 2; o > 0; o >>= 1) {
        if (t < o) {
            if (sv[t + o] > sv[t] || (sv[t + o] == sv[t] && si[t + o] < si[t])) { sv[t] = sv[t + o]; si[t] = si[t + o]; }
        }
        __syncthreads();
    }
    const int p = si[0];
    if (!(sv[0] > 0.0) || p >= n) {
        if (t == 0) status[0] = 1;
        return;
    }
    if (p != c) {
        for (int k = t; k < n; k += kGJ) {
            const double x = a[int64_t(c) * n + k];
            a[int64_t(c) * n + k] = a[int64_t(p) * n + k];
            a[int64_t(p) * n + k] = x;
            const double y = inv[int64_t(c) * n + k];
            inv[int64_t(c) * n + k] = inv[int64_t(p) * n + k];
            inv[int64_t(p) * n + k] = y;
        }
    }
    __syncthreads();
    const double pinv = 1.0 / a[int64_t(c) * n + c];
    __syncthreads();
    for (int k = t; k < n; k += kGJ) {
        a[int64_t(c) * n + k] *= pinv;
        inv[int64_t(c) * n + k] *= pinv;
    }
    for (int r = t; r < n; r += kGJ) colc[r] = (r == c) ? 0.0 : a[int64_t(r) * n + c];
}

__global__ void __launch_bounds__(kBlock) k_gj_elim(int n, int c, double *__restrict__ a, double *__restrict__ inv,
                                                    const double *__restrict__ colc, const int *status)
{
    if (status[0]) return;
    const int r = blockIdx.y;
    const double f = colc[r];
    if (f == 0.0) return;
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    if (k >= c) a[int64_t(r) * n + k] -= f * a[int64_t(c) * n + k];
    inv[int64_t(r) * n + k] -= f * inv[int64_t(c) * n + k];
}

__global__ void __launch_bounds__(kBlock) k_eye(int n, double *__restrict__ a)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(n) * n) a[i] = (i / n == i % n) ? 1.0 : 0.0;
}

void launch_gauss_jordan(int n, double *a, double *inv, double *colc, int *status, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_eye, dim3(nblocks(int64_t(n) * n)), dim3(kBlock), 0, s, n, inv);
    for (int c = 0; c < n; ++c) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kGJ), 0, s, n, c, a, inv, colc, status);
        hipLaunchKernelGGL(k_gj_elim, dim3(nblocks(n), n), dim3(kBlock), 0, s, n, c, a, inv, colc, status);
    }
}

__global__ void __launch_bounds__(kBlock) k_scale_sym(int n, double *__restrict__ a, const double *__restrict__ sc)
{
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < int64_t(n) * n) a[i] *= sc[i / n] * sc[i % n];
}

void launch_scale_sym(int n, double *a, const double *sc, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale_sym, dim3(nblocks(int64_t(n) * n)), dim3(kBlock), 0, s, n, a, sc);
}

// ---------------------------------------------------------------------------------
// Elementwise helpers.
// ---------------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBlock) k_convert(int n, const Tin *__restrict__ x, Tout *__restrict__ y,
                                                    double scale)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = Tout(double(x[i]) * scale);
}
template <typename Tin, typename Tout>
void launch_convert(int n, const Tin *x, Tout *y, double scale, hipStream_t s)
{
    hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(nblocks(n)), dim3(kBlock), 0, s, n, x, y, scale);
}

__global__ void __launch_bounds__(kBlock) k_axpby_d(int n, double a, const double *__restrict__ x, double b,
                                                    double *__restrict__ y)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    // b = 0 never reads y (it may be uninitialised memory, where 0 * NaN = NaN)
    if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}
void launch_axpby_d(int n, double a, const double *x, double b, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby_d, dim3(nblocks(n)), dim3(kBlock), 0, s, n, a, x, b, y);
}

__global__ void __launch_bounds__(kBlock) k_scale_inv_sqrt(int n, const double *__restrict__ nrm2, double *__restrict__ x)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const double sc = 1.0 / sqrt(*nrm2);
    if (i < n) x[i] *= sc;
}
void launch_scale_by_inv_sqrt(int n, const double *nrm2, double *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(nblocks(n)), dim3(kBlock), 0, s, n, nrm2, x);
}

// start vector entries u - 1/2 from SplitMix64 (seeded, independent of the disorder stream)
__global__ void __launch_bounds__(kBlock) k_random(int n, uint64_t seed, double *x)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    uint64_t z = seed + uint64_t(s + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[s] = double(z >> 11) * 0x1.0p-53 - 0.5;
}
void launch_random_vector(int n, uint64_t seed, double *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_random, dim3(nblocks(n)), dim3(kBlock), 0, s, n, seed, x);
}

// ---------------------------------------------------------------------------------
// Simplified QMR (Freund & Nachtigal) with device-resident scalars.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sqmr_init(int n, const T *__restrict__ b, T *__restrict__ r,
                                                      T *__restrict__ x, T *__restrict__ d)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    r[i] = b[i];
    x[i] = T(0);
    d[i] = T(0);
}
template <typename T>
void launch_sqmr_init(int n, const T *b, T *r, T *x, T *d, hipStream_t s)
{
    hipLaunchKernelGGL(k_sqmr_init<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, n, b, r, x, d);
}

__global__ void k_sqmr_params(SqmrState *st, double shift, double tol)
{
    if (threadIdx.x != 0) return;
    st->shift = shift;
    st->tol = tol;
}
void launch_sqmr_params(SqmrState *st, double shift, double tol, hipStream_t s)
{
    hipLaunchKernelGGL(k_sqmr_params, dim3(1), dim3(64), 0, s, st, shift, tol);
}

__global__ void k_sqmr_start(SqmrState *st, const double *rr, const double *rho)
{
    if (threadIdx.x != 0) return;
    st->tau = sqrt(*rr);
    st->tau0 = st->tau;
    st->rho = *rho;
    st->theta_old = 0.0;
    st->j = 0;
    st->breakdown = 0;
    st->done = (st->tau == 0.0 || st->rho == 0.0 || !isfinite(st->rho)) ? 1 : 0;
    st->done_next = st->done;
    st->done_prev = st->done;
}
void launch_sqmr_scalar_start(SqmrState *st, const double *rr, const double *rho, hipStream_t s)
{
    hipLaunchKernelGGL(k_sqmr_start, dim3(1), dim3(64), 0, s, st, rr, rho);
}

// scalar steps of simplified QMR, run by one thread after the reduction they need
__device__ inline void sqmr_alpha(SqmrState *st, double sigma)
{
    if (st->done) return;
    st->sigma = sigma;
    if (sigma == 0.0 || !isfinite(sigma)) {
        st->breakdown = 1;
        st->done = 1;
        st->done_next = 1;
        return;
    }
    st->alpha = st->rho / sigma;
}

__device__ inline void sqmr_theta(SqmrState *st, double rr)
{
    if (st->done) return;
    st->rr = rr;
    const double th = sqrt(rr) / st->tau;
    const double c2 = 1.0 / (1.0 + th * th);
    st->tau = st->tau * th * sqrt(c2);
    st->c1 = c2 * st->theta_old * st->theta_old;
    st->c2 = c2 * st->alpha;
    st->theta_old = th;
    st->theta = th;
    st->j += 1;
    if (st->tau * sqrt(double(st->j + 1)) <= st->tol * st->tau0 || !isfinite(st->tau)) st->done_next = 1;
}

// rn is read only when neither flag is set (then the reduction ran)
__device__ inline void sqmr_beta(SqmrState *st, const double *rn_p)
{
    if (!st->done && !st->done_next) {
        const double rn = *rn_p;
        if (rn == 0.0 || !isfinite(rn)) {
            st->breakdown = 1;
            st->done_next = 1;
        } else {
            st->beta = rn / st->rho;
            st->rho = rn;
        }
    }
    st->done_prev = st->done;
    st->done = st->done_next;
}

enum SqmrOp { kOpAlpha = 0, kOpTheta = 1, kOpBeta = 2 };

// out = sum of nparts partial sums (skipped, out untouched, when *skip), then one
// scalar step of simplified QMR by thread 0 (always run: it tests the flags itself)
template <int OP>
__global__ void __launch_bounds__(kBlock) k_final_sum_sqmr(int nparts, const double *__restrict__ partial,
                                                           double *__restrict__ out, const int *skip, SqmrState *st)
{
    __shared__ double sh[kBlock / 64];
    if (!*skip) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nparts; b += kBlock) a += partial[b];
        const double r = block_sum(a, sh);
        if (threadIdx.x == 0) *out = r;
    }
    if (threadIdx.x != 0) return;
    __threadfence_block();
    if (OP == kOpAlpha) sqmr_alpha(st, *out);
    else if (OP == kOpTheta) sqmr_theta(st, *out);
    else sqmr_beta(st, out);
}

// y -= Q c (ncols columns, ncols may be 0) and the partial sums of w . y, in one pass:
// the grid and the order of the products are those of k_multidot_partial with one
// column, so the partial sums are the same as a separate dot product's
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sub_qc_dot(int n, int ncols, const T *__restrict__ Q, int64_t ldq,
                                                       const double *__restrict__ c, T *__restrict__ y,
                                                       const T *__restrict__ w, double *__restrict__ partial,
                                                       const int *skip)
{
    if (skip && *skip) return;
    __shared__ double cs[128];
    __shared__ double sh[kBlock / 64];
    for (int t = threadIdx.x; t < ncols; t += kBlock) cs[t] = c[t];
    __syncthreads();
    double dot = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        double acc = 0.0;
        for (int k = 0; k < ncols; ++k) acc += double(Q[i + int64_t(k) * ldq]) * cs[k];
        const T v = ncols > 0 ? T(double(y[i]) - acc) : y[i];
        if (ncols > 0) y[i] = v;
        dot += double(w[i]) * double(v);
    }
    const double r = block_sum(dot, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <typename T>
void launch_sqmr_sub_dot_alpha(int n, int ncols, const T *Q, const double *c, T *t, const T *q, double *partial,
                               double *sigma, SqmrState *st, hipStream_t s)
{
    if (ncols > 128) throw std::invalid_argument("launch_sqmr_sub_dot_alpha: too many columns");
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_sub_qc_dot<T>, dim3(nb), dim3(kBlock), 0, s, n, ncols, Q, int64_t(n), c, t, q, partial,
                       &st->done);
    hipLaunchKernelGGL(k_final_sum_sqmr<kOpAlpha>, dim3(1), dim3(kBlock), 0, s, nb, partial, sigma, &st->done, st);
}

template <typename T>
void launch_sqmr_sub_dot_beta(int n, int ncols, const T *Y, const double *g, T *u, const T *r, double *partial,
                              double *rho, SqmrState *st, hipStream_t s)
{
    if (ncols > 128) throw std::invalid_argument("launch_sqmr_sub_dot_beta: too many columns");
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_sub_qc_dot<T>, dim3(nb), dim3(kBlock), 0, s, n, ncols, Y, int64_t(n), g, u, r, partial,
                       &st->done_next);
    hipLaunchKernelGGL(k_final_sum_sqmr<kOpBeta>, dim3(1), dim3(kBlock), 0, s, nb, partial, rho, &st->done_next, st);
}

// r -= alpha t, with the partial sums of |r|^2
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sqmr_update_r(int n, const SqmrState *st, const T *__restrict__ t,
                                                          T *__restrict__ r, double *__restrict__ partial)
{
    if (st->done) return;
    __shared__ double sh[kBlock / 64];
    const T a = T(st->alpha);
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const T v = r[i] - a * t[i];
        r[i] = v;
        acc += double(v) * double(v);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
template <typename T>
void launch_sqmr_update_r(int n, SqmrState *st, const T *t, T *r, double *partial, double *rr, hipStream_t s)
{
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_sqmr_update_r<T>, dim3(nb), dim3(kBlock), 0, s, n, st, t, r, partial);
    hipLaunchKernelGGL(k_final_sum_sqmr<kOpTheta>, dim3(1), dim3(kBlock), 0, s, nb, partial, rr, &st->done, st);
}

// The end of a step, in one pass over q: d = c1 d + c2 q and x += d (when the step was
// live before the beta step), then q = u + beta q (when it is still live after it).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sqmr_update_xdq(int n, const SqmrState *st, const T *__restrict__ u,
                                                            T *__restrict__ q, T *__restrict__ d, T *__restrict__ x)
{
    const bool xd = !st->done_prev, nq = !st->done;
    if (!xd && !nq) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const T qi = q[i];
    if (xd) {
        const T dv = T(st->c1) * d[i] + T(st->c2) * qi;
        d[i] = dv;
        x[i] += dv;
    }
    if (nq) q[i] = u[i] + T(st->beta) * qi;
}
template <typename T>
void launch_sqmr_update_xdq(int n, SqmrState *st, const T *u, T *q, T *d, T *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_sqmr_update_xdq<T>, dim3(nblocks(n)), dim3(kBlock), 0, s, n, st, u, q, d, x);
}

__global__ void k_small_matvec(int p, const double *__restrict__ M, const double *__restrict__ c,
                               double *__restrict__ out, const int *skip)
{
    if (skip && *skip) return;
    const int i = threadIdx.x;
    if (i >= p) return;
    double a = 0.0;
    for (int k = 0; k < p; ++k) a += M[i + k * p] * c[k];
    out[i] = a;
}
void launch_small_matvec(int p, const double *M, const double *c, double *out, const int *skip, hipStream_t s)
{
    if (p <= 0) return;
    hipLaunchKernelGGL(k_small_matvec, dim3(1), dim3(128), 0, s, p, M, c, out, skip);
}

// ---- explicit instantiations ------------------------------------------------------
#define JD_INST(T)                                                                                        \
    template void launch_stencil<T>(int, int, const T *, double, const T *, T *, hipStream_t, const int *,       \
                                    const T *);                                                                 \
    template void launch_stencil_state<T>(int, int, const double *, const SqmrState *, const T *, T *,         \
                                          hipStream_t, const double *);                                         \
    template void launch_copy<T>(int, const T *, T *, hipStream_t);                                       \
    template void launch_gather<T>(int, const int *, const T *, T *, hipStream_t, const int *);            \
    template void launch_scatter<T>(int, const int *, const T *, T *, hipStream_t, const int *);           \
    template void launch_down<T>(const DevLevel<T> &, T *, hipStream_t, const int *);                      \
    template void launch_up<T>(const DevLevel<T> &, const T *, T *, hipStream_t, const int *);             \
    template void launch_coarse<T>(int, int, int, const T *, const T *, T *, hipStream_t, const int *);    \
    template void launch_dinv_coarse<T>(int, const T *, const T *, const int *, int, int, const int *,      \
                                        const T *, const T *, T *, T *, hipStream_t, const int *);          \
    template void launch_multidot<T>(int, int, const T *, int64_t, const T *, double *, double *,          \
                                     hipStream_t, const int *);                                            \
    template void launch_dot<T>(int, const T *, const T *, double *, double *, hipStream_t, const int *);  \
    template void launch_sub_qc<T>(int, int, const T *, int64_t, const double *, T *, hipStream_t,        \
                                   const int *, double);                                                   \
    template void launch_sqmr_init<T>(int, const T *, T *, T *, T *, hipStream_t);                        \
    template void launch_sqmr_update_r<T>(int, SqmrState *, const T *, T *, double *, double *,           \
                                          hipStream_t);                                                    \
    template void launch_sqmr_update_xdq<T>(int, SqmrState *, const T *, T *, T *, T *, hipStream_t);      \
    template void launch_sqmr_sub_dot_alpha<T>(int, int, const T *, const double *, T *, const T *,        \
                                               double *, double *, SqmrState *, hipStream_t);              \
    template void launch_sqmr_sub_dot_beta<T>(int, int, const T *, const double *, T *, const T *,         \
                                              double *, double *, SqmrState *, hipStream_t);
JD_INST(float)
JD_INST(double)
template void launch_convert<double, float>(int, const double *, float *, double, hipStream_t);
template void launch_convert<float, double>(int, const float *, double *, double, hipStream_t);
template void launch_convert<double, double>(int, const double *, double *, double, hipStream_t);
template void launch_convert<float, float>(int, const float *, float *, double, hipStream_t);

}  // namespace jdmi
