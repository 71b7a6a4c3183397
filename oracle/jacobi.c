/*
 * O3 -- dense cyclic Jacobi eigensolver (oracle, test infrastructure only).
 *
 * The textbook two-sided Jacobi method for a real symmetric matrix (Jacobi 1846;
 * Golub & Van Loan, "Matrix Computations", section 8.5, the 2x2 symmetric Schur
 * decomposition and the cyclic-by-row sweep).  Used as brute force on tiny
 * lattices and for the small projected matrices of the oracle's Lanczos method.
 *
 * A (n x n, row-major, symmetric) is overwritten; on return its diagonal holds the
 * eigenvalues (also copied to w).  If vt != NULL, row p of vt is the unit
 * eigenvector for w[p].  Iteration stops when off(A) <= tol * ||A||_F or after
 * max_sweeps sweeps; the return value is the number of sweeps, or -1 if the
 * tolerance was not met.
 */
#include <math.h>
#include <stddef.h>

static double frob2(int n, const double *a, int offdiag_only)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (!offdiag_only || i != j) s += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    return s;
}

int oracle_jacobi_eig(int n, double *a, double *vt, double *w, double tol, int max_sweeps)
{
    if (vt)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) vt[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    const double fro = sqrt(frob2(n, a, 0));
    int sweep = 0, ok = 0;
    for (; sweep <= max_sweeps; ++sweep) {
        if (sqrt(frob2(n, a, 1)) <= tol * fro) { ok = 1; break; }
        if (sweep == max_sweeps) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double *ap = a + (size_t)p * n, *aq = a + (size_t)q * n;
                const double apq = ap[q];
                if (apq == 0.0) continue;
                /* 2x2 symmetric Schur: choose t = tan(theta) of smaller modulus */
                const double tau = (aq[q] - ap[p]) / (2.0 * apq);
                const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                              : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* rows p, q of J^T A J; by symmetry these are also columns p, q */
                const double app = ap[p], aqq = aq[q];
                for (int k = 0; k < n; ++k) {
                    if (k == p || k == q) continue;
                    const double akp = ap[k], akq = aq[k];
                    const double np_ = c * akp - s * akq, nq_ = s * akp + c * akq;
                    ap[k] = np_; aq[k] = nq_;
                    a[(size_t)k * n + p] = np_; a[(size_t)k * n + q] = nq_;
                }
                /* the zeroing rotation gives app - t apq and aqq + t apq exactly */
                ap[p] = app - t * apq;
                aq[q] = aqq + t * apq;
                ap[q] = 0.0; aq[p] = 0.0;
                if (vt) {
                    double *vp = vt + (size_t)p * n, *vq = vt + (size_t)q * n;
                    for (int k = 0; k < n; ++k) {
                        const double x = vp[k], y = vq[k];
                        vp[k] = c * x - s * y; vq[k] = s * x + c * y;
                    }
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
    return ok ? sweep : -1;
}
