"""O5 -- shift-and-invert Lanczos with full reorthogonalisation.

Section 4.1: Lanczos applied to (A - sigma I)^{-1} builds orthonormal v_1, v_2, ...
and a tridiagonal T with (A - sigma I)^{-1} V_m = V_m T_m + beta_m v_{m+1} e_m^T
(the recurrence of eq. (lanczos) with A replaced by the shifted inverse; the
paper's beta_{i+1} = v_{i+1} A v_i is read with the missing transpose,
v_{i+1}^T (A - sigma I)^{-1} v_i).  Eigenvalues mu of T_m approximate those of
(A - sigma I)^{-1}; lambda = sigma + 1/mu, so the largest |mu| give the
eigenvalues nearest sigma.  The paper's production runs restart implicitly
(ARPACK); the oracle does not restart and re-orthogonalises every new vector
twice against all previous ones (classical Gram-Schmidt, twice), which keeps
V_m orthonormal to working precision.  Eigenpairs of T_m come from the dense
Jacobi solver (O3).  Each returned pair is refined by its Rayleigh quotient and
accepted only when its residual, computed directly from A, is below the target.
"""
import numpy as np

from . import jacobi, lattice


def si_lanczos(L, eps, sigma, k, solve, tol=1e-12, max_steps=None, seed=12345,
               extra=2, bc="periodic", hop=None):
    """k + extra eigenpairs of A nearest sigma.

    ``solve(b)`` must return (A - sigma_f I)^{-1} b for a fixed sigma_f near sigma;
    ``solve.shift`` holds sigma_f.  Returns (lams, X, res) sorted by (|lam - sigma|, lam),
    with res the directly computed ||A x - lam x||_2 of each unit vector x.
    """
    n = L ** 3
    want = min(k + extra, n)
    sf = solve.shift
    anorm = lattice.inf_norm(eps, L, bc, hop)
    max_steps = min(n, max_steps or max(4 * want + 40, 80))
    rng = np.random.default_rng(seed)
    V = np.zeros((n, max_steps + 1))
    v = rng.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    alpha = []
    beta = []
    result = None
    for m in range(1, max_steps + 1):
        w = solve(V[:, m - 1])
        a = V[:, m - 1] @ w
        # full reorthogonalisation, classical Gram-Schmidt applied twice
        for _ in range(2):
            w -= V[:, :m] @ (V[:, :m].T @ w)
        b = np.linalg.norm(w)
        alpha.append(a)
        beta.append(b)
        if m >= want and (m % 5 == 0 or m == max_steps or b == 0.0):
            T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
            mu, S = jacobi.eigh(T)
            pick = np.argsort(-np.abs(mu), kind="stable")[:want]
            lams, X, res = [], [], []
            for p in pick:
                if mu[p] == 0.0:
                    continue
                x = V[:, :m] @ S[:, p]
                x /= np.linalg.norm(x)
                ax = lattice.matvec(L, eps, x, bc=bc, hop=hop)
                lam = x @ ax  # Rayleigh quotient
                lams.append(lam)
                X.append(x)
                res.append(np.linalg.norm(ax - lam * x))
            lams = np.array(lams)
            res = np.array(res)
            if len(lams) == want and np.all(res <= tol * anorm):
                result = (lams, np.array(X).T, res)
                break
        if b == 0.0:
            break
        V[:, m] = w / b
    if result is None:
        raise RuntimeError("shift-and-invert Lanczos did not converge")
    lams, X, res = result
    order = np.lexsort((lams, np.abs(lams - sigma)))
    return lams[order], X[:, order], res[order]
