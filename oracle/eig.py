"""O7 -- the result the hot path must reproduce, and the checks around it.

Problem statement (abstract; section 3; section 8.2): a few eigenpairs of the
Anderson matrix nearest a target sigma (the paper: the five nearest lambda = 0).
Definition used here: the k eigenvalues of A = -T + diag(eps) on the periodic
L^3 lattice with the smallest |lambda - sigma|, ties ordered by lambda, with unit
eigenvectors whose largest-modulus component is positive (lowest index on ties).
No preconditioner or iteration parameter enters this definition.  With bc="hardwall"
the same definition holds for the lattice with hard walls (section 8.2), and with
hop (random bond values, the off-diagonal model of section 8.2) for that model.

* n <= DENSE_MAX: all eigenpairs by dense Jacobi (O3), then selection;
* otherwise: shift-and-invert Lanczos (O5) on the exact multifrontal LDL^T (O4).
  If A - sigma I is numerically singular the factorisation shift becomes
  sigma_f = sigma + 1e-9 (1 + |sigma|); selection still uses sigma.
"""
import time

import numpy as np

from . import generator, jacobi, lanczos, lattice, ldlt

DENSE_MAX = 512


def select_nearest(lams, sigma, k):
    """Indices of the k values nearest sigma, ordered by (|lam - sigma|, lam)."""
    lams = np.asarray(lams)
    order = np.lexsort((lams, np.abs(lams - sigma)))
    return order[:k]


def normalise_signs(X):
    """Unit columns, largest-|x_i| component positive (first index on ties)."""
    X = np.array(X, dtype=np.float64, copy=True)
    for c in range(X.shape[1]):
        x = X[:, c] / np.linalg.norm(X[:, c])
        i = int(np.argmax(np.abs(x)))
        X[:, c] = -x if x[i] < 0 else x
    return X


class _Solver:
    def __init__(self, fact):
        self.fact = fact
        self.shift = fact.tau

    def __call__(self, b):
        return self.fact.solve(b)


def factor_near(L, eps, sigma, leaf=256, bc="periodic", hop=None):
    """Exact LDL^T of A - sigma_f I with the singular-shift retry."""
    anorm = lattice.inf_norm(eps, L, bc, hop)
    for sf in (sigma, sigma + 1e-9 * (1.0 + abs(sigma))):
        try:
            f = ldlt.LDLT(L, eps, sf, leaf=leaf, bc=bc, hop=hop)
        except ZeroDivisionError:
            continue
        if f.min_pivot > 1e-13 * anorm:
            return f
    return f


def nearest_eigenpairs(L, eps, sigma, k, tol=1e-12, method=None, timings=None, bc="periodic", hop=None):
    """(lams[k], X[n, k], res[k], anorm) -- the result definition above.

    ``timings`` (a dict, optional) receives the seconds of the factorisation and of the
    Lanczos iteration of the large path."""
    eps = np.asarray(eps, dtype=np.float64)
    n = L ** 3
    anorm = lattice.inf_norm(eps, L, bc, hop)
    if method is None:
        method = "dense" if n <= DENSE_MAX else "lanczos"
    if method == "dense":
        A = lattice.hamiltonian(L, eps, bc=bc, hop=hop).toarray()
        w, V = jacobi.eigh(A)
        idx = select_nearest(w, sigma, k)
        lams, X = w[idx], V[:, idx]
    else:
        t0 = time.time()
        f = factor_near(L, eps, sigma, bc=bc, hop=hop)
        t1 = time.time()
        lams, X, _ = lanczos.si_lanczos(L, eps, sigma, k, _Solver(f), tol=tol, bc=bc, hop=hop)
        if timings is not None:
            timings["factorisation_s"] = t1 - t0
            timings["lanczos_s"] = time.time() - t1
        idx = select_nearest(lams, sigma, k)
        lams, X = lams[idx], X[:, idx]
    X = normalise_signs(X)
    res = np.array([np.linalg.norm(lattice.matvec(L, eps, X[:, c], bc=bc, hop=hop) - lams[c] * X[:, c])
                    for c in range(X.shape[1])])
    return lams, X, res, anorm


def anderson_nearest(L, W, seed, sigma, k, model="anderson", **kw):
    """The definition for the seeded lattice: the diagonal model (box disorder of width W
    on the diagonal, couplings -1) or the off-diagonal model (constant diagonal 1.28,
    bonds uniform of width W; section 8.2)."""
    if model == "offdiag":
        eps, hop = generator.offdiag_model(L, W, seed)
        return nearest_eigenpairs(L, eps, sigma, k, hop=hop, **kw)
    return nearest_eigenpairs(L, generator.disorder(L, W, seed), sigma, k, **kw)


def count_in_window(L, eps, lo, hi, bc="periodic", hop=None):
    """Number of eigenvalues in [lo, hi) by two inertia counts (Sylvester)."""
    n_hi, z_hi = ldlt.count_below(L, eps, hi, bc=bc, hop=hop)
    n_lo, z_lo = ldlt.count_below(L, eps, lo, bc=bc, hop=hop)
    if z_hi or z_lo:
        raise ZeroDivisionError("window end is an eigenvalue")
    return n_hi - n_lo
