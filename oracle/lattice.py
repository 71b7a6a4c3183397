"""O2 -- the Anderson Hamiltonian on the periodic L x L x L lattice.

Section 3, eq. (eigenequation): every site couples to its six nearest neighbours
and carries the random potential eps on the diagonal.  The paper writes the
hopping as +1; the operator used throughout this project is
A = -T + diag(eps), T the 0/1 adjacency of the periodic lattice (hopping -1).
For even L the staggered gauge U = diag((-1)^{i+j+k}) maps one sign onto the
other (U T U = -T), so the spectra coincide; the tests check this.

Periodic boundary conditions (figure 1 caption; section 8.2): x_0 = x_L and
x_{L+1} = x_1 in every direction.  For L = 2 the +1 and -1 neighbours of a site
coincide, so the two couplings add up to one entry of -2.

Hard-wall boundary conditions (section 8.2, the variant of Table 6): the lattice is
embedded in zeros, x_0 = x_{L+1} = 0, so a site on a face has no coupling across it.
``bc`` selects "periodic" (default) or "hardwall" everywhere below.

Random couplings (the off-diagonal model of section 8.2): ``hop`` (shape (3, n)) gives
the value of the bond from site s to its +x, +y, +z neighbour, hop[d, s]; the matrix
entry of that bond is hop[d, s] itself, in both triangles (the constant -1 couplings of
the diagonal model are hop = -1 everywhere).  None keeps the constant coupling.
"""
import numpy as np
import scipy.sparse as sp

NEIGHBOURS = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def site_coords(L):
    s = np.arange(L ** 3)
    return s % L, (s // L) % L, s // (L * L)


def _check_bc(bc):
    if bc not in ("periodic", "hardwall"):
        raise ValueError(f"unknown boundary condition {bc!r}")


def _hamiltonian_bonds(L, eps, hop, bc):
    """CSR with one entry hop[d, s] per bond, placed in both triangles."""
    n = L ** 3
    i, j, k = site_coords(L)
    s = np.arange(n)
    rows, cols = [s], [s]
    vals = [np.asarray(eps, dtype=np.float64)]
    for d, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        ii, jj, kk = i + di, j + dj, k + dk
        keep = np.ones(n, bool) if bc == "periodic" else (ii < L) & (jj < L) & (kk < L)
        nb = ((ii % L) + L * ((jj % L) + L * (kk % L)))[keep]
        t = np.asarray(hop[d], dtype=np.float64)[keep]
        rows += [s[keep], nb]
        cols += [nb, s[keep]]
        vals += [t, t]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A.tocsr()


def hamiltonian(L, eps, hopping=-1.0, bc="periodic", hop=None):
    """CSR of A = hopping * T + diag(eps) (or the bond values hop); duplicate couplings
    accumulate."""
    _check_bc(bc)
    if hop is not None:
        return _hamiltonian_bonds(L, eps, hop, bc)
    n = L ** 3
    i, j, k = site_coords(L)
    s = np.arange(n)
    rows, cols = [s], [s]
    vals = [np.asarray(eps, dtype=np.float64)]
    for di, dj, dk in NEIGHBOURS:
        ii, jj, kk = i + di, j + dj, k + dk
        if bc == "periodic":
            keep = np.ones(n, bool)
        else:  # a neighbour outside the box is a zero of the embedding: no coupling
            keep = (ii >= 0) & (ii < L) & (jj >= 0) & (jj < L) & (kk >= 0) & (kk < L)
        rows.append(s[keep])
        cols.append(((ii % L) + L * ((jj % L) + L * (kk % L)))[keep])
        vals.append(np.full(int(keep.sum()), hopping))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()  # COO -> CSR sums duplicates


def _shift(X, step, axis, bc):
    """Y[.., m, ..] = X[.., m - step, ..] along axis: cyclic, or with zeros shifted in."""
    if bc == "periodic":
        return np.roll(X, step, axis)
    Y = np.zeros_like(X)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if step > 0:
        src[axis], dst[axis] = slice(0, X.shape[axis] - step), slice(step, None)
    else:
        src[axis], dst[axis] = slice(-step, None), slice(0, X.shape[axis] + step)
    Y[tuple(dst)] = X[tuple(src)]
    return Y


def matvec(L, eps, x, shift=0.0, hopping=-1.0, bc="periodic", hop=None):
    """y = (A - shift I) x, written out neighbour by neighbour."""
    _check_bc(bc)
    x = np.asarray(x, dtype=np.float64)
    X = x.reshape(L, L, L)  # axes (k, j, i)
    if hop is not None:
        # bond d of site s couples s and s + e_d: y_s += t_s x_{s+e}, y_{s+e} += t_s x_s
        y = (np.asarray(eps) - shift) * x
        for d, axis in ((0, 2), (1, 1), (2, 0)):
            T = np.asarray(hop[d], dtype=np.float64).reshape(L, L, L)
            if bc == "hardwall":  # the bonds of the last layer leave the box
                T = T.copy()
                idx = [slice(None)] * 3
                idx[axis] = L - 1
                T[tuple(idx)] = 0.0
            y += (T * _shift(X, -1, axis, bc)).reshape(-1)
            y += _shift(T * X, 1, axis, bc).reshape(-1)
        return y
    nb = (_shift(X, 1, 2, bc) + _shift(X, -1, 2, bc) + _shift(X, 1, 1, bc) + _shift(X, -1, 1, bc)
          + _shift(X, 1, 0, bc) + _shift(X, -1, 0, bc)).reshape(-1)
    return hopping * nb + (np.asarray(eps) - shift) * x


def degree(L, bc="periodic"):
    """Couplings of every site: 6 on the torus; 6 minus the faces a site lies on with
    hard walls (for L = 1 every coupling leaves the box)."""
    _check_bc(bc)
    if bc == "periodic":
        return np.full(L ** 3, 6)
    i, j, k = site_coords(L)
    d = np.zeros(L ** 3, dtype=np.int64)
    for c in (i, j, k):
        d += (c > 0).astype(np.int64) + (c < L - 1).astype(np.int64)
    return d


def inf_norm(eps, L=None, bc="periodic", hop=None):
    """||A||_inf = max_s (couplings of s + |eps_s|): 6 + max|eps| on the torus (six
    couplings of modulus 1 per row, any L >= 2); with hard walls the row sums differ
    and L is needed; with bond values, the largest row sum of their moduli."""
    eps = np.asarray(eps, dtype=np.float64)
    if hop is not None:
        if L is None:
            L = int(round(len(eps) ** (1.0 / 3.0)))
        A = hamiltonian(L, eps, bc=bc, hop=hop)
        return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))
    if bc == "periodic":
        return 6.0 + float(np.max(np.abs(eps))) if len(eps) else 6.0
    if L is None:
        L = int(round(len(eps) ** (1.0 / 3.0)))
    return float(np.max(degree(L, bc) + np.abs(eps)))


def clean_spectrum(L, bc="periodic"):
    """Closed form at W = 0: -2 (cos(2 pi a/L) + cos(2 pi b/L) + cos(2 pi c/L)),
    a, b, c = 0 .. L-1 (periodic); -2 sum cos(pi a/(L+1)), a = 1 .. L (hard walls:
    the sine modes of the open chain)."""
    _check_bc(bc)
    if bc == "periodic":
        c = np.cos(2.0 * np.pi * np.arange(L) / L)
    else:
        c = np.cos(np.pi * np.arange(1, L + 1) / (L + 1))
    return -2.0 * (c[:, None, None] + c[None, :, None] + c[None, None, :]).reshape(-1)
