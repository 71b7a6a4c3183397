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
"""
import numpy as np
import scipy.sparse as sp

NEIGHBOURS = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def site_coords(L):
    s = np.arange(L ** 3)
    return s % L, (s // L) % L, s // (L * L)


def hamiltonian(L, eps, hopping=-1.0):
    """CSR of A = hopping * T + diag(eps); duplicate couplings accumulate."""
    n = L ** 3
    i, j, k = site_coords(L)
    s = np.arange(n)
    rows, cols = [s], [s]
    vals = [np.asarray(eps, dtype=np.float64)]
    for di, dj, dk in NEIGHBOURS:
        rows.append(s)
        cols.append(((i + di) % L) + L * (((j + dj) % L) + L * ((k + dk) % L)))
        vals.append(np.full(n, hopping))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()  # COO -> CSR sums duplicates


def matvec(L, eps, x, shift=0.0, hopping=-1.0):
    """y = (A - shift I) x, written out neighbour by neighbour."""
    x = np.asarray(x, dtype=np.float64)
    X = x.reshape(L, L, L)  # axes (k, j, i)
    nb = (np.roll(X, 1, 2) + np.roll(X, -1, 2) + np.roll(X, 1, 1) + np.roll(X, -1, 1)
          + np.roll(X, 1, 0) + np.roll(X, -1, 0)).reshape(-1)
    return hopping * nb + (np.asarray(eps) - shift) * x


def inf_norm(eps):
    """||A||_inf = 6 + max|eps| (six couplings of modulus 1 per row, any L >= 2)."""
    return 6.0 + float(np.max(np.abs(eps))) if len(eps) else 6.0


def clean_spectrum(L):
    """Closed form at W = 0: -2 (cos(2 pi a/L) + cos(2 pi b/L) + cos(2 pi c/L))."""
    c = np.cos(2.0 * np.pi * np.arange(L) / L)
    return -2.0 * (c[:, None, None] + c[None, :, None] + c[None, None, :]).reshape(-1)
