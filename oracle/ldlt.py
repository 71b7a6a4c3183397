"""O4/O6 -- exact sparse LDL^T of A - tau I on the periodic lattice, and its inertia.

Reference for what is computed: the shift-and-invert methods of section 4.1 need
full-accuracy solves with A - sigma I, and a symmetric indefinite LDL^T with 1x1
and 2x2 pivots (section 5.1: Bunch-Kaufman pivoting restricted to dense blocks)
provides them.  By Sylvester's law of inertia, the signs of the 1x1 and 2x2 blocks
of D count the eigenvalues of A below tau.

How it is computed (textbook multifrontal method, no approximation):

* geometric nested dissection of the torus: a still-periodic direction is cut by
  two planes (a single plane does not disconnect a ring), an open direction by one
  plane through its middle; boxes of at most ``leaf`` sites are leaves;
* each tree node owns its separator (or leaf box); its front couples those
  variables to the ancestors they touch (the node's boundary);
* the fully summed block F11 of a front is factored by LAPACK's Bunch-Kaufman
  LDL^T (``dsytrf``), the boundary receives the Schur complement
  F22 - F12^T F11^{-1} F12, which is added into the parent front.

Inertia is additive over this block elimination (Haynsworth), so the total
count of negative eigenvalues is the sum over the fronts' D blocks.
"""
import numpy as np
import scipy.linalg
from scipy.linalg import lapack

from . import lattice


class _Node:
    __slots__ = ("own", "children", "bnd", "ldu", "ipiv", "f12", "first")

    def __init__(self, own):
        self.own = own
        self.children = []
        self.bnd = None
        self.ldu = None
        self.ipiv = None
        self.f12 = None
        self.first = None


def _region_sites(L, ivs):
    """Site indices of a box given three coordinate lists (x, y, z)."""
    xs, ys, zs = (np.asarray(v, dtype=np.int64) for v in ivs)
    return (xs[None, None, :] + L * (ys[None, :, None] + L * zs[:, None, None])).reshape(-1)


def nested_dissection(L, leaf=256, bc="periodic"):
    """Postorder list of nodes of a geometric nested-dissection tree of the torus (or,
    with hard walls, of the box: every direction open from the start)."""
    order = []

    def build(ivs, wrap):
        size = len(ivs[0]) * len(ivs[1]) * len(ivs[2])
        if size == 0:
            return None
        # pick the longest direction that can be cut (prefer still-periodic ones on ties)
        best = None
        for d in range(3):
            m = len(ivs[d])
            can = (m >= 4) if wrap[d] else (m >= 3)
            if can and (best is None or (m, wrap[d]) > (len(ivs[best]), wrap[best])):
                best = d
        if size <= leaf or best is None:
            node = _Node(_region_sites(L, ivs))
            order.append(node)
            return node
        d = best
        coords = ivs[d]
        m = len(coords)
        if wrap[d]:
            h = m // 2
            sep = [coords[0], coords[h]]
            parts = [coords[1:h], coords[h + 1:]]
        else:
            h = m // 2
            sep = [coords[h]]
            parts = [coords[:h], coords[h + 1:]]
        kids = []
        for part in parts:
            civs = list(ivs)
            civs[d] = part
            cw = list(wrap)
            cw[d] = False
            c = build(civs, cw)
            if c is not None:
                kids.append(c)
        sivs = list(ivs)
        sivs[d] = sep
        node = _Node(_region_sites(L, sivs))
        node.children = kids
        order.append(node)
        return node

    periodic = bc == "periodic"
    build([list(range(L))] * 3, [periodic] * 3)
    return order


def _neighbours(L, v, bc="periodic"):
    i = v % L
    j = (v // L) % L
    k = v // (L * L)
    out = []
    for di, dj, dk in lattice.NEIGHBOURS:
        ii, jj, kk = i + di, j + dj, k + dk
        nb = (ii % L) + L * ((jj % L) + L * (kk % L))
        if bc != "periodic":
            nb = nb[(ii >= 0) & (ii < L) & (jj >= 0) & (jj < L) & (kk >= 0) & (kk < L)]
        out.append(nb)
    return np.concatenate(out)


def _d_inertia(ldu, ipiv):
    """(#neg, #zero, #pos, min |eigenvalue| of a D block) from dsytrf's lower output."""
    m = ldu.shape[0]
    neg = zero = pos = 0
    dmin = np.inf
    k = 0
    while k < m:
        if ipiv[k] > 0:
            d = ldu[k, k]
            if d < 0:
                neg += 1
            elif d > 0:
                pos += 1
            else:
                zero += 1
            dmin = min(dmin, abs(d))
            k += 1
        else:
            a, b, c = ldu[k, k], ldu[k + 1, k], ldu[k + 1, k + 1]
            ev = np.linalg.eigvalsh(np.array([[a, b], [b, c]]))
            for e in ev:
                if e < 0:
                    neg += 1
                elif e > 0:
                    pos += 1
                else:
                    zero += 1
                dmin = min(dmin, abs(e))
            k += 2
    return neg, zero, pos, dmin


class LDLT:
    """Exact multifrontal LDL^T of A - tau I, A the Anderson matrix on the L^3 torus.

    ``keep_factors=False`` gives the inertia-only mode: each front is discarded as
    soon as its Schur complement has been passed on.
    """

    def __init__(self, L, eps, tau, leaf=256, keep_factors=True, bc="periodic", hop=None):
        self.L = L
        self.n = L ** 3
        self.tau = float(tau)
        self.bc = bc
        self.hop = hop
        self.eps = np.asarray(eps, dtype=np.float64)
        A = lattice.hamiltonian(L, self.eps, bc=bc, hop=hop)
        A = A - self.tau * _sp_eye(self.n)
        A = A.tocsr()
        self.nodes = nested_dissection(L, leaf, bc)
        owner = np.empty(self.n, dtype=np.int64)
        for t, node in enumerate(self.nodes):
            owner[node.own] = t
        # first descendant (postorder) of every node
        for t, node in enumerate(self.nodes):
            node.first = min([c.first for c in node.children], default=t)
        pos = -np.ones(self.n, dtype=np.int64)
        updates = {}
        self.neg = self.zero = self.pos = 0
        self.min_pivot = np.inf
        for t, node in enumerate(self.nodes):
            cand = [_neighbours(L, node.own, bc)] + [c.bnd for c in node.children]
            cand = np.unique(np.concatenate(cand))
            node.bnd = cand[owner[cand] > t]
            front = np.concatenate([node.own, node.bnd])
            m1, m = len(node.own), len(front)
            pos[front] = np.arange(m)
            F = np.zeros((m, m))
            # original entries in the rows of the owned variables (and their mirror
            # images in the boundary rows)
            for r_local, v in enumerate(node.own):
                lo, hi = A.indptr[v], A.indptr[v + 1]
                cols = A.indices[lo:hi]
                vals = A.data[lo:hi]
                keep = owner[cols] >= t
                cl = pos[cols[keep]]
                F[r_local, cl] += vals[keep]
                bmask = cl >= m1
                F[cl[bmask], r_local] += vals[keep][bmask]
            for c in node.children:
                U = updates.pop(id(c))
                ix = pos[c.bnd]
                F[np.ix_(ix, ix)] += U
            pos[front] = -1
            F11 = F[:m1, :m1]
            ldu, ipiv, info = lapack.dsytrf(F11, lower=1, lwork=max(1, 64 * m1))
            if info < 0:
                raise RuntimeError("dsytrf argument error")
            neg, zero, posv, dmin = _d_inertia(ldu, ipiv)
            self.neg += neg
            self.zero += zero
            self.pos += posv
            self.min_pivot = min(self.min_pivot, dmin)
            if zero:
                # exactly singular block: the factorization cannot continue
                raise ZeroDivisionError("singular pivot block in the exact LDL^T")
            if m > m1:
                F12 = F[:m1, m1:]
                # F11^{-1} F12 for many right-hand sides: LU with partial pivoting
                # (LAPACK getrf/getrs, level-3); the Bunch-Kaufman factors above give
                # the inertia and the one-vector solves.
                X = scipy.linalg.lu_solve(scipy.linalg.lu_factor(F11, check_finite=False),
                                          F12, check_finite=False)
                updates[id(node)] = F[m1:, m1:] - F12.T @ X
                del X
                if keep_factors:
                    node.f12 = np.ascontiguousarray(F12)
            if keep_factors:
                node.ldu, node.ipiv = ldu, ipiv
            del F
        self.keep = keep_factors

    def inertia(self):
        """(#negative, #zero, #positive) eigenvalues of A - tau I (Sylvester)."""
        return self.neg, self.zero, self.pos

    def solve(self, b, refine=2):
        """x = (A - tau I)^{-1} b: tree sweeps plus ``refine`` steps of iterative
        refinement with the same factors (residual recomputed from A itself)."""
        b = np.asarray(b, dtype=np.float64)
        x = self._sweep(b)
        for _ in range(refine):
            r = b - lattice.matvec(self.L, self.eps, x, shift=self.tau, bc=self.bc, hop=self.hop)
            x = x + self._sweep(r)
        return x

    def _sweep(self, b):
        if not self.keep:
            raise RuntimeError("factors were not kept")
        r = np.array(b, dtype=np.float64, copy=True)
        for node in self.nodes:  # postorder: eliminate towards the root
            y, _ = lapack.dsytrs(node.ldu, node.ipiv, r[node.own], lower=1)
            if node.f12 is not None:
                r[node.bnd] -= node.f12.T @ y
        x = np.empty_like(r)
        for node in reversed(self.nodes):  # root first: substitute back
            rhs = r[node.own]
            if node.f12 is not None:
                rhs = rhs - node.f12 @ x[node.bnd]
            x[node.own], _ = lapack.dsytrs(node.ldu, node.ipiv, rhs, lower=1)
        return x


def _sp_eye(n):
    import scipy.sparse as sp
    return sp.identity(n, format="csr")


def count_below(L, eps, tau, leaf=256, bc="periodic", hop=None):
    """Number of eigenvalues of A strictly below tau (inertia of A - tau I)."""
    f = LDLT(L, eps, tau, leaf=leaf, keep_factors=False, bc=bc, hop=hop)
    neg, zero, _ = f.inertia()
    return neg, zero
