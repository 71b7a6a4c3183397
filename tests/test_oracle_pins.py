"""Pins of the FP64 CPU oracle against facts fixed by the paper or by mathematics.

Each test names what it pins.  None of them calls the HIP path.
"""
import numpy as np
import pytest

from oracle import eig, generator, jacobi, lanczos, lattice, ldlt


# --- O1: SplitMix64 / box distribution ---------------------------------------------

def test_splitmix64_published_outputs():
    # Reference outputs of SplitMix64 (Steele, Lea & Flood 2014; Vigna's reference
    # implementation) for the stream seeded with 0: the first three outputs.
    out = generator.splitmix64(0, 3)
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert generator.splitmix64_scalar(0, 2) == 0x6E789E6AA1B965F4


def test_splitmix64_counter_based():
    # output m of seed s equals output 1 of seed s + (m-1)*gamma (counter form)
    s = 987654321
    a = generator.splitmix64(s, 10)
    for m in range(1, 11):
        assert int(a[m - 1]) == generator.splitmix64_scalar((s + (m - 1) * generator.GAMMA) % 2**64, 1)


def test_box_distribution():
    # section 3: eps iid uniform in the box [-w/2, w/2]
    W = 16.5
    e = generator.disorder(40, W, 7)
    assert e.min() >= -W / 2 and e.max() < W / 2
    n = e.size
    assert abs(e.mean()) < 5 * W / np.sqrt(12 * n)
    assert abs(e.var() - W * W / 12) < 0.02 * W * W / 12
    # two seeds give different, reproducible draws
    assert np.array_equal(e, generator.disorder(40, W, 7))
    assert not np.array_equal(e, generator.disorder(40, W, 8))


# --- O2/O3: operator and dense Jacobi ---------------------------------------------

@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
def test_clean_spectrum_closed_form(L):
    # W = 0: the spectrum of the periodic lattice is -2 (cos kx + cos ky + cos kz),
    # k = 2 pi a / L.  Odd L makes the sign of the hopping visible (non-bipartite).
    A = lattice.hamiltonian(L, np.zeros(L ** 3)).toarray()
    w, V = jacobi.eigh(A)
    assert np.allclose(w, np.sort(lattice.clean_spectrum(L)), atol=1e-12, rtol=0)
    assert np.allclose(A @ V, V * w, atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(L ** 3), atol=1e-12)


def test_hamiltonian_structure():
    for L in (2, 3, 5):
        e = generator.disorder(L, 12.0, 3)
        A = lattice.hamiltonian(L, e)
        assert abs(A - A.T).max() == 0
        assert np.array_equal(A.diagonal(), e)
        rowsum = np.asarray(abs(A).sum(axis=1)).ravel()
        assert np.allclose(rowsum, 6 + np.abs(e))  # six couplings of modulus 1
        assert np.isclose(lattice.inf_norm(e), abs(A).sum(axis=1).max())
        nnz_row = np.diff(A.indptr)
        assert set(nnz_row) == ({4} if L == 2 else {7})
    A2 = lattice.hamiltonian(2, np.zeros(8)).toarray()
    assert set(np.unique(A2)) == {0.0, -2.0}  # L = 2: the two neighbours coincide


def test_matvec_matches_csr():
    L = 7
    e = generator.disorder(L, 16.5, 1)
    x = np.random.default_rng(0).standard_normal(L ** 3)
    A = lattice.hamiltonian(L, e)
    assert np.allclose(lattice.matvec(L, e, x, shift=0.3), A @ x - 0.3 * x, atol=1e-13, rtol=0)


def test_jacobi_against_library_eigh():
    rng = np.random.default_rng(5)
    B = rng.standard_normal((60, 60))
    A = B + B.T
    w, V = jacobi.eigh(A)
    assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12)
    assert np.allclose(A @ V, V * w, atol=1e-11)
    assert np.allclose(V.T @ V, np.eye(60), atol=1e-12)


@pytest.mark.parametrize("L", [4, 6])
def test_gauge_and_hopping_sign_even_L(L):
    # even L: U = diag((-1)^{i+j+k}) gives U T U = -T, so spec H(eps) = -spec H(-eps)
    # and the +1 (paper) and -1 hopping conventions share one spectrum.
    e = generator.disorder(L, 16.5, 2)
    w = jacobi.eigh(lattice.hamiltonian(L, e).toarray(), vectors=False)[0]
    wm = jacobi.eigh(lattice.hamiltonian(L, -e).toarray(), vectors=False)[0]
    wp = jacobi.eigh(lattice.hamiltonian(L, e, hopping=+1.0).toarray(), vectors=False)[0]
    assert np.allclose(w, -wm[::-1], atol=1e-12)
    assert np.allclose(w, wp, atol=1e-12)


def test_gershgorin_bound():
    # section 3: the eigenvalues lie in [-6 - w/2, 6 + w/2]
    L, W = 6, 21.0
    e = generator.disorder(L, W, 4)
    w = jacobi.eigh(lattice.hamiltonian(L, e).toarray(), vectors=False)[0]
    assert w.min() >= -6 - W / 2 and w.max() <= 6 + W / 2


def test_translation_and_reflection_invariance():
    L = 6
    e = generator.disorder(L, 16.5, 9).reshape(L, L, L)
    w0 = jacobi.eigh(lattice.hamiltonian(L, e.ravel()).toarray(), vectors=False)[0]
    for f in (np.roll(e, 2, axis=0).ravel(), e[:, ::-1, :].ravel(), e.transpose(1, 0, 2).ravel()):
        w1 = jacobi.eigh(lattice.hamiltonian(L, f.copy()).toarray(), vectors=False)[0]
        assert np.allclose(w0, w1, atol=1e-12)


# --- O4/O6: exact sparse LDL^T and inertia ------------------------------------------

@pytest.mark.parametrize("L,seed", [(3, 0), (4, 1), (6, 2), (7, 3)])
def test_inertia_matches_dense_count(L, seed):
    e = generator.disorder(L, 16.5, seed)
    A = lattice.hamiltonian(L, e).toarray()
    w = jacobi.eigh(A, vectors=False)[0]
    for tau in (0.0, 0.41, -2.3, 5.0):
        f = ldlt.LDLT(L, e, tau, leaf=20)
        neg, zero, pos = f.inertia()
        assert neg == int((w < tau).sum()) and zero == 0 and neg + pos == L ** 3
        b = np.random.default_rng(1).standard_normal(L ** 3)
        x = f.solve(b)
        assert np.linalg.norm(A @ x - tau * x - b) <= 1e-12 * np.linalg.norm(b) * lattice.inf_norm(e)


@pytest.mark.parametrize("L", [8, 12, 16])
def test_inertia_closed_form_clean_lattice(L):
    # W = 0: count of eigenvalues below tau from the closed form, at sizes beyond
    # the dense path; tau placed away from every lattice eigenvalue.
    spec = lattice.clean_spectrum(L)
    for tau in (0.1234, -1.777, 3.05):
        assert np.min(np.abs(spec - tau)) > 1e-3
        neg, zero = ldlt.count_below(L, np.zeros(L ** 3), tau)
        assert zero == 0 and neg == int((spec < tau).sum())


def test_nested_dissection_partitions_sites():
    for L in (5, 8, 11):
        nodes = ldlt.nested_dissection(L, leaf=30)
        allv = np.concatenate([n.own for n in nodes])
        assert np.array_equal(np.sort(allv), np.arange(L ** 3))


# --- O5/O7: shift-and-invert Lanczos and the result definition ----------------------

def test_lanczos_matches_dense_jacobi():
    L = 8
    e = generator.disorder(L, 16.5, 0)
    l1, X1, r1, an = eig.nearest_eigenpairs(L, e, 0.0, 6, method="dense")
    l2, X2, r2, _ = eig.nearest_eigenpairs(L, e, 0.0, 6, method="lanczos")
    assert np.allclose(l1, l2, atol=1e-12, rtol=0)
    assert np.allclose(X1, X2, atol=1e-8)  # same sign convention
    assert r1.max() <= 1e-12 * an and r2.max() <= 1e-12 * an


def _chain(f):
    # 1D periodic chain with hopping -1 and diagonal f
    m = len(f)
    H = np.diag(f)
    for i in range(m):
        H[i, (i + 1) % m] -= 1.0
        H[(i + 1) % m, i] -= 1.0
    return H


@pytest.mark.parametrize("L,sigma", [(16, 0.3), (20, -0.7)])
def test_separable_diagonal_kronecker_sum(L, sigma):
    # eps_{ijk} = f_i + g_j + h_k makes A a Kronecker sum of three periodic chains:
    # its eigenvalues are all sums a + b + c of the chains' eigenvalues.
    rng = np.random.default_rng(L)
    f, g, h = (rng.uniform(-2.5, 2.5, L) for _ in range(3))
    eps = (f[None, None, :] + g[None, :, None] + h[:, None, None]).reshape(-1)
    ea, eb, ec = (jacobi.eigh(_chain(v), vectors=False)[0] for v in (f, g, h))
    sums = (ea[None, None, :] + eb[None, :, None] + ec[:, None, None]).reshape(-1)
    k = 8
    ref = sums[eig.select_nearest(sums, sigma, k)]
    lams, X, res, an = eig.nearest_eigenpairs(L, eps, sigma, k)
    assert np.allclose(lams, ref, atol=1e-11, rtol=0)
    assert res.max() <= 1e-12 * an


def test_window_count_by_inertia():
    L = 6
    e = generator.disorder(L, 16.5, 5)
    w = jacobi.eigh(lattice.hamiltonian(L, e).toarray(), vectors=False)[0]
    assert eig.count_in_window(L, e, -0.5, 0.7) == int(((w >= -0.5) & (w < 0.7)).sum())


def test_selection_order_rule():
    lams = np.array([0.3, -0.1, 0.1, -0.3, 0.05])
    idx = eig.select_nearest(lams, 0.0, 5)
    assert list(lams[idx]) == [0.05, -0.1, 0.1, -0.3, 0.3]


# --- planted mistakes: each plausible slip in the operator fails a pin above --------

@pytest.mark.parametrize("mistake", ["sign", "dropped_z", "wrong_index"])
def test_planted_mistakes_are_caught(monkeypatch, mistake):
    L = 5  # odd: the hopping sign changes the clean spectrum
    if mistake == "sign":
        A = lattice.hamiltonian(L, np.zeros(L ** 3), hopping=+1.0).toarray()
    elif mistake == "dropped_z":
        monkeypatch.setattr(lattice, "NEIGHBOURS", lattice.NEIGHBOURS[:4])
        A = lattice.hamiltonian(L, np.zeros(L ** 3)).toarray()
    else:
        # x and y swapped in the neighbour arithmetic only: the diagonal stays in
        # site order, so the operator no longer matches the stencil definition
        e = generator.disorder(L, 4.0, 1)
        orig = lattice.site_coords
        monkeypatch.setattr(lattice, "site_coords",
                            lambda L_: (lambda c: (c[1], c[0], c[2]))(orig(L_)))
        Aw = lattice.hamiltonian(L, e)
        monkeypatch.undo()
        x = np.random.default_rng(0).standard_normal(L ** 3)
        y = lattice.matvec(L, e, x)  # the stencil written out neighbour by neighbour
        assert not np.allclose(Aw @ x, y)
        assert np.allclose(lattice.hamiltonian(L, e) @ x, y)
        return
    w = jacobi.eigh(A, vectors=False)[0]
    assert not np.allclose(w, np.sort(lattice.clean_spectrum(L)), atol=1e-9)


@pytest.mark.parametrize("L,sigma", [(3, -6.0), (4, 6.0)])
def test_singular_shift_retry_clean_lattice(L, sigma):
    """The factorisation shift moves off sigma when A - sigma I is singular.

    At W = 0 the extreme eigenvalues of the periodic lattice are simple: -6 (the
    constant vector) and, for even L, +6 (the staggered vector (-1)^(i+j+k)); the
    closed form -2 sum cos(2 pi a / L) puts the nearest other eigenvalue 2 (L = 4) or
    3 (L = 3) away.  With sigma exactly on one of them the exact LDL^T of A - sigma I
    meets a zero (or rounding-sized) pivot, factor_near retries at
    sigma + 1e-9 (1 + |sigma|), solves with the retried factors are accurate, and
    shift-and-invert Lanczos with that shift returns the eigenvalue sigma itself with
    the closed-form eigenvector."""
    eps = np.zeros(L ** 3)
    anorm = lattice.inf_norm(eps)
    spec = np.sort(lattice.clean_spectrum(L))
    assert spec[0 if sigma < 0 else -1] == sigma
    f = eig.factor_near(L, eps, sigma)
    assert f.tau == sigma + 1e-9 * (1.0 + abs(sigma))
    assert f.min_pivot > 1e-13 * anorm
    b = np.random.default_rng(5).standard_normal(L ** 3)
    x = f.solve(b)
    # backward error of the solve with the retried shift, at rounding level
    r = lattice.matvec(L, eps, x, shift=f.tau) - b
    assert np.linalg.norm(r) <= 1e-12 * (anorm * np.linalg.norm(x) + np.linalg.norm(b))
    # With the shift 1e-9 from the eigenvalue, (A - sigma_f I)^{-1} has condition ~1e9
    # and the Lanczos vectors after the dominant one carry rounding of that size: the
    # Ritz vector's residual stalls near 1e-9 ||A||, while its Rayleigh quotient is
    # exact to rounding (the error is quadratic in the vector's)
    lams, X, res = lanczos.si_lanczos(L, eps, sigma, 1, eig._Solver(f), tol=1e-8, extra=0)
    assert abs(lams[0] - sigma) <= 1e-12
    i, j, k = lattice.site_coords(L)
    v = np.ones(L ** 3) if sigma < 0 else (-1.0) ** (i + j + k)
    v /= np.linalg.norm(v)
    c = abs(X[:, 0] @ v)
    assert np.sqrt(max(0.0, 1.0 - c * c)) <= 1e-8  # sine of the angle to the closed form
    assert res[0] <= 1e-8 * anorm


# --- hard-wall boundary conditions (section 8.2, Table 6) ---------------------------

@pytest.mark.parametrize("L", [1, 2, 3, 4, 5])
def test_hardwall_clean_spectrum_closed_form(L):
    # W = 0 with hard walls: the open chain's sine modes give -2 sum cos(pi a / (L+1)),
    # a = 1..L; L = 1 is a single uncoupled site
    A = lattice.hamiltonian(L, np.zeros(L ** 3), bc="hardwall").toarray()
    w, V = jacobi.eigh(A)
    assert np.allclose(w, np.sort(lattice.clean_spectrum(L, bc="hardwall")), atol=1e-12, rtol=0)
    assert np.allclose(A @ V, V * w, atol=1e-12)


def test_hardwall_structure_and_norm():
    for L in (2, 3, 5):
        e = generator.disorder(L, 12.0, 3)
        A = lattice.hamiltonian(L, e, bc="hardwall")
        assert abs(A - A.T).max() == 0
        assert np.array_equal(A.diagonal(), e)
        # 3 L^2 (L - 1) bonds, each stored twice
        assert A.nnz - L ** 3 == 6 * L * L * (L - 1)
        rowsum = np.asarray(abs(A).sum(axis=1)).ravel()
        assert np.allclose(rowsum, lattice.degree(L, "hardwall") + np.abs(e))
        assert np.isclose(lattice.inf_norm(e, L, "hardwall"), rowsum.max())
        x = np.random.default_rng(L).standard_normal(L ** 3)
        assert np.allclose(lattice.matvec(L, e, x, shift=0.3, bc="hardwall"), A @ x - 0.3 * x, atol=1e-13, rtol=0)


@pytest.mark.parametrize("L", [3, 5])
def test_hardwall_gauge_any_L(L):
    # the box without wrap is bipartite for every L: spec H(eps) = -spec H(-eps), and the
    # +1 and -1 hopping conventions share one spectrum (odd L too, unlike the torus)
    e = generator.disorder(L, 16.5, 2)
    w = jacobi.eigh(lattice.hamiltonian(L, e, bc="hardwall").toarray(), vectors=False)[0]
    wm = jacobi.eigh(lattice.hamiltonian(L, -e, bc="hardwall").toarray(), vectors=False)[0]
    wp = jacobi.eigh(lattice.hamiltonian(L, e, hopping=+1.0, bc="hardwall").toarray(), vectors=False)[0]
    assert np.allclose(w, -wm[::-1], atol=1e-12)
    assert np.allclose(w, wp, atol=1e-12)


@pytest.mark.parametrize("L,seed", [(3, 0), (5, 1), (7, 3)])
def test_hardwall_inertia_matches_dense_count(L, seed):
    e = generator.disorder(L, 16.5, seed)
    A = lattice.hamiltonian(L, e, bc="hardwall").toarray()
    w = jacobi.eigh(A, vectors=False)[0]
    for tau in (0.0, 0.41, -2.3):
        f = ldlt.LDLT(L, e, tau, leaf=20, bc="hardwall")
        neg, zero, pos = f.inertia()
        assert neg == int((w < tau).sum()) and zero == 0 and neg + pos == L ** 3
        b = np.random.default_rng(1).standard_normal(L ** 3)
        x = f.solve(b)
        assert np.linalg.norm(A @ x - tau * x - b) <= 1e-12 * np.linalg.norm(b) * lattice.inf_norm(e, L, "hardwall")


def test_hardwall_lanczos_matches_dense_and_differs_from_periodic():
    L = 8
    e = generator.disorder(L, 16.5, 0)
    l1, X1, r1, an = eig.nearest_eigenpairs(L, e, 0.0, 6, method="dense", bc="hardwall")
    l2, X2, r2, _ = eig.nearest_eigenpairs(L, e, 0.0, 6, method="lanczos", bc="hardwall")
    assert np.allclose(l1, l2, atol=1e-12, rtol=0)
    assert np.allclose(X1, X2, atol=1e-8)
    assert r1.max() <= 1e-12 * an and r2.max() <= 1e-12 * an
    lp = eig.nearest_eigenpairs(L, e, 0.0, 6, method="dense")[0]
    assert np.max(np.abs(lp - l1)) > 1e-3  # the boundary condition matters


def _open_chain(f):
    m = len(f)
    H = np.diag(f)
    for i in range(m - 1):
        H[i, i + 1] = H[i + 1, i] = -1.0
    return H


def test_hardwall_separable_kronecker_sum():
    # eps_{ijk} = f_i + g_j + h_k: a Kronecker sum of three open chains
    L, sigma, k = 16, 0.2, 8
    rng = np.random.default_rng(7)
    f, g, h = (rng.uniform(-2.5, 2.5, L) for _ in range(3))
    eps = (f[None, None, :] + g[None, :, None] + h[:, None, None]).reshape(-1)
    ea, eb, ec = (jacobi.eigh(_open_chain(v), vectors=False)[0] for v in (f, g, h))
    sums = (ea[None, None, :] + eb[None, :, None] + ec[:, None, None]).reshape(-1)
    ref = sums[eig.select_nearest(sums, sigma, k)]
    lams, X, res, an = eig.nearest_eigenpairs(L, eps, sigma, k, bc="hardwall")
    assert np.allclose(lams, ref, atol=1e-11, rtol=0)
    assert res.max() <= 1e-12 * an


def test_hardwall_inertia_closed_form():
    L = 12
    spec = lattice.clean_spectrum(L, bc="hardwall")
    for tau in (0.1234, -1.777):
        assert np.min(np.abs(spec - tau)) > 1e-3
        neg, zero = ldlt.count_below(L, np.zeros(L ** 3), tau, bc="hardwall")
        assert zero == 0 and neg == int((spec < tau).sum())


def test_stored_results_carry_inertia_certificates():
    """Every stored oracle result (tests/golden, written by make_golden.py from the oracle
    only) holds the Sylvester count of its window: exactly k eigenvalues lie within the
    half-way point between the k-th and the (k+1)-th distance to sigma (section 5.1)."""
    import glob
    import json
    import os
    files = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.json")))
    assert len(files) >= 7
    for path in files:
        with open(path) as fh:
            g = json.load(fh)
        c = g["certificate"]
        assert c["inertia_count"] == g["k"], path
        lo, hi = c["window"]
        lams = np.array(g["lams"])
        assert np.all((lams > lo) & (lams < hi)), path
        assert not (lo < g["next"] < hi), path
        assert len(c["kato_temple"]) == g["k"] and max(c["kato_temple"]) < 1e-12, path


# --- the off-diagonal ("inverse") model: random bond values (section 8.2, Table 6) --------

def test_hoppings_generator():
    L, W, seed = 5, 1.0, 3
    n = L ** 3
    t = generator.hoppings(L, W, seed)
    assert t.shape == (3, n)
    # bond (s, d) takes output n + 3 s + d + 1 of the stream: after the diagonal's outputs
    for s_, d in ((0, 0), (7, 2), (n - 1, 1)):
        u = (generator.splitmix64_scalar(seed, n + 3 * s_ + d + 1) >> 11) * 2.0 ** -53
        assert t[d, s_] == W * (u - 0.5)
    big = generator.hoppings(40, 1.0, 1)
    assert big.min() >= -0.5 and big.max() < 0.5 and abs(big.mean()) < 5e-3


@pytest.mark.parametrize("L,bc", [(2, "periodic"), (3, "periodic"), (5, "periodic"), (4, "hardwall")])
def test_bond_values_reduce_to_the_constant_coupling(L, bc):
    # hop = -1 on every bond is the diagonal model, entry by entry and product by product
    e = generator.disorder(L, 16.5, 6)
    hop = -np.ones((3, L ** 3))
    A0 = lattice.hamiltonian(L, e, bc=bc)
    A1 = lattice.hamiltonian(L, e, bc=bc, hop=hop)
    assert abs(A0 - A1).max() == 0
    x = np.random.default_rng(2).standard_normal(L ** 3)
    assert np.allclose(lattice.matvec(L, e, x, 0.2, bc=bc, hop=hop), lattice.matvec(L, e, x, 0.2, bc=bc),
                       atol=1e-13, rtol=0)
    assert lattice.inf_norm(e, L, bc, hop) == lattice.inf_norm(e, L, bc)


@pytest.mark.parametrize("L,bc", [(4, "periodic"), (5, "periodic"), (5, "hardwall")])
def test_bond_values_structure(L, bc):
    eps, hop = generator.offdiag_model(L, 1.0, 4)
    A = lattice.hamiltonian(L, eps, bc=bc, hop=hop)
    assert abs(A - A.T).max() == 0 and np.all(A.diagonal() == 1.28)
    x = np.random.default_rng(L).standard_normal(L ** 3)
    assert np.allclose(lattice.matvec(L, eps, x, -0.3, bc=bc, hop=hop), A @ x + 0.3 * x, atol=1e-13, rtol=0)
    # entry of the bond from site s to s + e_x is hop[0, s]
    s_ = 1 + L * (2 + L * 1)
    assert A[s_, s_ + 1] == hop[0, s_]
    assert np.isclose(lattice.inf_norm(eps, L, bc, hop), np.asarray(abs(A).sum(axis=1)).max())


def _open_chain_bonds(f, t):
    H = np.diag(f)
    for i in range(len(f) - 1):
        H[i, i + 1] = H[i + 1, i] = t[i]
    return H


def test_bond_values_kronecker_sum():
    # hard walls, eps_ijk = f_i + g_j + h_k and x-bonds depending on i only (y on j, z on k):
    # A is the Kronecker sum of three open chains with random bonds
    L, sigma, k = 14, 0.15, 6
    rng = np.random.default_rng(11)
    f, g, h = (rng.uniform(-1.5, 1.5, L) for _ in range(3))
    tx, ty, tz = (rng.uniform(-0.5, 0.5, L) for _ in range(3))
    eps = (f[None, None, :] + g[None, :, None] + h[:, None, None]).reshape(-1)
    ones = np.ones((L, L, L))
    hop = np.stack([(ones * tx[None, None, :]).reshape(-1), (ones * ty[None, :, None]).reshape(-1),
                    (ones * tz[:, None, None]).reshape(-1)])
    ea, eb, ec = (jacobi.eigh(_open_chain_bonds(v, t), vectors=False)[0] for v, t in ((f, tx), (g, ty), (h, tz)))
    sums = (ea[None, None, :] + eb[None, :, None] + ec[:, None, None]).reshape(-1)
    ref = sums[eig.select_nearest(sums, sigma, k)]
    lams, X, res, an = eig.nearest_eigenpairs(L, eps, sigma, k, bc="hardwall", hop=hop)
    assert np.allclose(lams, ref, atol=1e-11, rtol=0)
    assert res.max() <= 1e-12 * an


@pytest.mark.parametrize("L", [4, 6])
def test_offdiag_gauge_symmetry(L):
    # bipartite lattice (even L): flipping every bond sign leaves the spectrum, and a
    # constant diagonal c makes it symmetric about c
    eps, hop = generator.offdiag_model(L, 1.0, 5)
    w = jacobi.eigh(lattice.hamiltonian(L, eps, hop=hop).toarray(), vectors=False)[0]
    wf = jacobi.eigh(lattice.hamiltonian(L, eps, hop=-hop).toarray(), vectors=False)[0]
    assert np.allclose(w, wf, atol=1e-12)
    assert np.allclose(w - 1.28, -(w[::-1] - 1.28), atol=1e-12)


@pytest.mark.parametrize("L,seed", [(4, 0), (6, 2), (7, 3)])
def test_offdiag_inertia_and_lanczos(L, seed):
    eps, hop = generator.offdiag_model(L, 1.0, seed)
    A = lattice.hamiltonian(L, eps, hop=hop).toarray()
    w = jacobi.eigh(A, vectors=False)[0]
    for tau in (0.0, 1.1, 2.3):
        neg, zero, pos = ldlt.LDLT(L, eps, tau, leaf=20, hop=hop).inertia()
        assert neg == int((w < tau).sum()) and zero == 0
    l1, X1, r1, an = eig.nearest_eigenpairs(L, eps, 0.0, 4, method="dense", hop=hop)
    l2, X2, r2, _ = eig.nearest_eigenpairs(L, eps, 0.0, 4, method="lanczos", hop=hop)
    assert np.allclose(l1, l2, atol=1e-12, rtol=0) and np.allclose(X1, X2, atol=1e-8)
    assert r2.max() <= 1e-12 * an
