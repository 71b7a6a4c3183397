"""GPU parity of the hot path against the FP64 oracle, through the C ABI.

Every comparison uses seeded inputs; expected values come from ``oracle`` (live, or
stored in tests/golden by tests/golden/make_golden.py).
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_math_0508111_amd as jd  # noqa: E402
from oracle import eig, generator, lattice, ldlt  # noqa: E402
from tests import seeded_inputs  # noqa: E402

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U32 = np.finfo(np.float32).eps / 2


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def stream():
    return torch.cuda.current_stream()


# --- K1: disorder ---------------------------------------------------------------------

@pytest.mark.parametrize("L,W,seed", [(10, 16.5, 0), (7, 12.0, 3), (2, 16.5, 5), (33, 21.0, 11), (100, 16.5, 0)])
def test_gen_diag_bit_exact(L, W, seed):
    n = L ** 3
    e64 = torch.empty(n, dtype=torch.float64, device="cuda")
    e32 = torch.empty(n, dtype=torch.float32, device="cuda")
    jd.gen_diag(L, W, seed, e64, e32, stream=stream())
    torch.cuda.synchronize()
    ref = generator.disorder(L, W, seed)
    assert np.array_equal(e64.cpu().numpy(), ref)
    assert np.array_equal(e32.cpu().numpy(), ref.astype(np.float32))


# --- K2: stencil SpMV ---------------------------------------------------------------------

@pytest.mark.parametrize("L,shift", [(2, 0.0), (3, 0.7), (10, 0.0), (33, -0.25), (100, 0.0), (150, 0.1)])
def test_stencil_parity(L, shift):
    n = L ** 3
    eps = generator.disorder(L, 16.5, 1)
    x = seeded_inputs.vector(n, 7)
    ref = lattice.matvec(L, eps, x, shift=shift)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    jd.stencil_spmv(L, dev(eps), shift, dev(x), y, "fp64", stream=stream())
    torch.cuda.synchronize()
    scale = np.abs(eps - shift) * np.abs(x) + 6 * np.abs(x).max()
    assert np.all(np.abs(y.cpu().numpy() - ref) <= 8 * np.finfo(float).eps * scale)
    # binary32: error bound of 8 roundings of the inputs and the arithmetic
    y32 = torch.empty(n, dtype=torch.float32, device="cuda")
    jd.stencil_spmv(L, dev(eps, torch.float32), shift, dev(x, torch.float32), y32, "mixed", stream=stream())
    torch.cuda.synchronize()
    assert np.all(np.abs(y32.cpu().numpy().astype(np.float64) - ref) <= 16 * U32 * scale)


# --- multilevel preconditioner -------------------------------------------------------------

@pytest.mark.parametrize("L,cmax,sigma,flags", [(4, 8, 0.0, 0), (6, 16, 0.0, 0), (8, 40, 0.37, 0), (10, 60, -0.2, 0),
                                               (6, 16, 0.0, jd.JD_FLAG_LEVELS), (10, 60, -0.2, jd.JD_FLAG_LEVELS)])
def test_precond_exact_without_dropping(L, cmax, sigma, flags):
    # nothing dropped and every pivot accepted: the multilevel factorisation is exact,
    # so K^{-1} (A - sigma I) x = x, both through the explicit inverse factor and level by level
    W, seed = 16.5, 2
    P = jd.Precond(L, W, seed, sigma, drop_tol=-1.0, coarse_max=cmax, flags=flags)
    lv = P.levels()
    assert lv["levels"] >= 1
    eps = generator.disorder(L, W, seed)
    x = seeded_inputs.vector(L ** 3, 3)
    b = lattice.matvec(L, eps, x, shift=sigma)
    y = torch.empty(L ** 3, dtype=torch.float64, device="cuda")
    P.apply(dev(b), y, "fp64", stream=stream())
    torch.cuda.synchronize()
    assert np.linalg.norm(y.cpu().numpy() - x) <= 1e-9 * np.linalg.norm(x)
    P.close()


@pytest.mark.parametrize("L", [16, 24])
def test_inverse_factor_matches_level_by_level(L):
    # with nothing dropped from Z, P^T Z^T D^{-1} Z P is the level-by-level apply of the
    # same (incomplete) factorisation
    n = L ** 3
    Pz = jd.Precond(L, 16.5, 0, 0.0, z_drop=-1.0)
    Pl = jd.Precond(L, 16.5, 0, 0.0, flags=jd.JD_FLAG_LEVELS)
    assert Pz.levels() == Pl.levels()
    b = seeded_inputs.vector(n, 4)
    yz = torch.empty(n, dtype=torch.float64, device="cuda")
    yl = torch.empty(n, dtype=torch.float64, device="cuda")
    Pz.apply(dev(b), yz, stream=stream())
    Pl.apply(dev(b), yl, stream=stream())
    torch.cuda.synchronize()
    assert torch.linalg.norm(yz - yl).item() <= 1e-10 * torch.linalg.norm(yl).item()
    Pz.close()
    Pl.close()


@pytest.mark.parametrize("L", [16, 30])
def test_precond_symmetric_and_deterministic(L):
    P = jd.Precond(L, 16.5, 0, 0.0)
    n = L ** 3
    u, v = seeded_inputs.vector(n, 1), seeded_inputs.vector(n, 2)
    Ku = torch.empty(n, dtype=torch.float64, device="cuda")
    Kv = torch.empty(n, dtype=torch.float64, device="cuda")
    Ku2 = torch.empty(n, dtype=torch.float64, device="cuda")
    P.apply(dev(u), Ku, stream=stream())
    P.apply(dev(v), Kv, stream=stream())
    P.apply(dev(u), Ku2, stream=stream())
    torch.cuda.synchronize()
    a, b = v @ Ku.cpu().numpy(), u @ Kv.cpu().numpy()
    assert abs(a - b) <= 1e-11 * abs(a)
    assert torch.equal(Ku, Ku2)
    P.close()


# --- inner iteration: simplified QMR with the projected preconditioner ----------------------

def test_linear_solve_exact_preconditioner_one_step():
    L, sigma = 8, 0.21
    p = jd.Problem(L, 16.5, 4, sigma, drop_tol=-1.0, coarse_max=40)
    eps = generator.disorder(L, 16.5, 4)
    b = seeded_inputs.vector(L ** 3, 9)
    x = torch.zeros(L ** 3, dtype=torch.float64, device="cuda")
    its = p.linear_solve(sigma, dev(b), x, rtol=1e-12, maxit=10)
    torch.cuda.synchronize()
    ref = ldlt.LDLT(L, eps, sigma, leaf=64).solve(b)
    assert its <= 2
    assert np.linalg.norm(x.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    p.close()


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-10, 1e-9), ("mixed", 1e-5, 1e-4),
                                                ("mixed_factors", 1e-10, 1e-9)])
def test_linear_solve_projected(precision, rtol, tol):
    L, sigma = 16, 0.05
    n = L ** 3
    p = jd.Problem(L, 16.5, 1, sigma, precision=precision)
    eps = generator.disorder(L, 16.5, 1)
    Q = seeded_inputs.orthonormal_block(n, 3, 5)
    b = seeded_inputs.vector(n, 11)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    its = p.linear_solve(sigma, dev(b), x, Q=dev(Q), rtol=rtol, maxit=400)
    torch.cuda.synchronize()
    xs = x.cpu().numpy()
    proj = lambda v: v - Q @ (Q.T @ v)
    res = proj(lattice.matvec(L, eps, proj(xs), shift=sigma)) - proj(b)
    assert np.abs(Q.T @ xs).max() <= 1e-6 * np.linalg.norm(xs)
    assert np.linalg.norm(res) <= tol * np.linalg.norm(proj(b)) * 20
    assert 1 <= its < 400
    p.close()


# --- the solve: eigenpairs nearest sigma -----------------------------------------------------

def _check_pairs(L, W, seed, sigma, k, lams_ref, evals, evecs, resid, info, tol=1e-10, vec_ref=None):
    eps = generator.disorder(L, W, seed)
    anorm = lattice.inf_norm(eps)
    assert info["n_converged"] == k
    assert np.all(np.abs(evals - lams_ref) <= 1e-9), (evals, lams_ref)
    # residuals recomputed by the oracle's own product
    for c in range(k):
        x = evecs[:, c]
        r = np.linalg.norm(lattice.matvec(L, eps, x) - evals[c] * x)
        assert r <= tol * anorm * 1.0001, (c, r / anorm)
        assert abs(resid[c] - r / anorm) <= 1e-3 * max(r / anorm, 1e-16) + 1e-15
    G = evecs.T @ evecs
    assert np.abs(G - np.eye(k)).max() <= 1e-8
    if vec_ref is not None:
        for c in range(k):
            assert abs(abs(evecs[:, c] @ vec_ref[:, c]) - 1.0) <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_factors"])
def test_solve_small_live_oracle(precision):
    L, W, seed, sigma, k = 8, 16.5, 3, 0.0, 5
    ref, X, _, _ = eig.anderson_nearest(L, W, seed, sigma, k, method="dense")
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, vectors=True, precision=precision)
    _check_pairs(L, W, seed, sigma, k, ref, evals, evecs, resid, info, vec_ref=X)
    assert np.allclose(evecs, X, atol=1e-7)  # same sign convention


@pytest.mark.parametrize("L,W,seed,sigma,k", [(12, 12.0, 5, 0.3, 7), (15, 21.0, 8, -0.6, 4)])
def test_solve_ragged_live_oracle(L, W, seed, sigma, k):
    ref, X, _, _ = eig.anderson_nearest(L, W, seed, sigma, k)
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, vectors=True, precision="mixed")
    _check_pairs(L, W, seed, sigma, k, ref, evals, evecs, resid, info, vec_ref=X)


def _golden(name):
    with open(os.path.join(GOLD, name + ".json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name,precision", [("L10_W16.5_s0_k5", "fp64"), ("L10_W16.5_s0_k5", "mixed"),
                                            ("L20_W12_s1000000_k7", "mixed"), ("L30_W21_s1000001_k3", "mixed"),
                                            ("L40_W16.5_s1000002_k10", "mixed"), ("L50_W16.5_s0_k5", "fp64")])
def test_solve_against_stored_oracle(name, precision):
    g = _golden(name)
    evals, evecs, resid, info = jd.solve(g["L"], g["W"], g["seed"], g["sigma"], g["k"], 1e-10, vectors=True,
                                         precision=precision)
    _check_pairs(g["L"], g["W"], g["seed"], g["sigma"], g["k"], np.array(g["lams"]), evals, evecs, resid, info)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_eager(precision):
    # The inner iteration replayed as a captured HIP graph runs the same kernels in the
    # same order as the eager launches: identical iteration counts and eigenvalues.
    L, W, seed, sigma, k = 16, 16.5, 2, 0.0, 4
    ref, _, _, _ = eig.anderson_nearest(L, W, seed, sigma, k)
    e0, _, _, i0 = jd.solve(L, W, seed, sigma, k, 1e-10, precision=precision)
    e1, _, _, i1 = jd.solve(L, W, seed, sigma, k, 1e-10, precision=precision, flags=jd.JD_FLAG_GRAPHS)
    assert i0["status"] == 0 and i1["status"] == 0
    assert (i0["outer_its"], i0["inner_its"]) == (i1["outer_its"], i1["inner_its"])
    assert np.array_equal(e0, e1)
    assert np.max(np.abs(np.sort(e0) - np.sort(ref))) <= 1e-9


@pytest.mark.parametrize("L,W,seed,sigma,k", [(10, 21.0, 1000002, 0.9, 3), (8, 12.0, 1000005, 0.1, 7),
                                              (20, 21.0, 1000004, -0.2, 2)])
def test_solve_on_recycled_memory(L, W, seed, sigma, k):
    # Device memory handed out again after a free keeps its old contents.  Fill a large
    # block with NaN and release it to the runtime first: a solve must read nothing it
    # did not write (locking a vector once formed 0 * Q with Q not yet written).
    junk = torch.full((1 << 27,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    ref, _, _, _ = eig.anderson_nearest(L, W, seed, sigma, k)
    for precision in ("mixed", "fp64"):
        evals, _, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, precision=precision)
        assert info["status"] == 0 and info["n_converged"] == k
        assert np.max(np.abs(np.sort(evals) - np.sort(ref))) <= 1e-9


# --- edge cases -------------------------------------------------------------------------------

def test_solve_every_eigenpair_of_the_smallest_lattice():
    # L = 2: n = 8 and k = n (the whole spectrum; the last level is the whole matrix)
    L, W, seed, sigma = 2, 16.5, 11, 0.0
    ref, X, _, _ = eig.anderson_nearest(L, W, seed, sigma, 8, method="dense")
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, 8, 1e-10, vectors=True, precision="fp64")
    _check_pairs(L, W, seed, sigma, 8, ref, evals, evecs, resid, info, vec_ref=X)


@pytest.mark.parametrize("L,k,precision", [(3, 1, "fp64"), (5, 1, "mixed"), (6, 64, "fp64"), (7, 64, "mixed_factors")])
def test_solve_odd_lattices_and_the_largest_k(L, k, precision):
    W, seed, sigma = 12.0, 21, 0.25
    ref, X, _, _ = eig.anderson_nearest(L, W, seed, sigma, k, method="dense")
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, vectors=True, precision=precision)
    _check_pairs(L, W, seed, sigma, k, ref, evals, evecs, resid, info)


def test_partial_convergence_reports_what_converged():
    # an outer-iteration cap too small for k pairs: JD_ENOCONV, the converged pairs are
    # exact, the others NaN
    L, W, seed, sigma, k = 10, 16.5, 0, 0.0, 5
    ref, _, _, _ = eig.anderson_nearest(L, W, seed, sigma, k)
    evals, _, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, precision="fp64", max_outer=6)
    assert info["status"] == 1 and info["outer_its"] == 6 and info["n_converged"] < k
    got = evals[: info["n_converged"]]
    assert np.all(np.isnan(evals[info["n_converged"]:]))
    for v in got:  # each converged value is one of the wanted ones (or the next few)
        assert np.min(np.abs(eig.anderson_nearest(L, W, seed, sigma, k + 5)[0] - v)) <= 1e-9
    assert np.all(resid[: info["n_converged"]] <= 1e-10 * 1.0001)


def test_solve_options_setter():
    p = jd.Problem(12, 16.5, 3, 0.0, precision="fp64")
    ref = eig.anderson_nearest(12, 16.5, 3, 0.0, 4)[0]
    e0, _, _, i0 = p.solve(4, 1e-10)
    p.set_solve_options(jmin=12, jmax=40, max_inner=60, switch_tol=1e-6)
    e1, _, _, i1 = p.solve(4, 1e-10)
    assert i0["status"] == 0 and i1["status"] == 0
    assert np.max(np.abs(np.sort(e0) - np.sort(ref))) <= 1e-9 and np.max(np.abs(np.sort(e1) - np.sort(ref))) <= 1e-9
    with pytest.raises(jd.JdError):
        p.set_solve_options(jmax=121)
    for bad in (dict(jmin=120), dict(jmin=30, jmax=30)):
        with pytest.raises(jd.JdError):
            p.set_solve_options(**bad)
    # jmin alone, above the default jmax of this size (2 * max(k + 5, 10) = 20): the
    # restart then keeps 25 of at least 26 columns
    p.set_solve_options(jmin=25)
    e2, _, _, i2 = p.solve(4, 1e-10)
    assert i2["status"] == 0 and np.max(np.abs(np.sort(e2) - np.sort(ref))) <= 1e-9
    p.close()


def test_inner_tolerance_rate_option():
    # the j-th correction equation of a pair is solved to rate^j: rates other than the
    # default change the iteration path, and every path converges to the oracle's values
    ref = np.sort(eig.anderson_nearest(12, 16.5, 5, 0.0, 4)[0])
    p = jd.Problem(12, 16.5, 5, 0.0, precision="mixed")
    paths = []
    for rate in (0.0, 0.1, 0.8):  # 0: the default
        p.set_solve_options(inner_tol_rate=rate)
        e, _, _, info = p.solve(4, 1e-10)
        assert info["status"] == 0 and np.max(np.abs(np.sort(e) - ref)) <= 1e-9, rate
        paths.append((info["outer_its"], info["inner_its"]))
    p.close()
    assert len(set(paths)) > 1, paths
    # the same option through jd_solve's options
    e, _, _, info = jd.solve(12, 16.5, 5, 0.0, 4, 1e-10, precision="fp64", inner_tol_rate=0.1)
    assert info["status"] == 0 and np.max(np.abs(np.sort(e) - ref)) <= 1e-9


def test_search_space_set_at_setup_with_jmin_alone():
    # the same rule through jd_solve's options (L = 10, k = 5: default jmax 20)
    ref = eig.anderson_nearest(10, 16.5, 0, 0.0, 5)[0]
    evals, _, _, info = jd.solve(10, 16.5, 0, 0.0, 5, 1e-10, precision="mixed", jmin=25)
    assert info["status"] == 0 and np.max(np.abs(evals - ref)) <= 1e-9


def test_solve_after_a_stalled_setup():
    # W = 12 near the band centre: the multilevel setup stalls (kappa is raised) and the
    # solve takes the larger search space and longer inner solves.  Checked by the
    # properties that hold at any size: residuals recomputed by the oracle's own product,
    # orthonormal vectors, and the eigenvalues are the k nearest sigma among those the
    # oracle's exact inertia counts in a window around sigma.
    L, W, seed, sigma, k = 40, 12.0, 1000009, 0.9233143873275735, 4
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, vectors=True, precision="mixed")
    assert info["status"] == 0 and info["n_converged"] == k
    eps = generator.disorder(L, W, seed)
    anorm = lattice.inf_norm(eps)
    for c in range(k):
        x = evecs[:, c]
        r = np.linalg.norm(lattice.matvec(L, eps, x) - evals[c] * x)
        assert r <= 1e-10 * anorm * 1.0001
    assert np.abs(evecs.T @ evecs - np.eye(k)).max() <= 1e-8
    # no eigenvalue is missing between sigma and the farthest returned one: the exact
    # LDL^T inertia counts as many eigenvalues in that window as were returned
    lo, hi = np.min(evals) - 1e-9, np.max(evals) + 1e-9
    radius = max(sigma - lo, hi - sigma)
    assert eig.count_in_window(L, eps, sigma - radius, sigma + radius) == k


# --- hard-wall boundary conditions (section 8.2, Table 6) ---------------------------------

@pytest.mark.parametrize("L,shift", [(2, 0.0), (3, 0.7), (33, -0.25), (100, 0.0)])
def test_stencil_parity_hardwall(L, shift):
    n = L ** 3
    eps = generator.disorder(L, 16.5, 1)
    x = seeded_inputs.vector(n, 7)
    ref = lattice.matvec(L, eps, x, shift=shift, bc="hardwall")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    jd.stencil_spmv(L, dev(eps), shift, dev(x), y, "fp64", stream=stream(), bc="hardwall")
    torch.cuda.synchronize()
    scale = np.abs(eps - shift) * np.abs(x) + 6 * np.abs(x).max()
    assert np.all(np.abs(y.cpu().numpy() - ref) <= 8 * np.finfo(float).eps * scale)
    y32 = torch.empty(n, dtype=torch.float32, device="cuda")
    jd.stencil_spmv(L, dev(eps, torch.float32), shift, dev(x, torch.float32), y32, "mixed", stream=stream(),
                    bc="hardwall")
    torch.cuda.synchronize()
    assert np.all(np.abs(y32.cpu().numpy().astype(np.float64) - ref) <= 16 * U32 * scale)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_solve_hardwall_against_stored_oracle(precision):
    g = _golden("L30_W16.5_s0_k5_hardwall")
    assert g["bc"] == "hardwall" and g["certificate"]["inertia_count"] == g["k"]
    L, W, seed, sigma, k = g["L"], g["W"], g["seed"], g["sigma"], g["k"]
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, vectors=True, precision=precision,
                                         bc="hardwall")
    assert info["n_converged"] == k and np.max(np.abs(evals - np.array(g["lams"]))) <= 1e-9
    eps = generator.disorder(L, W, seed)
    for c in range(k):
        r = np.linalg.norm(lattice.matvec(L, eps, evecs[:, c], bc="hardwall") - evals[c] * evecs[:, c])
        assert r <= 1e-10 * g["anorm"] * 1.0001
    assert abs(info["anorm"] - g["anorm"]) <= 1e-15 * g["anorm"]


@pytest.mark.parametrize("L,W,seed,sigma,k,precision", [(8, 16.5, 3, 0.0, 5, "fp64"), (12, 12.0, 5, 0.3, 6, "mixed"),
                                                        (15, 21.0, 8, -0.6, 4, "mixed_factors"),
                                                        (7, 16.5, 1, 0.2, 64, "fp64")])
def test_solve_hardwall_live_oracle(L, W, seed, sigma, k, precision):
    eps = generator.disorder(L, W, seed)
    ref, X, _, anorm = eig.nearest_eigenpairs(L, eps, sigma, k, bc="hardwall")
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, vectors=True, precision=precision,
                                         bc="hardwall")
    assert info["n_converged"] == k and abs(info["anorm"] - anorm) <= 1e-15 * anorm
    assert np.all(np.abs(evals - ref) <= 1e-9), (evals, ref)
    for c in range(k):
        x = evecs[:, c]
        r = np.linalg.norm(lattice.matvec(L, eps, x, bc="hardwall") - evals[c] * x)
        assert r <= 1e-10 * anorm * 1.0001
    assert np.abs(evecs.T @ evecs - np.eye(k)).max() <= 1e-8
    if k <= 8:
        for c in range(k):
            assert abs(abs(evecs[:, c] @ X[:, c]) - 1.0) <= 1e-8


# --- shift-and-invert Lanczos on the same kernels (section 4.1; section 8.2, Tables 2-3) ----

@pytest.mark.parametrize("L,W,seed,sigma,k,precision,bc", [(10, 16.5, 0, 0.0, 5, "fp64", "periodic"),
                                                           (16, 12.0, 4, 0.35, 6, "mixed_factors", "periodic"),
                                                           (12, 21.0, 7, -0.4, 4, "fp64", "hardwall"),
                                                           (2, 16.5, 11, 0.0, 8, "fp64", "periodic")])
def test_si_lanczos_against_oracle(L, W, seed, sigma, k, precision, bc):
    eps = generator.disorder(L, W, seed)
    ref, X, _, anorm = eig.nearest_eigenpairs(L, eps, sigma, k, bc=bc)
    p = jd.Problem(L, W, seed, sigma, precision=precision, bc=bc)
    evals, evecs, resid, info = p.lanczos(k, 1e-10, vectors=True)
    p.close()
    assert info["status"] == 0 and info["n_converged"] == k
    assert np.all(np.abs(evals - ref) <= 1e-9), (evals, ref)
    for c in range(k):
        x = evecs[:, c]
        r = np.linalg.norm(lattice.matvec(L, eps, x, bc=bc) - evals[c] * x)
        assert r <= 1e-10 * anorm * 1.0001
    assert np.abs(evecs.T @ evecs - np.eye(k)).max() <= 1e-8
    # inner solves to 1e-10 take more steps per product than the correction equations of
    # Jacobi-Davidson (the comparison of section 8.2)
    assert info["outer_its"] >= 1 and info["inner_its"] >= info["outer_its"]


def test_si_lanczos_restarts_and_rejects_binary32():
    # a basis of 20 for k = 8 forces restarts
    L, W, seed, sigma, k = 14, 16.5, 2, 0.1, 8
    ref = eig.anderson_nearest(L, W, seed, sigma, k)[0]
    p = jd.Problem(L, W, seed, sigma, precision="fp64", jmax=20)
    evals, _, resid, info = p.lanczos(k)
    assert info["status"] == 0 and np.max(np.abs(evals - ref)) <= 1e-9
    assert info["outer_its"] > 20
    p.set_precision("mixed")
    with pytest.raises(jd.JdError) as e:
        p.lanczos(k)
    assert e.value.code == jd.JD_ENOTIMPL
    p.close()


# --- the off-diagonal model: random bond values (section 8.2, Table 6) ---------------------

@pytest.mark.parametrize("L,W,seed", [(2, 1.0, 5), (7, 1.0, 3), (40, 1.0, 0)])
def test_gen_hop_bit_exact(L, W, seed):
    n = L ** 3
    h64 = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    h32 = torch.empty(3 * n, dtype=torch.float32, device="cuda")
    jd.gen_hop(L, W, seed, h64, h32, stream=stream())
    torch.cuda.synchronize()
    ref = generator.hoppings(L, W, seed).reshape(-1)
    assert np.array_equal(h64.cpu().numpy(), ref)
    assert np.array_equal(h32.cpu().numpy(), ref.astype(np.float32))


@pytest.mark.parametrize("L,bc,shift", [(2, "periodic", 0.0), (3, "periodic", 0.4), (3, "hardwall", 0.0),
                                        (33, "periodic", -0.2), (64, "hardwall", 0.1)])
def test_stencil_parity_offdiag(L, bc, shift):
    n = L ** 3
    eps, hop = generator.offdiag_model(L, 1.0, 2)
    x = seeded_inputs.vector(n, 9)
    ref = lattice.matvec(L, eps, x, shift=shift, bc=bc, hop=hop)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    jd.stencil_spmv(L, dev(eps), shift, dev(x), y, "fp64", stream=stream(), bc=bc, hop=dev(hop.reshape(-1)))
    torch.cuda.synchronize()
    scale = np.abs(eps - shift) * np.abs(x) + 6 * 0.5 * np.abs(x).max()
    assert np.all(np.abs(y.cpu().numpy() - ref) <= 12 * np.finfo(float).eps * scale)
    y32 = torch.empty(n, dtype=torch.float32, device="cuda")
    jd.stencil_spmv(L, dev(eps, torch.float32), shift, dev(x, torch.float32), y32, "mixed", stream=stream(), bc=bc,
                    hop=dev(hop.reshape(-1), torch.float32))
    torch.cuda.synchronize()
    assert np.all(np.abs(y32.cpu().numpy().astype(np.float64) - ref) <= 24 * U32 * scale)


@pytest.mark.parametrize("L,seed,sigma,k,precision,bc", [(8, 3, 0.0, 5, "fp64", "periodic"),
                                                         (12, 5, 0.3, 6, "mixed", "periodic"),
                                                         (11, 8, -0.2, 4, "mixed_factors", "hardwall")])
def test_solve_offdiag_live_oracle(L, seed, sigma, k, precision, bc):
    eps, hop = generator.offdiag_model(L, 1.0, seed)
    ref, X, _, anorm = eig.nearest_eigenpairs(L, eps, sigma, k, bc=bc, hop=hop)
    evals, evecs, resid, info = jd.solve(L, 1.0, seed, sigma, k, 1e-10, vectors=True, precision=precision, bc=bc,
                                         model="offdiag")
    assert info["n_converged"] == k and abs(info["anorm"] - anorm) <= 1e-14 * anorm
    assert np.all(np.abs(evals - ref) <= 1e-9), (evals, ref)
    for c in range(k):
        x = evecs[:, c]
        r = np.linalg.norm(lattice.matvec(L, eps, x, bc=bc, hop=hop) - evals[c] * x)
        assert r <= 1e-10 * anorm * 1.0001
    assert np.abs(evecs.T @ evecs - np.eye(k)).max() <= 1e-8


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_solve_offdiag_against_stored_oracle(precision):
    g = _golden("L30_W1_s0_k5_offdiag")
    assert g["model"] == "offdiag" and g["certificate"]["inertia_count"] == g["k"]
    L, W, seed, sigma, k = g["L"], g["W"], g["seed"], g["sigma"], g["k"]
    evals, evecs, resid, info = jd.solve(L, W, seed, sigma, k, 1e-10, vectors=True, precision=precision,
                                         model="offdiag")
    assert info["n_converged"] == k and np.max(np.abs(evals - np.array(g["lams"]))) <= 1e-9
    eps, hop = generator.offdiag_model(L, W, seed)
    for c in range(k):
        r = np.linalg.norm(lattice.matvec(L, eps, evecs[:, c], hop=hop) - evals[c] * evecs[:, c])
        assert r <= 1e-10 * g["anorm"] * 1.0001


# --- the dense tall-skinny products of Rayleigh-Ritz on the matrix cores (section 4.2) --------

@pytest.mark.parametrize("n,m,mout", [(1, 1, 1), (17, 3, 2), (1000, 16, 16), (4099, 17, 65), (70001, 90, 30),
                                      (33333, 90, 89), (5000, 120, 120), (129, 5, 0)])
def test_block_product_against_library_matmul(n, m, mout):
    rng = np.random.default_rng(n + m + mout)
    V = rng.standard_normal((m, n))   # stored transposed: column-major n x m on the device
    S = rng.standard_normal((mout, m))
    dV = torch.as_tensor(V, device="cuda").t()
    dS = torch.as_tensor(S, device="cuda").t()
    dO = torch.full((mout, n), float("nan"), dtype=torch.float64, device="cuda").t()
    jd.block_product(dV, dS, dO, stream=stream())
    torch.cuda.synchronize()
    ref = V.T @ S.T
    bound = 2 * m * np.finfo(float).eps * (np.abs(V.T) @ np.abs(S.T))
    assert np.all(np.abs(dO.cpu().numpy() - ref) <= bound + 1e-300)
