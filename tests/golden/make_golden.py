"""Writes the stored oracle results under tests/golden/ (calls only ``oracle``).

    python tests/golden/make_golden.py [name ...]

Each JSON file holds the k eigenvalues of the Anderson matrix nearest sigma
(section 3, eq. (eigenequation), periodic lattice, hopping -1, SplitMix64 box
disorder), as computed by the FP64 oracle: shift-and-invert Lanczos on an exact
multifrontal LDL^T (and, where n <= 1000, also dense Jacobi), with an inertia
certificate: the exact LDL^T counts k eigenvalues in the window that the stored
values and the next one delimit (``--certify NAME ...`` adds it to stored results).
Large cases take minutes and several GB of host memory.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eig, generator, jacobi, lattice  # noqa: E402

CASES = {
    # lattice 10^3, W 16.5, seed 0, 5 nearest 0 (the small plain-FP64 configuration)
    "L10_W16.5_s0_k5": dict(L=10, W=16.5, seed=0, sigma=0.0, k=5, dense=True),
    # lattice 50^3, W 16.5, seed 0, 5 nearest 0 (plain FP64 on the GPU)
    "L50_W16.5_s0_k5": dict(L=50, W=16.5, seed=0, sigma=0.0, k=5),
    # lattice 100^3, W 16.5, seed 0, 10 nearest 0 (mixed precision)
    "L100_W16.5_s0_k10": dict(L=100, W=16.5, seed=0, sigma=0.0, k=10),
    # serving-mix style requests (L in 20..60, W in {12, 16.5, 21}, sigma in [-1, 1])
    "L20_W12_s1000000_k7": dict(L=20, W=12.0, seed=1000000, sigma=0.35, k=7),
    "L30_W21_s1000001_k3": dict(L=30, W=21.0, seed=1000001, sigma=-0.62, k=3),
    "L40_W16.5_s1000002_k10": dict(L=40, W=16.5, seed=1000002, sigma=0.11, k=10),
    # a hard serving request: W = 12 near the band centre, the largest lattice of the mix
    "L60_W12_s1000041_k7": dict(L=60, W=12.0, seed=1000041, sigma=0.6205487042125981, k=7),
    # hard-wall boundary conditions (section 8.2, Table 6)
    "L30_W16.5_s0_k5_hardwall": dict(L=30, W=16.5, seed=0, sigma=0.0, k=5, bc="hardwall"),
    # the off-diagonal model (section 8.2, Table 6): diagonal 1.28, bonds on [-1/2, 1/2]
    "L30_W1_s0_k5_offdiag": dict(L=30, W=1.0, seed=0, sigma=0.0, k=5, model="offdiag"),
}


def _model(c):
    """(eps, hop) of a case: the diagonal model, or the off-diagonal one."""
    if c.get("model", "anderson") == "offdiag":
        return generator.offdiag_model(c["L"], c["W"], c["seed"])
    return generator.disorder(c["L"], c["W"], c["seed"]), None


def _machine():
    import os
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        threads = os.cpu_count()
    return f"{threads} threads, {model}"


def certify(out, eps, hop=None):
    """Inertia certificate of a stored result (Sylvester's law on the exact LDL^T).

    rho is halfway between the k-th and the (k+1)-th distance to sigma; the window
    [sigma - rho, sigma + rho) must hold exactly k eigenvalues.  Each returned value
    theta_i with residual r_i (unit vector) has an eigenvalue within r_i; with the
    window count and disjoint intervals that eigenvalue is the i-th nearest, and
    Kato-Temple bounds its distance to theta_i by r_i^2 / delta_i, delta_i a lower
    bound of the distance from theta_i to every other eigenvalue."""
    sigma, k = out["sigma"], out["k"]
    lams, res = np.array(out["lams"]), np.array(out["res"])
    d_k, d_next = abs(lams[-1] - sigma), abs(out["next"] - sigma)
    rho = 0.5 * (d_k + d_next)
    t0 = time.time()
    count = eig.count_in_window(out["L"], eps, sigma - rho, sigma + rho, bc=out.get("bc", "periodic"), hop=hop)
    assert count == k, (count, k)
    iv = [(lams[i] - res[i], lams[i] + res[i]) for i in range(k)]
    kt = []
    for i in range(k):
        others = [abs(lams[i] - lams[j]) - res[j] for j in range(k) if j != i]
        # eigenvalues outside the window are at least rho - |theta_i - sigma| away
        delta = min(others + [rho - abs(lams[i] - sigma)])
        assert res[i] < delta
        kt.append(float(res[i] ** 2 / delta))
    for i in range(k):
        for j in range(i + 1, k):
            assert iv[i][1] < iv[j][0] or iv[j][1] < iv[i][0], (i, j)
    out["certificate"] = dict(rho=rho, window=[sigma - rho, sigma + rho], inertia_count=count,
                              kato_temple=kt, seconds=round(time.time() - t0, 1),
                              cite="section 5.1 (inertia of the LDL^T factors); section 4.1 "
                                   "(shift-and-invert with exact factorisations)")
    return out


def run(name, c):
    t0 = time.time()
    eps, hop = _model(c)
    tm = {}
    bc = c.get("bc", "periodic")
    lams, X, res, anorm = eig.nearest_eigenpairs(c["L"], eps, c["sigma"], c["k"] + 1,
                                                 method="lanczos", timings=tm, bc=bc, hop=hop)
    out = dict(c)
    out.pop("dense", None)
    out.update(lams=[float(v) for v in lams[:c["k"]]], next=float(lams[c["k"]]),
               res=[float(v) for v in res[:c["k"]]], anorm=anorm, method="si-lanczos",
               seconds=round(time.time() - t0, 1), factor_seconds=round(tm["factorisation_s"], 1),
               lanczos_seconds=round(tm["lanczos_s"], 1), machine=_machine(),
               cite="section 3 eq. (eigenequation); problem: k eigenvalues nearest sigma")
    if c.get("dense"):
        A = lattice.hamiltonian(c["L"], eps, bc=bc, hop=hop).toarray()
        w = jacobi.eigh(A, vectors=False)[0]
        idx = eig.select_nearest(w, c["sigma"], c["k"] + 1)
        out["lams_dense_jacobi"] = [float(v) for v in w[idx][:c["k"]]]
        assert np.allclose(out["lams_dense_jacobi"], out["lams"], atol=1e-12, rtol=0)
    certify(out, eps, hop)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, "done in", out["seconds"], "s", flush=True)


def certify_stored(name):
    """Add the inertia certificate to a stored result without recomputing its pairs."""
    path = os.path.join(HERE, name + ".json")
    with open(path) as fh:
        out = json.load(fh)
    eps, hop = _model(out)
    certify(out, eps, hop)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, "certified in", out["certificate"]["seconds"], "s", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--certify":
        for n in args[1:] or list(CASES):
            certify_stored(n)
        sys.exit(0)
    names = args or [n for n in CASES if not n.startswith("L100")]
    for n in names:
        run(n, CASES[n])
