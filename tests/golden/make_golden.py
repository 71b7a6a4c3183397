"""Writes the stored oracle results under tests/golden/ (calls only ``oracle``).

    python tests/golden/make_golden.py [name ...]

Each JSON file holds the k eigenvalues of the Anderson matrix nearest sigma
(section 3, eq. (eigenequation), periodic lattice, hopping -1, SplitMix64 box
disorder), as computed by the FP64 oracle: shift-and-invert Lanczos on an exact
multifrontal LDL^T (and, where n <= 1000, also dense Jacobi).  Large cases take
minutes and several GB of host memory.
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
}


def run(name, c):
    t0 = time.time()
    eps = generator.disorder(c["L"], c["W"], c["seed"])
    lams, X, res, anorm = eig.nearest_eigenpairs(c["L"], eps, c["sigma"], c["k"] + 1,
                                                 method="lanczos")
    out = dict(c)
    out.pop("dense", None)
    out.update(lams=[float(v) for v in lams[:c["k"]]], next=float(lams[c["k"]]),
               res=[float(v) for v in res[:c["k"]]], anorm=anorm, method="si-lanczos",
               seconds=round(time.time() - t0, 1),
               cite="section 3 eq. (eigenequation); problem: k eigenvalues nearest sigma")
    if c.get("dense"):
        A = lattice.hamiltonian(c["L"], eps).toarray()
        w = jacobi.eigh(A, vectors=False)[0]
        idx = eig.select_nearest(w, c["sigma"], c["k"] + 1)
        out["lams_dense_jacobi"] = [float(v) for v in w[idx][:c["k"]]]
        assert np.allclose(out["lams_dense_jacobi"], out["lams"], atol=1e-12, rtol=0)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, "done in", out["seconds"], "s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or [n for n in CASES if not n.startswith("L100")]
    for n in names:
        run(n, CASES[n])
