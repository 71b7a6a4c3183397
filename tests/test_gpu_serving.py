"""Serving (continuous batching) on the GPU: results identical alone and in the mix,
admission by the HBM budget, checked against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_math_0508111_amd as jd  # noqa: E402
from oracle import eig, generator, lattice  # noqa: E402

REQS = [(12, 16.5, 1000000, 0.3, 4), (16, 12.0, 1000001, -0.5, 6), (10, 21.0, 1000002, 0.9, 3),
        (14, 16.5, 1000003, 0.0, 5), (20, 21.0, 1000004, -0.2, 2), (8, 12.0, 1000005, 0.1, 7)]


def test_results_identical_alone_and_in_the_mix():
    alone = [jd.solve(L, W, s, sg, k, 1e-10, precision="mixed")[0] for (L, W, s, sg, k) in REQS]
    srv = jd.Server(workers=4)
    tickets = [srv.submit(jd.Server.request(L, W, s, sg, k)) for (L, W, s, sg, k) in REQS * 2]
    results = [srv.wait(t) for t in tickets]
    srv.close()
    for i, r in enumerate(results):
        assert r["status"] == 0 and r["n_converged"] == r["k"], r["error"]
        assert np.array_equal(r["evals"], alone[i % len(REQS)])  # bit for bit
    # and against the oracle
    for (L, W, s, sg, k), r in zip(REQS, results):
        ref = eig.anderson_nearest(L, W, s, sg, k)[0]
        assert np.all(np.abs(r["evals"] - ref) <= 1e-9)
        assert np.all(r["resid"] <= 1e-10 * 1.0001)


def test_admission_by_hbm_budget():
    reqs = [jd.Server.request(L, W, s, sg, k) for (L, W, s, sg, k) in REQS]
    fp = max(jd.Server.footprint(r) for r in reqs)
    # a budget for one request at a time: everything is served, one after the other
    srv = jd.Server(hbm_budget_bytes=fp, workers=4)
    tickets = [srv.submit(r) for r in reqs]
    res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == 0 for r in res), [(r["status"], r["error"], r["n_converged"], r["k"]) for r in res]
    assert max(r["queued_s"] for r in res) > 0.0
    # a request larger than the whole budget is refused at submission
    big = jd.Server.request(60, 16.5, 1, 0.0, 10)
    with pytest.raises(jd.JdError):
        srv.submit(big)
    srv.close()


def test_poll_and_unknown_ticket():
    srv = jd.Server(workers=2)
    t = srv.submit(jd.Server.request(8, 16.5, 3, 0.0, 3))
    r = None
    while r is None:
        r = srv.poll(t)
    assert r["status"] == 0
    with pytest.raises(jd.JdError):
        srv.poll(t)  # released after it was returned
    srv.close()


@pytest.mark.parametrize("L,W,k", [(20, 12.0, 10), (40, 16.5, 1), (40, 12.0, 10)])
def test_footprint_estimate_covers_the_device_memory(L, W, k):
    # admission reserves the estimate: the memory a request really holds must not exceed it
    req = jd.Server.request(L, W, 1000000 + L, 0.1, k)
    _, _, _, info = jd.solve(L, W, 1000000 + L, 0.1, k, 1e-10, precision="mixed")
    assert info["status"] == 0
    assert 0 < info["device_bytes"] <= jd.Server.footprint(req)
