"""Device memory from the caller (jd_set_allocator) through the C ABI.

PyTorch's caching allocator serves every device buffer of a setup, a solve and the
serving workers; each buffer goes back to it, and the results are bit-identical to
those with the library's own hipMalloc.
"""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_math_0508111_amd as jd  # noqa: E402
from oracle import eig  # noqa: E402


class CountingTorchAllocator:
    def __init__(self):
        self.lock = threading.Lock()
        self.allocs = self.frees = 0
        self.live = {}
        self.threads = set()

    def alloc(self, nbytes, stream):
        p = torch.cuda.caching_allocator_alloc(nbytes, stream=stream)
        with self.lock:
            self.allocs += 1
            self.live[p] = nbytes
            self.threads.add(threading.get_ident())
        return p

    def free(self, ptr, _stream):
        with self.lock:
            self.frees += 1
            assert self.live.pop(ptr, None) is not None, "freed a buffer the hook did not allocate"
        torch.cuda.caching_allocator_delete(ptr)


@pytest.fixture
def hook():
    h = CountingTorchAllocator()
    jd.set_allocator(h.alloc, h.free)
    try:
        yield h
    finally:
        jd.set_allocator(None, None)


def test_problem_and_solve_memory_from_the_hook(hook):
    L, W, seed, sigma, k = 12, 16.5, 3, 0.0, 4
    ref = eig.anderson_nearest(L, W, seed, sigma, k)[0]
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    p = jd.Problem(L, W, seed, sigma, precision="mixed")
    n_setup, f_setup = hook.allocs, hook.frees  # the setup's temporaries are freed already
    assert n_setup > f_setup >= 0
    held = torch.cuda.memory_allocated() - before
    assert held >= p.info()["device_bytes"] > 0
    evals, _, _, info = p.solve(k, 1e-10)
    assert info["status"] == 0 and np.max(np.abs(evals - ref)) <= 1e-9
    assert hook.allocs > n_setup  # the solve's search space and work vectors too
    assert hook.frees - f_setup == hook.allocs - n_setup  # the solve returned its buffers
    p.close()
    assert not hook.live and hook.frees == hook.allocs
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    # the same arithmetic as with the library's own allocations
    jd.set_allocator(None, None)
    e2, _, _, i2 = jd.solve(L, W, seed, sigma, k, 1e-10, precision="mixed")
    assert np.array_equal(evals, e2) and i2["outer_its"] == info["outer_its"]


def test_serving_workers_use_the_hook(hook):
    reqs = [(10, 16.5, 1000000 + i, 0.1 * i, 3) for i in range(4)] + [(14, 21.0, 1000010, -0.3, 5)]
    srv = jd.Server(workers=4)
    try:
        tickets = [srv.submit(jd.Server.request(*r, precision="mixed")) for r in reqs]
        res = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    assert hook.allocs > 0 and not hook.live and hook.frees == hook.allocs
    assert len(hook.threads - {threading.get_ident()}) >= 1  # called from worker threads
    for r, out in zip(reqs, res):
        assert out["status"] == 0, out["error"]
        ref = eig.anderson_nearest(*r)[0]
        assert np.max(np.abs(out["evals"] - ref)) <= 1e-9


def test_failing_hook_reports_enomem():
    jd.set_allocator(lambda nbytes, stream: 0, lambda ptr, stream: None)
    try:
        with pytest.raises(jd.JdError) as e:
            jd.Problem(8, 16.5, 0, 0.0)
        assert e.value.code == jd.JD_ENOMEM
    finally:
        jd.set_allocator(None, None)
