"""The allocation-free linear solve (jd_problem_linear_solve_noalloc) through the C ABI.

Checked against jd_problem_linear_solve, the entry point it is a variant of: the same
kernels in the same order on the same inputs, so the same step count and a bitwise
identical solution; two calls in a row, the second on a smaller problem with a narrower
projection; no device allocation (jd_set_allocator's hook counts none) and a clear
error when a call needs more than the static scratch holds.
"""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_math_0508111_amd as jd  # noqa: E402
from oracle import generator, lattice  # noqa: E402
from tests import seeded_inputs  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


class Counter:
    def __init__(self):
        self.lock = threading.Lock()
        self.allocs = 0

    def alloc(self, nbytes, stream):
        with self.lock:
            self.allocs += 1
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def free(self, ptr, _stream):
        torch.cuda.caching_allocator_delete(ptr)


def _pair(prob, L, sigma, Q, b, rtol, maxit):
    n = L ** 3
    x_ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    x_na = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    it_ref = prob.linear_solve(sigma, dev(b), x_ref, Q=None if Q is None else dev(Q), rtol=rtol, maxit=maxit)
    cnt = Counter()
    jd.set_allocator(cnt.alloc, cnt.free)
    try:
        it_na = prob.linear_solve(sigma, dev(b), x_na, Q=None if Q is None else dev(Q), rtol=rtol, maxit=maxit,
                                  noalloc=True)
    finally:
        jd.set_allocator(None, None)
    torch.cuda.synchronize()
    assert cnt.allocs == 0
    return it_ref, x_ref.cpu().numpy(), it_na, x_na.cpu().numpy()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matches_the_allocating_solve(precision):
    # second case: smaller n and a narrower projection; binary32 inner vectors reach a
    # relative residual of about 1e-5
    rtols = (1e-5, 1e-5) if precision == "mixed" else (1e-9, 1e-10)
    cases = [(14, 16.5, 1, 0.05, 3, rtols[0]), (8, 21.0, 2, -0.3, 1, rtols[1])]
    for L, W, seed, sigma, p, rtol in cases:
        n = L ** 3
        prob = jd.Problem(L, W, seed, sigma, precision=precision)
        Q = seeded_inputs.orthonormal_block(n, p, 5 + p)
        b = seeded_inputs.vector(n, 11 + L)
        it_ref, x_ref, it_na, x_na = _pair(prob, L, sigma, Q, b, rtol, 300)
        assert it_na == it_ref and 1 <= it_na < 300, (it_ref, it_na)
        assert np.array_equal(x_na, x_ref)
        # and it is a solution of the projected system (oracle's own product)
        eps = generator.disorder(L, W, seed)
        proj = lambda v: v - Q @ (Q.T @ v)
        res = proj(lattice.matvec(L, eps, proj(x_na), shift=sigma)) - proj(b)
        assert np.linalg.norm(res) <= 20 * 10 * rtol * np.linalg.norm(proj(b))
        prob.close()


def test_noalloc_without_projection_and_the_size_limit():
    L, sigma = 12, 0.1
    prob = jd.Problem(L, 16.5, 3, sigma, precision="fp64")
    b = seeded_inputs.vector(L ** 3, 4)
    it_ref, x_ref, it_na, x_na = _pair(prob, L, sigma, None, b, 1e-9, 200)
    assert it_na == it_ref and np.array_equal(x_na, x_ref)
    prob.close()
    # L = 40 in binary64 with 64 projection columns needs about 70 MB of scratch
    L = 40
    n = L ** 3
    prob = jd.Problem(L, 16.5, 3, sigma, precision="fp64")
    Q = torch.zeros((n, 64), dtype=torch.float64, device="cuda")
    Q[torch.arange(64, device="cuda") * 17, torch.arange(64, device="cuda")] = 1.0
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(jd.JdError) as e:
        prob.linear_solve(sigma, dev(seeded_inputs.vector(n, 1)), x, Q=Q, noalloc=True)
    assert e.value.code == jd.JD_EINVAL and "scratch" in str(e.value)
    prob.close()
