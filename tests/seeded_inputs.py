"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds none of the method's arithmetic: only reproducible random vectors and the
request parameters of the workloads.
"""
import numpy as np


def vector(n, seed, dtype=np.float64):
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


def orthonormal_block(n, p, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, p)))
    return np.ascontiguousarray(q)


def serving_requests(count, seed=1, first_disorder_seed=1000000):
    """Mixed solve requests: L in {20..60}, W in {12, 16.5, 21}, sigma ~ U[-1, 1],
    k in 1..10, disorder seed first_disorder_seed + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        out.append(dict(L=int(rng.choice([20, 30, 40, 50, 60])), W=float(rng.choice([12.0, 16.5, 21.0])),
                        seed=first_disorder_seed + i, sigma=float(rng.uniform(-1.0, 1.0)),
                        k=int(rng.integers(1, 11))))
    return out


def poisson_arrivals(count, rate, seed=2):
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))
