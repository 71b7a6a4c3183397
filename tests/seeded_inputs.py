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
