"""O3 -- Python wrapper of the dense cyclic Jacobi eigensolver in ``jacobi.c``.

The shared object is built with gcc on first use (or by the project's build step);
it is part of the oracle and is loaded only by tests, the smoke check and the
benchmark's CPU baseline.
"""
import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_LIB = os.path.join(_HERE, "_jacobi.so")
_lib = None


def build_oracle_c():
    """Compile jacobi.c into _jacobi.so (plain gcc, -O2, no fast-math)."""
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"])
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle_c()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_jacobi_eig.restype = ctypes.c_int
        lib.oracle_jacobi_eig.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        _lib = lib
    return _lib


def eigh(A, vectors=True, tol=1e-15, max_sweeps=60):
    """Eigen-decomposition of a dense symmetric matrix by cyclic Jacobi.

    Returns (w, V) with A V = V diag(w), columns of V orthonormal, w ascending.
    """
    a = np.array(A, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    if n == 0:
        return np.zeros(0), np.zeros((0, 0))
    if not np.allclose(a, a.T, rtol=0, atol=0):
        raise ValueError("matrix is not symmetric")
    w = np.empty(n)
    vt = np.empty((n, n)) if vectors else None
    sweeps = _load().oracle_jacobi_eig(n, a.ctypes.data, vt.ctypes.data if vectors else None,
                                       w.ctypes.data, tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not reach the off-diagonal tolerance")
    order = np.argsort(w, kind="stable")
    return w[order], (vt[order].T.copy() if vectors else None)
