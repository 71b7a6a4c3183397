"""Shift-and-invert Jacobi-Davidson for the 3D Anderson model on MI355X (gfx950).

Thin ctypes binding of ``libjdmi.so`` (declared in ``include/jd.h``).  It only
marshals arguments: every step of the solve runs in the library's HIP kernels and
host setup.  Device arrays are passed as torch CUDA tensors (their data pointers);
host outputs are numpy arrays.  If the library is missing this module raises on
first use; there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjdmi.so")

JD_OK, JD_ENOCONV, JD_EINVAL, JD_ENOMEM, JD_EDEVICE, JD_ESETUP, JD_ENOTIMPL = 0, 1, -1, -2, -3, -4, -5
JD_FP64, JD_MIXED, JD_MIXED_FACTORS = 0, 1, 2
JD_BC_PERIODIC, JD_BC_HARDWALL = 0, 1
_BC = {"periodic": JD_BC_PERIODIC, "hardwall": JD_BC_HARDWALL, JD_BC_PERIODIC: JD_BC_PERIODIC,
       JD_BC_HARDWALL: JD_BC_HARDWALL}
JD_MODEL_ANDERSON, JD_MODEL_OFFDIAG = 0, 1
_MODEL = {"anderson": JD_MODEL_ANDERSON, "offdiag": JD_MODEL_OFFDIAG, JD_MODEL_ANDERSON: JD_MODEL_ANDERSON,
          JD_MODEL_OFFDIAG: JD_MODEL_OFFDIAG}
JD_FLAG_GRAPHS = 1
JD_FLAG_LEVELS = 2
_PREC = {"fp64": JD_FP64, "mixed": JD_MIXED, "mixed_factors": JD_MIXED_FACTORS, JD_FP64: JD_FP64,
         JD_MIXED: JD_MIXED, JD_MIXED_FACTORS: JD_MIXED_FACTORS}


class JdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"jd error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("drop_tol", ctypes.c_double), ("kappa", ctypes.c_double),
                ("agg_tau", ctypes.c_double), ("schur_tol", ctypes.c_double), ("coarse_max", ctypes.c_int),
                ("max_levels", ctypes.c_int), ("z_drop", ctypes.c_double), ("jmin", ctypes.c_int), ("jmax", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int), ("switch_tol", ctypes.c_double),
                ("flags", ctypes.c_int), ("z_parts", ctypes.c_int), ("bc", ctypes.c_int),
                ("model", ctypes.c_int), ("inner_tol_min", ctypes.c_double), ("inner_tol_rate", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("W", ctypes.c_double), ("seed", ctypes.c_uint64), ("sigma", ctypes.c_double),
                ("k", ctypes.c_int), ("tol", ctypes.c_double), ("precision", ctypes.c_int), ("flags", ctypes.c_int),
                ("bc", ctypes.c_int), ("model", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("k", ctypes.c_int), ("n_converged", ctypes.c_int),
                ("outer_its", ctypes.c_int), ("inner_its", ctypes.c_int), ("evals", ctypes.c_double * 64),
                ("resid", ctypes.c_double * 64), ("queued_s", ctypes.c_double), ("setup_s", ctypes.c_double),
                ("solve_s", ctypes.c_double), ("latency_s", ctypes.c_double), ("device_bytes", ctypes.c_size_t),
                ("error", ctypes.c_char * 160)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("evals", "resid", "error")}
        d["error"] = self.error.decode(errors="replace")
        d["evals"] = np.array(self.evals[: self.k])
        d["resid"] = np.array(self.resid[: self.k])
        return d


class Info(ctypes.Structure):
    _fields_ = [("n_converged", ctypes.c_int), ("outer_its", ctypes.c_int), ("inner_its", ctypes.c_int),
                ("levels", ctypes.c_int), ("n_2x2", ctypes.c_int), ("coarse_n", ctypes.c_int),
                ("setup_s", ctypes.c_double), ("solve_s", ctypes.c_double), ("fill", ctypes.c_double),
                ("anorm", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = ["jd_solve", "jd_setup", "jd_problem_solve", "jd_problem_info", "jd_problem_set_precision", "jd_problem_set_solve_options", "jd_problem_free", "jd_gen_diag",
           "jd_stencil_spmv", "jd_precond_create", "jd_precond_apply", "jd_precond_levels", "jd_precond_free", "jd_problem_precond", "jd_precond_factor_nnz",
           "jd_precond_factor_product", "jd_precond_segments",
           "jd_problem_linear_solve", "jd_last_error", "jd_version", "jd_server_create", "jd_server_submit",
           "jd_server_poll", "jd_server_wait", "jd_server_footprint", "jd_server_destroy",
           "jd_host_matching", "jd_host_split_cycles", "jd_host_factor", "jd_host_precond_apply", "jd_set_allocator",
           "jd_problem_linear_solve_noalloc", "jd_problem_lanczos", "jd_gen_hop", "jd_block_product"]

_lib = None


def lib():
    """Load libjdmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_math_0508111_amd.build` first")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, U64, DP = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)
    OP, IP = ctypes.POINTER(Options), ctypes.POINTER(Info)
    sig = {
        "jd_solve": (I, [I, D, U64, D, I, D, P, P, P, OP, IP]),
        "jd_setup": (I, [I, D, U64, D, OP, ctypes.POINTER(P)]),
        "jd_problem_solve": (I, [P, I, D, P, P, P, P, IP]),
        "jd_problem_lanczos": (I, [P, I, D, D, P, P, P, IP]),
        "jd_problem_info": (I, [P, IP]),
        "jd_problem_set_precision": (I, [P, I]),
        "jd_problem_set_solve_options": (I, [P, OP]),
        "jd_problem_free": (None, [P]),
        "jd_gen_diag": (I, [I, D, U64, P, P, P]),
        "jd_stencil_spmv": (I, [I, I, I, P, P, D, P, P, P]),
        "jd_gen_hop": (I, [I, D, U64, P, P, P]),
        "jd_block_product": (I, [I, I, I, P, ctypes.c_int64, P, I, P, ctypes.c_int64, P]),
        "jd_precond_create": (I, [I, D, U64, D, OP, ctypes.POINTER(P)]),
        "jd_precond_apply": (I, [P, I, P, P, P]),
        "jd_precond_levels": (I, [P, I, P, P, P]),
        "jd_precond_free": (None, [P]),
        "jd_problem_precond": (I, [P, ctypes.POINTER(P)]),
        "jd_precond_factor_nnz": (I, [P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(I)]),
        "jd_precond_factor_product": (I, [P, I, I, P, P, P]),
        "jd_precond_segments": (I, [P, I, P, P, P]),
        "jd_problem_linear_solve": (I, [P, D, P, I, P, P, D, I, ctypes.POINTER(I)]),
        "jd_problem_linear_solve_noalloc": (I, [P, D, P, I, P, P, D, I, ctypes.POINTER(I)]),
        "jd_server_create": (I, [ctypes.c_size_t, I, I, ctypes.POINTER(P)]),
        "jd_server_submit": (I, [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
        "jd_server_poll": (I, [P, ctypes.c_uint64, ctypes.POINTER(Result)]),
        "jd_server_wait": (I, [P, ctypes.c_uint64, ctypes.POINTER(Result)]),
        "jd_server_footprint": (ctypes.c_size_t, [ctypes.POINTER(Request)]),
        "jd_server_destroy": (None, [P]),
        "jd_set_allocator": (I, [P, P, P]),
        "jd_last_error": (ctypes.c_char_p, []),
        "jd_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc, allow_partial=False):
    if rc == JD_OK or (allow_partial and rc == JD_ENOCONV):
        return rc
    raise JdError(rc, lib().jd_last_error().decode())


def make_options(precision="fp64", stream=None, **kw):
    o = Options()
    o.precision = _PREC[precision]
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, _BC[v] if k == "bc" else _MODEL[v] if k == "model" else v)
    if stream is not None:
        o.stream = ctypes.c_void_p(_stream_ptr(stream))
    return o


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# element type of the device vectors of the step entry points, per precision code
_VEC_DTYPE = {JD_FP64: "torch.float64", JD_MIXED: "torch.float32"}


def _dev(t, dtype, numel, name):
    """Device pointer of tensor t after checking what the kernels will assume of it: a
    contiguous GPU tensor of `dtype` ("torch.float64"/"torch.float32"; None: the ABI
    rejects the precision itself) holding at least `numel` elements.  A wrong element
    type or a short tensor would otherwise send the kernels past the allocation."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name}: a GPU tensor is required")
    if dtype is not None and str(t.dtype) != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {numel} needed")
    return ctypes.c_void_p(t.data_ptr())


def _host(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def solve(L, W, seed, sigma, k, tol=1e-10, vectors=False, precision="fp64", **opts):
    """k eigenpairs of the Anderson matrix nearest sigma (jd_solve)."""
    n = L ** 3
    evals = np.full(k, np.nan)
    resid = np.full(k, np.nan)
    evecs = np.empty((k, n)) if vectors else None
    info = Info()
    o = make_options(precision, **opts)
    rc = lib().jd_solve(L, float(W), seed, float(sigma), k, float(tol), _host(evals),
                        _host(evecs), _host(resid), ctypes.byref(o), ctypes.byref(info))
    _check(rc, allow_partial=True)
    return evals, (evecs.T if vectors else None), resid, dict(info.as_dict(), status=rc)


class Problem:
    """jd_setup / jd_problem_solve: setup once, factors resident on the device."""

    def __init__(self, L, W, seed, sigma, precision="fp64", **opts):
        self.L, self.n = L, L ** 3
        self._opts = make_options(precision, **opts)
        h = ctypes.c_void_p()
        _check(lib().jd_setup(L, float(W), seed, float(sigma), ctypes.byref(self._opts), ctypes.byref(h)))
        self._h = h

    def set_precision(self, precision):
        _check(lib().jd_problem_set_precision(self._h, _PREC[precision]))

    def set_solve_options(self, **opts):
        """jd_problem_set_solve_options: jmin, jmax, max_outer, max_inner, switch_tol, inner_tol_min,
        inner_tol_rate, flags."""
        o = make_options(**opts)
        _check(lib().jd_problem_set_solve_options(self._h, ctypes.byref(o)))

    def precond(self):
        """A view of the problem's preconditioner (it holds a reference to the problem)."""
        h = ctypes.c_void_p()
        _check(lib().jd_problem_precond(self._h, ctypes.byref(h)))
        v = Precond(self.L, 0.0, 0, 0.0, _handle=h)
        v._owner = self  # the view reads the problem's factors: keep the problem alive
        return v

    def info(self):
        i = Info()
        _check(lib().jd_problem_info(self._h, ctypes.byref(i)))
        return i.as_dict()

    def solve(self, k, tol=1e-10, vectors=False, device_out=None):
        evals = np.full(k, np.nan)
        resid = np.full(k, np.nan)
        evecs = np.empty((k, self.n)) if vectors else None
        info = Info()
        d_out = _dev(device_out, "torch.float64", self.n * k, "device_out")
        rc = lib().jd_problem_solve(self._h, k, float(tol), _host(evals), _host(evecs), d_out,
                                    _host(resid), ctypes.byref(info))
        _check(rc, allow_partial=True)
        return evals, (evecs.T if vectors else None), resid, dict(info.as_dict(), status=rc)

    def lanczos(self, k, tol=1e-10, inner_tol=1e-10, vectors=False):
        """jd_problem_lanczos: the same pairs by shift-and-invert Lanczos."""
        evals = np.full(k, np.nan)
        resid = np.full(k, np.nan)
        evecs = np.empty((k, self.n)) if vectors else None
        info = Info()
        rc = lib().jd_problem_lanczos(self._h, k, float(tol), float(inner_tol), _host(evals), _host(evecs),
                                      _host(resid), ctypes.byref(info))
        _check(rc, allow_partial=True)
        return evals, (evecs.T if vectors else None), resid, dict(info.as_dict(), status=rc)

    def linear_solve(self, shift, b, x, Q=None, rtol=1e-8, maxit=200, noalloc=False):
        """Q: (n, p) device tensor of orthonormal columns (laid out column-major for the ABI).
        noalloc: jd_problem_linear_solve_noalloc (static scratch, allocates nothing)."""
        its = ctypes.c_int(0)
        if Q is not None and (len(Q.shape) != 2 or int(Q.shape[0]) != self.n):
            raise ValueError(f"Q: shape {tuple(Q.shape)}, expected ({self.n}, p)")
        p = 0 if Q is None else int(Q.shape[1])
        Qc = None if Q is None else Q.t().contiguous()
        qp = _dev(Qc, "torch.float64", self.n * p, "Q")
        bp = _dev(b, "torch.float64", self.n, "b")
        xp = _dev(x, "torch.float64", self.n, "x")
        fn = lib().jd_problem_linear_solve_noalloc if noalloc else lib().jd_problem_linear_solve
        _check(fn(self._h, float(shift), qp, p, bp, xp, float(rtol), int(maxit), ctypes.byref(its)))
        return its.value

    def close(self):
        if self._h:
            lib().jd_problem_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Precond:
    """jd_precond_create / jd_precond_apply: the multilevel ILDL^T preconditioner alone."""

    def __init__(self, L, W, seed, sigma, _handle=None, **opts):
        self.L, self.n = L, L ** 3
        if _handle is not None:
            self._h = _handle
            return
        self._opts = make_options("fp64", **opts)
        h = ctypes.c_void_p()
        _check(lib().jd_precond_create(L, float(W), seed, float(sigma), ctypes.byref(self._opts), ctypes.byref(h)))
        self._h = h

    def factor_nnz(self):
        nnz = ctypes.c_longlong()
        _check(lib().jd_precond_factor_nnz(self._h, ctypes.byref(nnz), None))
        return nnz.value

    def factor_product(self, x, y, transpose=False, precision="mixed", stream=None):
        """x = y = None: the timing form (the products on the workspace's values)."""
        pr = _PREC[precision]
        dt = _VEC_DTYPE.get(pr)
        _check(lib().jd_precond_factor_product(self._h, pr, int(transpose), _dev(x, dt, self.n, "x"),
                                               _dev(y, dt, self.n, "y"), _stream_ptr(stream)))

    def segments(self, cap=64):
        lb = np.zeros(cap, np.int32)
        rows = np.zeros(cap, np.int32)
        nnz = np.zeros(cap, np.int64)
        ns = lib().jd_precond_segments(self._h, cap, _host(lb), _host(rows), _host(nnz))
        if ns < 0:
            _check(ns)
        ns = min(ns, cap)
        return dict(segments=ns, lev_begin=lb[:ns].tolist(), rows=rows[:ns].tolist(), nnz=nnz[:ns].tolist())

    def apply(self, x, y, precision="fp64", stream=None):
        pr = _PREC[precision]
        dt = _VEC_DTYPE.get(pr)
        _check(lib().jd_precond_apply(self._h, pr, _dev(x, dt, self.n, "x"), _dev(y, dt, self.n, "y"),
                                      _stream_ptr(stream)))

    def levels(self, cap=256):
        while True:
            sizes = np.zeros(cap, np.int32)
            nb = np.zeros(cap, np.int32)
            nnz = np.zeros(cap, np.int64)
            nl = lib().jd_precond_levels(self._h, cap, _host(sizes), _host(nb), _host(nnz))
            if nl < 0:
                _check(nl)
            if nl + 1 <= cap:
                return dict(levels=nl, sizes=sizes[:nl + 1].tolist(), nB=nb[:nl].tolist(), nnzG=nnz[:nl].tolist())
            cap = nl + 1

    def close(self):
        if self._h:
            lib().jd_precond_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gen_diag(L, W, seed, eps64, eps32=None, stream=None):
    n = int(L) ** 3
    _check(lib().jd_gen_diag(L, float(W), seed, _dev(eps64, "torch.float64", n, "eps64"),
                             _dev(eps32, "torch.float32", n, "eps32"), _stream_ptr(stream)))


def block_product(V, S, out, stream=None):
    """out = V S (jd_block_product); V (n, m), S (m, mout), out (n, mout): device float64
    tensors whose transposes are contiguous (column-major storage)."""
    n, m = int(V.shape[0]), int(V.shape[1])
    mout = int(S.shape[1])
    if int(S.shape[0]) != m or tuple(out.shape) != (n, mout):
        raise ValueError("shapes do not match: V (n, m), S (m, mout), out (n, mout)")
    for t, name in ((V, "V"), (S, "S"), (out, "out")):
        if not t.t().is_contiguous():
            raise ValueError(f"{name}: column-major storage expected (its transpose contiguous)")
    _check(lib().jd_block_product(n, m, mout, _dev(V.t(), "torch.float64", n * m, "V"), n,
                                  _dev(S.t(), "torch.float64", m * mout, "S"), m,
                                  _dev(out.t(), "torch.float64", n * mout, "out"), n, _stream_ptr(stream)))


def gen_hop(L, W, seed, hop64, hop32=None, stream=None):
    n = int(L) ** 3
    _check(lib().jd_gen_hop(L, float(W), seed, _dev(hop64, "torch.float64", 3 * n, "hop64"),
                            _dev(hop32, "torch.float32", 3 * n, "hop32"), _stream_ptr(stream)))


def stencil_spmv(L, eps, shift, x, y, precision="fp64", stream=None, bc="periodic", hop=None):
    n = int(L) ** 3
    pr = _PREC[precision]
    dt = _VEC_DTYPE.get(pr)
    _check(lib().jd_stencil_spmv(L, _BC[bc], pr, _dev(eps, dt, n, "eps"), _dev(hop, dt, 3 * n, "hop"), float(shift),
                                 _dev(x, dt, n, "x"), _dev(y, dt, n, "y"), _stream_ptr(stream)))


def version():
    return lib().jd_version().decode()


# C signatures of jd_set_allocator's callbacks
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_allocator = None  # the installed callbacks (kept alive while the library may call them)
_retired = []      # earlier callbacks: buffers obtained through them still return through them


def set_allocator(alloc=None, free=None):
    """jd_set_allocator with Python callables alloc(bytes, stream) -> int device pointer
    (0 on failure) and free(ptr, stream); both None restores hipMalloc/hipFree.
    The callables run on library threads too (serving workers) and must be thread-safe."""
    global _allocator
    if (alloc is None) != (free is None):
        raise ValueError("alloc and free must be given together")
    if alloc is None:
        cb = (None, None)
    else:
        def _a(nbytes, stream, _ctx):
            try:
                return int(alloc(int(nbytes), int(stream or 0))) or None
            except Exception:
                return None

        def _f(ptr, stream, _ctx):
            free(int(ptr), int(stream or 0))
        cb = (ALLOC_FN(_a), FREE_FN(_f))
    _check(lib().jd_set_allocator(ctypes.cast(cb[0], ctypes.c_void_p) if cb[0] else None,
                                  ctypes.cast(cb[1], ctypes.c_void_p) if cb[1] else None, None))
    if _allocator is not None:
        _retired.append(_allocator)
    _allocator = cb if cb[0] else None


def use_torch_allocator(enable=True):
    """Route the library's device memory through PyTorch's caching allocator
    (torch.cuda.caching_allocator_alloc / caching_allocator_delete), on the stream the
    library's work uses; enable=False restores hipMalloc/hipFree."""
    if not enable:
        set_allocator(None, None)
        return
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def free(ptr, _stream):
        torch.cuda.caching_allocator_delete(ptr)
    set_allocator(alloc, free)


class Server:
    """jd_server_*: independent solve requests served concurrently (one stream per worker)."""

    def __init__(self, hbm_budget_bytes=0, workers=0, setup_threads=0):
        h = ctypes.c_void_p()
        _check(lib().jd_server_create(int(hbm_budget_bytes), int(workers), int(setup_threads), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def request(L, W, seed, sigma, k, tol=1e-10, precision="mixed", flags=0, bc="periodic", model="anderson"):
        return Request(int(L), float(W), int(seed), float(sigma), int(k), float(tol), _PREC[precision], int(flags),
                       _BC[bc], _MODEL[model])

    def submit(self, req):
        t = ctypes.c_uint64()
        _check(lib().jd_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        r = Result()
        rc = lib().jd_server_poll(self._h, ticket, ctypes.byref(r))
        if rc < 0:
            _check(rc)
        return r.as_dict() if rc == 0 else None

    def wait(self, ticket):
        r = Result()
        _check(lib().jd_server_wait(self._h, ticket, ctypes.byref(r)))
        return r.as_dict()

    @staticmethod
    def footprint(req):
        return lib().jd_server_footprint(ctypes.byref(req))

    def close(self):
        if self._h:
            lib().jd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
