"""CPU checks of the Python binding's argument marshalling (no GPU, no library calls).

The library is replaced by a stub that records its calls, and device tensors by stand-ins
with the attributes the binding reads.  The binding must hand the kernels only
contiguous GPU tensors of the element type and length the entry point assumes, and raise
before the call otherwise.
"""
import ctypes

import pytest

torch = pytest.importorskip("torch")

import paper_math_0508111_amd as jd  # noqa: E402


class StubLib:
    def __init__(self, returns=None):
        self.calls = []
        self.owned = []
        self.returns = returns or {}

    def __getattr__(self, name):
        if name.startswith("__"):
            raise AttributeError(name)

        def f(*args):
            self.calls.append((name, args))
            r = self.returns.get(name, 0)
            return r(*args) if callable(r) else r
        return f

    def jd_last_error(self):
        return b"stub"


class Dev:
    """Stand-in for a device tensor."""

    def __init__(self, dtype, numel, cuda=True, contiguous=True, shape=None, ptr=0x10000):
        self.dtype, self.is_cuda, self._n, self._c, self._p = dtype, cuda, numel, contiguous, ptr
        self.shape = shape if shape is not None else (numel,)

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        return self._p

    def t(self):
        return Dev(self.dtype, self._n, self.is_cuda, False, (self.shape[1], self.shape[0]), self._p)

    def contiguous(self):
        return Dev(self.dtype, self._n, self.is_cuda, True, self.shape, self._p + 8)


F64, F32 = torch.float64, torch.float32


@pytest.fixture
def stub(monkeypatch):
    s = StubLib()
    monkeypatch.setattr(jd, "_lib", s)
    yield s
    # stand-in handles must never reach the real library's *_free
    for obj in s.owned:
        obj._h = None


def fake_precond(stub, L):
    P = jd.Precond(L, 0.0, 0, 0.0, _handle=ctypes.c_void_p(0x1234))
    stub.owned.append(P)
    return P


def _ptr_value(a):
    return None if a is None else a.value


def test_gen_diag_checks(stub):
    L, n = 5, 125
    jd.gen_diag(L, 16.5, 0, Dev(F64, n, ptr=0x100), Dev(F32, n, ptr=0x200))
    name, args = stub.calls[-1]
    assert name == "jd_gen_diag" and _ptr_value(args[3]) == 0x100 and _ptr_value(args[4]) == 0x200
    jd.gen_diag(L, 16.5, 0, Dev(F64, n), None)
    assert stub.calls[-1][1][4] is None
    for bad in (Dev(F32, n), Dev(F64, n - 1), Dev(F64, n, cuda=False), Dev(F64, n, contiguous=False)):
        with pytest.raises(ValueError):
            jd.gen_diag(L, 16.5, 0, bad, None)
    with pytest.raises(ValueError):
        jd.gen_diag(L, 16.5, 0, Dev(F64, n), Dev(F64, n))
    assert len(stub.calls) == 2


@pytest.mark.parametrize("precision,dt,wrong", [("fp64", F64, F32), ("mixed", F32, F64)])
def test_stencil_checks(stub, precision, dt, wrong):
    L, n = 4, 64
    jd.stencil_spmv(L, Dev(dt, n), 0.0, Dev(dt, n), Dev(dt, n), precision)
    assert stub.calls[-1][0] == "jd_stencil_spmv"
    for args in ((Dev(wrong, n), Dev(dt, n), Dev(dt, n)), (Dev(dt, n), Dev(dt, n - 1), Dev(dt, n)),
                 (Dev(dt, n), Dev(dt, n), Dev(wrong, n))):
        with pytest.raises(ValueError):
            jd.stencil_spmv(L, args[0], 0.0, args[1], args[2], precision)
    assert len(stub.calls) == 1


def test_stencil_unknown_precision_goes_to_the_library(stub):
    # the ABI itself rejects JD_MIXED_FACTORS for this entry point
    stub.returns["jd_stencil_spmv"] = jd.JD_EINVAL
    with pytest.raises(jd.JdError):
        jd.stencil_spmv(3, Dev(F64, 27), 0.0, Dev(F64, 27), Dev(F64, 27), "mixed_factors")


def test_precond_apply_and_factor_product_checks(stub):
    L, n = 6, 216
    P = fake_precond(stub, L)
    P.apply(Dev(F64, n), Dev(F64, n), "fp64")
    P.apply(Dev(F32, n), Dev(F32, n), "mixed")
    P.factor_product(Dev(F32, n), Dev(F32, n), transpose=True)
    P.factor_product(Dev(F64, n), Dev(F64, n), precision="fp64")
    assert [c[0] for c in stub.calls] == ["jd_precond_apply"] * 2 + ["jd_precond_factor_product"] * 2
    with pytest.raises(ValueError):
        P.apply(Dev(F32, n), Dev(F32, n), "fp64")
    with pytest.raises(ValueError):
        P.apply(Dev(F64, n), Dev(F64, n - 1), "fp64")
    with pytest.raises(ValueError):
        P.factor_product(Dev(F64, n), Dev(F64, n))  # default precision: binary32 vectors
    assert len(stub.calls) == 4


def test_levels_grows_its_buffers(stub):
    stub.returns["jd_precond_levels"] = lambda h, cap, *a: 300
    P = fake_precond(stub, 4)
    lv = P.levels(cap=256)
    caps = [c[1][1] for c in stub.calls if c[0] == "jd_precond_levels"]
    assert caps == [256, 301]
    assert lv["levels"] == 300 and len(lv["sizes"]) == 301 and len(lv["nB"]) == 300


def test_problem_checks_and_view_lifetime(stub):
    L, n, k = 5, 125, 3
    prob = jd.Problem(L, 16.5, 0, 0.0)
    prob.solve(k, device_out=Dev(F64, n * k, ptr=0x500))
    assert _ptr_value(stub.calls[-1][1][5]) == 0x500
    with pytest.raises(ValueError):
        prob.solve(k, device_out=Dev(F64, n * k - 1))
    with pytest.raises(ValueError):
        prob.solve(k, device_out=Dev(F32, n * k))
    # Q is passed column-major: the binding transposes and copies it
    prob.linear_solve(0.0, Dev(F64, n), Dev(F64, n), Q=Dev(F64, n * 2, shape=(n, 2), ptr=0x700))
    name, args = stub.calls[-1]
    assert name == "jd_problem_linear_solve" and _ptr_value(args[2]) == 0x708 and args[3] == 2
    with pytest.raises(ValueError):
        prob.linear_solve(0.0, Dev(F64, n), Dev(F64, n), Q=Dev(F64, n * 2, shape=(2, n)))
    with pytest.raises(ValueError):
        prob.linear_solve(0.0, Dev(F32, n), Dev(F64, n))
    with pytest.raises(ValueError):
        prob.linear_solve(0.0, Dev(F64, n), Dev(F64, n, cuda=False))
    view = prob.precond()
    assert view._owner is prob and view.n == n
