"""The no-allocation TT-matvec (t2s2_tt_matvec_noalloc) against the allocating
entry point t2s2_tt_matvec: same kernels, so the results must be bitwise
equal; two calls in a row (the second smaller), plus a rejected oversize
operator and a call after it.  The small general operator is also checked
against the oracle's TT-matvec (exact algebra, 1e-13 relative)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_04732_amd as t2s2  # noqa: E402
from paper_2506_04732_amd import TT, _lib  # noqa: E402
from oracle import tt as ott  # noqa: E402


def _say(*a):
    print("[case]", *a, flush=True)


class _TTM:
    """TTMStruct over device copies of numpy cores [R0][n][n][R1] (kept alive)."""

    def __init__(self, cores):
        import torch
        self.d = len(cores)
        self.bufs = [torch.from_numpy(np.ascontiguousarray(c).ravel()).cuda() for c in cores]
        self.n = (C.c_int * self.d)(*[c.shape[1] for c in cores])
        self.r = (C.c_int * (self.d + 1))(*([cores[0].shape[0]] + [c.shape[3] for c in cores]))
        self.c = (C.c_void_p * self.d)(*[b.data_ptr() for b in self.bufs])
        self.s = _lib.TTMStruct(self.d, self.n, self.r, C.cast(self.c, C.POINTER(C.c_void_p)))


def _pair(op, x):
    a = t2s2.ttm_matvec(op, x).to_numpy()
    b = t2s2.ttm_matvec(op, x, noalloc=True).to_numpy()
    return a, b


def test_noalloc_matvec_equals_allocating_matvec():
    rng = np.random.default_rng(5)
    # call 1: the problem's rank-2 operator, 4D N = 32, ragged ranks
    _say("noalloc call 1: 4D N=32 problem operator")
    p = t2s2.Problem(4, 32, 1e-2, rng.standard_normal(4), 1, rank_cap=8)
    xs = [rng.standard_normal(s) for s in [(1, 30, 20), (20, 30, 35), (35, 30, 17), (17, 30, 1)]]
    a, b = _pair(p.operator(), TT.from_numpy(xs))
    for ca, cb in zip(a, b):
        assert ca.shape == cb.shape and np.array_equal(ca, cb)
    # call 2, smaller: a general rank-3 TT-matrix, 2D
    _say("noalloc call 2: general 2D operator")
    A = [rng.standard_normal((1, 5, 5, 3)), rng.standard_normal((3, 7, 7, 1))]
    op = _TTM(A)
    x = [rng.standard_normal((1, 5, 2)), rng.standard_normal((2, 7, 1))]
    a, b = _pair(op.s, TT.from_numpy(x))
    for ca, cb in zip(a, b):
        assert np.array_equal(ca, cb)
    yo = ott.matvec(A, x)
    for cb, co in zip(b, yo):
        assert np.abs(cb - co).max() <= 1e-13 * np.abs(co).max()
    # an operator core beyond the static scratch is rejected before any work
    _say("noalloc oversize")
    big = _TTM([rng.standard_normal((1, 64, 64, 6)), rng.standard_normal((6, 64, 64, 6)),
                rng.standard_normal((6, 64, 64, 1))])
    xb = TT.from_numpy([rng.standard_normal(s) for s in [(1, 64, 1), (1, 64, 1), (1, 64, 1)]])
    with pytest.raises(t2s2.T2S2Error) as e:
        t2s2.ttm_matvec(big.s, xb, noalloc=True)
    assert e.value.code == t2s2.T2S2_EINVAL
    # and a call after it still matches
    _say("noalloc call 3: after the rejection")
    a, b = _pair(op.s, TT.from_numpy(x))
    for ca, cb in zip(a, b):
        assert np.array_equal(ca, cb)
