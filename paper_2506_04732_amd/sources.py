"""Separable TT right-hand sides on a problem's collocation grid.

Binding of t2s2_source_gaussians / t2s2_source_manufactured: the 1D factors
are evaluated at the collocation nodes and assembled into the block-diagonal
TT cores (rank = number of terms) by the library's kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np

from . import TT, Problem, _stream
from ._lib import check, lib


def _out(problem: Problem, s: int) -> TT:
    d = problem.d
    ranks = [1] + [s if d > 1 else 1] * (d - 1) + [1]
    return TT.empty_like_ranks(problem.m, ranks)


def gaussians(problem: Problem, amp: Sequence[float], centre, width: Sequence[float]) -> TT:
    """f(x) = sum_t amp[t] prod_l exp(-(x_l - centre[t][l])^2 / (2 width[t]^2))."""
    a = np.ascontiguousarray(amp, dtype=np.float64)
    c = np.ascontiguousarray(centre, dtype=np.float64).reshape(a.size, problem.d)
    w = np.ascontiguousarray(width, dtype=np.float64)
    if w.size != a.size:
        raise ValueError("amp, centre and width must describe the same number of terms")
    f = _out(problem, a.size)
    fs = f._struct()
    dp = C.POINTER(C.c_double)
    check(lib().t2s2_source_gaussians(problem._h, int(a.size), a.ctypes.data_as(dp), c.ctypes.data_as(dp),
                                      w.ctypes.data_as(dp), C.byref(fs), _stream()))
    f._read_ranks()
    return f


def manufactured(problem: Problem) -> TT:
    """Source of u = prod_l sin(pi x_l) exp(x_l) (vanishes on the boundary)."""
    f = _out(problem, problem.d)
    fs = f._struct()
    check(lib().t2s2_source_manufactured(problem._h, C.byref(fs), _stream()))
    f._read_ranks()
    return f


CROSS_RATIONAL, CROSS_EXP_DIST, CROSS_SIN_LINEAR = 0, 1, 2


def cross(problem: Problem, kind: int, amp: float, aux: float, w: Sequence[float], c: Sequence[float] = None,
          tol: float = 1e-10, r0: int = 2, rmax: int = 64, seed: int = 0):
    """t2s2_source_cross: a non-separable source sampled on the collocation
    grid by TT-cross with MaxVol.  kind 0: amp / (1 + sum w_l (x_l - c_l)^2);
    1: amp exp(-sqrt(aux + sum w_l (x_l - c_l)^2)); 2: amp sin(aux + sum w_l x_l).
    Returns (TT, {"rank", "sample_error"})."""
    d = problem.d
    wv = np.ascontiguousarray(w, dtype=np.float64).reshape(d)
    cv = np.zeros(d) if c is None else np.ascontiguousarray(c, dtype=np.float64).reshape(d)
    par = np.concatenate([[float(amp), float(aux)], wv, cv])
    f = TT.empty(problem.m, int(rmax))
    fs = f._struct()
    rk, err = C.c_int(), C.c_double()
    check(lib().t2s2_source_cross(problem._h, int(kind), par.ctypes.data_as(C.POINTER(C.c_double)), float(tol),
                                  int(r0), int(rmax), C.c_ulonglong(seed), C.byref(fs), C.byref(rk), C.byref(err),
                                  _stream()))
    f._read_ranks()
    return f, {"rank": rk.value, "sample_error": err.value}
