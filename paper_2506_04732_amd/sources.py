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
