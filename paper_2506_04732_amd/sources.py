"""TT right-hand sides sampled on a problem's collocation grid (input preparation).

Separable sources f(x) = sum_m prod_l g_ml(x_l) have an exact TT of rank equal
to the number of terms (block-diagonal cores); the 1D factors are evaluated at
the collocation nodes returned by the library (t2s2_problem_colloc).  This is
workload construction on the host, not part of the solve.
"""
from __future__ import annotations

from typing import Callable, List, Sequence

import numpy as np

from . import TT, Problem


def separable_cores(factors: List[List[np.ndarray]]) -> List[np.ndarray]:
    """Block-diagonal TT cores of sum_m outer(factors[m][0], ..., factors[m][d-1])."""
    s = len(factors)
    d = len(factors[0])
    cores = []
    for l in range(d):
        n = factors[0][l].size
        if d == 1:
            cores.append(np.sum([f[0] for f in factors], axis=0).reshape(1, n, 1))
            continue
        r0 = 1 if l == 0 else s
        r1 = 1 if l == d - 1 else s
        c = np.zeros((r0, n, r1))
        for m in range(s):
            c[0 if l == 0 else m, :, 0 if l == d - 1 else m] = factors[m][l]
        cores.append(c)
    return cores


def gaussian_factors(problem: Problem, amp, centre, width) -> List[List[np.ndarray]]:
    """f = sum_m amp_m prod_l exp(-(x_l - c_ml)^2 / (2 w_m^2)) on the collocation grid."""
    thetas = [problem.colloc(l) for l in range(problem.d)]
    out = []
    for m in range(len(amp)):
        fac = []
        for l, th in enumerate(thetas):
            v = np.exp(-(th - centre[m][l]) ** 2 / (2.0 * width[m] ** 2))
            fac.append(amp[m] * v if l == 0 else v)
        out.append(fac)
    return out


def sin_exp_factors(problem: Problem) -> List[List[np.ndarray]]:
    """Source of the manufactured solution u = prod_l sin(pi x_l) exp(x_l):
    f = sum_l (-eps phi'' + beta_l phi')(x_l) prod_{k != l} phi(x_k)."""
    thetas = [problem.colloc(l) for l in range(problem.d)]
    pi = np.pi
    phi = lambda t: np.sin(pi * t) * np.exp(t)
    dphi = lambda t: np.exp(t) * (np.sin(pi * t) + pi * np.cos(pi * t))
    d2phi = lambda t: np.exp(t) * ((1 - pi ** 2) * np.sin(pi * t) + 2 * pi * np.cos(pi * t))
    out = []
    for l in range(problem.d):
        out.append([(-problem.eps * d2phi(th) + problem.beta[l] * dphi(th)) if k == l else phi(th)
                    for k, th in enumerate(thetas)])
    return out


def source_tt(problem: Problem, factors: List[List[np.ndarray]], device="cuda") -> TT:
    return TT.from_numpy(separable_cores(factors), device=device)
