"""Pins of the oracle's space-time collocation (variable separable advection)."""
from functools import reduce

import numpy as np
from numpy.polynomial import legendre as npleg

from oracle import collocation as col
from oracle import metrics
from oracle import mol
from oracle import spacetime as st

VANISH = npleg.legsub([1.0], npleg.poly2leg([0, 0, 1]))       # 1 - x^2


def _poly_case(rng, N, kinds, eps, betas, T, rho):
    """u = prod over dimensions of a polynomial of degree <= N_l - 1 (space:
    vanishing at +-1); f and g of it.  Returns (ops, f_rows, g_full, u_full)."""
    ops = st.build_ops(N, kinds, eps, betas, T, rho)
    d = len(N)
    fac, der1, der2, vals_x = [], [], [], []
    for l, op in enumerate(ops):
        if op["kind"] == st.TIME:
            c = rng.uniform(-1, 1, size=N[l])             # polynomial in s, degree N - 1
            fac.append(npleg.legval(op["rows"], c))
            der1.append(npleg.legval(op["rows"], npleg.legder(c)) * 2.0 / T)
            der2.append(None)
            vals_x.append(npleg.legval(op["x"], c))
        else:
            c = npleg.legmul(VANISH, rng.uniform(-1, 1, size=N[l] - 2))
            fac.append(npleg.legval(op["rows"], c))
            der1.append(npleg.legval(op["rows"], npleg.legder(c)))
            der2.append(npleg.legval(op["rows"], npleg.legder(c, 2)))
            vals_x.append(npleg.legval(op["x"], c))
    f = 0.0
    bi = iter(betas)
    for l, op in enumerate(ops):
        if op["kind"] == st.TIME:
            term = der1[l]
        else:
            b = npleg.legval(op["rows"], np.asarray(next(bi)))
            term = -eps * der2[l] + b * der1[l]
        f = f + reduce(np.multiply.outer, [term if k == l else fac[k] for k in range(d)])
    f = f + rho * reduce(np.multiply.outer, fac)
    u = reduce(np.multiply.outer, vals_x)
    return ops, f, u, u


def test_polynomial_solution_reproduced_with_variable_beta():
    rng = np.random.default_rng(21)
    N, kinds = [9, 7, 8], [st.SPACE, st.SPACE, st.TIME]
    betas = [[0.4, 0.6, 0.3], [-0.2, 0.9]]              # beta_1 changes sign, beta_2 does not
    ops, f, g, u = _poly_case(rng, N, kinds, 3e-2, betas, T=0.7, rho=0.5)
    uh = st.solve_dense(ops, f, g)
    assert metrics.rel_frobenius(uh, u) < 1e-11
    # the data matter: a wrong time scale breaks it
    ops2 = st.build_ops(N, kinds, 3e-2, betas, T=1.4, rho=0.5)
    assert metrics.rel_frobenius(st.solve_dense(ops2, f, g), u) > 1e-3


def test_space_time_matches_fine_crank_nicolson():
    # constant beta: u(T) of the space-time solve vs 800 Crank-Nicolson steps
    N, Nt, eps, T = 10, 14, 5e-2, 0.5
    beta = [0.8, -0.4]
    ops = st.build_ops([N, N, Nt], [st.SPACE, st.SPACE, st.TIME], eps, [[beta[0]], [beta[1]]], T)
    cops = col.build_ops(2, N, eps, beta)
    x = [op["x"] for op in cops]
    u0 = np.multiply.outer(np.exp(-4 * (x[0] - 0.2) ** 2) * (1 - x[0] ** 2),
                           np.exp(-3 * (x[1] + 0.1) ** 2) * (1 - x[1] ** 2))
    g = np.multiply.outer(u0, np.ones(Nt))
    u = st.solve_dense(ops, np.zeros((N - 2, N - 2, Nt - 1)), g)
    uT = u[:, :, -1][1:-1, 1:-1]
    steps = 800
    uc = mol.march(cops, u0[1:-1, 1:-1], T / steps, 0.5, steps)
    assert metrics.rel_frobenius(uT, uc) < 1e-6
