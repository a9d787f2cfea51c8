"""Closed-form data of the separable Dirichlet test problems (workloads.dirichlet_problem).

u = prod_l u_l(x_l) solves -eps Lap u + beta . grad u = f with
f = sum_l (-eps u_l'' + beta_l u_l')(x_l) prod_{k != l} u_k(x_k)  (a sum of d
separable terms) and Dirichlet data g = u on the boundary.  Each side of a
test evaluates these on its own nodes; nothing here belongs to the method.
"""
from functools import reduce

import numpy as np
from numpy.polynomial import legendre as npleg


def factor(prob, l, x, k=0):
    """k-th derivative of u_l at the points x."""
    x = np.asarray(x, dtype=np.float64)
    if prob.meta["kind"] == "poly":
        c = prob.meta["coef"][l]
        return npleg.legval(x, npleg.legder(c, k) if k else c)
    a, b = prob.meta["a"][l], prob.meta["b"][l]
    return b * a ** k * np.exp(a * x)


def rhs_terms(prob, thetas):
    """f as d separable terms, each a list of d vectors on the collocation grids."""
    d = prob.d
    terms = []
    for l in range(d):
        fac = []
        for k in range(d):
            if k == l:
                fac.append(-prob.eps * factor(prob, k, thetas[k], 2) + prob.beta[k] * factor(prob, k, thetas[k], 1))
            else:
                fac.append(factor(prob, k, thetas[k]))
        terms.append(fac)
    return terms


def boundary_factors(prob, gll):
    """u_l at the GLL nodes: g = their outer product (TT rank 1)."""
    return [factor(prob, l, gll[l]) for l in range(prob.d)]


def full(factors):
    return reduce(np.multiply.outer, factors)


def block_tt(terms):
    """Cores of sum_t outer(terms[t]) (block-diagonal, rank = number of terms)."""
    s, d = len(terms), len(terms[0])
    if d == 1:
        return [sum(np.asarray(t[0], dtype=np.float64) for t in terms).reshape(1, -1, 1)]
    cores = []
    for l in range(d):
        n = len(terms[0][l])
        r0, r1 = (1 if l == 0 else s), (1 if l == d - 1 else s)
        c = np.zeros((r0, n, r1))
        for t in range(s):
            c[0 if l == 0 else t, :, 0 if l == d - 1 else t] = terms[t][l]
        cores.append(c)
    return cores
