"""Space-time collocation with variable separable advection (oracle, FP64).

TEST INFRASTRUCTURE ONLY.

Paper passages followed: Overview (the unified space-time formulation
handles time as one more dimension; superconsistency is applied to the
spatial dimensions only), Eq. pblm:time:A-C (du/dt - eps Lap u + beta . grad
u + rho u = b, u = g on the spatial boundary, u(., 0) = f_0).  Readings (the
paper does not print them):

* time t in [0, T] is the reference coordinate s in [-1, 1] mapped by
  t = T (s + 1) / 2, so d/dt = (2 / T) d/ds; the unknowns are the values at
  the GLL nodes s_1 .. s_n (the value at s_0 = -1 is the initial condition)
  and the rows are collocated at the n Gauss points, the zeros of P_n;
* beta_l(x_l) is a Legendre series evaluated at the collocation nodes; the
  spatial node set follows one advection value per dimension (the largest
  |beta_l| over the GLL nodes, with its sign, or positive if beta_l changes
  sign there);
* reaction rho is constant.

The full system on the tensor GLL grid has identity rows u = g wherever a
spatial index is 0 or N - 1 or the time index is 0, and collocation rows
elsewhere; it is assembled densely and solved by LU (tiny grids only).

Pins (tests/test_oracle_spacetime.py): a solution that is a polynomial of
degree <= N_l - 1 in every variable (vanishing on the spatial boundary) is
reproduced exactly with variable beta and rho != 0; with constant beta the
value at t = T agrees with a fine Crank-Nicolson march of ``mol``.
"""
from __future__ import annotations

from functools import reduce
from typing import List, Sequence

import numpy as np
from numpy.polynomial import legendre as npleg

from .spectral import SCHEME_SC, collocation_nodes, gauss_nodes, gll_nodes, lagrange_matrices

SPACE, TIME = 0, 1


def node_advection(coef, x) -> float:
    v = npleg.legval(x, np.asarray(coef, dtype=np.float64))
    if v.max() > 0.0 and v.min() < 0.0:
        return float(np.abs(v).max())
    return float(v[np.argmax(np.abs(v))])


def build_ops(N: Sequence[int], kinds: Sequence[int], eps: float, beta_coefs, T: float = 1.0, rho: float = 0.0,
              scheme: int = SCHEME_SC) -> List[dict]:
    """Per dimension: x (GLL nodes, reference), rows (collocation nodes,
    reference), E and M (rows x N), kind, and the physical row coordinates."""
    d = len(N)
    coefs = iter(beta_coefs)
    ops = []
    for l in range(d):
        n = N[l] - 1
        x = gll_nodes(n)
        if kinds[l] == TIME:
            s = gauss_nodes(n)
            E, D1, _ = lagrange_matrices(x, s)
            M = (2.0 / T) * D1 + (rho / d) * E
            ops.append({"x": x, "rows": s, "E": E, "M": M, "kind": TIME, "phys": 0.5 * T * (s + 1.0),
                        "phys_x": 0.5 * T * (x + 1.0)})
        else:
            c = next(coefs)
            th = collocation_nodes(n, eps, node_advection(c, x), scheme)
            E, D1, D2 = lagrange_matrices(x, th)
            M = -eps * D2 + npleg.legval(th, np.asarray(c, dtype=np.float64))[:, None] * D1 + (rho / d) * E
            ops.append({"x": x, "rows": th, "E": E, "M": M, "kind": SPACE, "phys": th, "phys_x": x})
    return ops


def interior_mask(op) -> np.ndarray:
    N = op["x"].size
    v = np.ones(N)
    v[0] = 0.0
    if op["kind"] == SPACE:
        v[-1] = 0.0
    return v


def assemble_full(ops) -> np.ndarray:
    d = len(ops)
    Es, Ms = [], []
    for op in ops:
        N = op["x"].size
        m = op["E"].shape[0]
        Ef, Mf = np.zeros((N, N)), np.zeros((N, N))
        Ef[1:1 + m] = op["E"]
        Mf[1:1 + m] = op["M"]
        Es.append(Ef)
        Ms.append(Mf)
    A = sum(reduce(np.kron, [Ms[k] if k == l else Es[k] for k in range(d)]) for l in range(d))
    interior = reduce(np.kron, [interior_mask(op) for op in ops])
    A[np.diag_indices_from(A)] += 1.0 - interior
    return A


def solve_dense(ops, f_rows: np.ndarray, g_full: np.ndarray) -> np.ndarray:
    """u on the full grid: f at the collocation rows, g elsewhere."""
    Ns = [op["x"].size for op in ops]
    b = np.array(g_full, dtype=np.float64).reshape(Ns).copy()
    inner = tuple(slice(1, 1 + op["E"].shape[0]) for op in ops)
    b[inner] = f_rows
    return np.linalg.solve(assemble_full(ops), b.reshape(-1)).reshape(Ns)


def unknowns(ops, u_full: np.ndarray) -> np.ndarray:
    """The unknown part of a full-grid tensor (interior space, t > 0)."""
    return u_full[tuple(slice(1, 1 + op["E"].shape[0]) for op in ops)]
