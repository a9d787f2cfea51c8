"""Method-of-lines time stepping of the collocation system (oracle, FP64).

TEST INFRASTRUCTURE ONLY.

Paper passages followed: Overview (the method-of-lines formulation with
backward Euler and Crank-Nicolson beside the space-time one), Eq.
pblm:time:A (du/dt - eps Lap u + beta . grad u + rho u = b), Eq.
ttss-backward-Euler and Eq. ttss-Crank-Nicolson.  Both are theta-schemes,

    (u^{k+1} - u^k) / dt + theta A u^{k+1} + (1 - theta) A u^k = b_step,

theta = 1 (backward Euler) and 1/2 (Crank-Nicolson), A = -eps Lap + beta .
grad + rho.  In collocation form on the interior unknowns (homogeneous
Dirichlet data; u on the GLL grid, rows at the collocation nodes, E the
Lagrange evaluation matrix, L the interior collocation operator of
``collocation.apply_interior``):

    (E + theta dt (L + rho E)) u^{k+1} = (E - (1 - theta) dt (L + rho E)) u^k + dt b_step.

This module assembles both matrices densely and solves by LU: the plain
definition, for tiny grids only.

Pins (tests/test_oracle_mol.py): a tensor-product polynomial of degree <=
N - 1 per dimension (vanishing on the boundary) times (1 + t) is reproduced
exactly by both schemes (the spatial collocation and the time step are both
exact for it); against the exact semi-discrete solution exp(-t E^{-1}(L +
rho E)) u^0 (scipy's expm) the error falls as dt for backward Euler and as
dt^2 for Crank-Nicolson; many backward Euler steps with a constant source
reach the steady solution of ``collocation.solve_schur``.
"""
from __future__ import annotations

from functools import reduce
from typing import Sequence

import numpy as np

from .collocation import interior_factors


def dense_matrices(ops: Sequence[dict]):
    """(E, L): the interior evaluation matrix (x)_l E_l and the interior
    collocation operator sum_l E_1 x .. M_l .. x E_d, both dense."""
    Es, Ms = interior_factors(ops)
    d = len(ops)
    E = reduce(np.kron, Es)
    L = sum(reduce(np.kron, [Ms[k] if k == l else Es[k] for k in range(d)]) for l in range(d))
    return E, L


def theta_step(ops: Sequence[dict], u: np.ndarray, dt: float, theta: float, rho: float = 0.0,
               b_step: np.ndarray = None) -> np.ndarray:
    """One theta-scheme step on the interior values u (shape (N_l - 2)_l)."""
    E, L = dense_matrices(ops)
    A = L + rho * E
    lhs = E + theta * dt * A
    rhs = (E - (1.0 - theta) * dt * A) @ u.reshape(-1)
    if b_step is not None:
        rhs = rhs + dt * np.asarray(b_step, dtype=np.float64).reshape(-1)
    return np.linalg.solve(lhs, rhs).reshape(u.shape)


def march(ops, u0, dt, theta, steps, rho=0.0, source=None):
    """`steps` steps from u0; source(k) -> b_step of step k (or None)."""
    u = np.asarray(u0, dtype=np.float64)
    for k in range(steps):
        u = theta_step(ops, u, dt, theta, rho, None if source is None else source(k))
    return u
