"""Tensor-product collocation system and full-format solves (oracle, FP64).

TEST INFRASTRUCTURE ONLY.

Paper passages followed:

* Overview (i): the d-dimensional method is the tensor product of the 1D
  discretisations; unknowns are nodal values on the tensor GLL grid.
* Overview (ii)-(iii) and Fig. 3: the superconsistent condition is applied
  independently per dimension, so the collocation grid is Cartesian.
* Eq. advection-diffusion with Eq. pblm:time:B: -eps Lap u + beta . grad u = f
  inside, u = g on the boundary.

Reading of the boundary treatment (the paper never writes the rows out):
rows whose multi-index lies on the boundary of the representation grid are
identity rows u = g; every other row collocates the PDE at the tensor
collocation point (theta_{j_1}, ..., theta_{j_d}):

    sum_l [ (x)_{k<l} E_k ] (x) M_l (x) [ (x)_{k>l} E_k ] u = f(theta_j),

with E_k the Lagrange evaluation matrix and M_l = -eps D2_l + beta_l D1_l of
``spectral.operator_1d``.  With g = 0 only interior columns survive, which
gives the interior system  L_int u_int = f  used by the TT solver.

Solvers:
* ``solve_dense``  -- assembles the full N^d x N^d matrix, numpy LU.
* ``solve_schur``  -- interior system as a Kronecker sum after factoring out
  (x) E_k:  L_int = ((x) E_k)(sum_l I (x) .. K_l .. (x) I),  K_l = E_l^{-1} M_l;
  complex Schur K_l = Q_l T_l Q_l^H, unitary transforms along each mode and
  back substitution on the triangular Kronecker sum.

* ``lift_rhs``     -- with Dirichlet data g != 0 the boundary values are
  known, so the collocation rows applied to them move to the right-hand side:
  b = f - L_rows (g with its interior values set to 0), L_rows the m^d x N^d
  row block on all GLL columns; then ``solve_schur(ops, b)`` gives the
  interior values.

Pins (tests/test_oracle_collocation.py): the two solvers agree and each has a
small backward error; exponential convergence to the manufactured solution;
the 1D special case equals ``spectral.solve_1d``; a d-D product of 1D
closed-form solutions is reproduced (exact separable case); with non-zero
boundary data a tensor-product polynomial of degree <= N-1 per dimension is
reproduced exactly by the dense solve, and lift + Schur equals the dense
solve.
"""
from __future__ import annotations

from functools import reduce
from typing import List, Sequence

import numpy as np
import scipy.linalg as sla

from .spectral import operator_1d, SCHEME_SC


def build_ops(d: int, N, eps: float, beta, scheme: int = SCHEME_SC) -> List[dict]:
    Ns = [int(N)] * d if np.isscalar(N) else [int(v) for v in N]
    beta = np.asarray(beta, dtype=np.float64)
    return [operator_1d(Ns[l], eps, float(beta[l]), scheme) for l in range(d)]


def interior_factors(ops: Sequence[dict]):
    """(E_int, M_int) per dimension: columns of the interior GLL nodes only."""
    return [op["E"][:, 1:-1] for op in ops], [op["M"][:, 1:-1] for op in ops]


def _row_operator(mat_rows: np.ndarray) -> np.ndarray:
    """N x N operator whose interior rows are ``mat_rows`` and boundary rows zero."""
    m, N = mat_rows.shape
    R = np.zeros((N, N))
    R[1:-1, :] = mat_rows
    return R


def assemble_full(ops: Sequence[dict]) -> np.ndarray:
    """Full (prod N) x (prod N) collocation matrix with identity boundary rows."""
    d = len(ops)
    Es = [_row_operator(op["E"]) for op in ops]
    Ms = [_row_operator(op["M"]) for op in ops]
    L = None
    for l in range(d):
        factors = [Ms[k] if k == l else Es[k] for k in range(d)]
        term = reduce(np.kron, factors)
        L = term if L is None else L + term
    interior = reduce(np.kron, [np.r_[0.0, np.ones(op["x"].size - 2), 0.0] for op in ops])
    L[np.diag_indices_from(L)] += (1.0 - interior)
    return L


def full_rhs(ops: Sequence[dict], f_interior: np.ndarray, g_full: np.ndarray = None) -> np.ndarray:
    """Right-hand side of the full system: f on interior rows, g on boundary rows."""
    Ns = [op["x"].size for op in ops]
    b = np.zeros(Ns) if g_full is None else np.array(g_full, dtype=np.float64).reshape(Ns).copy()
    # boundary rows carry g; interior rows are overwritten with f
    inner = tuple(slice(1, -1) for _ in ops)
    b[inner] = f_interior
    return b.reshape(-1)


def solve_dense(ops: Sequence[dict], f_interior: np.ndarray, g_full: np.ndarray = None) -> np.ndarray:
    """Dense LU solve of the full collocation system; returns u on the GLL grid."""
    A = assemble_full(ops)
    b = full_rhs(ops, f_interior, g_full)
    Ns = [op["x"].size for op in ops]
    return np.linalg.solve(A, b).reshape(Ns)


def mode_product(T: np.ndarray, A: np.ndarray, mode: int) -> np.ndarray:
    """Multiply tensor T along ``mode`` by matrix A: out[.., j, ..] = sum_i A[j,i] T[.., i, ..]."""
    Tm = np.moveaxis(T, mode, 0)
    out = np.tensordot(A, Tm, axes=(1, 0))
    return np.moveaxis(out, 0, mode)


def apply_interior(ops: Sequence[dict], u_int: np.ndarray) -> np.ndarray:
    """L_int u_int in full format (mode products, no Kronecker matrix formed)."""
    Es, Ms = interior_factors(ops)
    d = len(ops)
    out = np.zeros([E.shape[0] for E in Es], dtype=np.result_type(u_int, np.float64))
    for l in range(d):
        t = u_int
        for k in range(d):
            t = mode_product(t, Ms[k] if k == l else Es[k], k)
        out = out + t
    return out


def _tri_kron_sum_solve(Ts: List[np.ndarray], rhs: np.ndarray, shift: complex = 0.0) -> np.ndarray:
    """Solve (shift I + sum_l I (x) .. T_l .. (x) I) y = rhs, T_l upper triangular.

    Back substitution along the first mode; each slice is a (d-1)-mode
    problem with its shift increased by the diagonal entry of T_1.
    """
    T = Ts[0]
    m = T.shape[0]
    y = np.zeros_like(rhs)
    if len(Ts) == 1:
        return sla.solve_triangular(T + shift * np.eye(m), rhs, lower=False)
    for i in range(m - 1, -1, -1):
        r = rhs[i] - np.tensordot(T[i, i + 1:], y[i + 1:], axes=(0, 0))
        y[i] = _tri_kron_sum_solve(Ts[1:], r, shift + T[i, i])
    return y


def solve_schur(ops: Sequence[dict], f_interior: np.ndarray) -> np.ndarray:
    """Interior solve with g = 0 via complex Schur forms of K_l = E_l^{-1} M_l."""
    Es, Ms = interior_factors(ops)
    d = len(ops)
    g = np.asarray(f_interior, dtype=np.complex128)
    Qs, Ts = [], []
    for l in range(d):
        g = mode_product(g, np.linalg.inv(Es[l]), l)
        K = np.linalg.solve(Es[l], Ms[l])
        T, Q = sla.schur(K.astype(np.complex128), output="complex")
        Qs.append(Q)
        Ts.append(T)
    for l in range(d):
        g = mode_product(g, Qs[l].conj().T, l)
    y = _tri_kron_sum_solve(Ts, g)
    for l in range(d):
        y = mode_product(y, Qs[l], l)
    return y.real


def lift_rhs(ops: Sequence[dict], f_interior: np.ndarray, g_full: np.ndarray) -> np.ndarray:
    """Interior right-hand side for Dirichlet data g (Eq. pblm:time:B): b = f - L_rows g_b,
    g_b = g with interior values zeroed, L_rows = sum_l E_1 x .. M_l .. x E_d on all GLL columns."""
    gb = np.array(g_full, dtype=np.float64).copy()
    gb[tuple(slice(1, -1) for _ in ops)] = 0.0
    d = len(ops)
    out = None
    for l in range(d):
        t = gb
        for k in range(d):
            t = mode_product(t, ops[k]["M"] if k == l else ops[k]["E"], k)
        out = t if out is None else out + t
    return np.asarray(f_interior, dtype=np.float64) - out


def embed_interior(u_int: np.ndarray) -> np.ndarray:
    """Pad an interior solution with zero boundary values (g = 0)."""
    return np.pad(u_int, 1)


# ---- manufactured and analytic data (Results: manufactured-solution method) ----

def sin_exp(x):
    return np.sin(np.pi * x) * np.exp(x)


def sin_exp_d1(x):
    return np.exp(x) * (np.sin(np.pi * x) + np.pi * np.cos(np.pi * x))


def sin_exp_d2(x):
    return np.exp(x) * ((1.0 - np.pi ** 2) * np.sin(np.pi * x) + 2.0 * np.pi * np.cos(np.pi * x))


def manufactured_rhs_factors(ops: Sequence[dict], eps: float, beta) -> List[List[np.ndarray]]:
    """f = sum_l (-eps phi'' + beta_l phi')(x_l) prod_{k != l} phi(x_k) for phi = sin(pi x) e^x,
    as a list of d separable terms, each a list of d vectors on the collocation grids."""
    d = len(ops)
    terms = []
    for l in range(d):
        fac = []
        for k in range(d):
            t = ops[k]["theta"]
            if k == l:
                fac.append(-eps * sin_exp_d2(t) + beta[l] * sin_exp_d1(t))
            else:
                fac.append(sin_exp(t))
        terms.append(fac)
    return terms


def gauss_rhs_factors(ops: Sequence[dict], amp, centre, width) -> List[List[np.ndarray]]:
    """Separable Gaussian-mixture source sampled on the collocation grids."""
    terms = []
    for m in range(len(amp)):
        fac = []
        for k, op in enumerate(ops):
            v = np.exp(-(op["theta"] - centre[m, k]) ** 2 / (2.0 * width[m] ** 2))
            fac.append(amp[m] * v if k == 0 else v)
        terms.append(fac)
    return terms


def separable_full(terms: List[List[np.ndarray]]) -> np.ndarray:
    """Full tensor sum_terms outer(fac_1, ..., fac_d)."""
    out = None
    for fac in terms:
        t = reduce(np.multiply.outer, fac)
        out = t if out is None else out + t
    return out
