"""How closely two FP64 evaluations of ||b - L x|| / ||b|| can agree.

Two independent FP64 constructions of the collocation operator (the
library's and the oracle's) differ by ~1e-13 relative in D1 and D2 at
N ~ 48: the entries of the Lagrange derivative matrices move by about
N^2 ulp when a node moves by one ulp, so the discrete operator itself is
only defined to that level.  ``node_rounding_gap`` measures, with the oracle
alone, how much the residual of a given TT x changes when every interior GLL
node and every collocation node moves by one ulp (seeded directions):
||(L' - L) x|| / ||b||.  ``evaluation_floor`` is the rounding floor of the
evaluation itself: u times the summed norms of the Kronecker-sum terms of
L x that cancel.
"""
import numpy as np

from oracle import spectral as sp
from oracle import tt as ott


def node_rounding_gap(ops, eps, beta, x, b, seed=0):
    rng = np.random.default_rng(seed)
    Es, Ms, Es2, Ms2 = [], [], [], []
    for l, op in enumerate(ops):
        xg, th = op["x"], op["theta"]
        xg2 = xg.copy()
        xg2[1:-1] = np.nextafter(xg[1:-1], np.where(rng.random(xg.size - 2) < 0.5, -2.0, 2.0))
        th2 = np.nextafter(th, np.where(rng.random(th.size) < 0.5, -2.0, 2.0))
        E2, D12, D22 = sp.lagrange_matrices(xg2, th2)
        Es.append(op["E"][:, 1:-1])
        Ms.append(op["M"][:, 1:-1])
        Es2.append(E2[:, 1:-1])
        Ms2.append((-eps * D22 + float(beta[l]) * D12)[:, 1:-1])
    y1 = ott.matvec(ott.kron_sum_ttm(Es, Ms), x)
    y2 = ott.matvec(ott.kron_sum_ttm(Es2, Ms2), x)
    return ott.norm(ott.add(y1, y2, 1.0, -1.0)) / ott.norm(b)


def evaluation_floor(Es, Ms, x, b):
    terms = 0.0
    for l in range(len(Es)):
        cores = [np.einsum("pi,aib->apb", Ms[k] if k == l else Es[k], x[k]) for k in range(len(Es))]
        terms += ott.norm(cores)
    return np.finfo(np.float64).eps * terms / ott.norm(b)


def agreement_bound(ops, eps, beta, Es, Ms, x, b, rho):
    """|rho_library - rho_oracle| must stay below this: 1e-4 of rho, or 4x the
    node-rounding gap, or 64x the evaluation floor, whichever is largest."""
    return max(1e-4 * rho, 4.0 * node_rounding_gap(ops, eps, beta, x, b), 64.0 * evaluation_floor(Es, Ms, x, b))
