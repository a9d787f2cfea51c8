"""TT-cross approximation of function-generated tensors (oracle, FP64).

TEST INFRASTRUCTURE ONLY.

Paper passage followed: Methods, the closing paragraph on cross
approximation (a TT is computed from a small subset of the tensor's entries,
the rows and columns chosen by the MaxVol algorithm; used for the source
term).  The paper cites the methods (Oseledets & Tyrtyshnikov 2010; Goreinov
et al. 2010) without printing them.  Reading used here:

* ``maxvol(A)``: for a tall n x r matrix, start from the r rows chosen by
  Gaussian elimination with partial pivoting, then repeatedly swap in the row
  i and column j of the largest |B_ij|, B = A A[rows]^{-1}, while it exceeds
  1 + tol (each swap multiplies |det A[rows]| by |B_ij|).
* alternating cross with nested index sets: left sets I_l (multi-indices of
  dimensions < l) and right sets J_l (dimensions > l) of size r_l.  A
  left-to-right half sweep takes at core l the fiber tensor
  C(a, i, b) = f(I_{l-1}[a], i, J_l[b]), its QR factor Q, the MaxVol rows of
  Q (they extend I_{l-1} by one index to I_l) and the core Q Q[rows]^{-1};
  the last core is the fiber tensor itself.  Right-to-left is the mirror
  image.  The result interpolates f on the chosen crosses.
* rank adaptivity: start at rank r0 with random right sets; after each pair
  of half sweeps compare with f on random sample points; if the relative
  error exceeds tol, double the ranks (old index sets kept, random ones
  added), up to rmax.

Pins (tests/test_oracle_cross.py): MaxVol's submatrix dominates (|B| <= 1 +
tol) and its volume is within the r^{r/2} (1 + tol)^r factor of the largest
volume found by brute force; tensors of exact TT rank r (a TT evaluated
entrywise; sin of a linear form, rank 2) are recovered exactly; a smooth
non-separable function is approximated within the requested tolerance on
the full tensor.
"""
from __future__ import annotations

from typing import Callable, List, Sequence

import numpy as np
import scipy.linalg as sla


def maxvol(A: np.ndarray, tol: float = 0.01, max_iters: int = 200) -> np.ndarray:
    n, r = A.shape
    if n <= r:
        return np.arange(n)
    # A = P L U (partial pivoting): row k of P^T A = L U is row argmax_j P[j, k] of A
    P, _, _ = sla.lu(A)
    rows = np.argmax(P, axis=0)[:r].copy()
    B = np.linalg.solve(A[rows].T, A.T).T
    for _ in range(max_iters):
        i, j = np.unravel_index(np.argmax(np.abs(B)), B.shape)
        if abs(B[i, j]) <= 1.0 + tol:
            break
        rows[j] = i
        bj = B[:, j].copy()
        bi = B[i, :].copy()
        bi[j] -= 1.0
        B -= np.outer(bj, bi / B[i, j])
    return rows


def _fiber(fun, grids, left: np.ndarray, l: int, right: np.ndarray) -> np.ndarray:
    """C(a, i, b) = f(left[a], i, right[b]); left: (ra, l) ints, right: (rb, d-l-1) ints."""
    d = len(grids)
    ra, rb, n = left.shape[0], right.shape[0], len(grids[l])
    idx = np.empty((ra, n, rb, d), dtype=np.int64)
    idx[..., :l] = left[:, None, None, :]
    idx[..., l] = np.arange(n)[None, :, None]
    idx[..., l + 1:] = right[None, None, :, :]
    pts = np.stack([grids[k][idx[..., k]] for k in range(d)], axis=-1)
    return fun(pts)


def _feasible(ns, r):
    d = len(ns)
    out = [1]
    for l in range(1, d):
        out.append(int(min(r, np.prod(ns[:l], dtype=np.float64), np.prod(ns[l:], dtype=np.float64))))
    return out + [1]


def cross(fun: Callable, grids: Sequence[np.ndarray], rank: int, sweeps: int = 2, seed: int = 0,
          right_sets: List[np.ndarray] = None) -> List[np.ndarray]:
    """Fixed-rank alternating cross; returns TT cores.  fun maps an array of
    points (..., d) to values (...)."""
    rng = np.random.default_rng(seed)
    d = len(grids)
    ns = [len(g) for g in grids]
    rs = _feasible(ns, rank)
    J = [None] * (d + 1)
    J[d] = np.zeros((1, 0), dtype=np.int64)
    for l in range(d - 1, 0, -1):
        old = right_sets[l] if right_sets is not None and right_sets[l] is not None else np.zeros((0, d - l), np.int64)
        cand = [tuple(v) for v in old]
        seen = set(cand)
        while len(cand) < rs[l]:
            v = tuple(int(rng.integers(0, ns[k])) for k in range(l, d))
            if v not in seen:
                seen.add(v)
                cand.append(v)
        J[l] = np.asarray(cand[:rs[l]], dtype=np.int64).reshape(-1, d - l)
    I = [None] * (d + 1)
    I[0] = np.zeros((1, 0), dtype=np.int64)
    cores = [None] * d
    for half in range(2 * sweeps):
        if half % 2 == 0:
            for l in range(d - 1):
                C = _fiber(fun, grids, I[l], l, J[l + 1])
                ra, n, rb = C.shape
                Q, _ = np.linalg.qr(C.reshape(ra * n, rb))
                rows = maxvol(Q)
                cores[l] = np.linalg.solve(Q[rows].T, Q.T).T.reshape(ra, n, len(rows))
                I[l + 1] = np.concatenate([I[l][rows // n], (rows % n)[:, None]], axis=1)
            cores[d - 1] = _fiber(fun, grids, I[d - 1], d - 1, J[d])
        else:
            for l in range(d - 1, 0, -1):
                C = _fiber(fun, grids, I[l], l, J[l + 1])
                ra, n, rb = C.shape
                Q, _ = np.linalg.qr(C.reshape(ra, n * rb).T)
                cols = maxvol(Q)
                cores[l] = np.linalg.solve(Q[cols].T, Q.T).reshape(len(cols), n, rb)
                J[l] = np.concatenate([(cols // rb)[:, None], J[l + 1][cols % rb]], axis=1)
            cores[0] = _fiber(fun, grids, I[0], 0, J[1])
    return cores


def tt_at(cores, idx: np.ndarray) -> np.ndarray:
    """TT entries at multi-indices idx (S, d)."""
    v = np.ones((idx.shape[0], 1))
    for l, c in enumerate(cores):
        v = np.einsum("sa,sab->sb", v, c[:, idx[:, l], :].transpose(1, 0, 2))
    return v[:, 0]


def cross_adaptive(fun, grids, tol: float, r0: int = 2, rmax: int = 64, samples: int = 1000, seed: int = 0):
    """Double the rank until the relative error on random samples is <= tol."""
    rng = np.random.default_rng(seed + 1)
    d = len(grids)
    idx = np.stack([rng.integers(0, len(g), size=samples) for g in grids], axis=1)
    fv = fun(np.stack([grids[k][idx[:, k]] for k in range(d)], axis=1))
    r = r0
    while True:
        cores = cross(fun, grids, r, seed=seed)
        err = np.linalg.norm(tt_at(cores, idx) - fv) / np.linalg.norm(fv)
        if err <= tol or r >= rmax:
            return cores, {"rank": r, "sample_error": float(err)}
        r = min(2 * r, rmax)
