"""Tensor-train format and TT arithmetic (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Paper passages followed (Methods, "Tensor Train representation"):

* Eq. TT-format:elementwise / TT-format:slice: a d-way tensor is a product of
  cores G_l of size r_{l-1} x n_l x r_l with r_0 = r_d = 1; an entry is the
  product of the selected slices.  Layout here: core l is a C-contiguous
  array ``[r_{l-1}, n_l, r_l]``; full tensors are in C order (i_1 slowest).
* Eq. tt-matrix-format: a TT-matrix has cores L_l of size
  R_{l-1} x n_l x n_l x R_l, stored ``[R_{l-1}, n_row, n_col, R_l]``.
* TT decomposition paragraph: TT-SVD by sequential truncated SVDs of the
  unfoldings; error bounded by eps sqrt(d-1) ||A||_F; exact when ranks equal
  unfolding ranks; quasi-optimal with constant sqrt(d-1).
* Rounding paragraph: rndg(A) with ||A - rndg(A)||_F <= eps ||A||_F.
* Structure-preserving operations: scalar multiple, sum (ranks add),
  TT-matrix times TT (ranks multiply), inner product.

Truncation rule (not printed in the paper): for an unfolding with singular
values s_1 >= s_2 >= ..., keep the smallest r with sqrt(sum_{j>r} s_j^2) <=
delta, at least 1 and at most ``rmax``; delta = eps ||A||_F / sqrt(d-1).  This
is the rule under which the paper's error bounds hold.

Pins (tests/test_oracle_tt.py): the worked slice-product example of Fig. 2,
exact recovery of exact-rank tensors, both error bounds, Eckart-Young in 2D
(the 2D TT-SVD equals the best rank-r approximation), the TT-matrix product
equal to the dense Kronecker matrix-vector product, inner products and norms
against the full tensors.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

Cores = List[np.ndarray]


def ranks(cores: Sequence[np.ndarray]) -> List[int]:
    return [cores[0].shape[0]] + [c.shape[-1] for c in cores]


def full(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Contract a TT vector to its full tensor (n_1, ..., n_d)."""
    out = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])
    shape = [cores[0].shape[1]]
    for c in cores[1:]:
        out = out @ c.reshape(c.shape[0], -1)
        shape.append(c.shape[1])
        out = out.reshape(-1, c.shape[2])
    return out.reshape(shape)


def element(cores: Sequence[np.ndarray], idx: Sequence[int]) -> float:
    """A(i_1..i_d) = G_1(i_1) G_2(i_2) ... G_d(i_d) (product of slice matrices)."""
    v = np.ones((1, 1))
    for c, i in zip(cores, idx):
        v = v @ c[:, i, :]
    return float(v[0, 0])


def _trunc_rank(s: np.ndarray, delta: float, rmax: int) -> int:
    tail = np.sqrt(np.cumsum((s[::-1] ** 2))[::-1])  # tail[k] = ||s[k:]||
    r = s.size
    for k in range(1, s.size + 1):
        t = tail[k] if k < s.size else 0.0
        if t <= delta:
            r = k
            break
    return max(1, min(r, rmax))


def tt_svd(A: np.ndarray, eps: float = 0.0, rmax: int = 10 ** 9) -> Cores:
    """TT-SVD: sequential truncated SVDs of the unfoldings."""
    shape = A.shape
    d = len(shape)
    nrm = np.linalg.norm(A)
    delta = eps * nrm / np.sqrt(max(d - 1, 1))
    cores = []
    C = A.reshape(1, -1)
    r_prev = 1
    for l in range(d - 1):
        C = C.reshape(r_prev * shape[l], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        r = _trunc_rank(s, delta, rmax)
        cores.append(U[:, :r].reshape(r_prev, shape[l], r))
        C = s[:r, None] * Vt[:r]
        r_prev = r
    cores.append(C.reshape(r_prev, shape[-1], 1))
    return cores


def orthogonalize_right(cores: Sequence[np.ndarray]) -> Cores:
    """Right-to-left QR sweep: cores 2..d become right-orthonormal."""
    cores = [c.copy() for c in cores]
    for l in range(len(cores) - 1, 0, -1):
        r0, n, r1 = cores[l].shape
        Q, R = np.linalg.qr(cores[l].reshape(r0, n * r1).T)
        k = Q.shape[1]
        cores[l] = Q.T.reshape(k, n, r1)
        cores[l - 1] = np.tensordot(cores[l - 1], R.T, axes=(2, 0))
    return cores


def orthogonalize_left(cores: Sequence[np.ndarray]) -> Cores:
    """Left-to-right QR sweep: cores 1..d-1 become left-orthonormal."""
    cores = [c.copy() for c in cores]
    for l in range(len(cores) - 1):
        r0, n, r1 = cores[l].shape
        Q, R = np.linalg.qr(cores[l].reshape(r0 * n, r1))
        k = Q.shape[1]
        cores[l] = Q.reshape(r0, n, k)
        cores[l + 1] = np.tensordot(R, cores[l + 1], axes=(1, 0))
    return cores


def norm(cores: Sequence[np.ndarray]) -> float:
    """Frobenius norm via left orthogonalisation (norm of the last core)."""
    oc = orthogonalize_left(cores)
    return float(np.linalg.norm(oc[-1]))


def round_tt(cores: Sequence[np.ndarray], eps: float, rmax: int = 10 ** 9) -> Cores:
    """rndg: right-to-left orthogonalisation, then left-to-right truncated SVDs
    with delta = eps ||A||_F / sqrt(d-1)."""
    d = len(cores)
    oc = orthogonalize_right(cores)
    nrm = np.linalg.norm(oc[0])
    delta = eps * nrm / np.sqrt(max(d - 1, 1))
    for l in range(d - 1):
        r0, n, r1 = oc[l].shape
        U, s, Vt = np.linalg.svd(oc[l].reshape(r0 * n, r1), full_matrices=False)
        r = _trunc_rank(s, delta, rmax)
        oc[l] = U[:, :r].reshape(r0, n, r)
        oc[l + 1] = np.tensordot(s[:r, None] * Vt[:r], oc[l + 1], axes=(1, 0))
    return oc


def add(x: Sequence[np.ndarray], y: Sequence[np.ndarray], alpha: float = 1.0, beta: float = 1.0) -> Cores:
    """alpha x + beta y by block concatenation of cores (ranks add)."""
    d = len(x)
    out = []
    for l in range(d):
        a, b = x[l], y[l]
        if l == 0:
            a, b = alpha * a, beta * b
        if d == 1:
            out.append(a + b)
        elif l == 0:
            out.append(np.concatenate([a, b], axis=2))
        elif l == d - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            c = np.zeros((a.shape[0] + b.shape[0], a.shape[1], a.shape[2] + b.shape[2]))
            c[:a.shape[0], :, :a.shape[2]] = a
            c[a.shape[0]:, :, a.shape[2]:] = b
            out.append(c)
    return out


def dot(x: Sequence[np.ndarray], y: Sequence[np.ndarray]) -> float:
    """<x, y> by sweeping the 2-index environment from left to right."""
    env = np.ones((1, 1))
    for a, b in zip(x, y):
        t = np.tensordot(env, a, axes=(0, 0))          # (ry, n, rx')
        env = np.tensordot(t, b, axes=([0, 1], [0, 1]))  # (rx', ry')
    return float(env[0, 0])


def rel_diff(x: Sequence[np.ndarray], y: Sequence[np.ndarray]) -> float:
    """||x - y|| / ||y|| via the concatenated TT (no Gram expansion)."""
    return norm(add(x, y, 1.0, -1.0)) / norm(y)


def separable_to_tt(terms: List[List[np.ndarray]]) -> Cores:
    """Exact TT of sum_m outer(v_m1, ..., v_md): block-diagonal cores of rank = #terms."""
    s = len(terms)
    d = len(terms[0])
    cores = []
    for l in range(d):
        n = terms[0][l].size
        if d == 1:
            cores.append(sum(t[0] for t in terms).reshape(1, n, 1))
        elif l == 0:
            c = np.zeros((1, n, s))
            for m in range(s):
                c[0, :, m] = terms[m][l]
            cores.append(c)
        elif l == d - 1:
            c = np.zeros((s, n, 1))
            for m in range(s):
                c[m, :, 0] = terms[m][l]
            cores.append(c)
        else:
            c = np.zeros((s, n, s))
            for m in range(s):
                c[m, :, m] = terms[m][l]
            cores.append(c)
    return cores


# ---------------------------------------------------------------- TT-matrices

def kron_sum_ttm(Es: Sequence[np.ndarray], Ms: Sequence[np.ndarray]) -> Cores:
    """Rank-2 TT-matrix of sum_l E_1 (x) .. (x) M_l (x) .. (x) E_d (Eq. tt-matrix-format).

    Bond state 0 = "the M factor has been placed to the left", 1 = "not yet".
    First core [M_1, E_1], middle cores [[E, 0], [M, E]], last core [E_d; M_d].
    """
    d = len(Es)
    cores = []
    for l in range(d):
        E, M = Es[l], Ms[l]
        n0, n1 = E.shape
        if d == 1:
            c = M.reshape(1, n0, n1, 1).copy()
        elif l == 0:
            c = np.zeros((1, n0, n1, 2))
            c[0, :, :, 0] = M
            c[0, :, :, 1] = E
        elif l == d - 1:
            c = np.zeros((2, n0, n1, 1))
            c[0, :, :, 0] = E
            c[1, :, :, 0] = M
        else:
            c = np.zeros((2, n0, n1, 2))
            c[0, :, :, 0] = E
            c[1, :, :, 0] = M
            c[1, :, :, 1] = E
        cores.append(c)
    return cores


def ttm_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Dense matrix of a TT-matrix (rows: output multi-index, C order)."""
    out = np.ones((1, 1, 1))  # (rows, cols, R)
    for c in cores:
        R0, n0, n1, R1 = c.shape
        t = np.tensordot(out, c, axes=(2, 0))       # (rows, cols, n0, n1, R1)
        t = t.transpose(0, 2, 1, 3, 4)              # (rows, n0, cols, n1, R1)
        out = t.reshape(out.shape[0] * n0, out.shape[1] * n1, R1)
    return out[:, :, 0]


def matvec(A: Sequence[np.ndarray], x: Sequence[np.ndarray]) -> Cores:
    """y = A x in TT: Y_l[(a,alpha), i', (b,beta)] = sum_i A_l[a,i',i,b] X_l[alpha,i,beta]."""
    out = []
    for Ac, Xc in zip(A, x):
        R0, n0, n1, R1 = Ac.shape
        r0, _, r1 = Xc.shape
        y = np.einsum("apib,xiy->axpby", Ac, Xc)
        out.append(y.reshape(R0 * r0, n0, R1 * r1))
    return out


def residual_norm(A: Sequence[np.ndarray], x: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    """||b - A x||_2 / ||b||_2 in exact TT arithmetic (concatenation + orthogonalisation)."""
    r = add(b, matvec(A, x), 1.0, -1.0)
    return norm(r) / norm(b)


def compression_ratio(cores: Sequence[np.ndarray]) -> float:
    """TT storage / full storage (Results: compression ratio)."""
    return float(sum(c.size for c in cores)) / float(np.prod([c.shape[1] for c in cores], dtype=np.float64))
