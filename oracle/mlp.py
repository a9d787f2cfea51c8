"""FP64 reference of the learned warm start's network and loss (test infrastructure).

Only tests/, the graft entry's smoke check and bench.py's cpu_baseline leg
use this module; the library never does.

The paper trains nothing: the network is a systems addition that maps an
instance's parameters to initial TT cores (the TT format of Methods,
Eq. TT-format:elementwise).  Definitions written out here:

* Multilayer perceptron with widths w_0 .. w_L: H_0 = X (batch x w_0),
  Z_k = H_k W_k^T + b_k, H_{k+1} = tanh(Z_k) for k < L - 1, output
  Y = Z_{L-1} (linear).  Parameters are one flat vector holding, per layer,
  W_k (w_{k+1} x w_k, row-major) then b_k (w_{k+1}).
* Backward pass by the chain rule: with G = dLoss/dY,
  dW_k = G_k^T H_k, db_k = column sums of G_k, G_{k-1} = (G_k W_k) * (1 - H_k^2).
* TT fitting loss of one sample: the output vector is read as TT cores of
  uniform interior rank r (core l is [r_{l-1}][n_l][r_l], boundary ranks 1,
  cores stored one after another), P the predicted and T the target TT:
      loss = ||P - T||^2 / ||T||^2 = (<P,P> - 2 <P,T> + <T,T>) / <T,T>,
  which depends only on the represented tensors, not on the cores' gauge
  (the TT representation is not unique, Methods).  The inner products are
  the left-to-right contractions of the TT format; the gradient with respect
  to core l contracts the left and right environments of the other cores.
* Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


# ------------------------------------------------------------------ network
def param_count(widths: Sequence[int]) -> int:
    return int(sum(widths[k + 1] * widths[k] + widths[k + 1] for k in range(len(widths) - 1)))


def unpack(params: np.ndarray, widths: Sequence[int]) -> List[Tuple[np.ndarray, np.ndarray]]:
    out, o = [], 0
    for k in range(len(widths) - 1):
        wi, wo = widths[k], widths[k + 1]
        W = params[o:o + wo * wi].reshape(wo, wi)
        o += wo * wi
        b = params[o:o + wo]
        o += wo
        out.append((W, b))
    return out


def forward(params: np.ndarray, widths: Sequence[int], X: np.ndarray):
    """Returns Y and the list of layer inputs H_0 .. H_{L-1}."""
    layers = unpack(params, widths)
    H = [np.asarray(X, dtype=np.float64)]
    for k, (W, b) in enumerate(layers):
        Z = H[-1] @ W.T + b
        if k < len(layers) - 1:
            H.append(np.tanh(Z))
        else:
            return Z, H
    raise ValueError("need at least one layer")


def backward(params: np.ndarray, widths: Sequence[int], H: List[np.ndarray], dY: np.ndarray) -> np.ndarray:
    """Gradient of sum(dY * Y) with respect to the flat parameter vector."""
    layers = unpack(params, widths)
    grads = [None] * len(layers)
    G = np.asarray(dY, dtype=np.float64)
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        grads[k] = (G.T @ H[k], G.sum(axis=0))
        if k > 0:
            G = (G @ W) * (1.0 - H[k] ** 2)
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def adam(params, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ TT loss
def core_shapes(n: Sequence[int], r: int) -> List[Tuple[int, int, int]]:
    d = len(n)
    ranks = [1] + [r] * (d - 1) + [1]
    return [(ranks[l], n[l], ranks[l + 1]) for l in range(d)]


def output_size(n: Sequence[int], r: int) -> int:
    return int(sum(a * b * c for a, b, c in core_shapes(n, r)))


def split_cores(y: np.ndarray, n: Sequence[int], r: int) -> List[np.ndarray]:
    out, o = [], 0
    for sh in core_shapes(n, r):
        sz = sh[0] * sh[1] * sh[2]
        out.append(np.asarray(y[o:o + sz], dtype=np.float64).reshape(sh))
        o += sz
    return out


def _left_envs(A: List[np.ndarray], B: List[np.ndarray]) -> List[np.ndarray]:
    """E_0 = 1, E_{l+1}[b, c] = sum_{a, a', i} A_l[a, i, b] E_l[a, a'] B_l[a', i, c]."""
    E = [np.ones((1, 1))]
    for a, b in zip(A, B):
        E.append(np.einsum("aib,ac,cid->bd", a, E[-1], b))
    return E


def _right_envs(A: List[np.ndarray], B: List[np.ndarray]) -> List[np.ndarray]:
    """F_d = 1, F_l[a, c] = sum_{b, b', i} A_l[a, i, b] F_{l+1}[b, b'] B_l[c, i, b']."""
    d = len(A)
    F = [None] * (d + 1)
    F[d] = np.ones((1, 1))
    for l in range(d - 1, -1, -1):
        F[l] = np.einsum("aib,bd,cid->ac", A[l], F[l + 1], B[l])
    return F


def inner(A: List[np.ndarray], B: List[np.ndarray]) -> float:
    return float(_left_envs(A, B)[-1][0, 0])


def tt_fit_loss(y: np.ndarray, target: np.ndarray, n: Sequence[int], r: int):
    """(loss, dloss/dy) of one sample; y and target are flat core vectors."""
    P = split_cores(y, n, r)
    T = split_cores(target, n, r)
    Lpp, Rpp = _left_envs(P, P), _right_envs(P, P)
    Lpt, Rpt = _left_envs(P, T), _right_envs(P, T)
    pp, pt, tt = Lpp[-1][0, 0], Lpt[-1][0, 0], _left_envs(T, T)[-1][0, 0]
    loss = (pp - 2.0 * pt + tt) / tt
    grads = []
    for l in range(len(P)):
        g_pp = 2.0 * np.einsum("ac,cid,bd->aib", Lpp[l], P[l], Rpp[l + 1])
        g_pt = np.einsum("ac,cid,bd->aib", Lpt[l], T[l], Rpt[l + 1])
        grads.append(((g_pp - 2.0 * g_pt) / tt).ravel())
    return float(loss), np.concatenate(grads)
