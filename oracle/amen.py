"""Alternating TT linear solver with residual enrichment (oracle, FP64).

TEST INFRASTRUCTURE ONLY.

Paper passages followed: Results, "Superconsistent Stabilization" (AMEn solves
a local problem per TT core; a direct local solve costs O((r_{l-1} n_l r_l)^3);
the paper calls its sweeps "swaps") and Fig. 6 (residual, rank and compression
per swap; ranks grow each swap until a stationary point).  The paper cites the
AMEn method but does not print it.  Reading used here (one-site AMEn with
residual-based enrichment, alternating sweep directions):

1.  x and an auxiliary residual approximation z (rank ``kick``) start
    right-orthonormal; interfaces (projections of A and b onto the left and
    right bases of x, and of the residual onto the bases of z) are built.
2.  At core l the Galerkin-projected local system
        B u = f,  B = Phi_L (x) A_l (x) Phi_R,  f = Psi_L (x) b_l (x) Psi_R
    is solved exactly: by dense LU of the assembled local matrix
    (``local_solver="dense"``, or ``"auto"`` while r_{l-1} n_l r_l <=
    ``dense_max``), or, for a Kronecker-sum operator, by the complex Schur
    forms of its three factors (``local_solver="kron"``, ``local_solve_kron``).
    A local system too large for dense LU without Kronecker factors is an
    error (no iterative local solver: unpreconditioned GMRES stalls on these
    non-normal systems).
3.  The new core is split by a truncated SVD, delta = tol ||u|| / sqrt(d)
    (Frobenius tail rule), rank <= ``rank_cap``.
4.  Enrichment: the local residual projected onto the old-side basis of x
    and the far-side basis of z (``kick`` columns) is appended to the kept
    singular vectors; a QR restores orthonormality and the coefficients move
    to the neighbouring core.  z's core is the residual projected on z's bases.
5.  Interfaces of x and z are advanced; the direction alternates each sweep.
6.  Stop when the exact TT residual ||b - A x|| / ||b|| (``tt.residual_norm``)
    meets ``target`` and the largest local relative residual seen before the
    local solves of a sweep is below 10 ``tol`` (or, with
    ``stop_on_residual``, on the residual test alone: the stopping rule of
    the GPU solve, which the timing of the same workload uses), or after
    ``max_sweeps``.

What pins it: tests/test_oracle_amen.py checks the result against the
full-format dense LU and Schur solves (agreement to 1e-10 relative at tol
1e-12), and the returned residual against ``tt.residual_norm``.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import tt


# ---- interface updates -------------------------------------------------------
# Left interfaces are indexed [test, (operator bond), trial]; right interfaces
# the same.  "test" cores are x or z (projection basis), "trial" cores are x.

def _left_op(Phi, Y, A, X):
    """Phi'[b', B, b] = sum Phi[a', A, a] Y[a', i', b'] A[A, i', i, B] X[a, i, b]."""
    t = np.tensordot(Phi, X, axes=(2, 0))              # a', A, i, b
    t = np.tensordot(t, A, axes=([1, 2], [0, 2]))      # a', b, i', B
    t = np.tensordot(Y, t, axes=([0, 1], [0, 2]))      # b', b, B
    return t.transpose(0, 2, 1)


def _right_op(Phi, Y, A, X):
    """Phi'[a', A, a] = sum Phi[b', B, b] Y[a', i', b'] A[A, i', i, B] X[a, i, b]."""
    t = np.tensordot(X, Phi, axes=(2, 2))              # a, i, b', B
    t = np.tensordot(A, t, axes=([2, 3], [1, 3]))      # A, i', a, b'
    t = np.tensordot(Y, t, axes=([1, 2], [1, 3]))      # a', A, a
    return t


def _left_vec(Psi, Y, B):
    """Psi'[b', t] = sum Psi[a', s] Y[a', i, b'] B[s, i, t]."""
    t = np.tensordot(Psi, B, axes=(1, 0))              # a', i, t
    return np.tensordot(Y, t, axes=([0, 1], [0, 1]))   # b', t


def _right_vec(Psi, Y, B):
    """Psi'[a', s] = sum Psi[b', t] Y[a', i, b'] B[s, i, t]."""
    t = np.tensordot(B, Psi, axes=(2, 1))              # s, i, b'
    return np.tensordot(Y, t, axes=([1, 2], [1, 2]))   # a', s


# ---- local operator ----------------------------------------------------------

def local_apply(PhiL, A, PhiR, u):
    """y[a', i', b'] = sum PhiL[a', A, a] A[A, i', i, B] PhiR[b', B, b] u[a, i, b]."""
    t = np.tensordot(PhiL, u, axes=(2, 0))             # a', A, i, b
    t = np.tensordot(t, A, axes=([1, 2], [0, 2]))      # a', b, i', B
    t = np.tensordot(t, PhiR, axes=([1, 3], [2, 1]))   # a', i', b'
    return t


def local_rhs(PsiL, B, PsiR):
    t = np.tensordot(PsiL, B, axes=(1, 0))             # a', i, t
    return np.tensordot(t, PsiR, axes=(2, 1))          # a', i, b'


def local_dense(PhiL, A, PhiR):
    r0, n, r1 = PhiL.shape[0], A.shape[1], PhiR.shape[0]
    B = np.einsum("pAa,AijB,qBb->piqajb", PhiL, A, PhiR)
    return B.reshape(r0 * n * r1, r0 * n * r1)


def kron_sum_dense(KL, K, KR):
    """Dense Kronecker sum KL (+) K (+) KR on u[a, i, b] flattened row-major:
    the local operator of the scaled (Kronecker-sum) system at one core, with
    the left and right interfaces KL, KR (Results, stabilisation subsection:
    one local problem per core).  Plain definition, for small sizes."""
    r1, m, r2 = KL.shape[0], K.shape[0], KR.shape[0]
    I1, Im, I2 = np.eye(r1), np.eye(m), np.eye(r2)
    return np.kron(np.kron(KL, Im), I2) + np.kron(np.kron(I1, K), I2) + np.kron(np.kron(I1, Im), KR)


def _split_interface_left(Phi):
    """(L-part, E-part) of a left x-A-x interface; the boundary interface is (0, 1)."""
    if Phi.shape[1] == 1:
        return np.zeros((1, 1)), np.ones((1, 1))
    return Phi[:, 0, :], Phi[:, 1, :]


def _split_interface_right(Phi):
    """(E-part, L-part) of a right x-A-x interface; the boundary interface is (1, 0)."""
    if Phi.shape[1] == 1:
        return np.ones((1, 1)), np.zeros((1, 1))
    return Phi[:, 0, :], Phi[:, 1, :]


def local_solve_kron(PhiL, PhiR, E, M, f):
    """Exact solve of the local system of the rank-2 Kronecker-sum operator.

    With L_L, E_L (left) and E_R, L_R (right) the two blocks of each interface,
    the local operator is L_L (x) E (x) E_R + E_L (x) M (x) E_R + E_L (x) E (x) L_R
    = (E_L (x) E (x) E_R)(K_L (+) K (+) K_R), K_* = E_*^{-1} L_*, K = E^{-1} M.
    The Kronecker sum is solved with complex Schur forms and back substitution
    (same construction as ``collocation.solve_schur``).
    """
    from .collocation import mode_product, _tri_kron_sum_solve
    import scipy.linalg as sla
    LL, EL = _split_interface_left(PhiL)
    ER, LR = _split_interface_right(PhiR)
    g = f.astype(np.complex128)
    Ks = [np.linalg.solve(EL, LL), np.linalg.solve(E, M), np.linalg.solve(ER, LR)]
    g = mode_product(g, np.linalg.inv(EL), 0)
    g = mode_product(g, np.linalg.inv(E), 1)
    g = mode_product(g, np.linalg.inv(ER), 2)
    Qs, Ts = [], []
    for k in range(3):
        T, Q = sla.schur(Ks[k].astype(np.complex128), output="complex")
        Qs.append(Q)
        Ts.append(T)
        g = mode_product(g, Q.conj().T, k)
    y = _tri_kron_sum_solve(Ts, g)
    for k in range(3):
        y = mode_product(y, Qs[k], k)
    return y.real


def _random_tt(rng, ns, r):
    d = len(ns)
    rs = [1] + [r] * (d - 1) + [1]
    return [rng.standard_normal((rs[l], ns[l], rs[l + 1])) for l in range(d)]


def solve(A: Sequence[np.ndarray], b: Sequence[np.ndarray], x0: Optional[Sequence[np.ndarray]] = None,
          tol: float = 1e-10, target: float = 1e-8, max_sweeps: int = 30, kick: int = 4,
          rank_cap: int = 200, dense_max: int = 3000, seed: int = 0, verbose: bool = False,
          local_solver: str = "auto", kron_factors=None, stop_on_residual: bool = False):
    """Solve A x = b in TT format.  Returns (x cores, info dict)."""
    rng = np.random.default_rng(seed)
    d = len(A)
    ns = [c.shape[2] for c in A]
    x = [c.copy() for c in x0] if x0 is not None else _random_tt(rng, ns, 2)
    z = _random_tt(rng, ns, kick)
    x = tt.orthogonalize_right(x)
    z = tt.orthogonalize_right(z)

    one3 = np.ones((1, 1, 1))
    one2 = np.ones((1, 1))
    # interfaces: index l holds the interface between cores l-1 and l (0..d)
    XAX = [None] * (d + 1)
    XB = [None] * (d + 1)
    ZAX = [None] * (d + 1)
    ZB = [None] * (d + 1)
    XAX[0], XB[0], ZAX[0], ZB[0] = one3, one2, one3, one2
    XAX[d], XB[d], ZAX[d], ZB[d] = one3, one2, one3, one2
    for l in range(d - 1, 0, -1):
        XAX[l] = _right_op(XAX[l + 1], x[l], A[l], x[l])
        XB[l] = _right_vec(XB[l + 1], x[l], b[l])
        ZAX[l] = _right_op(ZAX[l + 1], z[l], A[l], x[l])
        ZB[l] = _right_vec(ZB[l + 1], z[l], b[l])

    history = []
    direction = +1
    converged = False
    sweeps = 0
    for sweep in range(max_sweeps):
        sweeps = sweep + 1
        max_res = 0.0
        order = range(d) if direction > 0 else range(d - 1, -1, -1)
        for l in order:
            PhiL, PhiR = XAX[l], XAX[l + 1]
            f = local_rhs(XB[l], b[l], XB[l + 1])
            fn = np.linalg.norm(f)
            u0 = x[l]
            res0 = np.linalg.norm(f - local_apply(PhiL, A[l], PhiR, u0)) / max(fn, 1e-300)
            max_res = max(max_res, res0)
            shape = u0.shape
            size = u0.size
            loc_tol = tol / np.sqrt(d)
            if res0 > loc_tol:
                if local_solver == "kron":
                    u = local_solve_kron(PhiL, PhiR, kron_factors[0][l], kron_factors[1][l], f)
                elif local_solver == "dense" or (local_solver == "auto" and size <= dense_max):
                    u = np.linalg.solve(local_dense(PhiL, A[l], PhiR), f.reshape(-1)).reshape(shape)
                else:
                    raise ValueError(f"local system of size {size} exceeds dense_max = {dense_max}: "
                                     "pass local_solver='kron' with the Kronecker factors")
            else:
                u = u0
            last = (direction > 0 and l == d - 1) or (direction < 0 and l == 0)
            if last:
                x[l] = u
                continue
            r0, n, r1 = shape
            unorm = np.linalg.norm(u)
            delta = tol * unorm / np.sqrt(d)
            if direction > 0:
                U, s, Vt = np.linalg.svd(u.reshape(r0 * n, r1), full_matrices=False)
                r = tt._trunc_rank(s, delta, rank_cap)
                U = U[:, :r]
                W = s[:r, None] * Vt[:r]                       # r x r1
                uk = (U @ W).reshape(r0, n, r1)
                # enrichment: residual with x-basis on the left, z-basis on the right
                kick_core = (local_rhs(XB[l], b[l], ZB[l + 1])
                             - local_apply(XAX[l], A[l], ZAX[l + 1], uk))
                Q, R = np.linalg.qr(np.concatenate([U, kick_core.reshape(r0 * n, -1)], axis=1))
                rn = Q.shape[1]
                x[l] = Q.reshape(r0, n, rn)
                V = R[:, :r] @ W                                 # rn x r1
                x[l + 1] = np.tensordot(V, x[l + 1], axes=(1, 0))
                # z core: residual with z-bases on both sides
                zc = (local_rhs(ZB[l], b[l], ZB[l + 1]) - local_apply(ZAX[l], A[l], ZAX[l + 1], uk))
                zq, _ = np.linalg.qr(zc.reshape(zc.shape[0] * n, -1))
                z[l] = zq.reshape(zc.shape[0], n, zq.shape[1])
                if z[l + 1].shape[0] != zq.shape[1]:
                    z[l + 1] = rng.standard_normal((zq.shape[1], z[l + 1].shape[1], z[l + 1].shape[2]))
                XAX[l + 1] = _left_op(XAX[l], x[l], A[l], x[l])
                XB[l + 1] = _left_vec(XB[l], x[l], b[l])
                ZAX[l + 1] = _left_op(ZAX[l], z[l], A[l], x[l])
                ZB[l + 1] = _left_vec(ZB[l], z[l], b[l])
            else:
                U, s, Vt = np.linalg.svd(u.reshape(r0, n * r1), full_matrices=False)
                r = tt._trunc_rank(s, delta, rank_cap)
                Vt = Vt[:r]
                W = U[:, :r] * s[None, :r]                       # r0 x r
                uk = (W @ Vt).reshape(r0, n, r1)
                kick_core = (local_rhs(ZB[l], b[l], XB[l + 1])
                             - local_apply(ZAX[l], A[l], XAX[l + 1], uk))
                Q, R = np.linalg.qr(np.concatenate([Vt.T, kick_core.reshape(-1, n * r1).T], axis=1))
                rn = Q.shape[1]
                x[l] = Q.T.reshape(rn, n, r1)
                V = W @ R[:, :r].T                               # r0 x rn
                x[l - 1] = np.tensordot(x[l - 1], V, axes=(2, 0))
                zc = (local_rhs(ZB[l], b[l], ZB[l + 1]) - local_apply(ZAX[l], A[l], ZAX[l + 1], uk))
                zq, _ = np.linalg.qr(zc.reshape(-1, n * zc.shape[2]).T)
                z[l] = zq.T.reshape(zq.shape[1], n, zc.shape[2])
                if z[l - 1].shape[2] != zq.shape[1]:
                    z[l - 1] = rng.standard_normal((z[l - 1].shape[0], z[l - 1].shape[1], zq.shape[1]))
                XAX[l] = _right_op(XAX[l + 1], x[l], A[l], x[l])
                XB[l] = _right_vec(XB[l + 1], x[l], b[l])
                ZAX[l] = _right_op(ZAX[l + 1], z[l], A[l], x[l])
                ZB[l] = _right_vec(ZB[l + 1], z[l], b[l])
        res = tt.residual_norm(A, x, b)
        rk = tt.ranks(x)
        history.append({"sweep": sweeps, "max_local_res": max_res, "residual": res, "max_rank": max(rk)})
        if verbose:
            print(history[-1], flush=True)
        direction = -direction
        if max_res < tol and res <= target:
            converged = True
            break
        if res <= target and (max_res < 10 * tol or stop_on_residual):
            converged = True
            break
    return x, {"converged": converged, "sweeps": sweeps, "history": history,
               "residual": history[-1]["residual"], "ranks": tt.ranks(x)}
