"""Pins for the oracle's TT solver: agreement with the full-format solves."""
import numpy as np
import pytest

import workloads
from oracle import amen
from oracle import collocation as col
from oracle import metrics
from oracle import spectral as sp
from oracle import tt


def _system(p):
    ops = col.build_ops(p.d, p.N, p.eps, p.beta, p.scheme)
    Es, Ms = col.interior_factors(ops)
    A = tt.kron_sum_ttm(Es, Ms)
    if p.source == "sin_exp":
        terms = col.manufactured_rhs_factors(ops, p.eps, p.beta)
    else:
        terms = col.gauss_rhs_factors(ops, p.gauss.amp, p.gauss.centre, p.gauss.width)
    return ops, Es, Ms, A, terms


@pytest.mark.parametrize("local_solver", ["auto", "kron"])
def test_amen_2d_manufactured_matches_dense_lu(local_solver):
    p = workloads.manufactured_2d()
    ops, Es, Ms, A, terms = _system(p)
    b = tt.separable_to_tt(terms)
    x, info = amen.solve(A, b, tol=1e-12, target=1e-11, local_solver=local_solver,
                         kron_factors=(Es, Ms), max_sweeps=12)
    u_dense = col.solve_dense(ops, col.separable_full(terms))
    assert metrics.rel_frobenius(col.embed_interior(tt.full(x)), u_dense) < 1e-10
    assert abs(info["residual"] - tt.residual_norm(A, x, b)) < 1e-14
    assert info["residual"] < 1e-11


def test_amen_3d_gauss_matches_schur():
    p = workloads.gauss_problem(3, 12, 2e-3, 4, seed=0, tol=1e-12, rank_cap=12)
    ops, Es, Ms, A, terms = _system(p)
    b = tt.separable_to_tt(terms)
    x, info = amen.solve(A, b, tol=1e-12, target=1e-11, local_solver="kron",
                         kron_factors=(Es, Ms), max_sweeps=15)
    u = col.solve_schur(ops, col.separable_full(terms))
    assert metrics.rel_frobenius(tt.full(x), u) < 1e-10


def test_local_kron_solve_equals_dense_local_solve():
    """The Kronecker-sum local solve equals LU on the assembled local matrix."""
    p = workloads.gauss_problem(3, 8, 1e-2, 2, seed=3, tol=1e-10, rank_cap=8)
    ops, Es, Ms, A, terms = _system(p)
    rng = np.random.default_rng(0)
    x = tt.orthogonalize_right([rng.standard_normal(s) for s in [(1, 6, 3), (3, 6, 4), (4, 6, 1)]])
    q, _ = np.linalg.qr(x[0].reshape(6, 3))
    x0 = q.reshape(1, 6, 3)
    PhiL = amen._left_op(np.ones((1, 1, 1)), x0, A[0], x0)
    PhiR = amen._right_op(np.ones((1, 1, 1)), x[2], A[2], x[2])
    f = rng.standard_normal((3, 6, 4))
    u_kron = amen.local_solve_kron(PhiL, PhiR, Es[1], Ms[1], f)
    u_lu = np.linalg.solve(amen.local_dense(PhiL, A[1], PhiR), f.ravel()).reshape(3, 6, 4)
    np.testing.assert_allclose(u_kron, u_lu, atol=1e-11 * np.abs(u_lu).max())


def test_amen_transport_dominated_is_oscillation_free():
    """Transport-dominated 3D problem with a smooth separable exact solution
    u = prod_l phi_l(x_l) (phi_l: closed form of Eq. adv-diff-1d, boundary
    layers at the outflow faces).  The superconsistent TT solution has the
    exact solution's derivative sign-change count along the mid-axis; plain
    collocation exceeds it (Results, Superconsistent Stabilization)."""
    d, N, eps = 3, 16, 1e-4
    beta = np.array([1.0, 0.7, 0.5])
    out = {}
    for scheme in (sp.SCHEME_SC, sp.SCHEME_PLAIN):
        ops = col.build_ops(d, N, eps, beta, scheme)
        Es, Ms = col.interior_factors(ops)
        A = tt.kron_sum_ttm(Es, Ms)
        terms = [[np.ones(N - 2) if k == l else sp.closed_form_1d(ops[k]["theta"], eps, beta[k])
                  for k in range(d)] for l in range(d)]
        b = tt.separable_to_tt(terms)
        x, info = amen.solve(A, b, tol=1e-10, target=1e-8, local_solver="kron",
                             kron_factors=(Es, Ms), max_sweeps=12)
        out[scheme] = col.embed_interior(tt.full(x))
    expected = metrics.sign_changes(sp.closed_form_1d(np.linspace(-1, 1, 2001), eps, beta[0]))
    assert expected == 1
    assert not metrics.is_oscillatory(out[sp.SCHEME_SC], expected)
    assert metrics.is_oscillatory(out[sp.SCHEME_PLAIN], expected)


def test_kron_sum_dense_matches_interface_assembly_and_spectrum():
    """kron_sum_dense against the assembly from rank-2 interfaces
    (local_dense with the Kronecker-sum TT-matrix core [[I, 0], [K, I]] and
    identity E-blocks), and its spectrum against the closed form: the
    eigenvalues of a Kronecker sum are the sums of the factors' eigenvalues."""
    rng = np.random.default_rng(31)
    KL, K, KR = rng.standard_normal((4, 4)), rng.standard_normal((3, 3)), rng.standard_normal((5, 5))
    PhiL = np.stack([KL, np.eye(4)], axis=1)          # (L-part, E-part)
    PhiR = np.stack([np.eye(5), KR], axis=1)          # (E-part, L-part)
    A = np.zeros((2, 3, 3, 2))
    A[0, :, :, 0] = np.eye(3)
    A[1, :, :, 0] = K
    A[1, :, :, 1] = np.eye(3)
    B = amen.kron_sum_dense(KL, K, KR)
    assert np.max(np.abs(B - amen.local_dense(PhiL, A, PhiR))) <= 1e-14
    sums = (np.linalg.eigvals(KL)[:, None, None] + np.linalg.eigvals(K)[None, :, None]
            + np.linalg.eigvals(KR)[None, None, :]).ravel()
    ev = np.linalg.eigvals(B)
    # every eigenvalue of B is one of the sums (matched greedily)
    rest = list(sums)
    for z in ev:
        k = int(np.argmin(np.abs(np.array(rest) - z)))
        assert abs(rest[k] - z) <= 1e-9 * max(1.0, abs(z))
        rest.pop(k)
