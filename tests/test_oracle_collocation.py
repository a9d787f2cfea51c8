"""Pins for the oracle's tensor-product collocation system and full-format solves."""
import numpy as np
import pytest

import workloads
from oracle import collocation as col
from oracle import metrics
from oracle import spectral as sp


def _manufactured(N, d=2):
    p = workloads.manufactured_2d(N)
    beta = p.beta if d == 2 else np.linspace(1.0, 0.4, d)
    ops = col.build_ops(d, N, p.eps, beta)
    f = col.separable_full(col.manufactured_rhs_factors(ops, p.eps, beta))
    grids = np.meshgrid(*[op["x"] for op in ops], indexing="ij")
    exact = np.ones_like(grids[0])
    for g in grids:
        exact = exact * col.sin_exp(g)
    return ops, f, exact


def test_dense_and_schur_agree_and_are_backward_stable():
    ops, f, _ = _manufactured(16)
    u_dense = col.solve_dense(ops, f)
    u_schur = col.embed_interior(col.solve_schur(ops, f))
    assert metrics.rel_frobenius(u_schur, u_dense) < 1e-12
    A = col.assemble_full(ops)
    b = col.full_rhs(ops, f)
    for u in (u_dense, u_schur):
        berr = np.linalg.norm(A @ u.ravel() - b) / (np.linalg.norm(A, 2) * np.linalg.norm(u))
        assert berr < 1e-14


def test_schur_matches_dense_3d_gauss():
    p = workloads.gauss_problem(3, 9, 2e-2, 3, seed=4, tol=1e-12, rank_cap=9)
    ops = col.build_ops(3, 9, p.eps, p.beta)
    f = col.separable_full(col.gauss_rhs_factors(ops, p.gauss.amp, p.gauss.centre, p.gauss.width))
    u_dense = col.solve_dense(ops, f)
    u_schur = col.embed_interior(col.solve_schur(ops, f))
    assert metrics.rel_frobenius(u_schur, u_dense) < 1e-12


def test_apply_interior_equals_assembled_rows():
    ops, _, _ = _manufactured(7, d=3)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((5, 5, 5))
    A = col.assemble_full(ops)
    full_u = np.pad(u, 1)
    lhs = (A @ full_u.ravel()).reshape(7, 7, 7)[1:-1, 1:-1, 1:-1]
    np.testing.assert_allclose(col.apply_interior(ops, u), lhs, atol=1e-11 * np.abs(lhs).max())


def test_manufactured_exponential_convergence():
    errs = {}
    for N in (8, 12, 16, 20):
        ops, f, exact = _manufactured(N)
        errs[N] = metrics.rel_frobenius(col.solve_dense(ops, f), exact)
    assert errs[8] > 1e-4 and errs[12] < 1e-5 and errs[16] < 1e-8 and errs[20] < 1e-12
    assert errs[12] / errs[8] < 1e-2 and errs[16] / errs[12] < 1e-2


def test_one_dimension_reduces_to_1d_solver():
    ops = col.build_ops(1, 12, 1e-3, [1.0])
    f = np.ones(10)
    u = col.solve_dense(ops, f)
    r = sp.solve_1d(12, 1e-3, 1.0, lambda t: np.ones_like(t))
    np.testing.assert_allclose(u, r["u"], atol=1e-12)


def _separable_boundary_layer(d, N, eps, beta, scheme):
    """u = prod_l phi_l(x_l), phi_l the 1D closed form for (eps, beta_l):
    -eps Lap u + beta.grad u = sum_l prod_{k != l} phi_k(x_k), u = 0 on the boundary."""
    ops = col.build_ops(d, N, eps, beta, scheme)
    terms = []
    for l in range(d):
        terms.append([np.ones_like(ops[k]["theta"]) if k == l else
                      sp.closed_form_1d(ops[k]["theta"], eps, beta[k]) for k in range(d)])
    f = col.separable_full(terms)
    grids = np.meshgrid(*[op["x"] for op in ops], indexing="ij")
    exact = np.ones_like(grids[0])
    for k, g in enumerate(grids):
        exact = exact * sp.closed_form_1d(g, eps, beta[k])
    return ops, f, exact


def test_separable_closed_form_is_reproduced_diffusive():
    ops, f, exact = _separable_boundary_layer(3, 18, 0.5, [1.0, 0.5, 0.8], sp.SCHEME_SC)
    assert metrics.rel_frobenius(col.embed_interior(col.solve_schur(ops, f)), exact) < 1e-11


def test_superconsistent_has_no_oscillation_in_2d_transport_regime():
    beta = [1.0, 0.6]
    eps, N = 1e-4, 17
    ops, f, exact = _separable_boundary_layer(2, N, eps, beta, sp.SCHEME_SC)
    u_sc = col.embed_interior(col.solve_schur(ops, f))
    fine = np.linspace(-1, 1, 2001)
    expected = metrics.sign_changes(sp.closed_form_1d(fine, eps, beta[0]))
    assert not metrics.is_oscillatory(u_sc, expected)
    ops_p, f_p, _ = _separable_boundary_layer(2, N, eps, beta, sp.SCHEME_PLAIN)
    u_plain = col.embed_interior(col.solve_schur(ops_p, f_p))
    assert metrics.is_oscillatory(u_plain, expected)


# ---- non-zero Dirichlet data (Eq. pblm:time:B with g != 0) ----------------
import dirichlet_data as dd  # noqa: E402


@pytest.mark.parametrize("d,N", [(1, 9), (2, 8), (3, 6)])
def test_dirichlet_polynomial_reproduced_exactly(d, N):
    # u of degree <= N - 1 per dimension: E, D1, D2 are exact on it, so the
    # collocation solution with g = u on the boundary is u itself
    prob = workloads.dirichlet_problem(d, N, 2e-2, seed=11, kind="poly")
    ops = col.build_ops(d, N, prob.eps, prob.beta)
    f = col.separable_full(dd.rhs_terms(prob, [op["theta"] for op in ops]))
    u_exact = dd.full(dd.boundary_factors(prob, [op["x"] for op in ops]))
    u = col.solve_dense(ops, f, u_exact)
    assert metrics.rel_frobenius(u, u_exact) < 1e-11
    inner = tuple(slice(1, -1) for _ in range(d))
    u_lift = col.solve_schur(ops, col.lift_rhs(ops, f, u_exact))
    assert metrics.rel_frobenius(u_lift, u_exact[inner]) < 1e-11
    # the boundary data matter: solving with g = 0 misses u by O(1)
    assert metrics.rel_frobenius(col.solve_dense(ops, f), u_exact) > 1e-2


def test_dirichlet_lift_and_schur_equal_dense_solve():
    prob = workloads.dirichlet_problem(3, [10, 8, 9], 5e-3, seed=12, kind="exp")
    ops = col.build_ops(3, prob.N, prob.eps, prob.beta)
    f = col.separable_full(dd.rhs_terms(prob, [op["theta"] for op in ops]))
    g = dd.full(dd.boundary_factors(prob, [op["x"] for op in ops]))
    g_noisy = g.copy()
    g_noisy[1:-1, 1:-1, 1:-1] += 1.0          # interior values of g are ignored
    u = col.solve_dense(ops, f, g)
    np.testing.assert_array_equal(col.solve_dense(ops, f, g_noisy), u)
    u_lift = col.solve_schur(ops, col.lift_rhs(ops, f, g_noisy))
    assert metrics.rel_frobenius(u_lift, u[1:-1, 1:-1, 1:-1]) < 1e-11
    # boundary values of the dense solution are g
    assert np.max(np.abs(u[0] - g[0])) < 1e-13 and np.max(np.abs(u[:, :, -1] - g[:, :, -1])) < 1e-13
