"""Pins for the oracle's 1D ingredients (Overview (i)-(ii), Eq. adv-diff-1d, Fig. 1).

Every check compares against something other than the oracle's own formulas:
closed forms, exact integrals, polynomials evaluated by numpy's Chebyshev and
Legendre classes, or the analytic solution of Eq. adv-diff-1d.
"""
import numpy as np
import pytest
from numpy.polynomial import Chebyshev, Legendre

from oracle import spectral as sp
from oracle import metrics


@pytest.mark.parametrize("n,expected", [
    (2, [0.0]),
    (3, [-1 / np.sqrt(5), 1 / np.sqrt(5)]),
    (4, [-np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7)]),
])
def test_gll_closed_forms(n, expected):
    x = sp.gll_nodes(n)
    assert x[0] == -1.0 and x[-1] == 1.0
    np.testing.assert_allclose(x[1:-1], expected, atol=1e-15)


@pytest.mark.parametrize("n", [3, 7, 16, 31, 47])
def test_gll_interior_are_zeros_of_legendre_derivative(n):
    x = sp.gll_nodes(n)
    dP = Legendre.basis(n).deriv()
    scale = np.abs(dP(np.linspace(-1, 1, 2001))).max()
    assert np.abs(dP(x[1:-1])).max() < 1e-13 * scale
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)


@pytest.mark.parametrize("n", [4, 9, 20])
def test_gll_quadrature_exact_to_degree_2n_minus_1(n):
    x, w = sp.gll_nodes(n), sp.gll_weights(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13
    # degree 2n is not integrated exactly: the discrete norm of P_n is 2/n,
    # the continuous one 2/(2n+1)
    Pn = Legendre.basis(n)(x)
    assert abs(np.dot(w, Pn * Pn) - 2.0 / n) < 1e-13


@pytest.mark.parametrize("n", [5, 12, 31])
def test_gauss_zeros(n):
    z = sp.gauss_nodes(n)
    assert np.abs(Legendre.basis(n)(z)).max() < 1e-13
    assert z.size == n


@pytest.mark.parametrize("n,eps,beta", [(7, 1e-2, 1.0), (15, 1e-4, 0.5), (31, 2e-3, -0.8), (23, 1.0, 0.3)])
def test_lagrange_matrices_exact_on_polynomials(n, eps, beta):
    """E p(x) = p(theta), D1 p(x) = p'(theta), D2 p(x) = p''(theta) for deg p <= n."""
    x = sp.gll_nodes(n)
    th = sp.sc_nodes(n, eps, beta)
    E, D1, D2 = sp.lagrange_matrices(x, th)
    u = np.finfo(float).eps
    for k in range(n + 1):
        p = Chebyshev.basis(k)
        # rounding level: a few hundred ulps of ||D|| ||p(x)|| (an O(1) error means a wrong matrix)
        for D, q in ((E, p), (D1, p.deriv()), (D2, p.deriv(2))):
            tol = 200 * u * (np.abs(D).sum(axis=1).max() * np.abs(p(x)).max() + np.abs(q(th)).max())
            assert np.abs(D @ p(x) - q(th)).max() < tol
    # a degree n+1 polynomial is not reproduced (the bound is sharp)
    p = Chebyshev.basis(n + 1)
    assert np.abs(E @ p(x) - p(th)).max() > 1e-8


def _q(n, eps, beta, t):
    return eps * Legendre.basis(n).deriv()(t) - beta * Legendre.basis(n)(t)


@pytest.mark.parametrize("n", [7, 16, 31])
@pytest.mark.parametrize("eps,beta", [(1e-2, 1.0), (1e-5, 1.0), (3e-1, 0.7), (1e-3, -1.0)])
def test_sc_nodes_interlace_and_solve_q(n, eps, beta):
    th = sp.sc_nodes(n, eps, beta)
    z = sp.gauss_nodes(n)
    assert th.size == n - 1
    assert np.all(th > z[:-1]) and np.all(th < z[1:])
    scale = np.abs(_q(n, eps, beta, np.linspace(-1, 1, 4001))).max()
    assert np.abs(_q(n, eps, beta, th)).max() < 1e-12 * scale


@pytest.mark.parametrize("n", [7, 20])
def test_sc_nodes_limits_and_symmetry(n):
    # diffusion dominated: zeros of P_n'
    np.testing.assert_allclose(sp.sc_nodes(n, 1e9, 1.0), sp.gll_nodes(n)[1:-1], atol=1e-8)
    # convection dominated: z_i + eps/beta
    eps = 1e-9
    th = sp.sc_nodes(n, eps, 1.0)
    np.testing.assert_allclose(th - sp.gauss_nodes(n)[:-1], eps, rtol=1e-3)
    # mirror symmetry in beta
    np.testing.assert_allclose(sp.sc_nodes(n, 1e-3, -0.6), -sp.sc_nodes(n, 1e-3, 0.6)[::-1], atol=1e-14)
    # beta = 0 is plain collocation
    np.testing.assert_allclose(sp.sc_nodes(n, 1e-3, 0.0), sp.gll_nodes(n)[1:-1])


def test_closed_form_satisfies_ode():
    eps, beta = 0.05, 1.0
    x = np.linspace(-0.999, 0.999, 50)
    h = 1e-4
    f = lambda t: sp.closed_form_1d(t, eps, beta)
    d1 = (f(x + h) - f(x - h)) / (2 * h)
    d2 = (f(x + h) - 2 * f(x) + f(x - h)) / h ** 2
    assert np.abs(beta * d1 - eps * d2 - 1.0).max() < 1e-4
    assert abs(f(np.array([-1.0]))[0]) < 1e-15 and abs(f(np.array([1.0]))[0]) < 1e-15


@pytest.mark.parametrize("n", [15, 23])
def test_1d_spectral_accuracy_diffusive(n):
    r = sp.solve_1d(n + 1, 1.0, 1.0, lambda t: np.ones_like(t))
    assert np.abs(r["u"] - sp.closed_form_1d(r["x"], 1.0, 1.0)).max() < 1e-12


@pytest.mark.parametrize("n", [7, 15, 31])
@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_1d_superconsistent_no_oscillation(n, eps):
    """Fig. 1: superconsistent nodes give a monotone-derivative profile like the
    exact solution (one sign change of the differences)."""
    r = sp.solve_1d(n + 1, eps, 1.0, lambda t: np.ones_like(t))
    exact_count = metrics.sign_changes(sp.closed_form_1d(np.linspace(-1, 1, 4001), eps, 1.0))
    assert exact_count == 1
    assert metrics.sign_changes(r["u"]) == exact_count


@pytest.mark.parametrize("n", [15, 31])
def test_1d_plain_collocation_oscillates(n):
    """Fig. 1 (c)-(d): plain collocation oscillates once convection dominates."""
    r = sp.solve_1d(n + 1, 1e-4, 1.0, lambda t: np.ones_like(t), scheme=sp.SCHEME_PLAIN)
    assert metrics.sign_changes(r["u"]) >= n - 2
    # and it is fine when diffusion dominates
    r = sp.solve_1d(n + 1, 1.0, 1.0, lambda t: np.ones_like(t), scheme=sp.SCHEME_PLAIN)
    assert metrics.sign_changes(r["u"]) == 1
