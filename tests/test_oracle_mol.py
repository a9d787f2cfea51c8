"""Pins of the oracle's method-of-lines steppers (Eq. ttss-backward-Euler,
Eq. ttss-Crank-Nicolson) on tiny grids."""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import legendre as npleg

from oracle import collocation as col
from oracle import mol


def _ops(d, N, eps, beta):
    return col.build_ops(d, N, eps, beta)


def _poly_factors(rng, N):
    # phi(x) = (1 - x^2) q(x), deg q = N - 3: degree N - 1, zero at +-1
    q = rng.uniform(-1, 1, size=N - 2)
    c = npleg.legmul(npleg.legsub([1.0], npleg.poly2leg([0, 0, 1])), q)
    return c


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_linear_in_time_polynomial_solution_is_exact(theta):
    # u = (1 + t) prod_l phi_l(x_l): du/dt = prod phi, so b(t) = prod phi + (1 + t) A prod phi;
    # the theta step's source is theta b(t_{k+1}) + (1 - theta) b(t_k)
    rng = np.random.default_rng(3)
    d, N, eps, rho, dt = 2, 9, 5e-2, 0.7, 0.1
    beta = np.array([0.8, -0.5])
    ops = _ops(d, N, eps, beta)
    cs = [_poly_factors(rng, N) for _ in range(d)]
    th = [op["theta"] for op in ops]
    xi = [op["x"][1:-1] for op in ops]
    phi_th = [npleg.legval(th[l], cs[l]) for l in range(d)]
    Aphi_terms = []
    for l in range(d):
        fac = [phi_th[k] for k in range(d)]
        fac[l] = -eps * npleg.legval(th[l], npleg.legder(cs[l], 2)) + beta[l] * npleg.legval(th[l], npleg.legder(cs[l]))
        Aphi_terms.append(fac)
    Aphi = col.separable_full(Aphi_terms) + rho * np.multiply.outer(*phi_th)
    P = np.multiply.outer(*phi_th)

    def b(t):
        return P + (1.0 + t) * Aphi

    u_exact = lambda t: (1.0 + t) * np.multiply.outer(*[npleg.legval(xi[l], cs[l]) for l in range(d)])
    steps = 5
    u = mol.march(ops, u_exact(0.0), dt, theta, steps, rho,
                  source=lambda k: theta * b((k + 1) * dt) + (1 - theta) * b(k * dt))
    assert np.linalg.norm(u - u_exact(steps * dt)) <= 1e-11 * np.linalg.norm(u_exact(steps * dt))


@pytest.mark.parametrize("theta,order", [(1.0, 1.0), (0.5, 2.0)])
def test_convergence_order_against_exact_semidiscrete_solution(theta, order):
    d, N, eps, rho = 2, 8, 2e-2, 0.3
    beta = np.array([1.0, 0.4])
    ops = _ops(d, N, eps, beta)
    E, L = mol.dense_matrices(ops)
    K = np.linalg.solve(E, L + rho * E)
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal((N - 2, N - 2))
    T = 0.4
    exact = (sla.expm(-T * K) @ u0.reshape(-1)).reshape(u0.shape)
    errs = []
    for steps in (20, 40, 80):
        u = mol.march(ops, u0, T / steps, theta, steps, rho)
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.15 for r in rates), (errs, rates)


def test_many_backward_euler_steps_reach_the_steady_solution():
    # constant source: u^k -> the steady state of A u = b
    d, N, eps = 2, 10, 5e-2
    beta = np.array([0.6, 0.9])
    ops = _ops(d, N, eps, beta)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((N - 2, N - 2))
    u_ss = col.solve_schur(ops, b)
    u = mol.march(ops, np.zeros_like(b), 5.0, 1.0, 30, 0.0, source=lambda k: b)
    assert np.linalg.norm(u - u_ss) <= 1e-10 * np.linalg.norm(u_ss)
