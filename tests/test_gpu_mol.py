"""GPU parity of the method-of-lines time steps (t2s2_mol_step; paper: Eq.
ttss-backward-Euler and Eq. ttss-Crank-Nicolson) and of the steady problem
with a reaction term against the oracle's dense steppers and solves.

Bar (FP64): relative L2 distance to the oracle after every step <= 1e-10
(each step solved to residual 1e-13, TT tolerance 1e-13); a linear-in-time
tensor-product polynomial solution is reproduced to 1e-10.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

pytestmark = pytest.mark.gpu

import paper_2506_04732_amd as t2s2  # noqa: E402
from paper_2506_04732_amd import TT  # noqa: E402
from oracle import collocation as col  # noqa: E402
from oracle import metrics  # noqa: E402
from oracle import mol  # noqa: E402
from oracle import tt as ott  # noqa: E402

STEP = dict(tol=1e-13, target=1e-13, max_sweeps=30, kick=4)


def _say(*a):
    print("[case]", *a, flush=True)


def _smooth_start(ops, seed):
    # u0 = sum of 2 separable bumps on the interior GLL nodes (TT rank 2)
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(2):
        c = rng.uniform(-0.4, 0.4, size=len(ops))
        terms.append([np.exp(-((op["x"][1:-1] - c[l]) ** 2) / 0.1) * (1 - op["x"][1:-1] ** 2)
                      for l, op in enumerate(ops)])
    return terms


def _block_tt(terms):
    s, d = len(terms), len(terms[0])
    if d == 1:
        return [sum(np.asarray(t[0], dtype=np.float64) for t in terms).reshape(1, -1, 1)]
    cores = []
    for l in range(d):
        n = len(terms[0][l])
        r0, r1 = (1 if l == 0 else s), (1 if l == d - 1 else s)
        c = np.zeros((r0, n, r1))
        for t in range(s):
            c[0 if l == 0 else t, :, 0 if l == d - 1 else t] = terms[t][l]
        cores.append(c)
    return cores


@pytest.mark.parametrize("theta,d,N", [(1.0, 2, 12), (0.5, 2, 12), (0.5, 3, 10), (1.0, 1, 16)])
def test_mol_steps_match_dense_stepper(theta, d, N):
    eps, rho, dt, steps = 2e-2, 0.3, 0.05, 8
    beta = np.array([1.0, -0.6, 0.4][:d])
    _say("mol", "BE" if theta == 1.0 else "CN", d, N)
    ops = col.build_ops(d, N, eps, beta)
    u0_terms = _smooth_start(ops, 7)
    u_or = col.separable_full(u0_terms)
    p = t2s2.MolProblem(d, N, eps, beta, dt=dt, theta=theta, rho=rho, rank_cap=24)
    u = TT.from_numpy(_block_tt(u0_terms), cap=24)
    for k in range(steps):
        r = p.step(u, **STEP)
        assert r.converged, (k, r.residual)
        u = r.x
        u_or = mol.theta_step(ops, u_or, dt, theta, rho)
        err = metrics.rel_frobenius(ott.full(u.to_numpy()), u_or)
        _say(f"step {k + 1}: rel. L2 error {err:.2e}, residual {r.residual:.2e}, sweeps {r.sweeps}, ranks {r.ranks}")
        assert err <= 1e-10


def test_mol_step_with_source_and_polynomial_exactness():
    # u = (1 + t) phi_1(x_1) phi_2(x_2), phi_l of degree N - 1 vanishing at +-1:
    # both schemes reproduce it exactly; source b_step = theta b(t_{k+1}) + (1 - theta) b(t_k)
    d, N, eps, rho, dt, theta = 2, 9, 5e-2, 0.7, 0.1, 0.5
    beta = np.array([0.8, -0.5])
    rng = np.random.default_rng(3)
    cs = [npleg.legmul(npleg.legsub([1.0], npleg.poly2leg([0, 0, 1])), rng.uniform(-1, 1, size=N - 2))
          for _ in range(d)]
    p = t2s2.MolProblem(d, N, eps, beta, dt=dt, theta=theta, rho=rho, rank_cap=16)
    th = [p.colloc(l) for l in range(d)]
    xi = [t2s2.nodes(N, eps, beta[l])[0][1:-1] for l in range(d)]
    phi = [npleg.legval(th[l], cs[l]) for l in range(d)]
    Aphi = []
    for l in range(d):
        fac = list(phi)
        fac[l] = -eps * npleg.legval(th[l], npleg.legder(cs[l], 2)) + beta[l] * npleg.legval(th[l], npleg.legder(cs[l]))
        Aphi.append(fac)
    Aphi.append([rho * phi[0], phi[1]])

    def b_terms(t):      # b(t) = phi + (1 + t) A phi, as separable terms
        return [list(phi)] + [[(1.0 + t) * f[0], f[1]] for f in Aphi]

    u = TT.from_numpy(_block_tt([[npleg.legval(xi[0], cs[0]), npleg.legval(xi[1], cs[1])]]), cap=16)
    _say("mol polynomial exactness CN")
    for k in range(4):
        bt = [[theta * f[0], f[1]] for f in b_terms((k + 1) * dt)] + \
             [[(1 - theta) * f[0], f[1]] for f in b_terms(k * dt)]
        r = p.step(u, TT.from_numpy(_block_tt(bt)), **STEP)
        assert r.converged
        u = r.x
    exact = (1.0 + 4 * dt) * np.multiply.outer(npleg.legval(xi[0], cs[0]), npleg.legval(xi[1], cs[1]))
    err = metrics.rel_frobenius(ott.full(u.to_numpy()), exact)
    _say(f"rel. L2 error vs exact {err:.2e}")
    assert err <= 1e-10


def test_reaction_steady_solve_matches_dense():
    d, N, eps, rho = 3, 10, 1e-2, 2.5
    beta = np.array([0.7, -0.2, 0.5])
    _say("reaction steady", d, N, rho)
    ops = col.build_ops(d, N, eps, beta)
    E, L = mol.dense_matrices(ops)
    rng = np.random.default_rng(9)
    terms = [[rng.standard_normal(N - 2) for _ in range(d)] for _ in range(2)]
    u = np.linalg.solve(L + rho * E, col.separable_full(terms).reshape(-1)).reshape([N - 2] * d)
    p = t2s2.Problem(d, N, eps, beta, rank_cap=24, rho=rho)
    r = p.solve(TT.from_numpy(_block_tt(terms)), tol=1e-13, target=1e-13, max_sweeps=30, kick=4)
    assert r.converged
    err = metrics.rel_frobenius(ott.full(r.x.to_numpy()), u)
    _say(f"rel. L2 error {err:.2e}")
    assert err <= 1e-10


def test_mol_step_rejects_steady_problem():
    p = t2s2.Problem(2, 8, 1e-2, [1.0, 0.5], rank_cap=8)
    u = TT.from_numpy([np.ones((1, 6, 1)), np.ones((1, 6, 1))])
    with pytest.raises(t2s2.T2S2Error) as e:
        t2s2.MolProblem.step(p, u)
    assert e.value.code == t2s2.T2S2_EINVAL
