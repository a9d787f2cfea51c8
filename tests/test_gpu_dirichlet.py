"""GPU parity of solves with non-zero Dirichlet data (Eq. pblm:time:B, u = g on
the boundary) against the oracle's dense LU of the full collocation system.

The library lifts the data into the interior right-hand side as a TT sum
(f - L_full g + L g_int, rounded at 1e-14); the oracle assembles the full
N^d x N^d system with identity boundary rows.  Bar: relative L2 distance of
the interior values <= 1e-10 (FP64, TT tolerance 1e-12); for tensor-product
polynomials of degree <= N - 1 also against the exact solution.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import dirichlet_data as dd  # noqa: E402
import paper_2506_04732_amd as t2s2  # noqa: E402
import workloads  # noqa: E402
from paper_2506_04732_amd import TT  # noqa: E402
from oracle import collocation as col  # noqa: E402
from oracle import metrics  # noqa: E402


def _say(*a):
    print("[case]", *a, flush=True)


def _gpu(prob):
    p = t2s2.Problem(prob.d, prob.N, prob.eps, prob.beta, prob.scheme, rank_cap=prob.rank_cap)
    thetas = [p.colloc(l) for l in range(prob.d)]
    gll = [t2s2.nodes(prob.N[l], prob.eps, prob.beta[l], prob.scheme)[0] for l in range(prob.d)]
    f = TT.from_numpy(dd.block_tt(dd.rhs_terms(prob, thetas)))
    g = TT.from_numpy(dd.block_tt([dd.boundary_factors(prob, gll)]))
    return p, f, g


def _oracle(prob):
    ops = col.build_ops(prob.d, prob.N, prob.eps, prob.beta, prob.scheme)
    f = col.separable_full(dd.rhs_terms(prob, [op["theta"] for op in ops]))
    g = dd.full(dd.boundary_factors(prob, [op["x"] for op in ops]))
    return col.solve_dense(ops, f, g), g


CASES = {
    "poly3d": lambda: workloads.dirichlet_problem(3, 8, 2e-2, seed=21, kind="poly", rank_cap=24),
    "exp3d": lambda: workloads.dirichlet_problem(3, 12, 5e-3, seed=22, kind="exp", rank_cap=24),
    "exp2d": lambda: workloads.dirichlet_problem(2, 16, 1e-2, seed=23, kind="exp", rank_cap=16),
    "exp1d": lambda: workloads.dirichlet_problem(1, 20, 1e-3, seed=24, kind="exp", rank_cap=4),
    "ragged": lambda: workloads.dirichlet_problem(4, [7, 10, 5, 8], 1e-2, seed=25, kind="exp", rank_cap=40),
}


@pytest.mark.parametrize("case", list(CASES))
def test_dirichlet_solve_matches_dense_lu(case):
    prob = CASES[case]()
    _say("dirichlet", case, prob.name)
    p, f, g = _gpu(prob)
    r = p.solve(f, g=g, tol=1e-12, target=1e-12, max_sweeps=30, kick=4)
    assert r.converged, (r.residual, r.history_residual)
    u, g_full = _oracle(prob)
    inner = tuple(slice(1, -1) for _ in range(prob.d))
    x = r.x.to_numpy()
    from oracle import tt as ott
    xi = ott.full(x)
    err = metrics.rel_frobenius(xi, u[inner])
    _say(f"rel. L2 error {err:.2e}, residual {r.residual:.2e}, sweeps {r.sweeps}, ranks {r.ranks}")
    assert err <= 1e-10
    if prob.meta["kind"] == "poly":
        assert metrics.rel_frobenius(xi, g_full[inner]) <= 1e-10
    # without the data the solution is a different one
    r0 = p.solve(f, tol=1e-12, target=1e-12, max_sweeps=30, kick=4)
    assert metrics.rel_frobenius(ott.full(r0.x.to_numpy()), u[inner]) > 1e-3


def test_dirichlet_batched_equals_single():
    probs = [CASES["exp3d"](), CASES["ragged"]()]
    _say("dirichlet batched", [q.name for q in probs])
    cap = 40
    for q in probs:
        q.rank_cap = cap
    pfg = [_gpu(q) for q in probs]
    opts = dict(tol=1e-12, target=1e-12, max_sweeps=30, kick=4, overlap=False)
    single = [p.solve(f, g=g, **opts) for p, f, g in pfg]
    batch = t2s2.solve_batched([p for p, _, _ in pfg], [f for _, f, _ in pfg], gs=[g for _, _, g in pfg],
                               workers=2, **opts)
    for s, b in zip(single, batch):
        assert s.converged and b.converged
        assert s.ranks == b.ranks
        for cs, cb in zip(s.x.to_numpy(), b.x.to_numpy()):
            assert np.array_equal(cs, cb)


def test_dirichlet_data_with_wrong_grid_is_rejected():
    prob = CASES["exp3d"]()
    p, f, g = _gpu(prob)
    with pytest.raises(t2s2.T2S2Error) as e:
        p.solve(f, g=f)          # interior-sized cores where GLL-sized ones are needed
    assert e.value.code == t2s2.T2S2_EINVAL
