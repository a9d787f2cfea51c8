"""Error paths of the C ABI that a caller must be able to see.

* A start x0 that does not fit the problem is rejected with T2S2_EINVAL
  before any device copy (wrong d, wrong mode sizes, ranks above the cap).
* Dense factorisations that stop at their iteration limit (Francis QR of an
  interface or 1D operator, one-sided Jacobi of a truncated SVD) return
  T2S2_EFACTOR.  The limit is lowered from the host
  (t2s2_debug_iteration_limits): the kernels still stop normally.
* The report's refinement-cap count and per-phase device times.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_04732_amd as t2s2  # noqa: E402
import workloads  # noqa: E402
from paper_2506_04732_amd import TT, sources  # noqa: E402


def _say(*a):
    print("[case]", *a, flush=True)


def _problem(cap=24):
    prob = workloads.gauss_problem(3, 16, 5e-3, 3, seed=9, tol=1e-12, rank_cap=cap)
    p = t2s2.Problem(prob.d, prob.N, prob.eps, prob.beta, prob.scheme, rank_cap=cap)
    f = sources.gaussians(p, prob.gauss.amp, prob.gauss.centre, prob.gauss.width)
    return p, f


@pytest.fixture
def limits():
    yield t2s2.debug_iteration_limits
    t2s2.debug_iteration_limits(0, 0)


def test_mismatched_start_is_rejected():
    _say("x0 mismatch")
    p, f = _problem()
    rng = np.random.default_rng(0)
    bad = {
        "wrong d": [rng.standard_normal(s) for s in [(1, 14, 2), (2, 14, 1)]],
        "wrong mode size": [rng.standard_normal(s) for s in [(1, 16, 2), (2, 16, 2), (2, 16, 1)]],
        "rank above cap": [rng.standard_normal(s) for s in [(1, 14, 30), (30, 14, 2), (2, 14, 1)]],
    }
    for name, cores in bad.items():
        with pytest.raises(t2s2.T2S2Error) as e:
            p.solve(f, x0=TT.from_numpy(cores), max_sweeps=2)
        assert e.value.code == t2s2.T2S2_EINVAL, name
    # a fitting start still works
    good = [rng.standard_normal(s) for s in [(1, 14, 2), (2, 14, 2), (2, 14, 1)]]
    r = p.solve(f, x0=TT.from_numpy(good), tol=1e-12, target=1e-11, max_sweeps=20)
    assert r.converged


def test_francis_limit_gives_efactor_in_local_solve_and_solve(limits):
    import torch
    _say("francis limit")
    rng = np.random.default_rng(1)
    r1, m, r2 = 40, 12, 36
    dev = "cuda"
    mk = lambda *s: torch.from_numpy(rng.standard_normal(s)).to(dev)
    Lint, K, Rint, g = mk(r1, r1), mk(m, m), mk(r2, r2), mk(r1, m, r2)
    u = t2s2.local_solve(Lint, K, Rint, g, method=t2s2.LOCAL_EIG)
    assert torch.isfinite(u).all()
    limits(francis_steps=1)
    for method in (t2s2.LOCAL_EIG, t2s2.LOCAL_HESS):
        with pytest.raises(t2s2.T2S2Error) as e:
            t2s2.local_solve(Lint, K, Rint, g, method=method)
        assert e.value.code == t2s2.T2S2_EFACTOR
    with pytest.raises(t2s2.T2S2Error) as e:
        t2s2.Problem(3, 12, 1e-2, [1.0, 0.5, 0.2])    # Schur form of K_l at set-up
    assert e.value.code == t2s2.T2S2_EFACTOR
    limits(0, 0)
    p, f = _problem()
    limits(francis_steps=1)
    with pytest.raises(t2s2.T2S2Error) as e:
        p.solve(f, tol=1e-12, target=1e-11, max_sweeps=4)
    assert e.value.code == t2s2.T2S2_EFACTOR
    limits(0, 0)
    r = p.solve(f, tol=1e-12, target=1e-11, max_sweeps=20)
    assert r.converged


def test_jacobi_limit_gives_efactor_in_rounding(limits):
    _say("jacobi limit")
    p, f = _problem()
    rng = np.random.default_rng(2)
    cores = [rng.standard_normal(s) for s in [(1, 14, 12), (12, 14, 12), (12, 14, 1)]]
    limits(jacobi_sweeps=1)
    with pytest.raises(t2s2.T2S2Error) as e:
        p.tt_round(TT.from_numpy(cores), 1e-8)
    assert e.value.code == t2s2.T2S2_EFACTOR
    limits(0, 0)
    x = p.tt_round(TT.from_numpy(cores), 1e-8)
    assert x.ranks[1] <= 12


def test_report_phases_and_refinement_counts():
    _say("report phases")
    p, f = _problem()
    r = p.solve(f, tol=1e-12, target=1e-11, max_sweeps=20)
    assert r.converged
    ph = r.phase_ms
    assert set(ph) == {"setup", "local_solve", "split", "interfaces", "residual"}
    assert all(v >= 0.0 for v in ph.values()) and ph["local_solve"] > 0 and ph["split"] > 0
    # device time of the phases is the stream's busy time inside the solve
    assert sum(ph.values()) <= r.time_ms * 1.05
    assert 0 <= r.refinement_capped <= r.local_systems
    # the eigenvector bases of the interfaces: ||V|| ||V^-1|| >= cond(V) >= 1
    assert np.isfinite(r.max_eig_cond) and r.max_eig_cond >= 1.0
