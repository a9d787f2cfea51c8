"""Plain collocation vs superconsistent collocation (Results: Superconsistent
Stabilization; the stability map of NEXT 4) on the GPU path.

The transport-dominated problem with the separable exact solution
u = prod_l phi_l(x_l), phi_l the closed form of beta_l phi' - eps phi'' = 1
(boundary layers at the outflow faces): f = sum_l prod_{k != l} phi_k.  The
oscillation count is the number of sign changes of the nodal differences
along the line through the grid centre in direction 1 (reading c13), taken
from the library's TT fiber (t2s2_tt_fiber).

* 3D N = 16: the GPU fiber equals the oracle's full-format (complex Schur)
  solution on that line to 1e-10 of its maximum, for both schemes, and so do
  the counts; the superconsistent count is the exact one (1), the plain one
  exceeds it.
* 6D points of the map (measured: superconsistent 0 of 30 grid points
  oscillatory, plain 19 of 30): a resolved point where neither oscillates and
  a transport-dominated point where only plain collocation does.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import paper_2506_04732_amd as t2s2  # noqa: E402
from paper_2506_04732_amd import TT  # noqa: E402
from oracle import collocation as col  # noqa: E402
from oracle import metrics  # noqa: E402
from oracle import spectral as sp  # noqa: E402


def _say(*a):
    print("[case]", *a, flush=True)


def _source_tt(p, d, N, eps, beta):
    th = [p.colloc(l) for l in range(d)]
    phis = [sp.closed_form_1d(th[l], eps, beta[l]) for l in range(d)]
    terms = [[np.ones(N - 2) if k == l else phis[k] for k in range(d)] for l in range(d)]
    cores = []
    for l in range(d):
        r0, r1 = (1 if l == 0 else d), (1 if l == d - 1 else d)
        c = np.zeros((r0, N - 2, r1))
        for t in range(d):
            c[0 if l == 0 else t, :, 0 if l == d - 1 else t] = terms[t][l]
        cores.append(c)
    return TT.from_numpy(cores), terms


def _line(p, x, d, N):
    return np.concatenate([[0.0], p.tt_fiber(x, 0, [N // 2 - 1] * d), [0.0]])


@pytest.mark.parametrize("scheme", [sp.SCHEME_SC, sp.SCHEME_PLAIN])
def test_3d_line_and_count_match_oracle(scheme):
    d, N, eps = 3, 16, 1e-4
    beta = np.array([1.0, 0.7, 0.5])
    _say("3D line", "SC" if scheme == sp.SCHEME_SC else "plain")
    p = t2s2.Problem(d, N, eps, beta, scheme, rank_cap=200)
    f, _ = _source_tt(p, d, N, eps, beta)
    r = p.solve(f, tol=1e-13, target=1e-12, max_sweeps=30, kick=8)
    assert r.converged, (r.residual, r.ranks)
    ops = col.build_ops(d, N, eps, beta, scheme)
    terms = [[np.ones(N - 2) if k == l else sp.closed_form_1d(ops[k]["theta"], eps, beta[k]) for k in range(d)]
             for l in range(d)]
    u = col.embed_interior(col.solve_schur(ops, col.separable_full(terms)))
    line_or = metrics.mid_axis_profile(u, 0)
    line = _line(p, r.x, d, N)
    dev = np.max(np.abs(line - line_or)) / np.max(np.abs(line_or))
    cnt, cnt_or = metrics.sign_changes(line), metrics.sign_changes(line_or)
    _say(f"line deviation {dev:.2e}, counts GPU {cnt} oracle {cnt_or}")
    assert dev <= 1e-10
    assert cnt == cnt_or
    exact = metrics.sign_changes(sp.closed_form_1d(np.linspace(-1, 1, 2001), eps, beta[0]))
    assert exact == 1
    if scheme == sp.SCHEME_SC:
        assert cnt == exact
    else:
        assert cnt > exact


@pytest.mark.parametrize("N,ratio,plain_oscillates", [(12, 1e-2, False), (24, 1e-3, True)])
def test_6d_map_points(N, ratio, plain_oscillates):
    d, eps = 6, 2.0 * ratio
    beta = np.full(d, 1.0 / np.sqrt(d))
    counts = {}
    for scheme in (sp.SCHEME_SC, sp.SCHEME_PLAIN):
        _say("6D map", N, ratio, "SC" if scheme == sp.SCHEME_SC else "plain")
        p = t2s2.Problem(d, N, eps, beta, scheme, rank_cap=64)
        f, _ = _source_tt(p, d, N, eps, beta)
        r = p.solve(f, tol=1e-10, target=1e-8, max_sweeps=20, kick=4, init_rank=4)
        assert r.converged, (r.residual, r.ranks)
        counts[scheme] = metrics.sign_changes(_line(p, r.x, d, N))
        _say(f"count {counts[scheme]}, ranks {r.ranks}")
    assert counts[sp.SCHEME_SC] == 1
    assert (counts[sp.SCHEME_PLAIN] > 1) == plain_oscillates
