"""Pins of the oracle's MaxVol and TT-cross (Methods, cross-approximation paragraph)."""
from functools import reduce
from itertools import combinations

import numpy as np
import pytest

from oracle import cross
from oracle import tt as ott


def test_maxvol_dominance_and_brute_force_volume():
    rng = np.random.default_rng(1)
    for n, r in [(8, 2), (9, 3), (12, 4)]:
        A = rng.standard_normal((n, r))
        rows = cross.maxvol(A, tol=0.01)
        assert len(set(rows.tolist())) == r
        B = np.linalg.solve(A[rows].T, A.T).T
        assert np.abs(B).max() <= 1.01 + 1e-12
        np.testing.assert_allclose(B[rows], np.eye(r), atol=1e-12)
        vol = abs(np.linalg.det(A[list(rows)]))
        best = max(abs(np.linalg.det(A[list(c)])) for c in combinations(range(n), r))
        assert vol <= best * (1 + 1e-12)
        assert vol >= best / (r ** (r / 2) * 1.01 ** r)


def test_exact_rank_tensor_from_tt_is_recovered():
    rng = np.random.default_rng(2)
    ns, ranks = [6, 7, 5, 6], [1, 3, 4, 2, 1]
    T = [rng.standard_normal((ranks[l], ns[l], ranks[l + 1])) for l in range(4)]
    grids = [np.arange(n, dtype=np.float64) for n in ns]

    def fun(pts):
        idx = pts.reshape(-1, 4).astype(np.int64)
        return cross.tt_at(T, idx).reshape(pts.shape[:-1])

    cores = cross.cross(fun, grids, 4, sweeps=2, seed=3)
    full, ref = ott.full(cores), ott.full(T)
    assert np.linalg.norm(full - ref) <= 1e-11 * np.linalg.norm(ref)


def test_sin_of_linear_form_has_rank_two():
    d, n = 5, 9
    grids = [np.linspace(-1, 1, n) for _ in range(d)]
    w = np.array([0.9, -0.4, 1.3, 0.2, -0.7])
    fun = lambda p: np.sin(0.3 + p @ w)
    cores = cross.cross(fun, grids, 2, sweeps=2, seed=4)
    assert max(c.shape[2] for c in cores) <= 2
    X = np.meshgrid(*grids, indexing="ij")
    ref = np.sin(0.3 + sum(w[k] * X[k] for k in range(d)))
    assert np.linalg.norm(ott.full(cores) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_adaptive_cross_of_smooth_nonseparable_function():
    d, n = 4, 10
    grids = [np.cos(np.pi * (np.arange(n) + 0.5) / n) for _ in range(d)]
    fun = lambda p: 1.0 / (1.0 + np.sum((p - 0.2) ** 2, axis=-1))
    cores, info = cross.cross_adaptive(fun, grids, tol=1e-8, r0=2, rmax=32)
    X = np.meshgrid(*grids, indexing="ij")
    ref = 1.0 / (1.0 + sum((X[k] - 0.2) ** 2 for k in range(d)))
    err = np.linalg.norm(ott.full(cores) - ref) / np.linalg.norm(ref)
    assert info["sample_error"] <= 1e-8 and err <= 1e-7
