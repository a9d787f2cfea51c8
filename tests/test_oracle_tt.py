"""Pins for the oracle's TT arithmetic (Methods, Tensor Train representation)."""
import json
import os
from functools import reduce

import numpy as np
import pytest

from oracle import metrics
from oracle import tt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_arithmetic.json")


def _rand_tt(rng, ns, rs):
    return [rng.standard_normal((rs[l], ns[l], rs[l + 1])) for l in range(len(ns))]


def test_worked_entry_is_product_of_slices():
    """Fig. 2: A(4,5,2,6,3,8) = G1(4) G2(5) G3(2) G4(6) G3(3) G6(8)."""
    g = json.load(open(GOLDEN))["worked_entry"]
    idx = [i - 1 for i in g["index_one_based"]]
    rng = np.random.default_rng(1)
    cores = _rand_tt(rng, [8] * 6, [1, 3, 2, 4, 3, 2, 1])
    full = tt.full(cores)
    prod = reduce(np.matmul, [cores[l][:, idx[l], :] for l in range(6)])[0, 0]
    assert abs(full[tuple(idx)] - prod) < 1e-12
    assert abs(tt.element(cores, idx) - prod) < 1e-12
    # brute-force sum over all bond indices (Eq. TT-format:elementwise)
    s = 0.0
    for a in np.ndindex(3, 2, 4, 3, 2):
        a = (0,) + a + (0,)
        s += np.prod([cores[l][a[l], idx[l], a[l + 1]] for l in range(6)])
    assert abs(s - prod) < 1e-12


def test_tt_svd_recovers_exact_ranks():
    rng = np.random.default_rng(2)
    cores = _rand_tt(rng, [5, 6, 4, 5], [1, 3, 4, 2, 1])
    A = tt.full(cores)
    rec = tt.tt_svd(A, eps=1e-14)
    assert tt.ranks(rec) == [1, 3, 4, 2, 1]
    assert np.linalg.norm(tt.full(rec) - A) < 1e-12 * np.linalg.norm(A)
    # the unfolding ranks are the TT ranks (Oseledets, Theorem 2.1)
    for l in range(1, 4):
        unf = A.reshape(int(np.prod(A.shape[:l])), -1)
        assert np.linalg.matrix_rank(unf) == tt.ranks(rec)[l]


@pytest.mark.parametrize("eps", [1e-1, 1e-3, 1e-6])
def test_tt_svd_error_bound(eps):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 5, 7, 4)) + 3 * tt.full(_rand_tt(rng, [6, 5, 7, 4], [1, 2, 2, 2, 1]))
    rec = tt.tt_svd(A, eps=eps)
    assert np.linalg.norm(tt.full(rec) - A) <= eps * np.linalg.norm(A) * (1 + 1e-12)


def test_tt_svd_2d_is_eckart_young():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((20, 15))
    s = np.linalg.svd(A, compute_uv=False)
    for r in (1, 3, 7):
        rec = tt.tt_svd(A, rmax=r)
        err = np.linalg.norm(tt.full(rec) - A)
        assert abs(err - np.sqrt(np.sum(s[r:] ** 2))) < 1e-12 * np.linalg.norm(A)


def test_tt_svd_quasi_optimality_bound():
    """||A - TT-SVD_r(A)|| <= sqrt(sum_l tail_l^2) <= sqrt(d-1) * best, with each
    unfolding tail a lower bound of the best error (Methods)."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((5, 6, 5, 4))
    rs = [2, 3, 2]
    rec = tt.tt_svd(A, rmax=3)
    rec_r = tt.tt_svd(A, rmax=10 ** 6)
    # exact TT of A, then rank-capped approximations per unfolding
    err = None
    cores = []
    C = A.reshape(1, -1)
    rp = 1
    for l, r in enumerate(rs):
        C = C.reshape(rp * A.shape[l], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        cores.append(U[:, :r].reshape(rp, A.shape[l], r))
        C = s[:r, None] * Vt[:r]
        rp = r
    cores.append(C.reshape(rp, A.shape[-1], 1))
    err = np.linalg.norm(tt.full(cores) - A)
    tails = []
    for l, r in enumerate(rs):
        s = np.linalg.svd(A.reshape(int(np.prod(A.shape[:l + 1])), -1), compute_uv=False)
        tails.append(np.sqrt(np.sum(s[r:] ** 2)))
    lower_best = max(tails)
    assert err <= np.sqrt(np.sum(np.square(tails))) * (1 + 1e-12)
    assert err <= np.sqrt(len(rs)) * np.sqrt(np.sum(np.square(tails)))
    assert err >= lower_best * (1 - 1e-12)
    assert tt.ranks(rec)[1:-1] == [3, 3, 3] or max(tt.ranks(rec)) <= 3
    assert np.linalg.norm(tt.full(rec_r) - A) < 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("eps", [1e-2, 1e-6, 1e-10])
def test_rounding_bound_and_rank_reduction(eps):
    rng = np.random.default_rng(6)
    x = _rand_tt(rng, [6, 7, 5, 6], [1, 3, 3, 3, 1])
    y = tt.add(x, x, 1.0, 2.0)                      # = 3x, ranks doubled
    assert tt.ranks(y) == [1, 6, 6, 6, 1]
    r = tt.round_tt(y, eps)
    assert max(tt.ranks(r)) <= 3
    np.testing.assert_allclose(tt.full(r), 3 * tt.full(x), atol=1e-10 * np.abs(tt.full(x)).max())
    z = tt.add(x, _rand_tt(rng, [6, 7, 5, 6], [1, 4, 4, 4, 1]))
    rz = tt.round_tt(z, eps)
    assert np.linalg.norm(tt.full(rz) - tt.full(z)) <= eps * np.linalg.norm(tt.full(z)) * (1 + 1e-10)


def test_matvec_equals_dense_kronecker_product():
    rng = np.random.default_rng(7)
    ns = [4, 5, 3]
    A = [rng.standard_normal((R0, n, n, R1)) for (R0, n, R1) in zip([1, 2, 3], ns, [2, 3, 1])]
    x = _rand_tt(rng, ns, [1, 2, 2, 1])
    dense = tt.ttm_full(A)
    y = tt.matvec(A, x)
    np.testing.assert_allclose(tt.full(y).ravel(), dense @ tt.full(x).ravel(), atol=1e-12)
    # explicit Kronecker construction of a rank-1 TT-matrix
    B = [rng.standard_normal((1, n, n, 1)) for n in ns]
    kron = reduce(np.kron, [b[0, :, :, 0] for b in B])
    np.testing.assert_allclose(tt.ttm_full(B), kron, atol=1e-13)


def test_kron_sum_ttm_matches_explicit_sum():
    rng = np.random.default_rng(8)
    d, n = 4, 3
    Es = [rng.standard_normal((n, n)) for _ in range(d)]
    Ms = [rng.standard_normal((n, n)) for _ in range(d)]
    explicit = sum(reduce(np.kron, [Ms[k] if k == l else Es[k] for k in range(d)]) for l in range(d))
    np.testing.assert_allclose(tt.ttm_full(tt.kron_sum_ttm(Es, Ms)), explicit, atol=1e-12)


def test_dot_norm_residual_against_full():
    rng = np.random.default_rng(9)
    ns = [5, 4, 6]
    x = _rand_tt(rng, ns, [1, 3, 2, 1])
    y = _rand_tt(rng, ns, [1, 2, 4, 1])
    assert abs(tt.dot(x, y) - np.sum(tt.full(x) * tt.full(y))) < 1e-11
    assert abs(tt.norm(x) - np.linalg.norm(tt.full(x))) < 1e-12 * np.linalg.norm(tt.full(x))
    A = [rng.standard_normal((R0, n, n, R1)) for (R0, n, R1) in zip([1, 2, 2], ns, [2, 2, 1])]
    res = tt.residual_norm(A, x, y)
    dense = np.linalg.norm(tt.full(y).ravel() - tt.ttm_full(A) @ tt.full(x).ravel()) / np.linalg.norm(tt.full(y))
    assert abs(res - dense) < 1e-12 * max(1.0, dense)
    assert abs(tt.rel_diff(x, y) - np.linalg.norm(tt.full(x) - tt.full(y)) / np.linalg.norm(tt.full(y))) < 1e-12


def test_separable_to_tt():
    rng = np.random.default_rng(10)
    terms = [[rng.standard_normal(n) for n in (3, 4, 5)] for _ in range(4)]
    full = sum(reduce(np.multiply.outer, t) for t in terms)
    cores = tt.separable_to_tt(terms)
    assert tt.ranks(cores) == [1, 4, 4, 1]
    np.testing.assert_allclose(tt.full(cores), full, atol=1e-12)


def test_paper_compression_and_storage_arithmetic():
    g = json.load(open(GOLDEN))
    c7 = g["compression_7d_spacetime"]
    v = metrics.compression_bound(c7["n"], c7["r"], c7["d"])
    assert int(np.floor(np.log10(v))) == c7["order_of_magnitude"] - 1 or \
        int(np.round(np.log10(v))) == c7["order_of_magnitude"]
    c6 = g["compression_6d_fig6"]
    v6 = metrics.compression_bound(c6["n"], c6["r"], c6["d"])
    assert int(np.round(np.log10(v6))) == c6["order_of_magnitude"] + 1 or \
        int(np.floor(np.log10(v6))) == c6["order_of_magnitude"]
    s = g["storage_example"]
    assert s["n"] * s["r"] ** 2 * s["d"] == s["tt_storage"]
    assert float(s["n"]) ** s["d"] == s["full_storage"]
    # the exact storage of such a TT is below that bound
    assert metrics.tt_storage(s["n"], s["r"], s["d"]) <= s["tt_storage"]


def test_compression_ratio_of_paper_sized_tts():
    # the paper's 7D space-time figure counts d cores of r x n x r entries
    g = json.load(open(GOLDEN))
    c7 = g["compression_7d_spacetime"]
    d, n, r = c7["d"], c7["n"], c7["r"]
    cores = [np.zeros((r, n, r)) for _ in range(d)]
    v = tt.compression_ratio(cores)
    assert abs(v / metrics.compression_bound(n, r, d) - 1.0) < 1e-14
    assert abs(np.log10(v) - c7["order_of_magnitude"]) < 1.0
    # with boundary ranks 1 it is the storage of metrics.tt_storage
    s = g["storage_example"]
    d, n, r = s["d"], s["n"], s["r"]
    cores = [np.zeros((1 if l == 0 else r, n, 1 if l == d - 1 else r)) for l in range(d)]
    assert tt.compression_ratio(cores) * float(n) ** d == metrics.tt_storage(n, r, d)
    assert tt.compression_ratio(cores) * s["full_storage"] <= s["tt_storage"]


def test_mid_axis_profile_and_oscillation_count():
    # u[i, j, k] = w[i] with w monotone except one dip: one extra sign change
    w = np.array([0.0, 1.0, 2.0, 1.5, 3.0, 4.0])
    u = np.broadcast_to(w[:, None, None], (6, 5, 4)).copy()
    u[:, 0, :] = -7.0                         # off the mid line: ignored
    np.testing.assert_array_equal(metrics.mid_axis_profile(u, 0), w)
    assert metrics.oscillation_count(u, 0) == 2
    assert metrics.is_oscillatory(u, 0) and not metrics.is_oscillatory(u, 2)
    # along axis 1 the line passes through index 3 of axis 0 (value 1.5)
    assert metrics.oscillation_count(u, 1) == 0


def test_metrics_sign_changes():
    assert metrics.sign_changes([0, 1, 2, 3, 2, 1, 0]) == 1
    assert metrics.sign_changes([0, 1, 0, 1, 0]) == 3
    assert metrics.sign_changes([0.0, 1.0, 1.0 + 1e-15, 2.0]) == 0
