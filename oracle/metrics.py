"""Diagnostics reported by the paper (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

* Relative Frobenius error ||f - f_n||_F / ||f||_F (Results, "Global Accuracy
  and Computational Cost").
* Oscillation count (Results, "Superconsistent Stabilization"): sign changes of
  the first derivative of the discrete solution along the mid-axis in the
  first direction, compared with the count of the regular solution.  Reading
  for the ambiguous "centre most degree of freedom": the other indices are
  N // 2; differences of consecutive nodal values stand for the derivative;
  differences below 1e-12 max|u| are ignored.
* Compression ratio: TT storage over full storage (Results; Methods remark on
  storage O(d n r^2) vs O(n^d)).

Pins: tests/test_oracle_tt.py -- test_metrics_sign_changes and
test_mid_axis_profile_and_oscillation_count (counts on hand-made profiles),
test_paper_compression_and_storage_arithmetic (the paper's printed
compression and storage figures from tests/golden/); the oscillation test
of the 2D collocation solve in tests/test_oracle_collocation.py.
"""
from __future__ import annotations

import numpy as np


def rel_frobenius(u, u_ref) -> float:
    u = np.asarray(u, dtype=np.float64)
    u_ref = np.asarray(u_ref, dtype=np.float64)
    return float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))


def sign_changes(values, rel_floor: float = 1e-12) -> int:
    """Number of sign changes of consecutive differences of a 1D profile."""
    v = np.asarray(values, dtype=np.float64)
    dv = np.diff(v)
    scale = np.max(np.abs(v)) if v.size else 0.0
    dv = dv[np.abs(dv) > rel_floor * scale]
    if dv.size < 2:
        return 0
    s = np.sign(dv)
    return int(np.count_nonzero(s[1:] != s[:-1]))


def mid_axis_profile(u_full: np.ndarray, axis: int = 0) -> np.ndarray:
    """Line through the grid centre along ``axis`` (other indices N // 2)."""
    idx = [n // 2 for n in u_full.shape]
    idx[axis] = slice(None)
    return u_full[tuple(idx)]


def oscillation_count(u_full: np.ndarray, axis: int = 0) -> int:
    return sign_changes(mid_axis_profile(u_full, axis))


def is_oscillatory(u_full: np.ndarray, expected: int, axis: int = 0) -> bool:
    return oscillation_count(u_full, axis) > expected


def tt_storage(n: int, r: int, d: int) -> int:
    """Storage of a TT tensor with all mode sizes n and inner ranks r (first and
    last cores are n x r)."""
    if d == 1:
        return n
    return 2 * n * r + (d - 2) * n * r * r


def compression_bound(n: int, r: int, d: int) -> float:
    """d n r^2 / n^d: the compression figure the paper quotes for a TT of
    maximal rank r, mode size n and d dimensions."""
    return float(d * n * r * r) / float(n) ** d
