"""CPU tests of libt2s2: exported symbols, host 1D builder against the oracle,
argument errors.  No GPU needed (the calls used here are host-only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2506_04732_amd as t2s2
from paper_2506_04732_amd import _lib
from oracle import spectral as sp

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "t2s2.h")


def test_library_exports_every_declared_symbol():
    decl = re.findall(r"^(?:int|void|const char\*)\s+(t2s2_\w+)\s*\(", open(HEADER).read(), re.M)
    assert len(decl) >= 12
    lib = t2s2.lib()
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(_lib.EXPORTED)


@pytest.mark.parametrize("N,eps,beta,scheme", [
    (4, 1e-2, 1.0, 1), (8, 1e-3, -0.4, 1), (16, 1e-2, 0.5, 1), (32, 2e-3, 0.7, 1), (33, 1e-6, 1.0, 1),
    (48, 1e-4, -1.0, 1), (64, 1e-1, 0.3, 1), (16, 1e-2, 0.0, 1), (20, 1e-3, 1.0, 0)])
def test_nodes_match_oracle(N, eps, beta, scheme):
    x, th = t2s2.nodes(N, eps, beta, scheme)
    np.testing.assert_allclose(x, sp.gll_nodes(N - 1), atol=4e-16)
    np.testing.assert_allclose(th, sp.collocation_nodes(N - 1, eps, beta, scheme), atol=2e-15)


@pytest.mark.parametrize("N,eps,beta,scheme", [(5, 1e-2, 1.0, 1), (16, 1e-2, 0.5, 1), (32, 2e-3, 0.7, 1),
                                                (46, 1e-4, -0.3, 1), (24, 1.0, 1.0, 0)])
def test_matrices_match_oracle(N, eps, beta, scheme):
    E, D1, D2 = t2s2.matrices_1d(N, eps, beta, scheme)
    x = sp.gll_nodes(N - 1)
    th = sp.collocation_nodes(N - 1, eps, beta, scheme)
    Eo, D1o, D2o = sp.lagrange_matrices(x, th)
    u = np.finfo(float).eps
    for A, B in ((E, Eo), (D1, D1o), (D2, D2o)):
        scale = np.abs(B).sum(axis=1).max()
        assert np.abs(A - B).max() < 500 * u * scale


@pytest.mark.parametrize("args", [(2, 1e-3, 1.0, 1), (3, 0.0, 1.0, 1), (8, -1.0, 1.0, 1),
                                  (8, 1e-3, float("nan"), 1), (8, 1e-3, 1.0, 7), (300, 1e-3, 1.0, 1)])
def test_nodes_reject_bad_arguments(args):
    with pytest.raises(t2s2.T2S2Error) as e:
        t2s2.nodes(*args)
    assert e.value.code == _lib.T2S2_EINVAL
    assert t2s2.lib().t2s2_last_error().decode() != ""


def test_last_error_cleared_on_success():
    with pytest.raises(t2s2.T2S2Error):
        t2s2.nodes(2, 1e-3, 1.0)
    t2s2.nodes(8, 1e-3, 1.0)
    assert t2s2.lib().t2s2_last_error().decode() == ""
