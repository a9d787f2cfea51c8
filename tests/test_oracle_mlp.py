"""Pins of the oracle's network, TT fitting loss and Adam step (oracle/mlp.py).

Each pin comes from outside the code under test: central finite differences
for every gradient, the full-tensor definition of the loss on tiny grids, the
gauge freedom of the TT format (Methods: the representation is not unique),
and Adam's first step, which moves every parameter by exactly lr times the
sign of its gradient.
"""
import numpy as np
import pytest

from oracle import mlp
from oracle import tt as ott


def _net(rng, widths):
    return rng.standard_normal(mlp.param_count(widths)) * 0.5


def test_param_layout_and_count():
    widths = [20, 256, 256, 256, 7392]
    # 20*256 + 256 + 2 * (256*256 + 256) + 256*7392 + 7392
    assert mlp.param_count(widths) == 20 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 7392 + 7392
    assert mlp.output_size([22] * 7, 8) == 22 * 8 + 5 * 8 * 22 * 8 + 8 * 22 == 7392


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    widths = [4, 6, 5, 3]
    p = _net(rng, widths)
    X = rng.standard_normal((7, 4))
    C = rng.standard_normal((7, 3))          # loss = sum(C * Y)
    Y, H = mlp.forward(p, widths, X)
    g = mlp.backward(p, widths, H, C)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (np.sum(C * mlp.forward(p + e, widths, X)[0]) - np.sum(C * mlp.forward(p - e, widths, X)[0])) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))


def test_network_is_affine_in_output_layer_and_odd_in_hidden():
    rng = np.random.default_rng(1)
    widths = [3, 5, 2]
    p = _net(rng, widths)
    X = rng.standard_normal((4, 3))
    layers = mlp.unpack(p, widths)
    # zero hidden biases: tanh is odd, so Y(-X) - b_out = -(Y(X) - b_out)
    layers[0][1][:] = 0.0
    Y1, _ = mlp.forward(p, widths, X)
    Y2, _ = mlp.forward(p, widths, -X)
    b_out = layers[1][1]
    np.testing.assert_allclose(Y2 - b_out, -(Y1 - b_out), atol=1e-14)


def _tiny_tt(rng, n, r):
    return rng.standard_normal(mlp.output_size(n, r))


def test_loss_equals_full_tensor_definition():
    rng = np.random.default_rng(2)
    n, r = [3, 4, 2, 3], 2
    y, t = _tiny_tt(rng, n, r), _tiny_tt(rng, n, r)
    loss, _ = mlp.tt_fit_loss(y, t, n, r)
    Pf = ott.full(mlp.split_cores(y, n, r))
    Tf = ott.full(mlp.split_cores(t, n, r))
    assert abs(loss - np.sum((Pf - Tf) ** 2) / np.sum(Tf ** 2)) <= 1e-13 * max(1.0, loss)


def test_loss_gradient_matches_finite_differences_and_vanishes_at_target():
    rng = np.random.default_rng(3)
    n, r = [3, 2, 4], 2
    y, t = _tiny_tt(rng, n, r), _tiny_tt(rng, n, r)
    _, g = mlp.tt_fit_loss(y, t, n, r)
    h = 1e-6
    fd = np.array([(mlp.tt_fit_loss(y + h * e, t, n, r)[0] - mlp.tt_fit_loss(y - h * e, t, n, r)[0]) / (2 * h)
                   for e in np.eye(y.size)])
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))
    l0, g0 = mlp.tt_fit_loss(t, t, n, r)
    assert abs(l0) <= 1e-14 and np.max(np.abs(g0)) <= 1e-13


def test_loss_is_gauge_invariant():
    rng = np.random.default_rng(4)
    n, r = [3, 4, 2, 3], 3
    y, t = _tiny_tt(rng, n, r), _tiny_tt(rng, n, r)
    P = mlp.split_cores(y, n, r)
    for l in range(len(P) - 1):
        A = rng.standard_normal((r, r)) + 3 * np.eye(r)
        P[l] = np.einsum("aib,bc->aic", P[l], A)
        P[l + 1] = np.einsum("cb,bid->cid", np.linalg.inv(A), P[l + 1])
    y2 = np.concatenate([c.ravel() for c in P])
    assert abs(mlp.tt_fit_loss(y, t, n, r)[0] - mlp.tt_fit_loss(y2, t, n, r)[0]) <= 1e-11


def test_adam_first_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    q, m, v = mlp.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(q, p - 1e-3 * np.sign(g), atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
