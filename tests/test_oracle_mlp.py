"""Pins of the FP64 network reference: central finite differences of the loss, and the
closed form of a network with all hidden weights zero."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def _params(seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=M.N_PARAMS) * 0.3


def test_parameter_count():
    assert M.N_PARAMS == 4801


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = _params(4)
    X = rng.normal(size=(40, 8))
    t = rng.normal(size=40)
    loss, g = M.loss_and_grad(P, X, t)
    idx = rng.choice(M.N_PARAMS, 200, replace=False)
    idx = np.concatenate([idx, [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4799, 4800]])
    h = 1e-6
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (M.loss_and_grad(Pp, X, t)[0] - M.loss_and_grad(Pm, X, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_constant_network_closed_form():
    # with W1 = W2 = W3 = 0 the network outputs b3; the loss is mean((b3 - t)^2) and only b3
    # has a gradient: 2 mean(b3 - t)
    P = np.zeros(M.N_PARAMS)
    P[-1] = 0.7
    t = np.array([0.1, 0.5, 2.0])
    loss, g = M.loss_and_grad(P, np.ones((3, 8)), t)
    assert np.isclose(loss, np.mean((0.7 - t) ** 2))
    assert np.isclose(g[-1], 2 * np.mean(0.7 - t))
    assert np.all(g[:-1][np.r_[0:512, 576:4672]] == 0)
    y = M.forward(P, np.ones((3, 8)))
    assert np.allclose(y, 0.7)


# ---------------------------------------------------------------------------------------
# SiLU at points where it has a closed form: silu(z) = z * sigmoid(z), sigmoid(1) = e/(1+e),
# sigmoid(-2) = 1/(1+e^2)
def test_silu_known_values():
    e = math.e
    assert M.silu(np.array(1.0)) == pytest.approx(e / (1.0 + e), rel=1e-15)
    assert M.silu(np.array(-2.0)) == pytest.approx(-2.0 / (1.0 + e * e), rel=1e-15)
    assert M.silu(np.array(0.0)) == 0.0
    assert M.silu(np.array(40.0)) == pytest.approx(40.0, rel=1e-15)
    assert abs(M.silu(np.array(-40.0))) < 1e-15


def test_forward_applies_silu_in_both_hidden_layers():
    # x0 = 1 feeds hidden unit 0 (z1 = 1, h1 = e/(1+e)); layer 2 scales it so that z2 = -2;
    # the output reads unit 0: y = silu(-2) = -2/(1+e^2).  A wrong activation in either
    # layer moves y.
    e = math.e
    W1 = np.zeros((8, 64)); W1[0, 0] = 1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = -2.0 * (1.0 + e) / e
    W3 = np.zeros(64); W3[0] = 1.0
    P = np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3, [0.0]])
    X = np.zeros((1, 8)); X[0, 0] = 1.0
    assert M.forward(P, X)[0] == pytest.approx(-2.0 / (1.0 + e * e), rel=1e-13)
    # and the same with the activation of layer 2 read from a bias alone (W2 = 0, b2 = -2)
    P2 = P.copy()
    P2[576:576 + 4096] = 0.0
    P2[576 + 4096] = -2.0
    assert M.forward(P2, X)[0] == pytest.approx(-2.0 / (1.0 + e * e), rel=1e-15)


# ---------------------------------------------------------------------------------------
# Adam (Kingma & Ba 2015, Algorithm 1), pinned by closed forms of its bias-corrected moments
def test_adam_first_step_moves_by_lr_times_sign():
    # m = v = 0, t = 1: m_hat = g, v_hat = g^2, so every weight moves by -lr g / (|g| + eps)
    rng = np.random.default_rng(5)
    P = rng.normal(size=M.N_PARAMS)
    g = rng.normal(size=M.N_PARAMS) * 10.0 ** rng.uniform(-4, 2, M.N_PARAMS)
    lr = 1e-3
    P1, m1, v1 = M.adam(P, np.zeros_like(P), np.zeros_like(P), g, 1, lr)
    assert np.allclose(P1 - P, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15)
    assert np.allclose(v1, 0.001 * g * g, rtol=1e-13)


def test_adam_constant_gradient_moves_by_lr_every_step():
    # with a constant gradient m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the corrected
    # moments are g and g^2 at every step and each step moves by -lr g / (|g| + eps)
    rng = np.random.default_rng(6)
    P = rng.normal(size=64)
    g = rng.normal(size=64)
    m, v = np.zeros(64), np.zeros(64)
    lr = 0.01
    for t in range(1, 31):
        Pn, m, v = M.adam(P, m, v, g, t, lr)
        assert np.allclose(Pn - P, -lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15), t
        P = Pn


def test_adam_alternating_gradient_second_step():
    # gradients g then -g: m_2 = -(1 - b1)^2 g, m_hat_2 = -(1 - b1) g / (1 + b1);
    # v_2 = (1 - b2)(1 + b2) g^2, v_hat_2 = g^2; the second step moves by
    # +lr (1 - b1) / (1 + b1) g / (|g| + eps)
    rng = np.random.default_rng(7)
    g = rng.normal(size=100)
    P0 = rng.normal(size=100)
    lr = 1e-2
    P1, m, v = M.adam(P0, np.zeros(100), np.zeros(100), g, 1, lr)
    P2, m, v = M.adam(P1, m, v, -g, 2, lr)
    assert np.allclose(P2 - P1, lr * (0.1 / 1.9) * g / (np.abs(g) + 1e-8), rtol=1e-10,
                       atol=1e-16)
