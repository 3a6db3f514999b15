"""Pins of the FP64 network reference: central finite differences of the loss, and the
closed form of a network with all hidden weights zero."""
import numpy as np

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
