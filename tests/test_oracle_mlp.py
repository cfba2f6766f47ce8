"""Pins of the oracle's MLP (10-64-64-3, tanh): backward pass against central finite
differences, and the forward pass against closed forms for special weights."""
import numpy as np

import coupling_pins as pins
import oracle

NP = oracle.NPARAM


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, NP)


def test_forward_special_cases():
    P = np.zeros(NP)
    b3 = P[NP - 3:]
    b3[:] = [0.5, -1.0, 2.0]
    x = np.random.default_rng(0).normal(size=(7, 10))
    assert np.array_equal(oracle.mlp_forward(P, x), np.tile(b3, (7, 1)))
    # one path: W1[0,0]=a, W2[0,0]=b, W3[0,0]=c -> y0 = c tanh(b tanh(a x0))
    P = np.zeros(NP)
    P[0] = 0.7
    off_w2 = 10 * 64 + 64
    P[off_w2] = -1.3
    off_w3 = off_w2 + 64 * 64 + 64
    P[off_w3] = 2.1
    y = oracle.mlp_forward(P, x)
    assert np.allclose(y[:, 0], 2.1 * np.tanh(-1.3 * np.tanh(0.7 * x[:, 0])), atol=1e-15)
    assert np.allclose(y[:, 1:], 0.0)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = _params(1)
    x = rng.normal(size=(13, 10))
    t = rng.normal(size=(13, 3))
    loss, g = oracle.mlp_loss_grad(P, x, t)
    y = oracle.mlp_forward(P, x)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-14
    idx = rng.choice(NP, 60, replace=False)
    idx = np.concatenate([idx, [0, 639, 640, 703, 704, NP - 4, NP - 1]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (oracle.mlp_loss_grad(Pp, x, t)[0] - oracle.mlp_loss_grad(Pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])



def test_predicted_force_is_the_previous_plus_the_scaled_change():
    pins.pin_learned_force_prediction()
