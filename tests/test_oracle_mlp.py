"""Pins of the learned-proposal oracle (CPU): the MLP's gradient against central finite
differences of its loss, closed forms of the forward pass, Adam against its two-step
closed form, and the BF16-rounding variant against the exact one."""
import math

import numpy as np

from oracle import oracle as O

N = 882832


def _init(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    P = np.zeros(N)
    for W, b in O.mlp_layer_views(P):
        W[:] = rng.normal(size=W.shape) * scale / math.sqrt(W.shape[0])
        b[:] = rng.normal(size=b.shape) * 0.1
    return P


def test_parameter_count():
    assert O.mlp_n_params() == N == 40 * 512 + 512 + 3 * (512 * 512 + 512) + 512 * 144 + 144


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    P = _init(1)
    X = rng.normal(size=(3, 40))
    Y = rng.normal(size=(3, 72))
    L, G = O.mlp_grad(P, X, Y)
    assert abs(L - O.mlp_loss(P, X, Y)) < 1e-12 * abs(L)
    offs = np.cumsum([0] + [fi * fo + fo for fi, fo in zip(O.MLP_DIMS[:-1], O.MLP_DIMS[1:])])
    idx = []
    for l in range(5):  # weights and biases of every layer
        idx += list(rng.integers(offs[l], offs[l + 1], 6))
        idx.append(offs[l + 1] - 1)
    for i in idx:
        h = 1e-5
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (O.mlp_loss(Pp, X, Y) - O.mlp_loss(Pm, X, Y)) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(abs(G).max(), 1e-12) + 1e-7 * abs(G[i]), (i, fd, G[i])


def test_forward_closed_forms():
    P = np.zeros(N)
    layers = O.mlp_layer_views(P)
    layers[-1][1][:] = np.linspace(-1, 1, 144)
    X = np.random.default_rng(2).normal(size=(4, 40))
    np.testing.assert_array_equal(O.mlp_forward(P, X), np.tile(np.linspace(-1, 1, 144), (4, 1)))
    # a single path: out[0] = silu^4(2 x_3) when every other weight and bias is zero
    P[:] = 0
    layers[0][0][3, 0] = 2.0
    for l in (1, 2, 3):
        layers[l][0][0, 0] = 1.0
    layers[4][0][0, 0] = 1.0
    silu = lambda z: z / (1 + math.exp(-z))
    out = O.mlp_forward(P, X)
    for r in range(4):
        want = silu(silu(silu(silu(2 * X[r, 3]))))
        assert abs(out[r, 0] - want) < 1e-14
        assert not out[r, 1:].any()


def test_loss_closed_form():
    P = np.zeros(N)
    b = O.mlp_layer_views(P)[-1][1]
    b[:72] = 0.5
    b[72:] = math.log(2.0)
    X = np.zeros((2, 40))
    Y = np.full((2, 72), 1.5)
    # mean of (y - m)^2 / (2 e^{2s}) + s = 1 / 8 + ln 2
    assert abs(O.mlp_loss(P, X, Y) - (1 / 8 + math.log(2))) < 1e-14


def test_adam_two_steps_closed_form():
    P, m, v = np.array([1.0, -2.0]), np.zeros(2), np.zeros(2)
    g1, g2 = np.array([0.3, -4.0]), np.array([-0.1, 2.0])
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    P1, m1, v1 = O.adam(P, m, v, g1, 1, lr, b1, b2, eps)
    np.testing.assert_allclose(P1, P - lr * g1 / (np.abs(g1) + eps), rtol=1e-14)
    P2, m2, v2 = O.adam(P1, m1, v1, g2, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    np.testing.assert_allclose(P2, P1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-13)


def test_bf16_variant_close_to_exact():
    rng = np.random.default_rng(3)
    P = _init(3)
    X = rng.normal(size=(8, 40))
    Y = rng.normal(size=(8, 72))
    a, b = O.mlp_forward(P, X), O.mlp_forward(P, X, bf16=True)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 2e-2
    _, G = O.mlp_grad(P, X, Y)
    _, Gb = O.mlp_grad(P, X, Y, bf16=True)
    cos = G @ Gb / (np.linalg.norm(G) * np.linalg.norm(Gb))
    assert cos > 0.999
