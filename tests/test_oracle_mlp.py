"""Pins of the reference network: gradients against central finite differences,
Adam against its closed form on a quadratic."""
import numpy as np

from oracle.mlp import adam_step, backward, forward, init_params, loss


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    p = init_params(7, 6, 5, seed=1)
    for k in p:                                   # non-zero biases, away from ReLU kinks
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    X = rng.standard_normal((9, 7))
    T = rng.standard_normal((9, 5))
    Y, cache = forward(p, X)
    g = backward(p, cache, Y, T)
    h = 1e-6
    for k in p:
        num = np.zeros_like(p[k])
        it = np.nditer(p[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = p[k][i]
            p[k][i] = old + h
            lp = loss(forward(p, X)[0], T)
            p[k][i] = old - h
            lm = loss(forward(p, X)[0], T)
            p[k][i] = old
            num[i] = (lp - lm) / (2 * h)
        err = np.abs(num - g[k]).max() / max(np.abs(num).max(), 1e-12)
        assert err < 1e-6, (k, err)


def test_adam_first_step_closed_form():
    p = {"w": np.array([1.0, -2.0])}
    g = {"w": np.array([0.5, -4.0])}
    st = {}
    adam_step(p, g, st, lr=0.1)
    # first step: m_hat = g, v_hat = g^2 -> update = lr * sign(g) (up to eps)
    np.testing.assert_allclose(p["w"], [1.0 - 0.1, -2.0 + 0.1], atol=1e-7)


def test_training_reduces_loss_on_a_linear_target():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((256, 8))
    A = rng.standard_normal((8, 4))
    T = X @ A
    p = init_params(8, 32, 4, seed=2)
    st = {}
    l0 = loss(forward(p, X)[0], T)
    for _ in range(300):
        Y, c = forward(p, X)
        adam_step(p, backward(p, c, Y, T), st, lr=1e-2)
    assert loss(forward(p, X)[0], T) < 0.05 * l0
