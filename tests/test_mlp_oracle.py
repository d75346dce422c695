"""The float64 selector-network oracle against finite differences and
closed forms."""
import numpy as np
import pytest

from oracle import mlp


def _theta(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for s in mlp.SHAPES:
        parts.append(rng.uniform(-0.5, 0.5, size=s))
    return mlp.pack(parts)


def test_param_count():
    # 64*16 + 64 + 64*64 + 64 + 7*64 + 7
    assert mlp.N_PARAMS == 5703


def test_zero_weights_closed_form():
    th = np.zeros(mlp.N_PARAMS)
    th[-7:] = np.arange(7)  # b3
    X = np.random.default_rng(0).standard_normal((5, 16))
    T = np.ones((5, 7))
    Y, cache = mlp.forward(th, X)
    assert np.array_equal(Y, np.tile(np.arange(7.0), (5, 1)))
    g = mlp.backward(th, cache, Y, T)
    # dL/db3 = 2 (b3 - 1) / 7 (mean over batch of identical rows)
    assert np.allclose(g[-7:], 2 * (np.arange(7) - 1) / 7)
    assert np.all(g[:-7] == 0)
    assert mlp.loss(Y, T) == np.mean((np.arange(7.0) - 1) ** 2)


def test_missing_targets_closed_form():
    """A NaN target (a variant without a time) adds nothing to the loss or
    the gradient; the denominator stays batch x outputs."""
    th = np.zeros(mlp.N_PARAMS)
    th[-7:] = np.arange(7)
    X = np.random.default_rng(1).standard_normal((4, 16))
    T = np.ones((4, 7))
    T[:, 6] = np.nan
    T[1, 2] = np.nan
    Y, cache = mlp.forward(th, X)
    g = mlp.backward(th, cache, Y, T)
    # b3[v] gets 2 (v - 1) / (4 * 7) from each row whose target v is present
    rows = np.array([4, 4, 3, 4, 4, 4, 0])
    assert np.allclose(g[-7:], rows * 2 * (np.arange(7) - 1) / 28)
    sq = (np.arange(7.0) - 1) ** 2
    assert np.isclose(mlp.loss(Y, T), (sq @ rows) / 28)


def test_gradient_finite_differences():
    th = _theta(1)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((7, 16))
    T = rng.standard_normal((7, 7))
    T[rng.random((7, 7)) < 0.2] = np.nan  # missing targets
    L, g = mlp.loss_and_grad(th, X, T)
    n = mlp.N_PARAMS
    idx = list(rng.choice(n, size=300, replace=False)) + list(range(n - 7, n))
    fd = mlp.grad_fd(th, X, T, h=1e-6, idx=idx)
    for i in idx:
        assert abs(fd[i] - g[i]) <= 1e-6 * max(1.0, abs(g[i])) * 10 + 1e-9, (i, fd[i], g[i])


def test_relu_derivative_zero_at_zero():
    # choose b1 so that z1 == 0 exactly for X = 0: the gradient must not pass
    th = _theta(3)
    W1n = 64 * 16
    th[W1n:W1n + 64] = 0.0
    X = np.zeros((1, 16))
    Y, cache = mlp.forward(th, X)
    g = mlp.backward(th, cache, Y, np.zeros((1, 7)))
    assert np.all(g[W1n:W1n + 64] == 0)


def test_adam_first_step():
    # first step: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + eps)
    th = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    th2, m, v = mlp.adam_step(th, g, np.zeros(4), np.zeros(4), 1, lr=0.1, eps=1e-8)
    assert np.allclose(th2, -0.1 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
