"""Pins of the FP64 proposal-scorer reference (oracle/proposer.py).

The gradient is pinned by central finite differences of the loss (brute force,
independent of the chain-rule code), the loss by closed forms at special
points, Adam by its first-step closed form; planted mistakes must fail.
"""
import numpy as np
import pytest

from oracle import proposer as P


def _problem(d=5, H=7, n=40, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.6, P.n_params(d, H))
    X = rng.normal(0.0, 1.0, (n, d))
    y = (rng.random(n) < 0.4).astype(np.float64)
    return p, X, y


def _fd_grad(p, X, y, d, H, h=1e-6):
    g = np.empty_like(p)
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        g[i] = (P.loss_and_grad(p + e, X, y, d, H)[0] - P.loss_and_grad(p - e, X, y, d, H)[0]) / (2 * h)
    return g


def _kink_free(p, X, d, H, margin=1e-3):
    W1, b1, W2, b2, _, _ = P.unpack(p, d, H)
    a1 = X @ W1.T + b1
    a2 = np.maximum(a1, 0) @ W2.T + b2
    return np.abs(a1).min() > margin and np.abs(a2).min() > margin


@pytest.mark.parametrize("seed", [0, 1, 3])
def test_gradient_matches_finite_differences(seed):
    d, H = 5, 7
    p, X, y = _problem(d, H, seed=seed)
    assert _kink_free(p, X, d, H)
    _, g = P.loss_and_grad(p, X, y, d, H)
    fd = _fd_grad(p, X, y, d, H)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.abs(fd).max())


@pytest.mark.parametrize("mutant", [1, 2, 3])
def test_planted_mistakes_fail_the_finite_difference_pin(mutant):
    d, H = 5, 7
    p, X, y = _problem(d, H, seed=0)
    _, g = P.loss_and_grad(p, X, y, d, H, _mutate=mutant)
    fd = _fd_grad(p, X, y, d, H)
    assert np.max(np.abs(g - fd)) > 1e-4


def test_zero_network_loss_is_log2_and_bias_gradient_closed_form():
    d, H = 4, 6
    p = np.zeros(P.n_params(d, H))
    rng = np.random.default_rng(3)
    X = rng.normal(size=(25, d))
    y = (rng.random(25) < 0.3).astype(np.float64)
    loss, g = P.loss_and_grad(p, X, y, d, H)
    assert abs(loss - np.log(2.0)) < 1e-15
    # z = 0 everywhere: dL/db3 = mean(1/2 - y); every other gradient is 0 (dead ReLUs, zero w3)
    assert abs(g[-1] - np.mean(0.5 - y)) < 1e-15
    assert np.all(g[:-1] == 0.0)


def test_large_logits_do_not_overflow_and_match_the_limit():
    d, H = 3, 4
    p = np.zeros(P.n_params(d, H))
    p[-1] = 800.0                       # z = 800 for every row
    X = np.zeros((4, d))
    y = np.array([1.0, 0.0, 1.0, 0.0])
    loss, g = P.loss_and_grad(p, X, y, d, H)
    # rows with y=1 cost log(1+e^-800) ~ 0, rows with y=0 cost ~800
    assert abs(loss - 400.0) < 1e-9
    assert abs(g[-1] - 0.5) < 1e-12    # mean(sigmoid(800) - y) = 1/2


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.normal(size=10)
    g = rng.normal(size=10)
    p1, m, v = P.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01, eps=0.0)
    # bias-corrected first moments equal g and g^2: the step is lr * sign(g)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
