"""Pins of the FP64 reference network: its gradient against central finite
differences of its own loss, GELU against its definition, and the AdamW step
against the closed forms of its first steps."""
import math

import numpy as np

from oracle import mlp


def _batch(rng, rows=7):
    X = np.zeros((rows, mlp.IN))
    k = rng.integers(3, 20, rows)
    for r in range(rows):
        X[r, :2 * k[r]] = rng.normal(0, 1, 2 * k[r])
        X[r, 2 * mlp.SLOTS:2 * mlp.SLOTS + k[r]] = 1.0
    X[:, 3 * mlp.SLOTS] = rng.integers(0, 2, rows)
    T = np.zeros((rows, mlp.OUT))
    T[:, :mlp.SLOTS] = rng.integers(0, 2, (rows, mlp.SLOTS))
    T[:, mlp.SLOTS:] = rng.uniform(0, 1, (rows, mlp.SLOTS))
    return X, T


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = mlp.init_params(3) * 0.5
    X, T = _batch(rng)
    _, g = mlp.loss_and_grad(theta, X, T, wf=0.7)
    idx = np.concatenate([rng.integers(0, mlp.NPARAMS, 40),
                          [mlp.NPARAMS - 1, 128 * 128, 128 * 128 + 128 + 5]])
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = eps
        lp, _ = mlp.loss_and_grad(theta + e, X, T, wf=0.7)
        lm, _ = mlp.loss_and_grad(theta - e, X, T, wf=0.7)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_gelu_definition():
    """The tanh form of GELU, written out per element; it stays within 5e-4 of
    the exact z * Phi(z) (normal CDF via erf), and its derivative matches
    central differences."""
    z = np.linspace(-8, 8, 3201)
    c = math.sqrt(2.0 / math.pi)
    ref = np.array([0.5 * v * (1 + math.tanh(c * (v + 0.044715 * v ** 3))) for v in z])
    np.testing.assert_allclose(mlp.gelu(z), ref, rtol=1e-14, atol=1e-15)
    exact = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in z])
    assert np.abs(mlp.gelu(z) - exact).max() <= 5e-4
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-8)


def test_masked_slots_do_not_contribute():
    rng = np.random.default_rng(2)
    theta = mlp.init_params(4)
    X, T = _batch(rng)
    X[:, 2 * mlp.SLOTS + 25:3 * mlp.SLOTS] = 0.0
    l1, _ = mlp.loss_and_grad(theta, X, T)
    T2 = T.copy()
    T2[:, 25:mlp.SLOTS] = 1 - T2[:, 25:mlp.SLOTS]
    T2[:, mlp.SLOTS + 25:] += 3.0
    l2, _ = mlp.loss_and_grad(theta, X, T2)
    assert l1 == l2


def test_adamw_first_steps_closed_form():
    """Step 1 of Adam moves every parameter by lr * g / (|g| + eps): the bias
    corrections turn the first moments back into g and g^2.  With a constant
    gradient every later step does the same.  The decoupled weight decay adds
    lr * wd * w, whatever the gradient (also where it is zero)."""
    rng = np.random.default_rng(5)
    w = rng.normal(0, 1, 50)
    g = rng.normal(0, 1e-2, 50)
    g[:5] = 0.0
    lr, wd, eps = 1e-3, 0.01, 1e-8
    m = v = np.zeros(50)
    w1, m, v = mlp.adamw_step(w, g, m, v, 1, lr, wd, eps=eps)
    np.testing.assert_allclose(w1, w - lr * (g / (np.abs(g) + eps) + wd * w), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14, atol=0)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14, atol=0)
    w2, m, v = mlp.adamw_step(w1, g, m, v, 2, lr, wd, eps=eps)
    np.testing.assert_allclose(w2, w1 - lr * (g / (np.abs(g) + eps) + wd * w1), rtol=0, atol=1e-15)
    # a sign flip of the gradient: m_hat = (0.09 g - 0.1 g) / 0.19, v_hat = g^2 (both steps' |g| equal)
    with np.errstate(divide="ignore", invalid="ignore"):   # the zero gradients, eps = 0
        w3, _, _ = mlp.adamw_step(w1, -g, 0.1 * g, 0.001 * g * g, 2, lr, 0.0, eps=0.0)
    mh = (0.9 * 0.1 * g - 0.1 * g) / (1 - 0.81)
    nz = g != 0
    np.testing.assert_allclose(w3[nz], w1[nz] - lr * mh[nz] / np.abs(g[nz]), rtol=1e-12)
