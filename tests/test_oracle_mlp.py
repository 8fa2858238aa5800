"""Pins of the FP64 network oracle: gradients against central finite
differences, Adam's closed-form first step, bf16 rounding rules, and that
training actually fits a smooth target."""
import numpy as np

from oracle import mlp_oracle as mo


def rand_setup(n=40, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, mo.N_PARAMS)
    X = rng.uniform(0, 1, (n, 8))
    X[:, 6:] = 0.0
    t = np.sin(3 * X[:, 0]) + X[:, 1] ** 2
    wts = rng.uniform(0.1, 1.0, n)
    wts /= wts.sum()
    return theta, X, t, wts


def test_parameter_count():
    assert mo.N_PARAMS == 8 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1 == 8961


def test_gradient_matches_finite_differences():
    theta, X, t, wts = rand_setup()
    L, g = mo.loss_and_grad(theta, X, t, wts)
    assert np.isclose(L, mo.loss(theta, X, t, wts))
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mo.N_PARAMS, 300, replace=False), [0, 575, 576, 8959, 8960]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mo.loss(theta + e, X, t, wts) - mo.loss(theta - e, X, t, wts)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2: the update is -lr * g / (|g| + eps)
    theta, X, t, wts = rand_setup()
    _, g = mo.loss_and_grad(theta, X, t, wts)
    new, m, v = mo.adam(theta, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    np.testing.assert_allclose(new - theta, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_training_fits_smooth_target():
    theta, X, t, wts = rand_setup(n=200)
    L0 = mo.loss(theta, X, t, wts)
    theta2, losses = mo.train(theta, X, t, wts, 400, 3e-3)
    assert losses[-1] < 0.05 * L0


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159265], dtype=np.float32)
    r = mo.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie -> even
    assert r[2] == 1.0 + 2 ** -7             # above half -> up
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-12
    theta, X, t, wts = rand_setup()
    y, _ = mo.forward(theta, X)
    yb = mo.forward_bf16(theta, X)
    assert np.max(np.abs(yb - y)) < 0.05 * (1 + np.max(np.abs(y)))
