"""Pins of the FP64 network oracle: central finite differences, and closed
forms for a network whose hidden layers are switched off."""
import numpy as np
import pytest

from oracle import mlp


def test_finite_differences():
    rng = np.random.default_rng(0)
    n_in, width, B = 5, 7, 11
    p = mlp.init_params(n_in, width, rng)
    X = rng.normal(size=(B, n_in))
    t = rng.normal(size=B)
    w = rng.uniform(0.2, 2.0, B)
    L, g = mlp.grad(p, X, t, w, n_in, width)
    assert L == pytest.approx(mlp.loss(p, X, t, w, n_in, width), rel=1e-14)
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        h = 1e-6 * max(1.0, abs(p[i]))
        e[i] = h
        fd = (mlp.loss(p + e, X, t, w, n_in, width) - mlp.loss(p - e, X, t, w, n_in, width)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-9)


def test_closed_form_constant_network():
    """All weights zero: y = b4; dL/db4 = 2 sum w (b4 - t) / sum w and
    dL/dW4 = dL/db4 * silu(silu(silu(b)))... with b = 0 -> silu(0) = 0, so
    only b4 receives a gradient."""
    n_in, width = 3, 4
    p = np.zeros(mlp.n_params(n_in, width))
    p[-1] = 0.7
    rng = np.random.default_rng(1)
    X = rng.normal(size=(6, n_in))
    t = rng.normal(size=6)
    w = rng.uniform(0.5, 1.5, 6)
    y = mlp.forward(p, X, n_in, width)
    np.testing.assert_array_equal(y, np.full(6, 0.7))
    L, g = mlp.grad(p, X, t, w, n_in, width)
    assert L == pytest.approx(np.sum(w * (0.7 - t) ** 2) / np.sum(w), rel=1e-15)
    assert g[-1] == pytest.approx(2 * np.sum(w * (0.7 - t)) / np.sum(w), rel=1e-15)
    np.testing.assert_array_equal(g[:-1], 0.0)


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    np.testing.assert_allclose(mlp.dsilu(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), rtol=1e-8, atol=1e-10)
    assert mlp.silu(0.0) == 0.0


def test_pack_roundtrip():
    rng = np.random.default_rng(2)
    p = mlp.init_params(4, 6, rng)
    np.testing.assert_array_equal(mlp.pack(mlp.unpack(p, 4, 6)), p)
    assert p.size == mlp.n_params(4, 6)


def test_skip_term_closed_form_and_finite_differences():
    """Skip connection y = net(x) + s x[col]: with every parameter zero the
    output is s x[col] exactly, the loss is the closed form and only b4
    gets a gradient, 2 sum w (s x[col] - t) / sum w; with random parameters
    the gradient still matches central finite differences."""
    n_in, width = 3, 4
    rng = np.random.default_rng(3)
    X = rng.normal(size=(6, n_in))
    t = rng.normal(size=6)
    w = rng.uniform(0.5, 1.5, 6)
    p = np.zeros(mlp.n_params(n_in, width))
    sk = (2, -0.5)
    y = mlp.forward(p, X, n_in, width, skip=sk)
    np.testing.assert_array_equal(y, -0.5 * X[:, 2])
    L, g = mlp.grad(p, X, t, w, n_in, width, skip=sk)
    assert L == pytest.approx(np.sum(w * (-0.5 * X[:, 2] - t) ** 2) / np.sum(w), rel=1e-15)
    assert g[-1] == pytest.approx(2 * np.sum(w * (-0.5 * X[:, 2] - t)) / np.sum(w), rel=1e-14)
    np.testing.assert_array_equal(g[:-1], 0.0)
    p = mlp.init_params(n_in, width, rng)
    L, g = mlp.grad(p, X, t, w, n_in, width, skip=sk)
    for i in rng.choice(p.size, 20, replace=False):
        e = np.zeros_like(p)
        h = 1e-6 * max(1.0, abs(p[i]))
        e[i] = h
        fd = (mlp.loss(p + e, X, t, w, n_in, width, skip=sk) - mlp.loss(p - e, X, t, w, n_in, width, skip=sk)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-9)
    # the skip term is the network's residual target: same gradient as a
    # network without it trained on t - s x[col]
    _, g0 = mlp.grad(p, X, t + 0.5 * X[:, 2], w, n_in, width)
    np.testing.assert_allclose(g, g0, rtol=1e-12, atol=1e-15)
