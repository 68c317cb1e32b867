"""Pins of the fp64 selector-network reference (CPU)."""
import numpy as np

from oracle import mlp_ref as M


def test_param_count():
    assert M.N_PARAMS == 4996


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = M.init_params(3) + rng.standard_normal(M.N_PARAMS) * 0.05
    x = rng.standard_normal((7, 8))
    t = rng.standard_normal((7, 4))
    mask = (rng.random((7, 4)) < 0.8).astype(float)
    g = M.grad(p, x, t, mask)
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (M.loss(p + e, x, t, mask) - M.loss(p - e, x, t, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_closed_forms():
    # zero weights: output is the last bias, and only the last bias has gradient
    p = np.zeros(M.N_PARAMS)
    d = M.unpack(p)
    d["b3"] = np.array([1.0, -2.0, 0.5, 3.0])
    p = M.pack(d)
    x = np.random.default_rng(2).standard_normal((5, 8))
    y, _ = M.forward(p, x)
    assert np.allclose(y, d["b3"])
    t = np.zeros((5, 4))
    g = M.unpack(M.grad(p, x, t))
    assert np.allclose(g["b3"], 2 * d["b3"] / 4)     # d/db of mean over 20 entries of b^2
    for name in ("W1", "b1", "W2", "b2", "W3"):
        assert not np.any(g[name])
    # a single ReLU path: y = w3 * relu(w2 * relu(w1 . x))
    d = M.unpack(np.zeros(M.N_PARAMS))
    d["W1"][0, 0] = 2.0
    d["W2"][0, 0] = 3.0
    d["W3"][0, 0] = 0.5
    y, _ = M.forward(M.pack(d), np.array([[1.5, 0, 0, 0, 0, 0, 0, 0], [-1.0, 0, 0, 0, 0, 0, 0, 0]]))
    assert np.allclose(y[:, 0], [0.5 * 3.0 * 2.0 * 1.5, 0.0])
