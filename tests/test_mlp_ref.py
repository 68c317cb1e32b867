"""Pins of the fp64 selector-network reference (CPU)."""
import numpy as np

from oracle import mlp_ref as M


def test_param_count():
    assert M.N_PARAMS == 4996


def test_parameter_layout():
    # the layout the library's header states: W1[64][8] b1[64] W2[64][64]
    # b2[64] W3[4][64] b3[4], row-major (out x in), in that order
    p = np.arange(M.N_PARAMS, dtype=np.float64)
    d = M.unpack(p)
    assert d["W1"][5, 3] == 5 * 8 + 3
    assert d["b1"][0] == 512 and d["b1"][63] == 575
    assert d["W2"][2, 7] == 576 + 2 * 64 + 7
    assert d["b2"][0] == 4672
    assert d["W3"][3, 63] == 4736 + 3 * 64 + 63
    assert list(d["b3"]) == [4992, 4993, 4994, 4995]
    assert np.array_equal(M.pack(d), p)


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
