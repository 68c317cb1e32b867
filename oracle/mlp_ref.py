"""fp64 reference of the kernel-selector network (test infrastructure only).

Network: x (8) -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2) (64)
-> y = W3 h2 + b3 (4).  Loss: sum(mask * (y - t)^2) / mask_count.  The
parameter vector is laid out as W1[64][8], b1[64], W2[64][64], b2[64],
W3[4][64], b3[4] (row-major, out x in), 4996 values.

Plain numpy: the forward pass and the chain rule written out layer by layer,
used to check the GPU kernels' outputs and gradients.
"""
import numpy as np

N_IN, N_HID, N_OUT = 8, 64, 4
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(p, x):
    """x: (B, 8) -> y: (B, 4), plus the intermediates."""
    P = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"].T + P["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(p, x, t, mask=None):
    y, _ = forward(p, x)
    m = np.ones_like(y) if mask is None else np.asarray(mask, dtype=np.float64)
    return float(np.sum(m * (y - t) ** 2) / np.sum(m))


def grad(p, x, t, mask=None):
    """Gradient of loss() w.r.t. the parameter vector (chain rule by hand)."""
    P = unpack(p)
    y, (x, z1, h1, z2, h2) = forward(p, x)
    m = np.ones_like(y) if mask is None else np.asarray(mask, dtype=np.float64)
    dy = 2.0 * m * (y - t) / np.sum(m)
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dz2 = (dy @ P["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def init_params(seed=0, scale=1.0):
    """He-style initialisation (deterministic)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            d[name] = rng.standard_normal(shape) * scale * np.sqrt(2.0 / shape[1])
        else:
            d[name] = np.zeros(shape)
    return pack(d)
