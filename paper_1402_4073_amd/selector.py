"""Training and evaluation driver of the kernel-variant selector.

The network's forward, backward and Adam steps run in the library's HIP
kernels (tq_mlp_grad, tq_mlp_adam); this module only moves arrays and loops
over epochs.  Targets are log run times of the four variants measured on the
GPU; queries whose variant could not run carry a zero mask for that target.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as tq


def normalisation(X: np.ndarray):
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 1e-6, std, 1.0)
    return mean.astype(np.float32), std.astype(np.float32)


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initial weights, zero biases (layout of tq.h)."""
    rng = np.random.default_rng(seed)
    parts = []
    for out_d, in_d in ((64, 8), (64, 64), (4, 64)):
        parts.append(rng.standard_normal((out_d, in_d)) * np.sqrt(2.0 / in_d))
        parts.append(np.zeros(out_d))
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def train(ctx: int, X: np.ndarray, T: np.ndarray, M: np.ndarray | None = None, epochs: int = 3000,
          lr: float = 3e-3, seed: int = 0, device: str = "cuda:0"):
    """Full-batch Adam on the GPU.  X: (B, 8) normalised features, T: (B, 4)
    targets.  Returns (params, loss history)."""
    B = X.shape[0]
    d = torch.device(device)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(d)
    t = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(d)
    m = None if M is None else torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).to(d)
    count = float(B * T.shape[1] if M is None else M.sum())
    p = torch.from_numpy(init_params(seed)).to(d)
    g = torch.zeros_like(p)
    mo = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = torch.zeros(1, dtype=torch.float32, device=d)
    hist = []
    for step in range(1, epochs + 1):
        tq.tq_mlp_grad(ctx, p, x, t, m, B, count, None, g, loss)
        tq.tq_mlp_adam(ctx, p, g, mo, v, p.numel(), lr, 0.9, 0.999, 1e-8, step)
        if step % 100 == 0 or step == 1:
            hist.append((step, float(loss.item())))
    torch.cuda.synchronize()
    return p.cpu().numpy(), hist


def predict(ctx: int, params: np.ndarray, X: np.ndarray, device: str = "cuda:0") -> np.ndarray:
    """Batched GPU inference (tq_mlp_forward) on normalised features."""
    d = torch.device(device)
    p = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).to(d)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(d)
    y = torch.zeros((X.shape[0], 4), dtype=torch.float32, device=d)
    tq.tq_mlp_forward(ctx, p, x, X.shape[0], y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


DEFAULT_WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(__file__), "data",
                                             "selector_mi355x.json")


def load_default(ctx: int, path: str = DEFAULT_WEIGHTS) -> dict:
    """Install the weights trained on this GPU model (see data/) into a context."""
    import json
    with open(path) as fh:
        w = json.load(fh)
    tq.tq_selector_set(ctx, np.array(w["params"], dtype=np.float32), np.array(w["mean"], dtype=np.float32),
                       np.array(w["std"], dtype=np.float32), np.array(w["lo"], dtype=np.float32),
                       np.array(w["hi"], dtype=np.float32), float(w["margin"]))
    return w


def regret(times: np.ndarray, chosen: np.ndarray) -> dict:
    """Workload regret sum(t_chosen)/sum(t_best) - 1 and mean per-query
    (t - t_best)/t_best, times in seconds (B, 4) with inf for unavailable."""
    best = times.min(axis=1)
    sel = times[np.arange(times.shape[0]), chosen]
    return {"workload": float(sel.sum() / best.sum() - 1.0),
            "per_query_mean": float(np.mean((sel - best) / best))}
