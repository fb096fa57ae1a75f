"""Training the constraint-proposal scorer of the learned form on the GPU.

Marshalling only: the training rows are written by the library's clip during
plain marches (am_prop_collect), and the loss, its gradient and the Adam
updates run in the library's kernels (am_prop_grad, am_prop_adam).  Training
is full-batch Adam on the mean binary cross-entropy of "this line carries an
edge of the cell's face".
"""
from __future__ import annotations

import time

import numpy as np

from .binding import Context

D, H = 32, 128
N_FEATURES = 8


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (fan-in of the features in use for W1), zero biases,
    b3 at the log-odds of a 1-in-10 label rate."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((H, D))
    W1[:, :N_FEATURES] = rng.normal(0.0, np.sqrt(2.0 / N_FEATURES), (H, N_FEATURES))
    W2 = rng.normal(0.0, np.sqrt(2.0 / H), (H, H))
    w3 = rng.normal(0.0, np.sqrt(1.0 / H), H)
    p = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, [np.log(1.0 / 9.0)]])
    return p.astype(np.float32)


def collect(ctx: Context, orig, dirs, cap: int, rho: float = 6.0, max_cells: int = 1 << 24):
    """Marches (plain form) from the rays and returns the training rows the
    clip wrote: (X [n][32] float32, y [n] uint8) device tensors, n <= cap."""
    torch = ctx.torch
    X = torch.empty((cap, D), dtype=torch.float32, device=ctx.device)
    y = torch.empty(cap, dtype=torch.uint8, device=ctx.device)
    ctx.prop_collect(X, y, rho=rho)
    try:
        ctx.seed_rays(orig, dirs)
        ctx.march(max_cells=max_cells)
        n = min(ctx.prop_collected(), cap)
    finally:
        ctx.prop_collect(None, None)
    return X[:n], y[:n]


def train(ctx: Context, X, y, steps: int = 300, lr: float = 3e-3, seed: int = 0, log_every: int = 0):
    """Full-batch Adam on the scorer; returns (host float32 params, losses)."""
    torch = ctx.torch
    p = torch.as_tensor(init_params(seed), device=ctx.device)
    g = torch.zeros_like(p)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    losses = []
    t0 = time.perf_counter()
    for it in range(1, steps + 1):
        loss = ctx.prop_grad(X, y, p, g)
        ctx.prop_adam(p, g, m, v, it, lr)
        losses.append(loss)
        if log_every and (it % log_every == 0 or it == 1):
            print(f"[train] step {it} loss {loss:.5f} ({time.perf_counter() - t0:.1f} s)", flush=True)
    torch.cuda.synchronize(ctx.device)
    return p.cpu().numpy(), losses
