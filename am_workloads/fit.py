"""Fit ReLU MLP fixtures to analytic signed distance targets (input generation).

The fitted nets stand in for the paper's per-shape SDF fits (the ShapeNet fits
behind Tables 1-4 are not available).  Fitting is plain PyTorch (on the CPU by
default, or on a GPU with --device; the wider fits were made that way) and has
nothing to do with the meshing method; the resulting weights are frozen files
under ``am_workloads/data`` whose SHA-256 is recorded in ``FIXTURES.sha256``.

    python -m am_workloads.fit c2        # 3->[90]x6->1, 8 spheres, seed 1
    python -m am_workloads.fit c3 --device cuda --out /tmp/fits   # 3->[256]x8->1, superquadrics

Recipe (one reading of the workload description):
    targets: union of 8 spheres (c ~ U[-0.5,0.5]^3, r ~ U[0.15,0.35]) or of 8
    superquadrics; 2^18 samples, half uniform in [-1,1]^3 and half near the
    surface (random primitive, random direction, radial jitter N(0, 0.05^2));
    W ~ N(0, 2/fan_in), b ~ N(0, 0.01^2); full-batch Adam (lr 1e-4,
    betas 0.9/0.999), L1 loss; stored as float32.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

from .nets import DATA_DIR, Net, he_mlp, mlp_net

SPECS = {
    # name: hidden widths, seed, target kind, steps
    "c2": dict(hidden=[90] * 6, seed=1, target="spheres", steps=3000),
    "c3": dict(hidden=[256] * 8, seed=2, target="superquadrics", steps=3000),
    "c5": dict(hidden=[512] * 8, seed=4, target="spheres", steps=3000),
}


def sphere_params(rng, n=8):
    c = rng.uniform(-0.5, 0.5, (n, 3))
    r = rng.uniform(0.15, 0.35, n)
    return c, r


def sphere_sdf(x, c, r):
    d = np.linalg.norm(x[:, None, :] - c[None], axis=-1) - r[None]
    return d.min(axis=1)


def superquadric_params(rng, n=8):
    c = rng.uniform(-0.5, 0.5, (n, 3))
    a = rng.uniform(0.15, 0.35, (n, 3))
    e = rng.uniform(0.4, 1.6, (n, 2))
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    R = np.empty((n, 3, 3))
    for i, (w, x, y, z) in enumerate(q):
        R[i] = [[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]]
    return c, a, e, R


def superquadric_sdf(x, c, a, e, R):
    out = np.full(x.shape[0], np.inf)
    for k in range(c.shape[0]):
        p = (x - c[k]) @ R[k]                      # R^T (x - c)
        e1, e2 = e[k]
        t = np.abs(p) / a[k] + 1e-12
        g = (t[:, 0] ** (2 / e2) + t[:, 1] ** (2 / e2)) ** (e2 / e1) + t[:, 2] ** (2 / e1)
        out = np.minimum(out, a[k].min() * (g ** (e1 / 2) - 1.0))
    return out


def make_samples(rng, kind, n_samples, prim):
    half = n_samples // 2
    xu = rng.uniform(-1.0, 1.0, (half, 3))
    idx = rng.integers(0, prim[0].shape[0], n_samples - half)
    dirs = rng.normal(0.0, 1.0, (n_samples - half, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    jitter = rng.normal(0.0, 0.05, n_samples - half)
    if kind == "spheres":
        c, r = prim
        xs = c[idx] + dirs * (r[idx] + jitter)[:, None]
    else:
        c, a = prim[0], prim[1]
        xs = c[idx] + dirs * (a[idx].mean(axis=1) + jitter)[:, None]
    x = np.concatenate([xu, xs], axis=0)
    y = sphere_sdf(x, *prim) if kind == "spheres" else superquadric_sdf(x, *prim)
    return x, y


def fit(name: str, steps: int | None = None, threads: int | None = None, log_every: int = 100,
        device: str = "cpu", out_dir: str | None = None):
    import torch
    spec = SPECS[name]
    steps = spec["steps"] if steps is None else steps
    if threads:
        torch.set_num_threads(threads)
    rng = np.random.default_rng(spec["seed"])
    Ws, bs = he_mlp(spec["hidden"], spec["seed"], 0.01)
    prim = sphere_params(rng) if spec["target"] == "spheres" else superquadric_params(rng)
    x, y = make_samples(rng, spec["target"], 1 << 18, prim)
    X = torch.tensor(x, dtype=torch.float32, device=device)
    Y = torch.tensor(y, dtype=torch.float32, device=device)
    params = []
    for W, b in zip(Ws, bs):
        params += [torch.tensor(W, dtype=torch.float32, device=device, requires_grad=True),
                   torch.tensor(b, dtype=torch.float32, device=device, requires_grad=True)]
    opt = torch.optim.Adam(params, lr=1e-4, betas=(0.9, 0.999))
    t0 = time.time()
    for it in range(steps):
        h = X
        for i in range(0, len(params) - 2, 2):
            h = torch.relu(h @ params[i].T + params[i + 1])
        out = (h @ params[-2].T + params[-1])[:, 0]
        loss = (out - Y).abs().mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        if it % log_every == 0 or it == steps - 1:
            print(f"[fit {name}] step {it} loss {loss.item():.5f} ({time.time() - t0:.0f}s)", flush=True)
    Wf = [p.detach().cpu().numpy().astype(np.float64) for p in params[0::2]]
    bf = [p.detach().cpu().numpy().astype(np.float64) for p in params[1::2]]
    net = mlp_net(Wf, bf)
    out_dir = out_dir or DATA_DIR
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"{name}.npz")
    net.save(path, dtype=np.float32)
    meta = os.path.join(out_dir, f"{name}_primitives.npz")
    np.savez(meta, **{f"p{i}": np.asarray(p) for i, p in enumerate(prim)})
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    print(f"[fit {name}] wrote {path} sha256 {digest} final loss {loss.item():.5f}", flush=True)
    return path, digest


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(SPECS))
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--device", default="cpu")
    ap.add_argument("--out", default=None, help="output folder (default: am_workloads/data)")
    a = ap.parse_args(argv)
    fit(a.name, a.steps, a.threads, device=a.device, out_dir=a.out)


if __name__ == "__main__":
    main()
