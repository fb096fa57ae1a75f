"""Fit ReLU MLP fixtures to analytic signed distance targets (input generation).

The fitted nets stand in for the paper's per-shape SDF fits (the ShapeNet fits
behind Tables 1-4 are not available).  Fitting is plain PyTorch (on the CPU by
default, or on a GPU with --device; the wider fits were made that way) and has
nothing to do with the meshing method; the resulting weights are frozen files
under ``am_workloads/data`` whose SHA-256 is recorded in ``FIXTURES.sha256``.

    python -m am_workloads.fit c2        # 3->[90]x6->1, 8 spheres, seed 1
    python -m am_workloads.fit c3 --device cuda --out /tmp/fits   # 3->[256]x8->1, superquadrics
    python -m am_workloads.fit c4 --device cuda   # 64-shape auto-decoder [x; z] -> [512]x8 -> 1
    python -m am_workloads.fit c4-boxes           # its per-shape domain boxes (CPU, FP64)

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


# ---------------------------------------------------------------------------
# The batched workload: one latent-conditioned decoder trained as an
# auto-decoder (one learned latent per shape, as in DeepSDF) on 64 sphere
# unions of very different sizes.
# ---------------------------------------------------------------------------

DECODER = dict(hidden=[512] * 8, latent=256, reinject=4, shapes=64, seed=3, steps=2500,
               points_per_shape=2048, pool_per_shape=16384, scale=(0.03, 0.6), clamp=0.1,
               lr=5e-4, lr_latent=1e-3, latent_std=0.01, latent_reg=1e-4)


def decoder_shapes(rng, n_shapes, scale):
    """Shape i: a union of k_i ~ U{1..8} spheres (centres U[-0.5, 0.5]^3, radii
    U[0.15, 0.35]) scaled about the origin by s_i, log-uniform over `scale`
    (draws in that order, shape by shape), then ordered by s_i."""
    shapes = []
    for _ in range(n_shapes):
        k = int(rng.integers(1, 9))
        c = rng.uniform(-0.5, 0.5, (k, 3))
        r = rng.uniform(0.15, 0.35, k)
        s = float(np.exp(rng.uniform(np.log(scale[0]), np.log(scale[1]))))
        shapes.append((c * s, r * s, s))
    # shape index = rank of the scale (smallest first)
    return sorted(shapes, key=lambda sh: sh[2])


def decoder_samples(rng, shape, n):
    """n SDF samples of one shape: half uniform in [-1, 1]^3, half near its
    surface (random sphere, random direction, radial jitter N(0, (0.05 s)^2))."""
    c, r, s = shape
    half = n // 2
    xu = rng.uniform(-1.0, 1.0, (half, 3))
    idx = rng.integers(0, c.shape[0], n - half)
    dirs = rng.normal(0.0, 1.0, (n - half, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    jit = rng.normal(0.0, 0.05 * s, n - half)
    xs = c[idx] + dirs * (r[idx] + jit)[:, None]
    x = np.concatenate([xu, xs], axis=0)
    return x, sphere_sdf(x, c, r)


def fit_decoder(steps: int | None = None, device: str = "cpu", out_dir: str | None = None, log_every: int = 100):
    """Trains [x; z] (3 + 256) -> [512] x 8 -> 1 with [x; z] entering layer 1
    and again layer 4, jointly with one latent per shape (init N(0, 0.01^2)):
    Adam on the clamped L1 loss |clamp(f) - clamp(sdf)| (clamp 0.1) plus
    1e-4 |z|^2, 2048 points per shape per step from a pool of 16384.
    He-normal weights, biases N(0, 0.01^2).  Stores the decoder and latents."""
    import torch
    P = DECODER
    steps = P["steps"] if steps is None else steps
    rng = np.random.default_rng(P["seed"])
    shapes = decoder_shapes(rng, P["shapes"], P["scale"])
    pools = [decoder_samples(rng, sh, P["pool_per_shape"]) for sh in shapes]
    X = torch.tensor(np.stack([p[0] for p in pools]), dtype=torch.float32, device=device)   # [S, pool, 3]
    Y = torch.tensor(np.stack([p[1] for p in pools]), dtype=torch.float32, device=device)   # [S, pool]
    S, D, H = P["shapes"], P["latent"], P["hidden"]
    n_in = 3 + D
    Ws, bs = [], []
    for l, h in enumerate(H + [1]):
        fan = n_in if l == 0 else H[l - 1] + (n_in if l + 1 == P["reinject"] else 0)
        Ws.append(torch.tensor(rng.normal(0.0, np.sqrt(2.0 / fan), (h, fan)), dtype=torch.float32, device=device,
                               requires_grad=True))
        bs.append(torch.tensor(rng.normal(0.0, 0.01, h), dtype=torch.float32, device=device, requires_grad=True))
    Z = torch.tensor(rng.normal(0.0, P["latent_std"], (S, D)), dtype=torch.float32, device=device,
                     requires_grad=True)
    opt = torch.optim.Adam([{"params": Ws + bs, "lr": P["lr"]}, {"params": [Z], "lr": P["lr_latent"]}])
    g = torch.Generator(device="cpu").manual_seed(P["seed"])
    cl = P["clamp"]
    t0 = time.time()

    def forward(x, z):
        inp = torch.cat([x, z], dim=-1)
        h = inp
        for l in range(len(H)):
            if l + 1 == P["reinject"]:
                h = torch.cat([h, inp], dim=-1)
            h = torch.relu(h @ Ws[l].T + bs[l])
        return (h @ Ws[-1].T + bs[-1])[..., 0]

    for it in range(steps):
        idx = torch.randint(0, X.shape[1], (S, P["points_per_shape"]), generator=g).to(device)
        x = torch.gather(X, 1, idx[..., None].expand(-1, -1, 3))
        y = torch.gather(Y, 1, idx)
        z = Z[:, None, :].expand(-1, x.shape[1], -1)
        f = forward(x, z)
        loss = (f.clamp(-cl, cl) - y.clamp(-cl, cl)).abs().mean() + P["latent_reg"] * (Z ** 2).sum(dim=1).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        if it % log_every == 0 or it == steps - 1:
            print(f"[fit c4] step {it} loss {loss.item():.5f} ({time.time() - t0:.0f}s)", flush=True)
    out_dir = out_dir or DATA_DIR
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "c4.npz")
    arrs = {f"W{l}": W.detach().cpu().numpy().astype(np.float32) for l, W in enumerate(Ws)}
    arrs.update({f"b{l}": b.detach().cpu().numpy().astype(np.float32) for l, b in enumerate(bs)})
    arrs["Z"] = Z.detach().cpu().numpy().astype(np.float32)
    arrs["reinject"] = np.asarray(P["reinject"])
    np.savez(path, **arrs)
    meta = os.path.join(out_dir, "c4_shapes.npz")
    centres = np.full((S, 8, 3), np.nan)
    radii = np.full((S, 8), np.nan)
    for i, (c, r, _) in enumerate(shapes):
        centres[i, :len(r)] = c
        radii[i, :len(r)] = r
    np.savez(meta, scale=np.asarray([sh[2] for sh in shapes]), spheres=np.asarray([len(sh[1]) for sh in shapes]),
             centres=centres, radii=radii)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    print(f"[fit c4] wrote {path} sha256 {digest} final loss {loss.item():.5f}", flush=True)
    return path, digest


# Per-shape domain boxes of the batched workload: shape s is marched in the
# box of half-size h_s (log-spaced over the shapes) centred on a point of its
# learned surface, so that the shapes' cell counts are uneven while the
# decoder stays one trained network.
C4_BOX_HALF = (1.2e-3, 0.125)


def decoder_forward(arrs, x, z):
    """The stored decoder on points x [n, 3] with latent z [D], in FP64."""
    reinject = int(arrs["reinject"])
    n_w = len([k for k in arrs.files if k.startswith("W")])
    inp = np.concatenate([x, np.broadcast_to(z, (x.shape[0], z.shape[0]))], axis=1)
    h = inp
    for l in range(n_w - 1):
        if l + 1 == reinject:
            h = np.concatenate([h, inp], axis=1)
        h = np.maximum(h @ arrs[f"W{l}"].astype(np.float64).T + arrs[f"b{l}"].astype(np.float64), 0.0)
    return (h @ arrs[f"W{n_w - 1}"].astype(np.float64).T + arrs[f"b{n_w - 1}"].astype(np.float64))[:, 0]


def c4_boxes(out_dir: str | None = None):
    """Writes c4_boxes.npz: for shape s, the centre p_s (a zero of its learned
    SDF, by bisection along +x from the first sphere centre of its target
    union where the SDF is negative), the half-size h_s = h_0 (h_1/h_0)^(s/63)
    and a seed segment p_s + h_s t e_x, t in [-a_s, a_s], whose ends have
    opposite signs (a_s = 0.5, halved until they do)."""
    out_dir = out_dir or DATA_DIR
    arrs = np.load(os.path.join(out_dir, "c4.npz"), allow_pickle=False)
    meta = np.load(os.path.join(out_dir, "c4_shapes.npz"), allow_pickle=False)
    Z = arrs["Z"].astype(np.float64)
    S = Z.shape[0]
    h0, h1 = C4_BOX_HALF
    half = h0 * (h1 / h0) ** (np.arange(S) / (S - 1))
    centre = np.zeros((S, 3))
    seed_a = np.zeros(S)
    ex = np.array([1.0, 0.0, 0.0])
    for s in range(S):
        z = Z[s]
        f = lambda x: decoder_forward(arrs, np.atleast_2d(x), z)[0]
        found = False
        for k in range(int(meta["spheres"][s])):
            c, r = meta["centres"][s, k], float(meta["radii"][s, k])
            if not f(c) < 0.0:
                continue
            lo, hi = 0.0, 3.0 * r
            if not f(c + hi * ex) > 0.0:
                continue
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if mid <= lo or mid >= hi:
                    break
                if f(c + mid * ex) < 0.0:
                    lo = mid
                else:
                    hi = mid
            p = c + lo * ex
            a = 0.5
            while a > 1e-6 and not (f(p - a * half[s] * ex) < 0.0 < f(p + a * half[s] * ex)):
                a *= 0.5
            if a > 1e-6:
                centre[s], seed_a[s] = p, a
                found = True
                break
        if not found:
            raise RuntimeError(f"shape {s}: no sign change found along +x from its sphere centres")
    path = os.path.join(out_dir, "c4_boxes.npz")
    np.savez(path, centre=centre, half=half, seed_a=seed_a)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    print(f"[fit c4] wrote {path} sha256 {digest}", flush=True)
    return path, digest


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(SPECS) + ["c4", "c4-boxes"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--device", default="cpu")
    ap.add_argument("--out", default=None, help="output folder (default: am_workloads/data)")
    a = ap.parse_args(argv)
    if a.name == "c4":
        fit_decoder(a.steps, device=a.device, out_dir=a.out)
        c4_boxes(a.out)
    elif a.name == "c4-boxes":
        c4_boxes(a.out)
    else:
        fit(a.name, a.steps, a.threads, device=a.device, out_dir=a.out)


if __name__ == "__main__":
    main()
