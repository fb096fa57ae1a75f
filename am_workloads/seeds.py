"""Seeded ray sets for triggering (input generation only).

A ray is a segment ``o + t d, t in [0, 1]``; the seeding step bisects it for a
zero crossing of F (Sec. 4.3.2 of the paper uses dichotomy; the paper's runs
trigger from 1,024 surface points per shape, Table 3).  Segments are shortened
so they end inside the domain box [-1, 1]^3.
"""
from __future__ import annotations

import numpy as np


def fibonacci_dirs(n: int) -> np.ndarray:
    """n unit vectors spread over the sphere (golden-angle spiral)."""
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * i
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def clip_to_box(origins: np.ndarray, dirs: np.ndarray, t_max: float = 1.0, box: float = 1.0):
    """Scale each direction so that o + d stays in the box (t in [0, 1])."""
    origins = np.asarray(origins, np.float64)
    dirs = np.asarray(dirs, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        tp = np.where(dirs > 0, (box - origins) / dirs, np.inf)
        tn = np.where(dirs < 0, (-box - origins) / dirs, np.inf)
    t_exit = np.minimum(tp, tn).min(axis=1)
    t = np.minimum(t_max, t_exit * (1.0 - 1e-9))
    return origins, dirs * t[:, None]


def axis_ray():
    """One ray from the origin along +x (length 1)."""
    return np.zeros((1, 3)), np.array([[1.0, 0.0, 0.0]])


def centre_rays(centres: np.ndarray, per_centre: int = 128):
    """per_centre Fibonacci directions from each centre, clipped to the box."""
    d = fibonacci_dirs(per_centre)
    o = np.repeat(np.asarray(centres, np.float64), per_centre, axis=0)
    dd = np.tile(d, (len(centres), 1))
    return clip_to_box(o, dd)


def random_rays(n: int, seed: int, origin_scale: float = 0.1):
    """n rays from near the origin in uniformly random directions."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-origin_scale, origin_scale, (n, 3))
    d = rng.normal(0.0, 1.0, (n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return clip_to_box(o, d)
