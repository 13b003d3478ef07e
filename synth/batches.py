"""Seeded ray and point batches for the ray-batch and encoder entry points."""
from __future__ import annotations

import numpy as np


def random_rays(n: int, seed: int, distance: float = 2.0, spread: float = 0.35,
                center=(0.5, 0.5, 0.5)):
    """Origins on a sphere of radius `distance` about `center`; directions
    aimed at `center` plus a uniform offset of up to `spread` per axis, so a
    mix of hits, grazing rays and misses.  float32 [n, 3] each, unit dirs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.asarray(center, np.float64)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    o = c + distance * u
    tgt = c + rng.uniform(-spread, spread, size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def view_rays(origins, n: int, seed: int, spread: float = 0.73, center=(0.5, 0.5, 0.5)):
    """Training batches: each ray starts at one of `origins` (float [k, 3],
    e.g. camera positions), chosen uniformly, and aims at `center` plus a
    uniform offset of up to `spread` per axis (0.73 covers a 40-degree view
    of the unit cube from distance 2).  float32 [n, 3] each, unit dirs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    org = np.asarray(origins, np.float64).reshape(-1, 3)
    o = org[rng.integers(0, len(org), size=n)]
    d = np.asarray(center, np.float64) + rng.uniform(-spread, spread, size=(n, 3)) - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def surface_points(verts: np.ndarray, tris: np.ndarray, n: int, seed: int) -> np.ndarray:
    """Uniform barycentric samples on uniformly chosen triangles, float32 [n, 3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = rng.integers(0, len(tris), size=n)
    a, b = rng.uniform(size=n), rng.uniform(size=n)
    flip = a + b > 1.0
    a[flip], b[flip] = 1.0 - a[flip], 1.0 - b[flip]
    v = np.asarray(verts, np.float64)[np.asarray(tris)[t]]
    p = v[:, 0] + a[:, None] * (v[:, 1] - v[:, 0]) + b[:, None] * (v[:, 2] - v[:, 0])
    return np.clip(p, 0.0, 1.0).astype(np.float32)
