"""Seeded model parameters: level resolutions, MLP weights, feature values.

These stand in for trained i-NOLF parameters.  Feature values are drawn by a
counter-based generator keyed on (seed, level, vertex, feature), so the value
of a vertex does not depend on which other vertices exist; any consumer that
knows a vertex can obtain its feature without the full key list.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .mesh import _splitmix64

GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def level_resolutions(n_min: int, n_max: int, n_levels: int):
    """Geometric series N_l = round(n_min * b**l), b = (n_max/n_min)**(1/(L-1))."""
    if n_levels == 1:
        return [int(n_min)]
    b = (n_max / n_min) ** (1.0 / (n_levels - 1))
    return [int(round(n_min * b ** l)) for l in range(n_levels)]


def xavier_mlp(seed: int, d_in: int, hidden: int = 64, d_out: int = 4, n_hidden: int = 2):
    """Bias-free MLP weights, Xavier-uniform U(+-sqrt(6/(fan_in+fan_out))),
    drawn from PCG64(seed) in layer order, each row-major [out][in], float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = [d_in] + [hidden] * n_hidden + [d_out]
    ws = []
    for fi, fo in zip(dims[:-1], dims[1:]):
        a = math.sqrt(6.0 / (fi + fo))
        ws.append(rng.uniform(-a, a, size=(fo, fi)).astype(np.float32))
    return ws


def _feature_chunk(seed, level, keys, F, kind, sigma):
    keys = np.asarray(keys, np.int64).astype(np.uint64)
    base = _splitmix64(np.array([seed], np.uint64) ^ (np.uint64(level) << np.uint64(40)))[0]
    out = np.empty((len(keys), F), np.float32)
    with np.errstate(over="ignore"):
        for f in range(F):
            h = _splitmix64((keys * np.uint64(F) + np.uint64(f)) * GOLDEN ^ base)
            if kind == "normal":
                u1 = ((h >> np.uint64(40)).astype(np.float64) + 0.5) * 2.0 ** -24
                u2 = (((h >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float64) + 0.5) * 2.0 ** -24
                z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
                out[:, f] = (sigma * z).astype(np.float32)
            elif kind == "uniform":
                u = (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
                out[:, f] = (sigma * (2.0 * u - 1.0)).astype(np.float32)
            else:
                raise ValueError(kind)
    return out


def feature_values(seed: int, level: int, keys, F: int = 2, kind: str = "normal",
                   sigma: float = 1e-2, threads: int | None = None) -> np.ndarray:
    """Feature vectors (float32 [n, F]) for the given linear vertex keys of one level.

    kind="normal": N(0, sigma^2) by Box-Muller on 24-bit uniforms;
    kind="uniform": U(-sigma, sigma) (sigma=1 is the "loud" variant that
    makes colour depend strongly on the encoding)."""
    keys = np.asarray(keys, np.int64).reshape(-1)
    n = len(keys)
    chunk = 1 << 20
    if n <= chunk:
        return _feature_chunk(seed, level, keys, F, kind, sigma)
    out = np.empty((n, F), np.float32)
    threads = threads or min(16, os.cpu_count() or 1)

    def job(s):
        out[s:s + chunk] = _feature_chunk(seed, level, keys[s:s + chunk], F, kind, sigma)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(job, range(0, n, chunk)))
    return out


def table_features(seed: int, level: int, vertices: np.ndarray, res: int, **kw) -> np.ndarray:
    """Feature vectors for integer vertex coordinates [n, 3] (x, y, z) of a
    level with resolution `res` (vertex coordinates run 0..res)."""
    v = np.asarray(vertices, np.int64)
    key = (v[:, 2] * (res + 1) + v[:, 1]) * (res + 1) + v[:, 0]
    return feature_values(seed, level, key, **kw)
