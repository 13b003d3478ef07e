"""Procedural proxy meshes (triangle soups inside the unit cube).

All vertex coordinates are rounded to multiples of 2**-VERTEX_FRAC_BITS.  Such
values are exact in FP32 and FP64 alike, so every consumer sees the very same
geometry, and scaled by an integer grid resolution they become integers, which
lets occupancy be decided in exact integer arithmetic.
"""
from __future__ import annotations

import itertools

import numpy as np

VERTEX_FRAC_BITS = 16
_MASK64 = (1 << 64) - 1


def quantize_vertices(v: np.ndarray) -> np.ndarray:
    """Round to the 2**-16 lattice, clip to [0, 1], return float32 (exact)."""
    s = float(1 << VERTEX_FRAC_BITS)
    q = np.clip(np.rint(np.asarray(v, np.float64) * s), 0, s) / s
    out = q.astype(np.float32)
    assert np.array_equal(out.astype(np.float64), q)
    return out


def _icosahedron():
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a, b in itertools.product((-1.0, 1.0), repeat=2):
        v += [(0.0, a, b * phi), (a, b * phi, 0.0), (b * phi, 0.0, a)]
    v = np.array(v, np.float64)
    faces = []
    for i, j, k in itertools.combinations(range(12), 3):
        d = [np.linalg.norm(v[i] - v[j]), np.linalg.norm(v[j] - v[k]), np.linalg.norm(v[i] - v[k])]
        if all(abs(x - 2.0) < 1e-9 for x in d):
            n = np.cross(v[j] - v[i], v[k] - v[i])
            faces.append((i, j, k) if np.dot(n, v[i] + v[j] + v[k]) > 0 else (i, k, j))
    assert len(faces) == 20
    return v, faces


def _geodesic(freq: int):
    """Unit-sphere geodesic grid: 20*freq**2 triangles, 10*freq**2+2 vertices."""
    base, faces = _icosahedron()
    index: dict = {}
    pos: list = []
    tris: list = []

    def vid(weights):
        # weights: {base vertex id: integer weight}, summing to freq
        key = tuple(sorted((k, w) for k, w in weights.items() if w))
        if key not in index:
            p = np.zeros(3)
            for k, w in key:
                p = p + base[k] * (w / freq)
            index[key] = len(pos)
            pos.append(p / np.linalg.norm(p))
        return index[key]

    for A, B, C in faces:
        def g(i, j):
            return vid({A: freq - i - j, B: i, C: j}) if A != B else None
        for i in range(freq):
            for j in range(freq - i):
                tris.append((g(i, j), g(i + 1, j), g(i, j + 1)))
                if i + j + 2 <= freq:
                    tris.append((g(i + 1, j), g(i + 1, j + 1), g(i, j + 1)))
    return np.array(pos, np.float64), np.array(tris, np.int32)


def icosphere(freq: int = 4, radius: float = 0.5, center=(0.5, 0.5, 0.5)):
    """Geodesic icosphere.  freq=4 gives 320 triangles (two midpoint
    subdivisions of the icosahedron); freq=71 gives 100,820."""
    u, tris = _geodesic(freq)
    v = np.asarray(center, np.float64) + radius * u
    return quantize_vertices(v), tris


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)).astype(np.uint64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _lattice(seed: int, i, j, k) -> np.ndarray:
    """Seeded lattice values in [-1, 1]."""
    h = _splitmix64(np.full(np.shape(i), seed, np.uint64))
    for c in (i, j, k):
        h = _splitmix64(h ^ np.asarray(c, np.int64).astype(np.uint64))
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 / 2.0 ** 53) - 1.0


def value_noise(p: np.ndarray, seed: int, octaves: int = 3, base_freq: float = 4.0,
                lacunarity: float = 2.0, gain: float = 0.5) -> np.ndarray:
    """Fractal value noise with quintic fade, normalised so |n| <= 1."""
    p = np.asarray(p, np.float64)
    total = np.zeros(len(p))
    norm = 0.0
    f, a = base_freq, 1.0
    for o in range(octaves):
        q = p * f
        c0 = np.floor(q).astype(np.int64)
        t = q - c0
        s = t * t * t * (t * (t * 6.0 - 15.0) + 10.0)
        acc = np.zeros(len(p))
        for dx, dy, dz in itertools.product((0, 1), repeat=3):
            w = ((s[:, 0] if dx else 1 - s[:, 0]) * (s[:, 1] if dy else 1 - s[:, 1])
                 * (s[:, 2] if dz else 1 - s[:, 2]))
            acc += w * _lattice(seed + o, c0[:, 0] + dx, c0[:, 1] + dy, c0[:, 2] + dz)
        total += a * acc
        norm += a
        f *= lacunarity
        a *= gain
    return total / norm


def displaced_sphere(freq: int = 71, base_radius: float = 0.45, amplitude: float = 0.05,
                     seed: int = 5, center=(0.5, 0.5, 0.5)):
    """Geodesic sphere (20*freq**2 triangles) whose radius is displaced by
    3-octave value noise evaluated at the undisplaced vertex."""
    u, tris = _geodesic(freq)
    c = np.asarray(center, np.float64)
    p0 = c + base_radius * u
    r = base_radius + amplitude * value_noise(p0, seed)
    return quantize_vertices(c + r[:, None] * u), tris
