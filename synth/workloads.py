"""The two single-object workloads, with their seeds.

tiny:   icosphere, 320 triangles, radius 0.5; 4 levels at 16/24/40/64; F=2;
        SH degree 4 (16 values); MLP 24-64-64-4; one 64x64 camera at distance
        2, vertical FOV 40 degrees, on Fibonacci direction 1 of 8.
object: 100,820-triangle sphere of base radius 0.45 displaced by 3-octave
        value noise (amplitude 0.05); 16 levels 16..2048; F=2; MLP 48-64-64-4;
        8 Fibonacci cameras at distance 2 (1920x1080 or 3840x2160).
Seeds: mesh 1, features 2, MLP 3, cameras 4, noise 5, loud features 6.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .camera import fibonacci_cameras
from .mesh import displaced_sphere, icosphere
from .params import level_resolutions, xavier_mlp

SEED_FEATURES, SEED_MLP, SEED_CAMERAS, SEED_NOISE, SEED_LOUD, SEED_SCENE = 2, 3, 4, 5, 6, 7
SH_DIM = 16


@dataclass
class Workload:
    name: str
    verts: np.ndarray
    tris: np.ndarray
    res: list
    F: int
    weights: list
    cameras: list
    dilate: int = 1
    psh_seed: int = 1
    feature_seed: int = SEED_FEATURES
    extra: dict = field(default_factory=dict)

    @property
    def d_in(self) -> int:
        return len(self.res) * self.F + SH_DIM


def workload_tiny() -> Workload:
    verts, tris = icosphere(4, 0.5)
    res = [16, 24, 40, 64]
    F = 2
    cams = fibonacci_cameras(8, 2.0, 64, 64)[1:2]
    return Workload("icosphere320_L4_64x64", verts, tris, res, F,
                    xavier_mlp(SEED_MLP, len(res) * F + SH_DIM), cams)


def workload_object(width: int = 3840, height: int = 2160, n_levels: int = 16,
                    n_max: int = 2048, freq: int = 71) -> Workload:
    verts, tris = displaced_sphere(freq, 0.45, 0.05, SEED_NOISE)
    res = level_resolutions(16, n_max, n_levels)
    F = 2
    cams = fibonacci_cameras(8, 2.0, width, height)
    return Workload(f"displaced_sphere{len(tris)}_L{n_levels}_{width}x{height}", verts, tris, res, F,
                    xavier_mlp(SEED_MLP, n_levels * F + SH_DIM), cams)


@dataclass
class SceneObject:
    """One object of a scene: a workload in its unit cube, placed by
    x_world = scale * rotation @ x_object + translation."""
    workload: Workload
    scale: float
    rotation: np.ndarray
    translation: np.ndarray


@dataclass
class SceneWorkload:
    name: str
    objects: list
    cameras: list


def random_rotation(rng) -> np.ndarray:
    """Uniformly distributed rotation (unit quaternion from three uniforms)."""
    u1, u2, u3 = rng.uniform(size=3)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    w, x, y, z = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3), \
        b * np.cos(2 * np.pi * u3)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _place(rng, box: float, smin: float, smax: float):
    s = float(rng.uniform(smin, smax))
    R = random_rotation(rng)
    # keep the rotated unit cube inside [0, box]^3
    corners = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], np.float64)
    w = s * corners @ R.T
    lo, hi = w.min(0), w.max(0)
    t = rng.uniform(-lo, box - hi)
    return s, R, t


def scene_tiny(n_objects: int = 3, width: int = 64, height: int = 64) -> SceneWorkload:
    """Parity scene: icospheres (320 triangles, 4 levels 16..64) with their own
    features and networks, scale 0.5..1.0, in a 2.5^3 box; one camera at
    distance 4.5 from the box centre."""
    rng = np.random.Generator(np.random.PCG64(SEED_SCENE))
    objs = []
    for k in range(n_objects):
        verts, tris = icosphere(4, 0.5)
        res = [16, 24, 40, 64]
        w = Workload(f"icosphere320_L4_obj{k}", verts, tris, res, 2,
                     xavier_mlp(SEED_MLP + 100 * (k + 1), len(res) * 2 + SH_DIM), [],
                     feature_seed=SEED_FEATURES + 100 * (k + 1))
        s, R, t = _place(rng, 2.5, 0.5, 1.0)
        objs.append(SceneObject(w, s, R, t))
    cams = fibonacci_cameras(8, 4.5, width, height, center=(1.25, 1.25, 1.25))[1:2]
    return SceneWorkload(f"scene{n_objects}_icosphere320_{width}x{height}", objs, cams)


def scene_objects(n_objects: int = 12, width: int = 3840, height: int = 2160, freq: int = 40) -> SceneWorkload:
    """Multi-object scene: displaced spheres (20 * freq^2 triangles, own noise,
    features and network each), 10 levels 16..512, scale 0.2..1.0 in a 4^3
    box; 8 Fibonacci cameras at distance 6 from the box centre."""
    rng = np.random.Generator(np.random.PCG64(SEED_SCENE))
    objs = []
    res = level_resolutions(16, 512, 10)
    for k in range(n_objects):
        verts, tris = displaced_sphere(freq, 0.45, 0.05, SEED_NOISE + 100 * (k + 1))
        w = Workload(f"displaced_sphere{len(tris)}_L10_obj{k}", verts, tris, res, 2,
                     xavier_mlp(SEED_MLP + 100 * (k + 1), len(res) * 2 + SH_DIM), [],
                     feature_seed=SEED_FEATURES + 100 * (k + 1))
        s, R, t = _place(rng, 4.0, 0.2, 1.0)
        objs.append(SceneObject(w, s, R, t))
    cams = fibonacci_cameras(8, 6.0, width, height, center=(2.0, 2.0, 2.0))
    return SceneWorkload(f"scene{n_objects}_displaced_sphere_L10_{width}x{height}", objs, cams)
