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

SEED_FEATURES, SEED_MLP, SEED_CAMERAS, SEED_NOISE, SEED_LOUD = 2, 3, 4, 5, 6
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
