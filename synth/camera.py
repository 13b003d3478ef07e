"""Camera poses (the inputs a client sends: a pose matrix and intrinsics).

A camera is stored as FP32 values exactly as the library receives them:
origin, an orthonormal right/up/forward frame, tan(fov_y / 2) and the image
size.  How rays are formed from it is the renderer's business, not this
module's.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Camera:
    origin: np.ndarray        # (3,) float32
    right: np.ndarray         # (3,) float32
    up: np.ndarray            # (3,) float32
    forward: np.ndarray       # (3,) float32
    tan_half_fov_y: np.float32
    width: int
    height: int

    def as_array(self) -> np.ndarray:
        """Packed float32[13]: origin, right, up, forward, tan_half_fov_y."""
        return np.concatenate([self.origin, self.right, self.up, self.forward,
                               np.array([self.tan_half_fov_y], np.float32)]).astype(np.float32)


def look_at_camera(eye, target=(0.5, 0.5, 0.5), fov_y_deg: float = 40.0,
                   width: int = 64, height: int = 64) -> Camera:
    """Pinhole camera at `eye` looking at `target`; world up is +z, or +y when
    the view axis is within ~2.6 degrees of z."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0]) if abs(f[2]) <= 0.999 else np.array([0.0, 1.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return Camera(eye.astype(np.float32), r.astype(np.float32), u.astype(np.float32),
                  f.astype(np.float32), np.float32(math.tan(math.radians(fov_y_deg) / 2.0)),
                  int(width), int(height))


def fibonacci_directions(n: int) -> np.ndarray:
    """n points of the Fibonacci sphere: z_k = 1-(2k+1)/n, phi_k = k*pi*(3-sqrt 5)."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def fibonacci_cameras(n: int = 8, distance: float = 2.0, width: int = 3840, height: int = 2160,
                      fov_y_deg: float = 40.0, center=(0.5, 0.5, 0.5)):
    c = np.asarray(center, np.float64)
    return [look_at_camera(c + distance * d, c, fov_y_deg, width, height)
            for d in fibonacci_directions(n)]


def random_cameras(n: int, seed: int, distance: float = 2.0, width: int = 3840, height: int = 2160,
                   fov_y_deg: float = 40.0, center=(0.5, 0.5, 0.5)):
    """Seeded uniform directions on the sphere of radius `distance`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    c = np.asarray(center, np.float64)
    return [look_at_camera(c + distance * x, c, fov_y_deg, width, height) for x in d]


SERVING_RESOLUTIONS = ((1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))


def orbit_requests(n_clients: int, duration_s: float, rate_hz: float, seed: int, distance: float = 2.0,
                   resolutions=((1920, 1080), (1280, 720), (3840, 2160), (800, 800)), center=(0.5, 0.5, 0.5),
                   fov_y_deg: float = 40.0, per_request: bool = False):
    """Client requests for a serving test: client k orbits `center` at
    `distance` about its own seeded axis at its own angular speed (0.5..2
    rad/s) and asks for frames at Poisson times of rate `rate_hz` within
    [0, duration_s).  The resolution is resolutions[k % len] for all of
    client k's frames, or, with per_request, drawn uniformly from
    `resolutions` for every request.  Returns a list of (client, arrival
    time, Camera), sorted by time."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.asarray(center, np.float64)
    out = []
    for k in range(n_clients):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        start = np.cross(axis, rng.normal(size=3))
        start /= np.linalg.norm(start)
        omega = rng.uniform(0.5, 2.0)
        W, H = resolutions[k % len(resolutions)]
        t = rng.exponential(1.0 / rate_hz)
        while t < duration_s:
            a = omega * t
            d = start * math.cos(a) + np.cross(axis, start) * math.sin(a)   # rotation of start about axis
            if per_request:
                W, H = resolutions[int(rng.integers(len(resolutions)))]
            out.append((k, float(t), look_at_camera(c + distance * d, c, fov_y_deg, W, H)))
            t += rng.exponential(1.0 / rate_hz)
    out.sort(key=lambda r: r[1])
    return out
