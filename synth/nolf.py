"""Inputs of the paper's own i-NOLF form: density and diffuse texture cubes,
feature-table key sets, network weights with the coarse-opacity input.

Data only: what a trained object would hold, made up from seeded fields.
The density is a shell around a noise-displaced sphere: with s the signed
distance estimate |p - c| - R(u) (R from 3-octave value noise on the
undisplaced sphere, as for the proxy mesh) sampled at the base-grid
vertices and blended trilinearly inside each base cell, the density at a
cube vertex is sigma_max * max(0, 1 - |s| / h), rounded to FP16.  A base
cell holds a cube when some vertex value is non-zero; every other cell is
empty.  The blend is done per axis as (1 - w) a + w b, so two cubes sharing
a face hold identical values on it, and a cube's face towards an empty cell
is zero: the cached field is continuous.  The diffuse cubes (colour c_d in
RGB and tint t) cover the same cells, from base-grid noise blended the same
way plus a small per-vertex hash term, also rounded to FP16.

Feature keys of a level of resolution N (a multiple of b) are the corners of
the level's cells inside non-empty base cells, so every point with non-zero
density has all 8 corners stored.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .camera import fibonacci_cameras
from .mesh import _splitmix64, value_noise
from .params import xavier_mlp
from .workloads import SEED_FEATURES, SEED_MLP, SEED_NOISE, SH_DIM

SEED_DIFFUSE = 8


def _base_field(b: int, center, r0: float, amp: float, seed: int):
    """Signed distance estimate at the (b+1)^3 base-grid vertices, [z, y, x]."""
    g = np.arange(b + 1, dtype=np.float64) / b
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    p = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    c = np.asarray(center, np.float64)
    v = p - c
    rad = np.linalg.norm(v, axis=1)
    u = v / np.maximum(rad, 1e-12)[:, None]
    R = r0 + amp * value_noise(c + r0 * u, seed)
    return (rad - R).reshape(b + 1, b + 1, b + 1), p.reshape(b + 1, b + 1, b + 1, 3)


def _corners(field, cz, cy, cx):
    """Corner values [n, 2(z), 2(y), 2(x), ...] of cells (cz, cy, cx)."""
    out = np.empty((len(cz), 2, 2, 2) + field.shape[3:], field.dtype)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                out[:, dz, dy, dx] = field[cz + dz, cy + dy, cx + dx]
    return out


def _blend(cor, r: int):
    """Per-axis blend of corner values [n, 2, 2, 2, C] to the (r+1)^3 cube
    vertices [n, r+1 (z), r+1 (y), r+1 (x), C]: x first, then y, then z."""
    w = np.arange(r + 1, dtype=np.float64) / r
    wx = w[None, None, None, :, None]
    A = (1.0 - wx) * cor[:, :, :, 0:1, :] + wx * cor[:, :, :, 1:2, :]          # [n, 2, 2, r+1, C]
    wy = w[None, None, :, None, None]
    B = (1.0 - wy) * A[:, :, 0:1] + wy * A[:, :, 1:2]                            # [n, 2, r+1, r+1, C]
    wz = w[None, :, None, None, None]
    return (1.0 - wz) * B[:, 0:1] + wz * B[:, 1:2]                               # [n, r+1, r+1, r+1, C]


def _f16(a):
    return np.asarray(a, np.float64).astype(np.float16).astype(np.float32)


@dataclass
class NolfWorkload:
    name: str
    b: int
    r: int
    index: np.ndarray        # int32 [b^3]
    density: np.ndarray      # float32 [n_cubes, (r+1)^3, 1], FP16 values
    diffuse: np.ndarray      # float32 [n_cubes, (r+1)^3, 4], FP16 values
    res: list
    F: int
    weights: list            # W1 [64, 2L+17], W2, W3
    cameras: list
    step: float
    sigma_max: float
    shell: float
    feature_seed: int = SEED_FEATURES
    psh_seed: int = 1

    @property
    def d_in(self) -> int:
        return len(self.res) * self.F + SH_DIM + 1

    def occupied_cells(self):
        """(cz, cy, cx) of non-empty base cells, in linear order."""
        k = np.nonzero(self.index >= 0)[0]
        b = self.b
        return k // (b * b), (k // b) % b, k % b

    def level_keys(self, level: int) -> np.ndarray:
        """Sorted linear keys (z*(N+1) + y)*(N+1) + x of the level's vertices
        that are corners of its cells inside non-empty base cells."""
        N, b = self.res[level], self.b
        q = N // b
        cz, cy, cx = self.occupied_cells()
        off = np.arange(q + 1)
        keys = []
        step = max(1, (1 << 22) // ((q + 1) ** 3))
        for s in range(0, len(cz), step):
            z = (cz[s:s + step, None] * q + off[None])[:, :, None, None]
            y = (cy[s:s + step, None] * q + off[None])[:, None, :, None]
            x = (cx[s:s + step, None] * q + off[None])[:, None, None, :]
            keys.append(np.unique(((z * (N + 1) + y) * (N + 1) + x).ravel()))
        return np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.int64)

    def is_key(self, level: int, v) -> np.ndarray:
        """Whether integer vertices v [n, 3] (x, y, z) of the level are keys."""
        N, b = self.res[level], self.b
        q = N // b
        v = np.asarray(v, np.int64).reshape(-1, 3)
        ok = np.zeros(len(v), bool)
        idx = self.index
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    c = (v - np.array([dx, dy, dz])) // q      # a base cell that has v on its closed box
                    inside = np.all((c >= 0) & (c < b) & (c * q <= v) & (v <= c * q + q), axis=1)
                    cc = np.clip(c, 0, b - 1)
                    ok |= inside & (idx[(cc[:, 2] * b + cc[:, 1]) * b + cc[:, 0]] >= 0)
        return ok


def make_nolf(name: str, b: int, r: int, res, step: float, shell: float, sigma_max: float, cameras,
              r0: float, amp: float = 0.05, center=(0.5, 0.5, 0.5), F: int = 2) -> NolfWorkload:
    for v in [b, r] + list(res):
        if v & (v - 1):
            raise ValueError("resolutions must be powers of two")
    if any(N % b for N in res):
        raise ValueError("level resolutions must be multiples of the base resolution")
    s, P = _base_field(b, center, r0, amp, SEED_NOISE)
    cell_min = np.full((b, b, b), np.inf)
    cell_max = np.full((b, b, b), -np.inf)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                sub = s[dz:dz + b, dy:dy + b, dx:dx + b]
                cell_min = np.minimum(cell_min, sub)
                cell_max = np.maximum(cell_max, sub)
    cz, cy, cx = np.nonzero((cell_min < shell) & (cell_max > -shell))
    S = _blend(_corners(s[..., None], cz, cy, cx), r)[..., 0]
    dens = _f16(sigma_max * np.maximum(0.0, 1.0 - np.abs(S) / shell))
    keep = dens.reshape(len(cz), -1).max(axis=1) > 0
    cz, cy, cx, dens = cz[keep], cy[keep], cx[keep], dens[keep]
    order = np.argsort((cz * b + cy) * b + cx, kind="stable")
    cz, cy, cx, dens = cz[order], cy[order], cx[order], dens[order]
    index = np.full(b ** 3, -1, np.int32)
    index[(cz * b + cy) * b + cx] = np.arange(len(cz), dtype=np.int32)
    # diffuse: base-grid noise per channel, blended, plus a per-vertex hash term
    noise = np.stack([value_noise(P.reshape(-1, 3), SEED_DIFFUSE + ch) for ch in range(4)], axis=1)
    noise = noise.reshape(b + 1, b + 1, b + 1, 4)
    D = _blend(_corners(noise, cz, cy, cx), r)                                     # [n, r+1, r+1, r+1, 4]
    loc = np.arange(r + 1)
    gz = (cz[:, None] * r + loc[None])[:, :, None, None]
    gy = (cy[:, None] * r + loc[None])[:, None, :, None]
    gx = (cx[:, None] * r + loc[None])[:, None, None, :]
    fine = b * r + 1
    gkey = ((gz * fine + gy) * fine + gx).astype(np.uint64)
    with np.errstate(over="ignore"):
        h = _splitmix64(gkey.ravel() ^ np.uint64(0xD1FF05E)).reshape(gkey.shape)
    jitter = ((h >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) * 2.0 - 1.0
    diff = np.empty_like(D)
    diff[..., :3] = np.clip(0.5 + 0.35 * D[..., :3] + 0.1 * jitter[..., None], 0.0, 1.0)
    diff[..., 3] = np.clip(0.5 + 0.4 * D[..., 3] + 0.1 * jitter, 0.0, 1.0)
    n = len(cz)
    w = NolfWorkload(name, b, r, index, dens.reshape(n, -1, 1), _f16(diff).reshape(n, -1, 4), list(res), F,
                     xavier_mlp(SEED_MLP, len(res) * F + SH_DIM + 1), cameras, float(step), float(sigma_max),
                     float(shell))
    _check_continuous(w, cz, cy, cx)
    return w


def _check_continuous(w: NolfWorkload, cz, cy, cx):
    """Shared faces hold equal values; faces towards empty cells are zero."""
    b, r = w.b, w.r
    V = w.density.reshape(-1, r + 1, r + 1, r + 1)
    for axis in range(3):
        c = [cz, cy, cx]
        nb = [a.copy() for a in c]
        nb[2 - axis] = nb[2 - axis] + 1
        inside = nb[2 - axis] < b
        k_nb = np.full(len(cz), -1)
        k_nb[inside] = w.index[(nb[0][inside] * b + nb[1][inside]) * b + nb[2][inside]]
        hi = np.take(V, [r], axis=3 - axis).squeeze(3 - axis)      # face at the upper end of this axis
        has = k_nb >= 0
        lo_nb = np.take(V[k_nb[has]], [0], axis=3 - axis).squeeze(3 - axis)
        assert np.array_equal(hi[has], lo_nb), "cube faces disagree"
        assert not hi[inside & ~has].any(), "a cube face towards an empty cell is not zero"
        lo = np.take(V, [0], axis=3 - axis).squeeze(3 - axis)
        pb = [a.copy() for a in c]
        pb[2 - axis] = pb[2 - axis] - 1
        inside = pb[2 - axis] >= 0
        k_pb = np.full(len(cz), -1)
        k_pb[inside] = w.index[(pb[0][inside] * b + pb[1][inside]) * b + pb[2][inside]]
        assert not lo[inside & (k_pb < 0)].any(), "a cube face towards an empty cell is not zero"


STEP_NGP = math.sqrt(3.0) / 1024.0


def nolf_tiny(width: int = 64, height: int = 64) -> NolfWorkload:
    """b=16, r=4 (fine grid 64), levels 16/32/64, shell half-width 2/16,
    sigma_max 128, step sqrt(3)/256; one camera at distance 2."""
    cams = fibonacci_cameras(8, 2.0, width, height)[1:2]
    return make_nolf(f"nolf_tiny_{width}x{height}", 16, 4, [16, 32, 64], math.sqrt(3.0) / 256.0, 2.0 / 16, 128.0,
                     cams, r0=0.3)


def nolf_object(width: int = 3840, height: int = 2160) -> NolfWorkload:
    """b=64, r=8 (fine grid 512), levels 64/128/256/512, shell half-width
    2/64, sigma_max 512, the instant-NGP step sqrt(3)/1024; 8 Fibonacci
    cameras at distance 2."""
    cams = fibonacci_cameras(8, 2.0, width, height)
    return make_nolf(f"nolf_sphere_b64r8_L4_{width}x{height}", 64, 8, [64, 128, 256, 512], STEP_NGP, 2.0 / 64, 512.0,
                     cams, r0=0.4)
