"""Per-level grid lookup with trilinear blending, FP64 (test infrastructure
only).

Sec. 4.1 ("Perfect Spatial Hashing Encoding"): a position x is scaled by the
grid resolution N, the vertex coordinate is p = floor(N x) (the text says
"round" but writes the floor; the floor is taken), the feature vectors of the
cell's eight corners are fetched and blended trilinearly.  Readings adopted:
  * x is first clamped to [0, 1]^3, and p to N - 1 per axis, so x = 1 puts
    full weight on the upper corner;
  * the floor is that of the exact real product N * x (x is an FP32 value, N
    an integer < 2**29, so the FP64 product is exact);
  * w = N x - p, corner c = (c_x, c_y, c_z) in {0,1}^3 has weight
    prod_i (c_i ? w_i : 1 - w_i);
  * the multiresolution encoding concatenates the levels in order, level 0
    (coarsest) first (Sec. 4.1, recalling i-NGP's concatenation).
The lookup is a plain dictionary from vertex to feature vector: what a
collision-free hash of the occupied vertices reaches.

Pins: an affine feature field is reproduced exactly (up to rounding); the
weights are a partition of unity; a query at a vertex returns that vertex's
feature; x = 1 selects the upper corner.
"""
from __future__ import annotations

import numpy as np

CORNERS = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], np.int64)


def grid_cell(x, N: int):
    """(p int64 [n, 3], w float64 [n, 3]) for FP32-valued positions x."""
    x = np.clip(np.asarray(x, np.float64).reshape(-1, 3), 0.0, 1.0)
    y = float(N) * x                       # exact: 24-bit x times integer N < 2**29
    p = np.minimum(np.floor(y), N - 1).astype(np.int64)
    return p, y - p


class FeatureGrid:
    """Dictionary of one level: integer vertex (x, y, z) -> feature vector."""

    def __init__(self, res: int, vertices, features):
        self.res = int(res)
        v = np.asarray(vertices, np.int64).reshape(-1, 3)
        f = np.asarray(features, np.float64)
        self.F = f.shape[1]
        self.table = {tuple(int(a) for a in vi): fi for vi, fi in zip(v, f)}

    def __call__(self, v):
        try:
            return self.table[tuple(int(a) for a in v)]
        except KeyError:
            raise KeyError(f"vertex {tuple(v)} of level N={self.res} is not occupied") from None


class FunctionGrid:
    """A level whose feature vector is given by a function of the vertex (for
    large levels where only the queried vertices are materialised)."""

    def __init__(self, res: int, F: int, fn, exists=None):
        self.res, self.F, self.fn, self.exists = int(res), int(F), fn, exists

    def lookup_many(self, verts):
        verts = np.asarray(verts, np.int64).reshape(-1, 3)
        if self.exists is not None:
            ok = self.exists(verts)
            if not np.all(ok):
                bad = verts[~ok][0]
                raise KeyError(f"vertex {tuple(bad)} of level N={self.res} is not occupied")
        return np.asarray(self.fn(verts), np.float64)


def trilinear_encode(x, grid) -> np.ndarray:
    """Blend the eight corner features of each position: float64 [n, F]."""
    p, w = grid_cell(x, grid.res)
    n = len(p)
    v = (p[:, None, :] + CORNERS[None]).reshape(-1, 3)          # [n*8, 3], corner-major per point
    if isinstance(grid, FunctionGrid):
        f = grid.lookup_many(v)
    else:
        f = np.array([grid(vi) for vi in v]).reshape(-1, grid.F)
    f = f.reshape(n, 8, grid.F)
    out = np.zeros((n, grid.F))
    for ci, c in enumerate(CORNERS):
        wc = np.prod(np.where(c[None, :] == 1, w, 1.0 - w), axis=1)
        out += wc[:, None] * f[:, ci]
    return out


def corner_vertices(x, N: int) -> np.ndarray:
    """The eight corner vertices of each position's cell: int64 [n, 8, 3]."""
    p, _ = grid_cell(x, N)
    return p[:, None, :] + CORNERS[None]


__all__ = ["grid_cell", "trilinear_encode", "FeatureGrid", "FunctionGrid", "corner_vertices", "CORNERS"]
