"""Brute-force closest hit of rays on the triangle proxy, FP64 (test
infrastructure only).

The paper finds one hit point per ray on a geometry proxy ("Lumigraph with
geometry proxies for fast ray querying", abstract and Sec. 1); this build's
proxy is a triangle mesh.  Plain definition: test every ray against every
triangle (Moeller-Trumbore, two-sided), keep the smallest t > 0, break ties
by the lowest triangle index; no hit is a miss (tri = -1, t = +inf).
Rays with a non-finite or zero direction, or a non-finite origin, miss.

Several answers are correct where the decision is within rounding: a ray
through (or within a hair of) a shared edge may hit either triangle, and a
ray grazing the silhouette may hit or miss.  Such rays are flagged
`ambiguous`: some triangle in front of the origin has its smallest
barycentric coordinate within `eps_bary` of zero, or is met at a grazing
angle, or the two nearest hits are within a relative `eps_t` in t.  All
other rays have one correct answer.

The cosine of the angle between each hit ray and the normal of the
triangle it hits is returned beside the hit (`cos`, NaN for a miss).  Near
grazing incidence the hit point moves by about t * (direction error) / cos
for a small change of the direction, so an FP32 ray determines it only to
~t * 2^-23 / |cos|; colour parity of the FP32 path is held where |cos| is
not small (the tests' reading), and reported elsewhere.

Pins: a ray aimed at a triangle's centroid along its normal hits that
triangle at the closed-form plane distance, with cos = 1; a ray at a known
angle to the normal gives that angle's cosine; an empty proxy gives misses.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class HitResult:
    tri: np.ndarray        # int64 [n], -1 = miss
    t: np.ndarray          # float64 [n], +inf = miss
    ambiguous: np.ndarray  # bool [n]
    cos: np.ndarray = None  # float64 [n]: |cos| of the incidence angle at the hit, NaN = miss

    @property
    def hit(self):
        return self.tri >= 0


def closest_hit(o, d, verts, tris, eps_bary: float = 2.0 ** -16, eps_t: float = 2.0 ** -16,
                max_pairs: int = 1 << 21) -> HitResult:
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    n = len(o)
    tri_out = np.full(n, -1, np.int64)
    t_out = np.full(n, np.inf)
    amb = np.zeros(n, bool)
    cos_out = np.full(n, np.nan)
    tris = np.asarray(tris, np.int64).reshape(-1, 3)
    if n == 0 or len(tris) == 0:
        return HitResult(tri_out, t_out, amb, cos_out)
    V = np.asarray(verts, np.float64)
    a = V[tris[:, 0]]
    e1 = V[tris[:, 1]] - a
    e2 = V[tris[:, 2]] - a
    nrm = np.linalg.norm(np.cross(e1, e2), axis=1)
    valid = np.all(np.isfinite(o), axis=1) & np.all(np.isfinite(d), axis=1) & np.any(d != 0, axis=1)
    idx_all = np.nonzero(valid)[0]
    T = len(tris)
    step = max(1, max_pairs // T)
    for s in range(0, len(idx_all), step):
        idx = idx_all[s:s + step]
        D = d[idx][:, None, :]
        O = o[idx][:, None, :]
        pvec = np.cross(D, e2[None])
        det = np.einsum("rtk,tk->rt", pvec, e1)
        nz = det != 0
        inv = np.where(nz, 1.0 / np.where(nz, det, 1.0), 0.0)
        tvec = O - a[None]
        u = np.einsum("rtk,rtk->rt", tvec, pvec) * inv
        qvec = np.cross(tvec, e1[None])
        v = np.einsum("rtk,rtk->rt", D, qvec) * inv
        t = np.einsum("tk,rtk->rt", e2, qvec) * inv
        m = np.minimum(np.minimum(u, v), 1.0 - u - v)
        hit = nz & (m >= 0) & (t > 0)
        tt = np.where(hit, t, np.inf)
        best = np.argmin(tt, axis=1)
        rows = np.arange(len(idx))
        tbest = tt[rows, best]
        got = np.isfinite(tbest)
        tri_out[idx] = np.where(got, best, -1)
        t_out[idx] = tbest
        # ambiguity
        dn = np.linalg.norm(d[idx], axis=1)[:, None]
        cosang = np.abs(det) / (nrm[None] * dn)
        cos_out[idx] = np.where(got, cosang[rows, best], np.nan)
        front = nz & (t > 0)
        near_edge = front & (np.abs(m) < eps_bary)
        grazing = (cosang < 1e-6) & (m > -eps_bary) & (t > 0)
        tt2 = tt.copy()
        tt2[rows, best] = np.inf
        second = tt2.min(axis=1)
        gap = np.where(got & np.isfinite(second), second - np.where(got, tbest, 0.0), np.inf)
        close_t = gap <= eps_t * np.abs(np.where(got, tbest, 0.0))
        amb[idx] = near_edge.any(axis=1) | grazing.any(axis=1) | close_t
    return HitResult(tri_out, t_out, amb, cos_out)
