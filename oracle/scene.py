"""Scenes of several i-NOLF objects, FP64 (test infrastructure only).

The paper renders scenes of several objects and merges them per pixel by
depth (Sec. 5, the frame composer composites the objects' frames by their
depth maps; Sec. 7, applications with several objects).  Each object is an
i-NOLF of its own (proxy, offset and feature tables, network) defined in its
unit cube and placed in the world by a similarity transform
    x_world = s R x_object + t     (s > 0 uniform scale, R a rotation).
Plain definition per ray (o, d) in the world:
  1. for every object, the ray in object space is o' = R^T (o - t) / s,
     d' = R^T d / s; the ray parameter is the same in both spaces, so the
     object's closest hit t (render.py) is directly comparable;
  2. the nearest hit over all objects wins; equal t goes to the lowest
     object index;
  3. the winning object shades the ray exactly as render.py does, from its
     object-space hit point and the unit object-space direction d'/|d'|.
A ray is ambiguous if its hit is ambiguous in any object it meets, or if two
objects' hits lie within a relative `eps_t` of each other.

Pins (tests): one object under the identity transform renders exactly as
render.py; rotating the scene and the rays by the same axis permutation
leaves the image unchanged; an object duplicated at the same place wins with
its lower index; a ray aimed along an icosphere vertex direction stops at the
transformed vertex (closed-form distance); an object in front hides one
behind.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .encode import trilinear_encode
from .hit import closest_hit
from .mlp import mlp_forward
from .sh import sh_real


@dataclass
class Instance:
    model: object                # render.Model
    scale: float
    rotation: np.ndarray         # [3, 3], orthonormal, det +1
    translation: np.ndarray      # [3]

    def to_object(self, o, d):
        R = np.asarray(self.rotation, np.float64)
        oo = (np.asarray(o, np.float64) - np.asarray(self.translation, np.float64)) @ R / self.scale
        dd = np.asarray(d, np.float64) @ R / self.scale
        return oo, dd


def render_scene_rays(instances, o, d, eps_t: float = 1e-4, **hit_kw) -> dict:
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    n = len(o)
    best_t = np.full(n, np.inf)
    best_obj = np.full(n, -1, np.int64)
    best_tri = np.full(n, -1, np.int64)
    amb = np.zeros(n, bool)
    ts = []
    for k, inst in enumerate(instances):
        oo, dd = inst.to_object(o, d)
        h = closest_hit(oo, dd, inst.model.verts, inst.model.tris, **hit_kw)
        ts.append(h.t)
        amb |= h.ambiguous
        better = h.hit & (h.t < best_t)          # strict: ties keep the lower index
        best_t[better] = h.t[better]
        best_obj[better] = k
        best_tri[better] = h.tri[better]
    if len(ts) > 1:
        T = np.stack(ts)                          # [K, n]
        both = np.isfinite(T) & np.isfinite(best_t)[None]
        gap = np.abs(np.where(both, T, 0.0) - np.where(both, best_t[None], 0.0))
        for k in range(len(ts)):
            amb |= both[k] & (best_obj != k) & (gap[k] <= eps_t * np.abs(np.where(both[k], best_t, 0.0)))
    rgba = np.zeros((n, 4))
    for k, inst in enumerate(instances):
        idx = np.nonzero(best_obj == k)[0]
        if len(idx) == 0:
            continue
        oo, dd = inst.to_object(o[idx], d[idx])
        x = np.clip(oo + best_t[idx, None] * dd, 0.0, 1.0)
        m = inst.model
        enc = np.concatenate([trilinear_encode(x, g) for g in m.grids], axis=1)
        inp = np.concatenate([enc, sh_real(dd, m.sh_degree)], axis=1)
        rgba[idx] = mlp_forward(inp, m.weights)
    return {"rgba": rgba, "t": best_t, "obj": best_obj, "tri": best_tri, "ambiguous": amb}


__all__ = ["Instance", "render_scene_rays"]
