"""The whole one-query-per-ray path, FP64 (test infrastructure only).

Per ray (Sec. 4.2 and the overview figure of the per-ray query):
  1. closest hit on the proxy (hit.py); a miss yields RGBA = (0, 0, 0, 0),
     not premultiplied and with no background;
  2. hit point x = o + t d, clamped to [0, 1]^3;
  3. encoding E(x): per level, trilinear blend of the eight corner features
     (encode.py), levels concatenated coarsest first;
  4. view encoding SH(d / |d|) (sh.py);
  5. network input [E_0 .. E_{L-1}, SH_0 .. SH_15]; RGBA = F_s(input)
     (mlp.py, Eq. 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .encode import FeatureGrid, FunctionGrid, trilinear_encode
from .hit import closest_hit
from .mlp import mlp_forward
from .occupancy import is_key, shell_keys
from .rays import camera_rays
from .sh import sh_real


@dataclass
class Model:
    verts: np.ndarray
    tris: np.ndarray
    grids: list                 # one FeatureGrid / FunctionGrid per level
    weights: list               # [W1, W2, W3]
    sh_degree: int = 4
    extra: dict = field(default_factory=dict)

    @classmethod
    def from_workload(cls, w, kind: str = "normal", sigma: float = 1e-2, materialize: bool = True,
                      check_keys: bool = True):
        """Build the oracle's model of a synthetic workload.  With
        `materialize`, every level's key set is computed (exact voxelisation)
        and stored in a dictionary; otherwise features are generated for the
        queried vertices only and, with `check_keys`, each queried vertex is
        checked to be occupied."""
        import synth
        grids = []
        for l, N in enumerate(w.res):
            if materialize:
                keys = shell_keys(w.verts, w.tris, N, w.dilate)
                feats = synth.table_features(w.feature_seed, l, keys, N, F=w.F, kind=kind, sigma=sigma)
                grids.append(FeatureGrid(N, keys, feats))
            else:
                fn = (lambda v, l=l, N=N: synth.table_features(w.feature_seed, l, v, N, F=w.F,
                                                               kind=kind, sigma=sigma))
                ex = ((lambda v, N=N: is_key(w.verts, w.tris, N, v, w.dilate)) if check_keys else None)
                grids.append(FunctionGrid(N, w.F, fn, ex))
        return cls(np.asarray(w.verts), np.asarray(w.tris), grids, [np.asarray(x) for x in w.weights])


def encode_points(model: Model, x) -> np.ndarray:
    """Concatenated multi-level encoding of positions x [n, 3]: [n, L*F]."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    if len(model.grids) == 0:
        return np.zeros((len(x), 0))
    return np.concatenate([trilinear_encode(x, g) for g in model.grids], axis=1)


def render_rays(model: Model, o, d, **hit_kw) -> dict:
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    n = len(o)
    hit = closest_hit(o, d, model.verts, model.tris, **hit_kw)
    rgba = np.zeros((n, 4))
    x = np.full((n, 3), np.nan)
    idx = np.nonzero(hit.hit)[0]
    enc = np.zeros((n, sum(g.F for g in model.grids)))
    if len(idx):
        xh = np.clip(o[idx] + hit.t[idx, None] * d[idx], 0.0, 1.0)
        x[idx] = xh
        e = encode_points(model, xh)
        enc[idx] = e
        inp = np.concatenate([e, sh_real(d[idx], model.sh_degree)], axis=1)
        rgba[idx] = mlp_forward(inp, model.weights)
    return {"rgba": rgba, "tri": hit.tri, "t": hit.t, "x": x, "enc": enc, "ambiguous": hit.ambiguous,
            "cos": hit.cos}


def render_camera(model: Model, cam, rows=None, cols=None, **hit_kw) -> dict:
    """Render all pixels of `cam` (row-major) or the listed pixels."""
    o, d = camera_rays(cam, rows, cols)
    return render_rays(model, o, d, **hit_kw)
