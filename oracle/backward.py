"""Gradient of the training loss, FP64 (test infrastructure only).

Sec. 4.2, Eq. 8: the loss is the mean over a batch of rays of the squared
error of colour and opacity, (1/N) sum_i (|c_i - c_gt|^2 + (alpha_i - alpha_gt)^2),
i.e. the mean squared RGBA error per ray.  Its gradient with respect to the
network weights and to the feature vector stored at each grid vertex is the
chain rule through the path of render.py (the hit point does not depend on
the parameters; a miss contributes nothing):
  dL/dy     = 2 (y - y_gt) / N
  dz3       = dL/dy * y (1 - y)                  sigmoid
  dW3       = sum_rays dz3 h2^T,   dh2 = W3^T dz3, dz2 = dh2 [z2 > 0]
  dW2       = sum_rays dz2 h1^T,   dh1 = W2^T dz2, dz1 = dh1 [z1 > 0]
  dW1       = sum_rays dz1 in^T,   d_in = W1^T dz1
  dfeature(v) += w_c(x) d_in[E_l]  for each corner v = p + c of each level l.

Pins: FP64 central finite differences of the loss (tests), away from ReLU
kinks.
"""
from __future__ import annotations

import numpy as np

from .encode import CORNERS, grid_cell, trilinear_encode
from .hit import closest_hit
from .sh import sh_real


def mse_loss(rgba, target) -> float:
    """Eq. 8: mean over rays of the squared RGBA error."""
    rgba = np.asarray(rgba, np.float64)
    target = np.asarray(target, np.float64)
    return float(np.mean(np.sum((rgba - target) ** 2, axis=1)))


def mse_grad(rgba, target) -> np.ndarray:
    rgba = np.asarray(rgba, np.float64)
    return 2.0 * (rgba - np.asarray(target, np.float64)) / len(rgba)


def backward_rays(model, o, d, d_rgba, **hit_kw) -> dict:
    """Gradients of sum_i <d_rgba_i, rgba_i> with respect to the weights and
    the per-vertex features.  Returns {"weights": [dW1, dW2, dW3],
    "features": [dict vertex -> dF per level], "rgba": forward output}."""
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    g_out = np.asarray(d_rgba, np.float64).reshape(-1, 4)
    W = [np.asarray(w, np.float64) for w in model.weights]
    hit = closest_hit(o, d, model.verts, model.tris, **hit_kw)
    idx = np.nonzero(hit.hit)[0]
    dW = [np.zeros_like(w) for w in W]
    dfeat = [dict() for _ in model.grids]
    rgba = np.zeros((len(o), 4))
    if len(idx) == 0:
        return {"weights": dW, "features": dfeat, "rgba": rgba}
    x = np.clip(o[idx] + hit.t[idx, None] * d[idx], 0.0, 1.0)
    enc = np.concatenate([trilinear_encode(x, g) for g in model.grids], axis=1)
    inp = np.concatenate([enc, sh_real(d[idx], model.sh_degree)], axis=1)
    z1 = inp @ W[0].T
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W[1].T
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W[2].T
    y = 1.0 / (1.0 + np.exp(-z3))
    rgba[idx] = y
    dz3 = g_out[idx] * y * (1.0 - y)
    dW[2] = dz3.T @ h2
    dz2 = (dz3 @ W[2]) * (z2 > 0)
    dW[1] = dz2.T @ h1
    dz1 = (dz2 @ W[1]) * (z1 > 0)
    dW[0] = dz1.T @ inp
    d_in = dz1 @ W[0]
    col = 0
    for l, g in enumerate(model.grids):
        dE = d_in[:, col:col + g.F]
        col += g.F
        p, w = grid_cell(x, g.res)
        for c in CORNERS:
            wc = np.prod(np.where(c[None, :] == 1, w, 1.0 - w), axis=1)
            for k in range(len(idx)):
                v = tuple(int(a) for a in (p[k] + c))
                dfeat[l][v] = dfeat[l].get(v, 0.0) + wc[k] * dE[k]
    return {"weights": dW, "features": dfeat, "rgba": rgba}


__all__ = ["mse_loss", "mse_grad", "backward_rays"]
