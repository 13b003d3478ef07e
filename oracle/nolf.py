"""The paper's own i-NOLF rendering, FP64 (test infrastructure only).

Only tests/, the smoke check and the bench's CPU baseline use this module;
it shares no code with the HIP path.

Sec. 4.2 gives the complete i-NOLF: the hit point comes from a march
through cached density texture cubes (not from a proxy mesh), the sample
with the largest blending weight is the hit point, the weights summed along
the ray give a coarse opacity alpha_c that is a further input of the
specular network F_s (which returns the specular colour c_s and the opacity
alpha), and a view-independent diffuse colour c_d with a specular tint t,
read from cached diffuse texture cubes, combine with it as
c = c_d + t * c_s (Eq. 6-7).

Texture cubes (Sec. 4.2, density and diffuse texture cubes): a base grid of
b^3 cells indexes a table of small dense cubes; cell (cx, cy, cz) holds cube
index[(cz*b + cy)*b + cx] or -1 (empty: value 0).  Cube k stores the values
at the (r+1)^3 vertices of an r^3 grid over its cell, vertex (i, j, k') at
((k'*(r+1) + j)*(r+1) + i), so that a lookup never leaves its cube.  The
value at x in [0,1]^3 is the trilinear blend
    g = b*x, c = min(floor(g), b-1), u = (g - c)*r, p = min(floor(u), r-1),
    w = u - p,  f(x) = sum_corners prod_i (w_i or 1-w_i) * V[k][p + corner].

March (Eq. 4 with the argmax reading):
  * the ray (o, unit d) is clipped to the unit cube: [t_in, t_out],
    t_in = max(entry, 0); no interval means a miss;
  * samples t_j = t_in + (j + 1/2) * step for j = 0, 1, ... while t_j < t_out;
  * sigma_j = density(x_j), x_j = o + t_j d clamped to [0,1]^3;
    alpha_j = 1 - exp(-sigma_j * step), w_j = T_j * alpha_j,
    T_{j+1} = T_j * exp(-sigma_j * step), T_0 = 1;
  * the march ends after the first sample whose updated T is below t_stop
    (the transmittance cut-off of instant-NGP marching, 1e-4);
  * hit: the sample with the largest w_j (the lowest j on ties), provided
    that weight is at least w_min = 1e-4; otherwise the ray misses (RGBA 0,
    depth +inf): a ray that only grazes the density's fringe has no
    surface; alpha_c = sum_j w_j.
Shading of a hit at x_h = x_{j*} with unit direction d:
    in = [E_0(x_h) .. E_{L-1}(x_h), SH16(d), alpha_c]
    (c_s, alpha) = sigmoid(MLP(in)),  (c_d, t) = diffuse(x_h)
    RGBA = (c_d + t * c_s, alpha).

A ray is flagged ambiguous (either answer is right within rounding) when its
two largest weights are within a relative 1e-3, when any updated T is
within a relative 1e-3 of t_stop (the march may end one sample earlier or
later), when its largest weight is within a relative 1e-2 of w_min (hit or
miss is then decided by rounding), or when the end of the sample range lies
within 1e-4 of a step of t_out.

Pins (tests): lookups reproduce trilinear (affine) vertex data exactly and
read 0 in empty cells; a constant-density slab gives the closed-form
weights, hit sample and alpha_c; with t = 0 the colour is c_d, and zero
network weights give c_s = alpha = 1/2; a brute-force per-sample loop over
tiny inputs equals the vectorised march.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .encode import trilinear_encode
from .mlp import mlp_forward
from .sh import sh_real

T_STOP = 1e-4
W_MIN = 1e-4


@dataclass
class Cubes:
    b: int
    r: int
    index: np.ndarray      # int [b^3]
    values: np.ndarray     # float [n_cubes, (r+1)^3, C]


def cube_lookup(cubes: Cubes, x) -> np.ndarray:
    """Trilinear value of the cube field at points x [n, 3] -> [n, C]."""
    b, r = cubes.b, cubes.r
    x = np.clip(np.asarray(x, np.float64).reshape(-1, 3), 0.0, 1.0)
    g = x * b
    c = np.minimum(np.floor(g), b - 1).astype(np.int64)
    u = (g - c) * r
    p = np.minimum(np.floor(u), r - 1).astype(np.int64)
    w = u - p
    k = np.asarray(cubes.index).reshape(-1)[(c[:, 2] * b + c[:, 1]) * b + c[:, 0]]
    C = cubes.values.shape[2]
    out = np.zeros((len(x), C))
    occ = k >= 0
    kk = k[occ]
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                wt = ((w[occ, 0] if dx else 1.0 - w[occ, 0]) * (w[occ, 1] if dy else 1.0 - w[occ, 1])
                      * (w[occ, 2] if dz else 1.0 - w[occ, 2]))
                v = ((p[occ, 2] + dz) * (r + 1) + (p[occ, 1] + dy)) * (r + 1) + (p[occ, 0] + dx)
                out[occ] += wt[:, None] * cubes.values[kk, v].astype(np.float64)
    return out


def unit_cube_interval(o, d):
    """[t_in, t_out] of rays (o, d) inside [0,1]^3 (t_in clipped at 0); empty
    intervals have t_in >= t_out."""
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (0.0 - o) / d
        t1 = (1.0 - o) / d
    lo = np.where(d == 0.0, np.where((o >= 0.0) & (o <= 1.0), -np.inf, np.inf), np.minimum(t0, t1))
    hi = np.where(d == 0.0, np.where((o >= 0.0) & (o <= 1.0), np.inf, -np.inf), np.maximum(t0, t1))
    return np.maximum(lo.max(axis=1), 0.0), hi.min(axis=1)


def march(density: Cubes, o, d, step: float, t_stop: float = T_STOP) -> dict:
    """The density march of every ray: hit sample, its t, alpha_c and the
    ambiguity flag (module docstring)."""
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    n = len(o)
    t_in, t_out = unit_cube_interval(o, d)
    span = np.where(t_out > t_in, (t_out - t_in) / step - 0.5, -1.0)
    n_samp = np.where(span >= 0.0, np.floor(span).astype(np.int64) + 1, 0)   # j with (j + 1/2) step < t_out - t_in
    n_samp = np.where((span >= 0.0) & (span == np.floor(span)), n_samp - 1, n_samp)
    amb = (span >= 0.0) & (np.abs(span - np.round(span)) < 1e-4)
    T = np.ones(n)
    alive = n_samp > 0
    best_w = np.zeros(n)
    second_w = np.zeros(n)
    best_t = np.full(n, np.inf)
    ac = np.zeros(n)
    near_stop = np.zeros(n, bool)   # some updated T within a relative 1e-3 of t_stop
    j = 0
    while alive.any():
        idx = np.nonzero(alive)[0]
        t = t_in[idx] + (j + 0.5) * step
        x = o[idx] + t[:, None] * d[idx]
        sigma = cube_lookup(density, x)[:, 0]
        a = -np.expm1(-sigma * step)
        w = T[idx] * a
        better = w > best_w[idx]
        second_w[idx] = np.where(better, best_w[idx], np.maximum(second_w[idx], w))
        best_w[idx] = np.where(better, w, best_w[idx])
        best_t[idx] = np.where(better, t, best_t[idx])
        ac[idx] += w
        T[idx] = T[idx] * np.exp(-sigma * step)
        near_stop[idx] |= np.abs(T[idx] / t_stop - 1.0) < 1e-3
        done = T[idx] < t_stop
        alive[idx[done]] = False
        j += 1
        alive &= j < n_samp
    hit = best_w >= W_MIN
    amb |= hit & (second_w >= (1.0 - 1e-3) * best_w)
    amb |= near_stop
    amb |= np.abs(best_w / W_MIN - 1.0) < 1e-2
    return {"hit": hit, "t": np.where(hit, best_t, np.inf), "alpha_c": ac, "ambiguous": amb,
            "n_samples": n_samp}


def march_loop(density: Cubes, o, d, step: float, t_stop: float = T_STOP):
    """One ray, plain per-sample loop (the brute-force form the pins compare
    the vectorised march with).  Returns (hit, t, alpha_c)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    t_in, t_out = (v[0] for v in unit_cube_interval(o[None], d[None]))
    T, best, bt, ac, j = 1.0, 0.0, np.inf, 0.0, 0
    while t_in < t_out:
        t = t_in + (j + 0.5) * step
        if not t < t_out:
            break
        s = cube_lookup(density, (o + t * d)[None])[0, 0]
        w = T * (1.0 - np.exp(-s * step))
        if w > best:
            best, bt = w, t
        ac += w
        T *= np.exp(-s * step)
        if T < t_stop:
            break
        j += 1
    return best >= W_MIN, (bt if best >= W_MIN else np.inf), ac


@dataclass
class NolfModel:
    density: Cubes
    diffuse: Cubes          # values [n_cubes, (r+1)^3, 4]: c_d (RGB), tint
    grids: list             # per-level feature grids (encode.trilinear_encode)
    weights: list           # W1 [64, 2L+17], W2 [64, 64], W3 [4, 64]
    step: float
    t_stop: float = T_STOP


def model_from_workload(w, kind: str = "normal", sigma: float = 1e-2) -> NolfModel:
    """The oracle's model of a synthetic i-NOLF workload: the cubes as given,
    each level's features generated for the queried vertices, which are
    checked to be keys."""
    import synth
    from .encode import FunctionGrid
    grids = []
    for l, N in enumerate(w.res):
        fn = (lambda v, l=l, N=N: synth.table_features(w.feature_seed, l, v, N, F=w.F, kind=kind, sigma=sigma))
        grids.append(FunctionGrid(N, w.F, fn, lambda v, l=l: w.is_key(l, v)))
    return NolfModel(Cubes(w.b, w.r, w.index, w.density), Cubes(w.b, w.r, w.index, w.diffuse), grids,
                     [np.asarray(x) for x in w.weights], w.step)


def shade(m: NolfModel, x, d, alpha_c) -> np.ndarray:
    """RGBA of hits at x with directions d and coarse opacities alpha_c."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    enc = [trilinear_encode(x, g) for g in m.grids]
    inp = np.concatenate(enc + [sh_real(d, 4), np.asarray(alpha_c, np.float64).reshape(-1, 1)], axis=1)
    out = mlp_forward(inp, m.weights)                     # sigmoid outputs: c_s (RGB), alpha
    diff = cube_lookup(m.diffuse, x)                      # c_d (RGB), tint
    rgba = np.empty((len(x), 4))
    rgba[:, :3] = diff[:, :3] + diff[:, 3:4] * out[:, :3]
    rgba[:, 3] = out[:, 3]
    return rgba


def render_nolf_rays(m: NolfModel, o, d) -> dict:
    o = np.asarray(o, np.float64).reshape(-1, 3)
    d = np.asarray(d, np.float64).reshape(-1, 3)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    h = march(m.density, o, d, m.step, m.t_stop)
    rgba = np.zeros((len(o), 4))
    idx = np.nonzero(h["hit"])[0]
    if len(idx):
        x = np.clip(o[idx] + h["t"][idx, None] * d[idx], 0.0, 1.0)
        rgba[idx] = shade(m, x, d[idx], h["alpha_c"][idx])
    return {"rgba": rgba, **h}


__all__ = ["Cubes", "NolfModel", "T_STOP", "W_MIN", "cube_lookup", "unit_cube_interval", "march", "march_loop",
           "model_from_workload", "shade", "render_nolf_rays"]
