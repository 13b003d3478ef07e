"""Shared set-up of the GPU tests: a device model of a synthetic workload and
comparison helpers.  Inputs come from `synth`; expected values from `oracle`."""
import numpy as np

import synth


def feature_fn(w, kind="normal", sigma=1e-2):
    return lambda l, lv: synth.feature_values(w.feature_seed, l, lv.keys, F=w.F, kind=kind, sigma=sigma)


def make_renderer(w, tables=("f32", "f16"), kind="normal", sigma=1e-2):
    import paper_2303_04086_amd as P
    return P.Renderer(w.verts, w.tris, w.res, w.weights, feature_fn(w, kind, sigma), tables=tables,
                      dilate=w.dilate, seed=w.psh_seed)


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


# Largest share of rays the oracle may flag ambiguous (hit, miss or the
# triangle decided within rounding; either answer is then correct).  The
# share is what the margin makes it: about 7 x margin per unit of hit area
# (the band along the three edges of each triangle) plus the silhouette.
# Identical FP32 rays on both sides, margin 2^-16: measured 3.3e-4 of random
# batch rays and 2.4e-4 of the tiny camera frame.  FP32 camera rays against
# FP64 camera rays at 4K, margin 1e-4: measured 1.7e-3 of hit rays.
AMB_IDENTICAL_RAYS = 1e-3
AMB_CAMERA_RAYS = 3e-3

# Grazing hits: an FP32 camera ray fixes its hit point only to about
# t * 2^-23 / |cos| (cos of the incidence angle), which the finest cell
# weights (N = 2048) amplify; at |cos| < 0.01 (within 0.6 degrees of
# grazing, ~1e-4 of a sphere's hit pixels) FP32 colour is reported rather
# than held to 1e-5.
GRAZING_COS = 0.01


def compare_hits(gpu_tri, ora, max_amb_frac=AMB_IDENTICAL_RAYS):
    """Triangle ids bit-exact on rays the oracle calls unambiguous, and no
    more than max_amb_frac of the rays ambiguous; returns the mask of rays
    whose hit/miss agrees."""
    gpu_tri = np.asarray(gpu_tri).reshape(-1)
    amb = ora["ambiguous"]
    clear = ~amb
    bad = np.nonzero(clear & (gpu_tri != ora["tri"]))[0]
    assert len(bad) == 0, f"{len(bad)} unambiguous rays differ, e.g. {bad[:5]} gpu={gpu_tri[bad[:5]]} oracle={ora['tri'][bad[:5]]}"
    assert amb.mean() <= max_amb_frac, amb.mean()
    return (gpu_tri >= 0) == (ora["tri"] >= 0)
