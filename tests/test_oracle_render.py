"""Pins of the oracle's whole per-ray path."""
import numpy as np

import oracle
import synth
from oracle.encode import FeatureGrid


def test_empty_proxy_gives_zero_alpha(tiny):
    m = oracle.Model(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), [], tiny.weights)
    out = oracle.render_camera(m, tiny.cameras[0])
    assert np.all(out["rgba"] == 0) and np.all(out["tri"] == -1)


def test_single_level_constant_features_reduce_to_direction_only(tiny):
    N = 8
    v = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    g = FeatureGrid(N, v, np.tile([[0.3, -0.2]], (len(v), 1)))
    w = synth.xavier_mlp(3, 2 + 16)
    m = oracle.Model(tiny.verts, tiny.tris, [g], w)
    out = oracle.render_camera(m, tiny.cameras[0])
    hit = out["tri"] >= 0
    _, d = oracle.camera_rays(tiny.cameras[0])
    inp = np.concatenate([np.tile([[0.3, -0.2]], (hit.sum(), 1)), oracle.sh_real(d[hit])], 1)
    assert np.allclose(out["rgba"][hit], oracle.mlp_forward(inp, w), atol=1e-15)
    assert np.all(out["rgba"][~hit] == 0)


def test_hits_lie_on_the_sphere_and_in_the_right_image_region(tiny, tiny_oracle):
    cam = tiny.cameras[0]
    out = oracle.render_camera(tiny_oracle, cam)
    hit = out["tri"] >= 0
    r = np.linalg.norm(out["x"][hit] - 0.5, axis=1)
    assert np.all((r > 0.5 * np.cos(np.pi / 5) - 1e-9) & (r <= 0.5 + 1e-9))  # inside circumsphere, outside insphere-ish
    img = hit.reshape(cam.height, cam.width)
    # the sphere is centred in the view: the hit mask is symmetric about the image centre
    assert abs(img[:32].sum() - img[32:].sum()) <= 0.05 * img.sum()
    assert abs(img[:, :32].sum() - img[:, 32:].sum()) <= 0.05 * img.sum()
    # radius 0.5 at distance 2, fov 40: disc radius = tan(asin(0.25)) / tan(20 deg) * 32 px
    rad = np.tan(np.arcsin(0.25)) / np.tan(np.radians(20)) * 32
    assert abs(img.sum() - np.pi * rad ** 2) < 0.06 * np.pi * rad ** 2
    assert out["ambiguous"].mean() < 0.01


def test_feature_dependence_through_levels(tiny):
    # a feature change at the corner vertices of a hit point changes that ray's colour only
    m = oracle.Model.from_workload(tiny)
    cam = tiny.cameras[0]
    out = oracle.render_camera(m, cam)
    k = int(np.nonzero(out["tri"] >= 0)[0][100])
    p, _ = oracle.grid_cell(out["x"][k:k + 1], m.grids[3].res)
    g = m.grids[3]
    for c in range(8):
        v = tuple(int(a) for a in (p[0] + [(c & 1), (c >> 1) & 1, (c >> 2) & 1]))
        g.table[v] = g.table[v] + 0.5
    out2 = oracle.render_camera(m, cam)
    changed = np.nonzero(np.any(out2["rgba"] != out["rgba"], axis=1))[0]
    assert k in changed.tolist()
