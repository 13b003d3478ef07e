"""Pins of the scene oracle (several objects merged per ray by depth)."""
import numpy as np
import pytest

import oracle
from oracle.scene import Instance, render_scene_rays
import synth


@pytest.fixture(scope="module")
def model(tiny):
    return oracle.Model.from_workload(tiny, kind="uniform", sigma=0.5)


def test_identity_transform_equals_single_object(model):
    o, d = synth.random_rays(400, 3)
    one = render_scene_rays([Instance(model, 1.0, np.eye(3), np.zeros(3))], o, d)
    ref = oracle.render_rays(model, o, d)
    assert np.array_equal(one["rgba"], ref["rgba"])
    assert np.array_equal(one["tri"], ref["tri"]) and np.array_equal(one["t"], ref["t"])
    assert np.all(one["obj"][ref["tri"] >= 0] == 0) and np.all(one["obj"][ref["tri"] < 0] == -1)


def test_axis_permutation_rotates_the_scene(model):
    """A rotation that permutes the axes is exact in floating point: rotating
    the object about the world origin and the rays with it gives the same
    colours (object-space rays are identical)."""
    P = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])  # det +1
    t = np.array([0.25, -0.5, 2.0])
    o, d = synth.random_rays(300, 4)
    base = render_scene_rays([Instance(model, 1.0, np.eye(3), t)], o + t, d)
    rot = render_scene_rays([Instance(model, 1.0, P, P @ t)], (o + t) @ P.T, d @ P.T)
    assert np.array_equal(base["rgba"], rot["rgba"]) and np.array_equal(base["obj"], rot["obj"])


def test_duplicate_object_goes_to_lower_index(model):
    o, d = synth.random_rays(300, 5)
    inst = Instance(model, 0.5, np.eye(3), np.array([1.0, 1.0, 1.0]))
    r = render_scene_rays([inst, inst], o * 0.5 + 1.0, d)
    hit = r["obj"] >= 0
    assert hit.sum() > 100 and np.all(r["obj"][hit] == 0)


def test_vertex_direction_distance(tiny, model):
    """Scale 0.5, translation t: a ray from far away aimed at a proxy vertex
    along the vertex's radial direction stops at that vertex (the vertex is
    the closest point of the convex icosphere along that line)."""
    s, t = 0.5, np.array([3.0, -1.0, 2.0])
    v = np.asarray(tiny.verts, np.float64)
    c = np.array([0.5, 0.5, 0.5])
    k = [0, 5, 17]
    dirs = (v[k] - c) / np.linalg.norm(v[k] - c, axis=1, keepdims=True)
    target = s * v[k] + t                   # world position of the vertices
    o = target + 3.0 * dirs                 # 3 world units outside, looking back
    r = render_scene_rays([Instance(model, s, np.eye(3), t)], o, -dirs)
    assert np.all(r["obj"] == 0)
    assert np.allclose(r["t"], 3.0, rtol=0, atol=1e-12)


def test_front_object_hides_back_object(model):
    back = Instance(model, 1.0, np.eye(3), np.array([0.0, 0.0, 0.0]))
    front = Instance(model, 1.0, np.eye(3), np.array([0.0, 0.0, 2.0]))
    o = np.tile([[0.5, 0.5, 10.0]], (3, 1))
    d = np.tile([[0.0, 0.0, -1.0]], (3, 1))
    r = render_scene_rays([back, front], o, d)
    assert np.all(r["obj"] == 1)
    assert np.allclose(r["t"], 10.0 - 3.0, atol=1e-12)   # top of the front sphere at z = 2 + 1
    r2 = render_scene_rays([back, front], o * [1, 1, -1] + [0, 0, 2.0], -d)
    assert np.all(r2["obj"] == 0)                          # from below, the back one is first
