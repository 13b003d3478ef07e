"""Pins of the oracle's ray generation and brute-force closest hit."""
import math

import numpy as np
import pytest

import oracle
import synth


def _cam(W, H, eye=(0.5, -1.5, 0.5), fov=40.0):
    return synth.look_at_camera(eye, (0.5, 0.5, 0.5), fov, W, H)


def test_centre_pixel_looks_forward():
    c = _cam(5, 3)
    o, d = oracle.camera_rays(c, [1], [2])
    f = c.forward.astype(np.float64)
    assert np.allclose(d[0], f / np.linalg.norm(f), atol=1e-15)
    assert np.allclose(o[0], c.origin.astype(np.float64))


def test_field_of_view_and_aspect():
    c = _cam(8, 4, fov=40.0)
    f = c.forward.astype(np.float64) / np.linalg.norm(c.forward.astype(np.float64))
    # top edge of the image, horizontally centred: half the vertical FOV, above the axis
    _, d = oracle.camera_rays(c, [-0.5], [3.5])
    assert abs(math.degrees(math.acos(d[0] @ f)) - 20.0) < 1e-5
    assert d[0] @ c.up.astype(np.float64) > 0
    # left edge, vertically centred: atan(tan(20 deg) * W / H), to the left
    _, d = oracle.camera_rays(c, [1.5], [-0.5])
    want = math.degrees(math.atan(math.tan(math.radians(20.0)) * 2.0))
    assert abs(math.degrees(math.acos(d[0] @ f)) - want) < 1e-5
    assert d[0] @ c.right.astype(np.float64) < 0


def test_row_major_and_mirror_symmetry():
    c = _cam(6, 4)
    o, d = oracle.camera_rays(c)
    assert d.shape == (24, 3)
    r, u = c.right.astype(np.float64), c.up.astype(np.float64)
    D = d.reshape(4, 6, 3)
    assert np.allclose(D @ r, -(D[::-1, ::-1] @ r), atol=1e-12)
    assert np.allclose(D @ u, -(D[::-1, ::-1] @ u), atol=1e-12)
    assert np.all(np.diff(D[:, 0] @ u) < 0)      # rows run top to bottom
    assert np.all(np.diff(D[0, :] @ r) > 0)      # columns run left to right


def test_centroid_rays_hit_own_triangle_at_plane_distance(tiny):
    V = tiny.verts.astype(np.float64)
    T = tiny.tris
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n *= np.sign(np.sum(n * ((a + b + c) / 3 - 0.5), axis=1))[:, None]   # outward
    cen = (a + b + c) / 3
    o = cen + 0.3 * n
    h = oracle.closest_hit(o, -n, V, T)
    assert np.array_equal(h.tri, np.arange(len(T)))
    assert np.allclose(h.t, 0.3, atol=1e-12)
    assert np.allclose(h.cos, 1.0, atol=1e-12)        # along the normal
    # oblique: t = n.(a - o) / n.d
    rng = np.random.default_rng(0)
    o = cen + 0.02 * n
    d = -n + 0.3 * rng.normal(size=n.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    h = oracle.closest_hit(o, d, V, T)
    ok = h.tri == np.arange(len(T))
    t_plane = np.sum(n * (a - o), axis=1) / np.sum(n * d, axis=1)
    assert np.allclose(h.t[ok], t_plane[ok], rtol=1e-12)
    assert ok.mean() > 0.7
    # incidence cosine: |n.d| of the unit normal and unit direction (a scaled direction gives the same)
    assert np.allclose(h.cos[ok], np.abs(np.sum(n * d, axis=1))[ok], atol=1e-12)
    h3 = oracle.closest_hit(o, 3.0 * d, V, T)
    assert np.allclose(h3.cos[ok], h.cos[ok], atol=1e-12)
    miss = oracle.closest_hit(o, n, V, T)             # pointing away from its own triangle, out of the sphere
    assert np.all(np.isnan(miss.cos[miss.tri < 0]))


def test_nearest_wins_two_sided_and_ties_lowest_index():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0],
                  [0, 0, 1], [1, 0, 1], [0, 1, 1]], np.float64)
    T = np.array([[3, 4, 5], [0, 1, 2], [0, 2, 1]], np.int32)   # tri 2 duplicates tri 1 reversed
    o = np.array([[0.2, 0.2, 2.0], [0.2, 0.2, -1.0], [0.2, 0.2, 0.5], [2.0, 2.0, 2.0],
                  [np.nan, 0, 0]])
    d = np.array([[0, 0, -1], [0, 0, 1], [0, 0, -1], [0, 0, -1], [0, 0, 1]], np.float64)
    h = oracle.closest_hit(o, d, V, T)
    assert h.tri.tolist() == [0, 1, 1, -1, -1]
    assert np.allclose(h.t[:3], [1.0, 1.0, 0.5])
    assert np.isinf(h.t[3]) and np.isinf(h.t[4])
    assert h.ambiguous[0] == False and h.ambiguous[1]   # ray 1: tris 1, 2 coincide -> equal t


def test_edge_ray_is_ambiguous():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float64)
    T = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    h = oracle.closest_hit([[0.5, 0.5, 1.0], [0.25, 0.25, 1.0]], [[0, 0, -1], [0, 0, -1]], V, T)
    assert h.ambiguous.tolist() == [True, False]
    assert h.tri[1] == 0 and h.tri[0] in (0, 1)


def test_empty_proxy_all_miss():
    h = oracle.closest_hit(np.zeros((4, 3)), np.ones((4, 3)), np.zeros((0, 3)), np.zeros((0, 3), np.int32))
    assert np.all(h.tri == -1) and np.all(np.isinf(h.t))
