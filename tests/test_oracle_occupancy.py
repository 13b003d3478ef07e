"""Pins of the oracle's occupancy (surface cells, dilation, corner keys)."""
from fractions import Fraction as Fr
import itertools

import numpy as np
import pytest

import oracle
from oracle.occupancy import is_key
from oracle.encode import corner_vertices
import synth


def _clip_overlap(tri, lo, hi):
    """Independent exact test: clip the triangle polygon against the six
    half-spaces of the closed box with rational arithmetic; overlap iff
    something is left."""
    poly = [tuple(Fr(c) for c in p) for p in tri]
    for ax in range(3):
        for bound, keep_ge in ((lo[ax], True), (hi[ax], False)):
            inside = (lambda p: p[ax] >= bound) if keep_ge else (lambda p: p[ax] <= bound)
            out = []
            for i in range(len(poly)):
                S, E = poly[i - 1], poly[i]
                if inside(E):
                    if not inside(S):
                        t = (bound - S[ax]) / (E[ax] - S[ax])
                        out.append(tuple(S[k] + t * (E[k] - S[k]) for k in range(3)))
                    out.append(E)
                elif inside(S):
                    t = (bound - S[ax]) / (E[ax] - S[ax])
                    out.append(tuple(S[k] + t * (E[k] - S[k]) for k in range(3)))
            poly = out
            if not poly:
                return False
    return True


def _brute_surface(verts, tris, N):
    V = [[Fr(float(c)) for c in v] for v in verts]
    cells = set()
    for t in tris:
        tri = [V[i] for i in t]
        for p in itertools.product(range(N), repeat=3):
            if _clip_overlap(tri, [Fr(c, N) for c in p], [Fr(c + 1, N) for c in p]):
                cells.add((p[2] * N + p[1]) * N + p[0])
    return np.array(sorted(cells), np.int64)


def _q(a):
    return synth.quantize_vertices(np.asarray(a, np.float64))


@pytest.mark.parametrize("N", [2, 3, 5])
def test_surface_cells_match_rational_clipping(N):
    rng = np.random.default_rng(N)
    verts = [_q(rng.uniform(0, 1, size=(3, 3))) for _ in range(6)]
    # special cases: a triangle lying in a cell face plane, one with a vertex
    # on a cell corner, a sliver along a cell edge, a tiny one inside a cell
    verts.append(_q([[0.1, 0.2, 0.5], [0.9, 0.3, 0.5], [0.4, 0.8, 0.5]]))
    verts.append(_q([[1 / 2, 1 / 2, 1 / 2], [0.9, 0.7, 0.2], [0.6, 0.1, 0.8]]))
    verts.append(_q([[0.0, 0.5, 0.5], [1.0, 0.5, 0.5], [0.5, 0.5 + 2 ** -16, 0.5]]))
    verts.append(_q([[0.41, 0.41, 0.41], [0.42, 0.41, 0.41], [0.41, 0.42, 0.415]]))
    V = np.concatenate(verts)
    T = np.arange(len(V), dtype=np.int32).reshape(-1, 3)
    for t in T:
        got = oracle.surface_cells(V, t[None], N)
        want = _brute_surface(V, t[None], N)
        assert np.array_equal(got, want), (N, V[t])


def test_keys_local_rule_matches_global_construction():
    V = _q([[0.13, 0.2, 0.31], [0.77, 0.35, 0.52], [0.42, 0.81, 0.66],
            [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    T = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    for N in (4, 7):
        keys = oracle.shell_keys(V, T, N, 1)
        allv = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
        local = allv[is_key(V, T, N, allv, 1)]
        order = np.lexsort((local[:, 0], local[:, 1], local[:, 2]))
        assert np.array_equal(keys, local[order])


def test_keys_canonical_order_and_range(tiny, tiny_keys):
    for N, k in zip(tiny.res, tiny_keys):
        lin = (k[:, 2] * (N + 1) + k[:, 1]) * (N + 1) + k[:, 0]
        assert np.all(np.diff(lin) > 0)
        assert k.min() >= 0 and k.max() <= N


def test_corners_of_surface_points_are_keys(tiny, tiny_keys):
    x = synth.surface_points(tiny.verts, tiny.tris, 3000, 11)
    for N, k in zip(tiny.res, tiny_keys):
        ks = set(map(tuple, k.tolist()))
        cv = corner_vertices(x, N).reshape(-1, 3)
        assert all(tuple(v) in ks for v in cv.tolist())
        # and a half-cell perturbation off the surface still lands in occupied cells
        xp = np.clip(x + np.random.default_rng(N).uniform(-0.5, 0.5, x.shape) / N, 0, 1).astype(np.float32)
        cv = corner_vertices(xp, N).reshape(-1, 3)
        assert all(tuple(v) in ks for v in cv.tolist())


def test_key_count_follows_sphere_area(tiny, tiny_keys):
    # dilated shell of a sphere: about 6 * area * N^2 corner keys as N grows
    # (a shell of thickness ~6 cells around the surface; curvature and the
    # clipping at the cube faces lower the count at coarse levels)
    ratios = [len(k) / (6.0 * np.pi * N * N) for N, k in zip(tiny.res, tiny_keys)]
    assert all(0.8 < r < 1.05 for r in ratios), ratios
    assert ratios == sorted(ratios) and ratios[-1] > 0.95


def test_empty_mesh_has_no_keys():
    k = oracle.shell_keys(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), 8)
    assert k.shape == (0, 3)
