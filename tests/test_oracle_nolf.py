"""Pins of the i-NOLF oracle (density-cube march, argmax hit, coarse
opacity, diffuse + tint composition; Sec. 4.2, Eq. 4-7) against closed
forms, brute force and special cases."""
import math

import numpy as np
import pytest

import synth
from oracle.nolf import (Cubes, NolfModel, T_STOP, cube_lookup, march, march_loop, model_from_workload,
                         render_nolf_rays, shade, unit_cube_interval)


def _dense_cubes(b, r, fn, occupied=None, C=1):
    """Cubes over every (or the given) base cell with vertex values fn(p) for
    the vertex position p in [0,1]^3."""
    cells = [(z, y, x) for z in range(b) for y in range(b) for x in range(b)]
    if occupied is not None:
        cells = [c for c in cells if occupied(c)]
    index = np.full(b ** 3, -1, np.int64)
    vals = np.zeros((len(cells), (r + 1) ** 3, C))
    loc = np.arange(r + 1)
    for k, (z, y, x) in enumerate(cells):
        index[(z * b + y) * b + x] = k
        Z, Y, X = np.meshgrid(loc, loc, loc, indexing="ij")
        p = np.stack([(x * r + X.ravel()) / (b * r), (y * r + Y.ravel()) / (b * r), (z * r + Z.ravel()) / (b * r)], 1)
        vals[k] = fn(p).reshape(len(p), C)
    return Cubes(b, r, index, vals)


def test_lookup_reproduces_affine_and_reads_zero_when_empty():
    a = np.array([0.3, -1.2, 2.5])
    cubes = _dense_cubes(4, 4, lambda p: p @ a + 0.7, occupied=lambda c: (c[0] + c[1] + c[2]) % 2 == 0)
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (4000, 3))
    x[:10] = [[0, 0, 0], [1, 1, 1], [0.5, 0.25, 0.75], [1, 0, 0], [0, 1, 1], [0.25, 0.5, 0.5], [0.999, 0.5, 0.5],
              [0.75, 0.75, 0.0], [0.125, 0.375, 0.625], [1.0, 1.0, 0.0]]
    got = cube_lookup(cubes, x)[:, 0]
    c = np.minimum(np.floor(x * 4), 3).astype(int)
    occ = (c.sum(axis=1) % 2) == 0
    assert np.allclose(got[occ], x[occ] @ a + 0.7, rtol=0, atol=1e-12)
    assert np.all(got[~occ] == 0.0)


def test_lookup_is_exact_at_vertices():
    rng = np.random.default_rng(1)
    b, r = 2, 4
    table = {}
    def fn(p):
        out = []
        for q in np.round(p * b * r).astype(int):
            out.append(table.setdefault(tuple(q), rng.normal()))
        return np.array(out)
    cubes = _dense_cubes(b, r, fn)
    keys = list(table)
    x = np.array(keys, np.float64) / (b * r)
    assert np.array_equal(cube_lookup(cubes, x)[:, 0], np.array([table[k] for k in keys]))


def test_unit_cube_interval_closed_form():
    o = np.array([[-1.0, 0.5, 0.5], [0.5, 0.5, 0.5], [2.0, 2.0, 2.0], [-1.0, 0.5, 2.0]])
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    t0, t1 = unit_cube_interval(o, d)
    assert t0[0] == 1.0 and t1[0] == 2.0
    assert t0[1] == 0.0 and t1[1] == 0.5
    assert t0[2] >= t1[2] and t0[3] >= t1[3]


@pytest.mark.parametrize("sigma0", [0.5, 3.0, 2000.0])
def test_constant_density_closed_form(sigma0):
    """Uniform density everywhere: w_j = exp(-s d j) (1 - exp(-s d)) is
    largest at j = 0; alpha_c = 1 - exp(-s d k) after k samples, where k is
    the sample count or the first k with exp(-s d k) < t_stop."""
    cubes = _dense_cubes(2, 2, lambda p: np.full(len(p), sigma0))
    step = 0.01
    o = np.array([[-0.5, 0.3, 0.6]])
    d = np.array([[1.0, 0.0, 0.0]])
    h = march(cubes, o, d, step)
    n_samp = 100  # (j + 1/2) * 0.01 < 1
    k_stop = math.floor(math.log(1 / T_STOP) / (sigma0 * step)) + 1
    k = min(n_samp, k_stop)
    assert h["hit"][0] and h["t"][0] == pytest.approx(0.5 + 0.005, abs=1e-15)
    assert h["alpha_c"][0] == pytest.approx(1 - math.exp(-sigma0 * step * k), rel=1e-12)
    assert h["n_samples"][0] == n_samp


def test_density_step_hits_first_dense_sample():
    """Density 0 for x < 1/2 and s for x >= 1/2: the hit is the first sample
    past x = 1/2 (it has the largest weight)."""
    sigma0 = 50.0
    cubes = _dense_cubes(4, 2, lambda p: np.full(len(p), sigma0), occupied=lambda c: c[2] >= 2)
    step = 0.013
    o = np.array([[-0.3, 0.41, 0.77]])
    d = np.array([[1.0, 0.0, 0.0]])
    h = march(cubes, o, d, step)
    t_in = 0.3
    j = math.ceil((0.8 - t_in) / step - 0.5)       # first j with t_in + (j + 1/2) step >= 0.8 (x = 1/2)
    assert h["t"][0] == pytest.approx(t_in + (j + 0.5) * step, abs=1e-12)
    # the march then runs until T < t_stop: k dense samples
    k = math.floor(math.log(1 / T_STOP) / (sigma0 * step)) + 1
    assert h["alpha_c"][0] == pytest.approx(1 - math.exp(-sigma0 * step * k), rel=1e-12)


def test_no_or_faint_density_is_a_miss():
    """No density, or a largest weight below w_min = 1e-4: a miss."""
    cubes = _dense_cubes(2, 2, lambda p: np.zeros(len(p)))
    h = march(cubes, np.array([[-1.0, 0.5, 0.5]]), np.array([[1.0, 0.0, 0.0]]), 0.05)
    assert not h["hit"][0] and np.isinf(h["t"][0]) and h["alpha_c"][0] == 0.0
    # density s: first weight 1 - exp(-s step) -- just below and just above 1e-4
    for s, hit in ((0.9e-4 / 0.05, False), (1.1e-4 / 0.05, True)):
        h = march(_dense_cubes(2, 2, lambda p: np.full(len(p), s)), np.array([[-1.0, 0.5, 0.5]]),
                  np.array([[1.0, 0.0, 0.0]]), 0.05)
        assert h["hit"][0] == hit and h["alpha_c"][0] > 0


def test_vectorised_march_equals_per_sample_loop():
    w = synth.nolf_tiny()
    cubes = Cubes(w.b, w.r, w.index, w.density)
    o, d = synth.random_rays(64, 3, spread=0.3)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    h = march(cubes, o, d, w.step)
    for i in range(len(o)):
        hit, t, ac = march_loop(cubes, o[i], d[i], w.step)
        assert hit == h["hit"][i]
        assert (t == h["t"][i]) or (np.isinf(t) and np.isinf(h["t"][i]))
        assert ac == pytest.approx(h["alpha_c"][i], rel=1e-12, abs=1e-15)
    assert h["hit"].sum() > 20


def test_composition_special_cases():
    """Tint 0 gives c = c_d; zero network weights give c_s = alpha = 1/2."""
    w = synth.nolf_tiny()
    m = model_from_workload(w)
    rng = np.random.default_rng(3)
    o, d = synth.random_rays(256, 4, spread=0.3)
    h = render_nolf_rays(m, o, d)
    idx = np.nonzero(h["hit"])[0][:64]
    dn = d / np.linalg.norm(d, axis=1, keepdims=True)
    x = np.clip(o[idx] + h["t"][idx, None] * dn[idx], 0, 1)
    cd = cube_lookup(m.diffuse, x)
    no_tint = NolfModel(m.density, Cubes(w.b, w.r, w.index, np.concatenate([w.diffuse[..., :3], 0 * w.diffuse[..., 3:]], 2)),
                        m.grids, m.weights, m.step)
    assert np.array_equal(shade(no_tint, x, d[idx], h["alpha_c"][idx])[:, :3], cd[:, :3])
    zero = NolfModel(m.density, m.diffuse, m.grids, [np.zeros_like(a) for a in m.weights], m.step)
    out = shade(zero, x, d[idx], h["alpha_c"][idx])
    assert np.allclose(out[:, :3], cd[:, :3] + 0.5 * cd[:, 3:4], rtol=0, atol=1e-15) and np.all(out[:, 3] == 0.5)
    assert rng is not None


def test_tiny_field_is_continuous_and_keys_cover_dense_points():
    """Either side of every interior cell face the density differs only by
    the step times its slope; every point with density > 0 has its eight
    level corners stored at every level (the generator asserts equal
    shared faces and zero faces towards empty cells)."""
    w = synth.nolf_tiny()
    cubes = Cubes(w.b, w.r, w.index, w.density)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (20000, 3))
    x[:, 0] = np.round(x[:, 0] * w.b) / w.b                     # on x faces of base cells
    eps = 1e-9
    lo = cube_lookup(cubes, x - [eps, 0, 0])[:, 0]
    hi = cube_lookup(cubes, x + [eps, 0, 0])[:, 0]
    slope = w.sigma_max / w.shell * 4                              # bound on the blended field's slope
    assert np.all(np.abs(hi - lo) <= slope * 2 * eps + 1e-9)
    pts = rng.uniform(0, 1, (50000, 3))
    dense = cube_lookup(cubes, pts)[:, 0] > 0
    from oracle.encode import corner_vertices
    for l, N in enumerate(w.res):
        v = corner_vertices(pts[dense], N).reshape(-1, 3)
        assert np.all(w.is_key(l, v))
        keys = w.level_keys(l)
        lin = (v[:, 2] * (N + 1) + v[:, 1]) * (N + 1) + v[:, 0]
        assert np.all(np.isin(lin, keys))


def test_tiny_render_statistics():
    w = synth.nolf_tiny()
    m = model_from_workload(w)
    import oracle
    o, d = oracle.camera_rays(w.cameras[0])
    h = render_nolf_rays(m, o, d)
    frac = h["hit"].mean()
    assert 0.1 < frac < 0.6
    assert h["ambiguous"].mean() < 0.02
    rgba = h["rgba"][h["hit"]]
    assert np.all(rgba[:, 3] > 0) and np.all(rgba[:, 3] < 1) and np.all(rgba[:, :3] >= 0)
    assert np.all(h["alpha_c"][h["hit"]] > 0) and np.all(h["alpha_c"] <= 1 + 1e-12)
