"""Pins of the oracle's grid lookup + trilinear blend, SH basis and network."""
import math

import numpy as np
import pytest

import oracle
from oracle.encode import FeatureGrid, grid_cell, trilinear_encode


def _dense_grid(N, fn):
    v = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    return FeatureGrid(N, v, fn(v.astype(np.float64)))


def test_affine_field_reproduced():
    A = np.array([[1.5, -0.25, 3.0], [0.125, 2.0, -1.0]])
    b = np.array([0.3, -0.7])
    for N in (5, 16):
        g = _dense_grid(N, lambda v: v @ A.T + b)
        x = np.random.default_rng(N).uniform(0, 1, (500, 3)).astype(np.float32)
        got = trilinear_encode(x, g)
        want = (N * x.astype(np.float64)) @ A.T + b
        assert np.allclose(got, want, atol=1e-12)


def test_partition_of_unity_and_vertex_values():
    N = 8
    g = _dense_grid(N, lambda v: np.stack([np.ones(len(v)), np.sin(v[:, 0] + 3 * v[:, 1] - v[:, 2])], 1))
    x = np.random.default_rng(1).uniform(0, 1, (300, 3)).astype(np.float32)
    assert np.allclose(trilinear_encode(x, g)[:, 0], 1.0, atol=1e-14)
    v = np.array([[3, 5, 1], [0, 0, 0], [8, 8, 8], [8, 0, 4]])
    xv = (v / N).astype(np.float32)
    got = trilinear_encode(xv, g)[:, 1]
    assert np.allclose(got, np.sin(v[:, 0] + 3 * v[:, 1] - v[:, 2]), atol=1e-15)


def test_upper_boundary_and_clamp():
    p, w = grid_cell(np.array([[1.0, 0.0, 1.5], [-0.2, 0.5, 1.0]], np.float32), 4)
    assert p.tolist() == [[3, 0, 3], [0, 2, 3]]
    assert w.tolist() == [[1.0, 0.0, 1.0], [0.0, 0.0, 1.0]]


def test_floor_is_exact_product():
    # an FP32 x whose FP32 product with N rounds up to an integer while the
    # exact product lies below it
    N = 1482
    rng = np.random.default_rng(7)
    found = 0
    for x in rng.uniform(0, 1, 400000).astype(np.float32):
        y32 = np.float32(N) * x
        if y32 == np.floor(y32) and float(N) * float(x) < float(y32):
            p, w = grid_cell(np.array([[x, 0, 0]], np.float32), N)
            assert p[0, 0] == int(y32) - 1 and 0.999 < w[0, 0] < 1.0
            found += 1
    assert found > 0


def _sh_closed_forms(v):
    x, y, z = v.T
    pi = math.pi
    c1 = math.sqrt(3 / (4 * pi))
    return np.stack([
        0.5 * math.sqrt(1 / pi) * np.ones_like(x),
        -c1 * y, c1 * z, -c1 * x,
        0.5 * math.sqrt(15 / pi) * x * y,
        -0.5 * math.sqrt(15 / pi) * y * z,
        0.25 * math.sqrt(5 / pi) * (3 * z * z - 1),
        -0.5 * math.sqrt(15 / pi) * x * z,
        0.25 * math.sqrt(15 / pi) * (x * x - y * y),
        -0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y),
        0.5 * math.sqrt(105 / pi) * x * y * z,
        -0.25 * math.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1),
        0.25 * math.sqrt(7 / pi) * (5 * z ** 3 - 3 * z),
        -0.25 * math.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1),
        0.25 * math.sqrt(105 / pi) * z * (x * x - y * y),
        -0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),
    ], 1)


def test_sh_closed_forms():
    v = np.random.default_rng(3).normal(size=(200, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    assert np.allclose(oracle.sh_real(v), _sh_closed_forms(v), atol=1e-13)
    # unnormalised input is normalised first
    assert np.allclose(oracle.sh_real(3.5 * v), _sh_closed_forms(v), atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    zq, wq = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phi = 2 * math.pi * np.arange(nphi) / nphi
    Z, P = np.meshgrid(zq, phi, indexing="ij")
    W = np.outer(wq, np.full(nphi, 2 * math.pi / nphi)).reshape(-1)
    s = np.sqrt(1 - Z ** 2)
    v = np.stack([s * np.cos(P), s * np.sin(P), Z], -1).reshape(-1, 3)
    Y = oracle.sh_real(v)
    G = (Y * W[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_matches_scipy():
    special = pytest.importorskip("scipy.special")
    if not hasattr(special, "sph_harm_y"):
        pytest.skip("scipy without sph_harm_y")
    v = np.random.default_rng(4).normal(size=(100, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    theta = np.arccos(v[:, 2])
    phi = np.arctan2(v[:, 1], v[:, 0])
    Y = oracle.sh_real(v)
    for l in range(4):
        for m in range(-l, l + 1):
            c = special.sph_harm_y(l, abs(m), theta, phi)
            want = c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag)
            assert np.allclose(Y[:, l * l + l + m], want, atol=1e-12), (l, m)


def test_mlp_zero_weights_half():
    w = [np.zeros((64, 24)), np.zeros((64, 64)), np.zeros((4, 64))]
    out = oracle.mlp_forward(np.random.default_rng(0).normal(size=(10, 24)), w)
    assert np.all(out == 0.5)


def test_mlp_hand_worked():
    W1 = np.array([[1.0, -1.0], [2.0, 0.0]])
    W2 = np.array([[1.0, 0.0], [0.0, -1.0]])
    W3 = np.array([[0.5, 7.0]])
    # W1 x = (2, 6); W2 h1 = (2, -6) -> relu (2, 0); W3 h2 = 1
    out = oracle.mlp_forward(np.array([[3.0, 1.0]]), [W1, W2, W3])
    assert abs(out[0, 0] - 0.7310585786300049) < 1e-15
    # a negative first-layer pre-activation is cut: x = (-1, 0) -> W1 x = (-1, -2)
    assert oracle.mlp_forward(np.array([[-1.0, 0.0]]), [W1, W2, W3])[0, 0] == 0.5
