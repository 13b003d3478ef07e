"""Pins of the oracle's loss gradient: FP64 central finite differences.

With h = 1e-6 and a loss of order 0.1, the difference quotient carries a
rounding error of about eps * L / h ~ 3e-11, so each comparison allows a
relative error of 1e-5 plus an absolute 1e-10."""
import copy

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def setup(tiny):
    m = oracle.Model.from_workload(tiny, kind="uniform", sigma=0.5)   # features that matter
    o, d = synth.random_rays(256, 31, spread=0.25)
    rng = np.random.default_rng(3)
    target = rng.uniform(0, 1, (256, 4))
    return m, o.astype(np.float64), d.astype(np.float64), target


def _loss(m, o, d, target):
    return oracle.mse_loss(oracle.render_rays(m, o, d)["rgba"], target)


def test_weight_gradient_matches_finite_differences(setup):
    m, o, d, target = setup
    rgba = oracle.render_rays(m, o, d)["rgba"]
    g = oracle.backward_rays(m, o, d, oracle.mse_grad(rgba, target))
    assert np.array_equal(g["rgba"], rgba)
    rng = np.random.default_rng(0)
    h = 1e-6
    worst = 0.0
    for layer in range(3):
        W = m.weights[layer]
        for _ in range(8):
            i, j = rng.integers(0, W.shape[0]), rng.integers(0, W.shape[1])
            mp = copy.copy(m)
            mp.weights = [w.astype(np.float64).copy() for w in m.weights]
            mp.weights[layer][i, j] += h
            lp = _loss(mp, o, d, target)
            mp.weights[layer][i, j] -= 2 * h
            lm = _loss(mp, o, d, target)
            fd = (lp - lm) / (2 * h)
            an = g["weights"][layer][i, j]
            worst = max(worst, abs(fd - an) - 1e-5 * abs(an))
    assert worst < 1e-10, worst


def test_feature_gradient_matches_finite_differences(setup):
    m, o, d, target = setup
    rgba = oracle.render_rays(m, o, d)["rgba"]
    g = oracle.backward_rays(m, o, d, oracle.mse_grad(rgba, target))
    h = 1e-6
    worst = 0.0
    for l in (0, 3):
        grid = m.grids[l]
        verts = sorted(g["features"][l], key=lambda v: -np.abs(g["features"][l][v]).max())[:6]
        for v in verts:
            for f in range(grid.F):
                old = grid.table[v].copy()
                grid.table[v] = old + np.eye(grid.F)[f] * h
                lp = _loss(m, o, d, target)
                grid.table[v] = old - np.eye(grid.F)[f] * h
                lm = _loss(m, o, d, target)
                grid.table[v] = old
                fd = (lp - lm) / (2 * h)
                an = g["features"][l][v][f]
                worst = max(worst, abs(fd - an) - 1e-5 * abs(an))
    assert worst < 1e-10, worst


def test_eq8_loss_hand_value():
    """Eq. 8's normalisation fixed by hand: L = (1/N) sum_i (|c_i - c_gt|^2 +
    (alpha_i - alpha_gt)^2), so the squared errors of a ray's four channels
    add and the sum over rays is divided by the number of rays (not by 4N).
    Ray 0: 3 x 0.5^2 + 1^2 = 1.75; ray 1: 1^2 = 1; L = 2.75 / 2 = 1.375.
    dL/dy = 2 (y - y_gt) / N."""
    rgba = np.array([[0.5, 0.5, 0.5, 1.0], [0.0, 0.0, 0.0, 0.0]])
    target = np.array([[0.0, 0.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0]])
    assert oracle.mse_loss(rgba, target) == 1.375
    assert np.array_equal(oracle.mse_grad(rgba, target), np.array([[0.5, 0.5, 0.5, 1.0], [-1.0, 0.0, 0.0, 0.0]]))
    # a perfect prediction costs nothing; one ray's error is shared by N
    assert oracle.mse_loss(target, target) == 0.0
    assert oracle.mse_loss(np.zeros((4, 4)), np.array([[1.0, 0, 0, 0]] + [[0.0] * 4] * 3)) == 0.25


def test_sigmoid_slope_at_zero():
    # zero weights: output 0.5 everywhere, dL/dz3 = dL/dy / 4, no gradient below
    w = synth.workload_tiny()
    m = oracle.Model(w.verts, w.tris, oracle.Model.from_workload(w).grids,
                     [np.zeros((64, 24)), np.zeros((64, 64)), np.zeros((4, 64))])
    o, d = synth.random_rays(16, 5, spread=0.1)
    gy = np.ones((16, 4))
    g = oracle.backward_rays(m, o, d, gy)
    assert np.all(g["weights"][0] == 0) and np.all(g["weights"][1] == 0) and np.all(g["weights"][2] == 0)
    assert all(len(f) == 0 or all(np.all(v == 0) for v in f.values()) for f in g["features"])


def test_adam_first_step_is_normalised_gradient():
    rng = np.random.default_rng(5)
    p, g = rng.normal(size=1000), rng.normal(size=1000)
    g[:10] = 0.0
    lr, eps = 1e-2, 1e-15
    p1, m1, v1 = oracle.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr, 0.9, 0.99, eps)
    assert np.allclose(p1 - p, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    assert np.array_equal(p1[:10], p[:10])
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.01 * g * g)


def test_adam_lazy_skips_zero_gradients():
    """Lazy (sparse) Adam: a zero gradient leaves value and moments as they
    are even with nonzero moments (a dense step would move both), and a
    nonzero gradient from zero moments at t = 1 gives the closed-form step
    lr * g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 0.5, 3.0])
    m = np.array([0.5, 0.0, -0.25, 0.0])
    v = np.array([0.25, 0.0, 0.5, 0.0])
    g = np.array([0.0, 2.0, 0.0, -0.5])
    lr, eps = 1e-2, 1e-15
    p1, m1, v1 = oracle.adam_step(p, g, m, v, 1, lr, 0.9, 0.99, eps, lazy=True)
    assert p1[0] == 1.0 and m1[0] == 0.5 and v1[0] == 0.25
    assert p1[2] == 0.5 and m1[2] == -0.25 and v1[2] == 0.5
    assert np.isclose(p1[1], -2.0 - lr * 2.0 / (2.0 + eps), rtol=1e-14)
    assert np.isclose(p1[3], 3.0 + lr * 0.5 / (0.5 + eps), rtol=1e-14)
    assert np.isclose(m1[1], 0.2) and np.isclose(v1[3], 0.01 * 0.25)
    # the dense step moves the zero-gradient entries: by -lr * m_hat / (sqrt(v_hat) + eps)
    q, _, _ = oracle.adam_step(p, g, m, v, 1, lr, 0.9, 0.99, eps)
    assert np.isclose(q[0], 1.0 - lr * (0.45 / 0.1) / (np.sqrt(0.99 * 0.25 / 0.01) + eps), rtol=1e-12)


def test_adam_constant_gradient_keeps_step():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 30):
        q, m, v = oracle.adam_step(p, g, m, v, t, 0.05, 0.9, 0.99, 1e-12)
        assert np.allclose(q - p, -0.05 * g / (np.abs(g) + 1e-12), rtol=1e-9)
        p = q
