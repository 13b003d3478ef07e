"""The seeded inputs have the shapes the workloads name."""
import numpy as np

import synth


def test_icosphere_counts_and_lattice():
    v, t = synth.icosphere(4, 0.5)
    assert t.shape == (320, 3) and v.shape == (162, 3)
    s = v.astype(np.float64) * 2 ** 16
    assert np.array_equal(s, np.rint(s))
    r = np.linalg.norm(v.astype(np.float64) - 0.5, axis=1)
    assert np.all(np.abs(r - 0.5) < 2e-5)
    # every edge is shared by exactly two triangles (closed surface)
    e = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert np.all(cnt == 2)


def test_displaced_sphere_counts_and_bounds():
    v, t = synth.displaced_sphere(71)
    assert t.shape == (100820, 3) and v.shape == (50412, 3)
    r = np.linalg.norm(v.astype(np.float64) - 0.5, axis=1)
    assert r.min() >= 0.40 - 1e-5 and r.max() <= 0.50 + 1e-5
    assert v.min() >= 0 and v.max() <= 1


def test_level_resolutions():
    assert synth.level_resolutions(16, 2048, 16) == [16, 22, 31, 42, 58, 81, 111, 154, 213, 294, 406,
                                                     562, 776, 1072, 1482, 2048]
    assert synth.level_resolutions(16, 512, 10)[-1] == 512


def test_feature_values_counter_based():
    keys = np.arange(1000, dtype=np.int64) * 7919
    a = synth.feature_values(2, 3, keys)
    b = synth.feature_values(2, 3, keys[::-1])[::-1]
    assert np.array_equal(a, b)                      # independent of the rest of the key set
    big = synth.feature_values(2, 0, np.arange(400000))
    assert abs(big.std() - 0.01) < 2e-4 and abs(big.mean()) < 1e-4
    loud = synth.feature_values(6, 0, np.arange(100000), kind="uniform", sigma=1.0)
    assert loud.min() >= -1 and loud.max() <= 1 and abs(loud.std() - 1 / np.sqrt(3)) < 5e-3


def test_xavier_bounds():
    w = synth.xavier_mlp(3, 24)
    assert [x.shape for x in w] == [(64, 24), (64, 64), (4, 64)]
    assert np.abs(w[0]).max() <= np.sqrt(6 / 88) and np.abs(w[2]).max() <= np.sqrt(6 / 68)


def test_fibonacci_camera_one():
    cams = synth.fibonacci_cameras(8, 2.0, 64, 64)
    d = (cams[1].origin.astype(np.float64) - 0.5) / 2.0
    assert np.allclose(d, [-0.5756, 0.5273, 0.625], atol=2e-4)
    for c in cams:
        B = np.stack([c.right, c.up, c.forward]).astype(np.float64)
        assert np.allclose(B @ B.T, np.eye(3), atol=1e-6)
