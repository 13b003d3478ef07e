"""GPU parity at the benchmark's full size: the 100,820-triangle displaced
sphere with 16 PSH levels (16..2048) rendered at 3840x2160 in the launch
configuration the benchmark times, checked on sampled pixels that the FP64
oracle computes one by one (its feature lookups are generated per queried
vertex; occupancy of the queried vertices is checked locally)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import make_renderer, psnr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EPS_CAMERA = 1e-4   # barycentric margin: FP32 camera rays vs FP64 rays


@pytest.fixture(scope="module")
def obj():
    w = synth.workload_object(3840, 2160)
    return w, make_renderer(w, tables=("f32", "f16"))


@pytest.fixture(scope="module")
def oracle_model(obj):
    return oracle.Model.from_workload(obj[0], materialize=False, check_keys=False)


def _sample(cam, tri, n_hit, n_any, seed):
    rng = np.random.default_rng(seed)
    hits = np.nonzero(tri >= 0)[0]
    idx = np.concatenate([rng.choice(hits, n_hit, replace=False), rng.integers(0, len(tri), n_any)])
    return idx // cam.width, idx % cam.width, idx


@pytest.mark.parametrize("cam_id", [0, 5])
def test_object_4k_sampled_parity(obj, oracle_model, cam_id):
    w, R = obj
    cam = w.cameras[cam_id]
    n = cam.width * cam.height
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    depth = torch.empty(n, device="cuda")
    rgba32 = R.render(cam, "fp32", "f32", tri=tri, depth=depth).reshape(-1, 4).cpu().numpy()
    rgba16 = R.render(cam, "fp16", "f16").reshape(-1, 4).cpu().numpy()
    tri = tri.cpu().numpy()
    hit_frac = (tri >= 0).mean()
    assert 0.12 < hit_frac < 0.25, hit_frac
    rows, cols, idx = _sample(cam, tri, 240, 60, cam_id)
    ora = oracle.render_camera(oracle_model, cam, rows, cols, eps_bary=EPS_CAMERA)
    clear = ~ora["ambiguous"]
    assert np.array_equal(tri[idx][clear], ora["tri"][clear])
    agree = (tri[idx] >= 0) == (ora["tri"] >= 0)
    e32 = np.abs(rgba32[idx][agree] - ora["rgba"][agree]).max()
    e16 = np.abs(rgba16[idx][agree] - ora["rgba"][agree]).max()
    hit = agree & (ora["tri"] >= 0)
    p16 = psnr(rgba16[idx][hit], ora["rgba"][hit])
    print(f"camera {cam_id}: hit fraction {hit_frac:.4f}, fp32 max abs {e32:.2e}, fp16 max abs {e16:.2e}, "
          f"fp16 PSNR {p16:.1f} dB, ambiguous {int(ora['ambiguous'].sum())}")
    assert e32 <= 1e-5
    assert e16 <= 2e-3 and p16 >= 50.0
    d = depth.cpu().numpy()[idx]
    assert np.allclose(d[hit & clear], ora["t"][hit & clear], rtol=1e-5)


def test_object_corner_keys_exist(obj):
    """Every corner the GPU path reads at every level is an occupied vertex
    (decided locally by exact overlap tests, not from the library's keys)."""
    w, R = obj
    cam = w.cameras[2]
    n = cam.width * cam.height
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    R.render(cam, "fp32", "f32", tri=tri)
    tri = tri.cpu().numpy()
    rows, cols, idx = _sample(cam, tri, 6, 0, 3)
    m = oracle.Model.from_workload(w, materialize=False, check_keys=True)
    out = oracle.render_camera(m, cam, rows, cols, eps_bary=EPS_CAMERA)   # raises KeyError if a corner is missing
    assert np.all(out["tri"] >= 0)


def test_object_render_deterministic(obj):
    w, R = obj
    a = R.render(w.cameras[1], "fp16", "f16").clone()
    b = R.render(w.cameras[1], "fp16", "f16").clone()
    assert torch.equal(a, b)
