"""GPU parity of multi-object scene rendering (inrf_render_scene) against the
FP64 scene oracle, through the C ABI.

The oracle receives the transforms exactly as the library does (FP32 values);
rays whose hit is within rounding of an edge, a silhouette or another
object's hit (the oracle's `ambiguous` flag, tolerance 1e-4 for camera rays,
whose FP32 generation moves the surface point by ~1e-7) may take either
answer.  Object and triangle ids are compared bit for bit on the others;
FP32 colours to 1e-5, FP16 to 2e-3, with features N(0, 0.01) as in the
single-object tests (the FP32 object-space ray moves x by ~1e-7 of its
distance, which larger features would amplify past 1e-5)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import make_renderer
from oracle.scene import Instance, render_scene_rays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
EPS = dict(eps_bary=1e-4, eps_t=1e-4)


def _placement32(o):
    return (float(np.float32(o.scale)), np.asarray(o.rotation, np.float32).astype(np.float64),
            np.asarray(o.translation, np.float32).astype(np.float64))


@pytest.fixture(scope="module")
def scene():
    import paper_2303_04086_amd as P
    sc = synth.scene_tiny(3)
    rs = [make_renderer(o.workload, tables=("f32", "f16")) for o in sc.objects]
    S = P.Scene(rs, [(o.scale, o.rotation, o.translation) for o in sc.objects])
    insts = []
    for o in sc.objects:
        s, R, t = _placement32(o)
        insts.append(Instance(oracle.Model.from_workload(o.workload), s, R, t))
    return sc, S, rs, insts


def _render(S, cam, precision="fp32", table="f32"):
    n = cam.width * cam.height
    depth = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    obj = torch.empty(n, dtype=torch.int32, device="cuda")
    rgba = S.render(cam, precision, table, depth=depth, tri=tri, obj=obj)
    torch.cuda.synchronize()
    return (rgba.cpu().numpy().reshape(-1, 4), depth.cpu().numpy(), tri.cpu().numpy(), obj.cpu().numpy())


@pytest.mark.parametrize("wh", [(64, 64), (37, 23)])
def test_scene_matches_oracle(scene, wh):
    sc, S, rs, insts = scene
    base = sc.cameras[0]
    cam = synth.look_at_camera(base.origin.astype(np.float64), (1.25, 1.25, 1.25), 40.0, *wh)
    rgba, depth, tri, obj = _render(S, cam)
    o, d = oracle.camera_rays(cam)
    ora = render_scene_rays(insts, o, d, **EPS)
    clear = ~ora["ambiguous"]
    bad = np.nonzero(clear & ((obj != ora["obj"]) | (tri != ora["tri"])))[0]
    assert len(bad) == 0, (bad[:5], obj[bad[:5]], ora["obj"][bad[:5]])
    assert ora["ambiguous"].mean() < 0.02
    per_obj = [int((ora["obj"] == k).sum()) for k in range(len(insts))]
    print(f"scene {wh}: hits per object {per_obj}, ambiguous {int(ora['ambiguous'].sum())}")
    assert all(c > 0 for c in per_obj) or wh != (64, 64)
    agree = obj == ora["obj"]
    hit = agree & (obj >= 0)
    assert np.abs(rgba[agree] - ora["rgba"][agree]).max() <= 1e-5
    assert np.all(np.isinf(depth[obj < 0])) and np.all(tri[obj < 0] == -1) and np.all(rgba[obj < 0] == 0)
    assert np.allclose(depth[hit], ora["t"][hit], rtol=1e-5, atol=0)
    rgba16 = _render(S, cam, "fp16", "f16")[0]
    assert np.abs(rgba16[agree] - ora["rgba"][agree]).max() <= 2e-3


def test_single_identity_object_equals_render(scene):
    import paper_2303_04086_amd as P
    sc, S, rs, insts = scene
    cam = synth.fibonacci_cameras(8, 2.0, 48, 40)[3]
    S1 = P.Scene([rs[0]], [(1.0, np.eye(3), np.zeros(3))])
    rgba, depth, tri, obj = _render(S1, cam)
    n = cam.width * cam.height
    d1 = torch.empty(n, device="cuda")
    t1 = torch.empty(n, dtype=torch.int32, device="cuda")
    ref = rs[0].render(cam, "fp32", "f32", depth=d1, tri=t1)
    torch.cuda.synchronize()
    assert np.array_equal(rgba, ref.cpu().numpy().reshape(-1, 4))
    assert np.array_equal(depth, d1.cpu().numpy()) and np.array_equal(tri, t1.cpu().numpy())
    assert np.array_equal(obj, np.where(tri >= 0, 0, -1))


def test_empty_scene_and_errors(scene):
    import paper_2303_04086_amd as P
    sc, S, rs, insts = scene
    cam = synth.look_at_camera((6.0, 1.0, 1.0), (1.25, 1.25, 1.25), 40.0, 17, 9)
    S0 = P.Scene([], [])
    rgba, depth, tri, obj = _render(S0, cam)
    assert not rgba.any() and np.all(obj == -1) and np.all(tri == -1) and np.all(np.isinf(depth))
    bad = P.Scene([rs[0]], [(1.0, np.diag([1.0, 1.0, 2.0]), np.zeros(3))])   # not a rotation
    with pytest.raises(P.InrfError):
        bad.render(cam)
    mirror = P.Scene([rs[0]], [(1.0, np.diag([1.0, 1.0, -1.0]), np.zeros(3))])  # determinant -1
    with pytest.raises(P.InrfError):
        mirror.render(cam)
    neg = P.Scene([rs[0]], [(-1.0, np.eye(3), np.zeros(3))])
    with pytest.raises(P.InrfError):
        neg.render(cam)
    assert P.lib().inrf_scene_workspace_size(17, 100) == -1


@pytest.fixture(scope="module")
def scene12():
    """The benchmark's scene: 12 displaced spheres (32,000 triangles each, own
    features and networks, 10 levels 16..512), scale 0.2-1.0 in a 4^3 box,
    rendered at 3840x2160."""
    import paper_2303_04086_amd as P
    sc = synth.scene_objects(12, 3840, 2160)
    rs = [make_renderer(o.workload, tables=("f32", "f16")) for o in sc.objects]
    S = P.Scene(rs, [(o.scale, o.rotation, o.translation) for o in sc.objects])
    insts = []
    for o in sc.objects:
        s, R, t = _placement32(o)
        insts.append(Instance(oracle.Model.from_workload(o.workload, materialize=False, check_keys=False), s, R, t))
    return sc, S, insts


def _scene_pixels(sc, cam, n_near, n_any, seed):
    """n_near pixels whose FP64 ray passes through some object's bounding
    ball (centre s R (0.5, 0.5, 0.5) + t, radius s / 2), then n_any uniform
    pixels; chosen from the camera and the placements alone."""
    rng = np.random.default_rng(seed)
    pool = rng.integers(0, cam.width * cam.height, 60 * n_near + 1000)
    o, d = oracle.camera_rays(cam, pool // cam.width, pool % cam.width)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    near = np.zeros(len(pool), bool)
    for ob in sc.objects:
        c = ob.scale * np.asarray(ob.rotation) @ np.full(3, 0.5) + np.asarray(ob.translation)
        v = c - o
        tca = np.sum(v * d, axis=1)
        near |= (np.sum(v * v, axis=1) - tca ** 2 < (0.5 * ob.scale) ** 2) & (tca > 0)
    sel = pool[near][:n_near]
    assert len(sel) == n_near
    return np.concatenate([sel, rng.integers(0, cam.width * cam.height, n_any)])


@pytest.mark.parametrize("cam_id", [0, 5])
def test_scene12_4k_sampled(scene12, cam_id):
    """The 12-object scene at 4K in the launch configuration the benchmark
    times, on 400 sampled pixels: object and triangle ids bit-exact on
    unambiguous rays, FP32 colour to 1e-5, FP16 to 2e-3 with PSNR >= 50 dB
    over hit pixels."""
    from gpu_helpers import psnr
    sc, S, insts = scene12
    cam = sc.cameras[cam_id]
    rgba, depth, tri, obj = _render(S, cam)
    rgba16 = _render(S, cam, "fp16", "f16")[0]
    pix = _scene_pixels(sc, cam, 320, 80, 40 + cam_id)
    o, d = oracle.camera_rays(cam, pix // cam.width, pix % cam.width)
    ora = render_scene_rays(insts, o, d, **EPS)
    clear = ~ora["ambiguous"]
    bad = np.nonzero(clear & ((obj[pix] != ora["obj"]) | (tri[pix] != ora["tri"])))[0]
    assert len(bad) == 0, (pix[bad[:5]], obj[pix][bad[:5]], ora["obj"][bad[:5]])
    agree = obj[pix] == ora["obj"]
    hit = agree & (ora["obj"] >= 0)
    per_obj = np.bincount(ora["obj"][ora["obj"] >= 0], minlength=12)
    e32 = np.abs(rgba[pix][agree] - ora["rgba"][agree]).max()
    e16 = np.abs(rgba16[pix][agree] - ora["rgba"][agree]).max()
    p16 = psnr(rgba16[pix][hit], ora["rgba"][hit])
    print(f"scene12 camera {cam_id}: {int(hit.sum())} sampled hits over {int((per_obj > 0).sum())} objects, "
          f"ambiguous {int(ora['ambiguous'].sum())}, fp32 {e32:.2e}, fp16 {e16:.2e} ({p16:.1f} dB)")
    assert hit.sum() >= 200 and (per_obj > 0).sum() >= 4
    assert ora["ambiguous"].mean() <= 0.01
    assert e32 <= 1e-5
    assert e16 <= 2e-3 and p16 >= 50.0
    assert np.allclose(depth[pix][hit & clear], ora["t"][hit & clear], rtol=1e-5, atol=0)
